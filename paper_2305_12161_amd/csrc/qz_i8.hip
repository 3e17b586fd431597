// qz_i8.hip -- kernels for the int8 layout: one signed byte (+1 / -1) per site,
// lattice index i = x + L*(y + L*z).  One launch per colour (the colour-p pass
// reads only colour 1-p, so it updates in place without races), the bond count
// of the state entering a sweep fused into its colour-0 pass.
#include "qz_device.hpp"
#include "qz_internal.hpp"

namespace qz {
namespace {

constexpr int kThreads = 256;

// Sum a per-thread 64-bit value over the block and add it to *acc (one atomic).
__device__ __forceinline__ void block_add_u64(unsigned long long v, unsigned long long *acc)
{
    __shared__ unsigned long long part[kThreads / 64];
    __syncthreads();   // a previous call may still be reading part[]
    v = wave_sum_u64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
        part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int k = 0; k < kThreads / 64; ++k)
            tot += part[k];
        if (tot)
            atomicAdd(acc, tot);
    }
}

__device__ __forceinline__ uint32_t wrap_up(uint32_t v, uint32_t L) { return v + 1 == L ? 0 : v + 1; }
__device__ __forceinline__ uint32_t wrap_dn(uint32_t v, uint32_t L) { return v == 0 ? L - 1 : v - 1; }

// Infinite-temperature start: thread b draws Philox block (b, 0, 0, 1) and
// writes the 128 sites i = 128b .. 128b+127 (+1 where the bit is set).
__global__ void __launch_bounds__(kThreads) k_i8_init(uint64_t N, uint32_t k0, uint32_t k1,
                                                      int8_t *s)
{
    const uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    const uint64_t base = b * 128;
    if (base >= N)
        return;
    const Words4 r = philox10((uint32_t)b, 0u, 0u, 1u, k0, k1);
    uint32_t *out = reinterpret_cast<uint32_t *>(s + base);
#pragma unroll
    for (int q = 0; q < 32; ++q) {          // 4 sites per 32-bit store; N % 8 == 0
        if (base + 4 * q >= N)
            break;
        const uint32_t bits = (r.w[q >> 3] >> ((q & 7) * 4)) & 0xFu;
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            v |= (((bits >> k) & 1u) ? 0x01u : 0xFFu) << (8 * k);
        out[q] = v;
    }
}

// Half-sweep number `which` (0 = first, 1 = second) of sweep t: thread per
// colour index j (consecutive lanes hold consecutive j, so a wave shares one
// Philox block and evaluates it once).  The colour updated is p = which in the
// 01 cycle; in the mixed cycle the first colour is bit 0 of Philox block
// (0, t, 2, 0) (Supplementary Methods I B: order drawn per sweep).
__global__ void __launch_bounds__(kThreads)
    k_i8_half(uint32_t L, uint64_t half_n, uint32_t k0, uint32_t k1, uint32_t t, uint32_t which,
              uint32_t mixed, int8_t *s, unsigned long long *bond_acc,
              unsigned long long *flip_acc)
{
    const uint32_t first = mixed ? (philox10(0u, t, 2u, 0u, k0, k1).w[0] & 1u) : 0u;
    const uint32_t p = which ^ first;
    const uint32_t H = L >> 1;
    unsigned long long acc = 0, flips = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * kThreads + threadIdx.x; j < half_n;
         j += (uint64_t)gridDim.x * kThreads) {
        const uint32_t xh = (uint32_t)(j % H);
        const uint64_t row = j / H;
        const uint32_t y = (uint32_t)(row % L), z = (uint32_t)(row / L);
        const uint32_t x = 2 * xh + ((p + y + z) & 1u);
        const uint64_t LL = (uint64_t)L * L;
        const uint64_t zo = (uint64_t)z * LL, yo = (uint64_t)y * L;
        const uint64_t i = zo + yo + x;
        const int8_t me = s[i];
        uint32_t a = 0;
        a += s[zo + yo + wrap_up(x, L)] != me;
        a += s[zo + yo + wrap_dn(x, L)] != me;
        a += s[zo + (uint64_t)wrap_up(y, L) * L + x] != me;
        a += s[zo + (uint64_t)wrap_dn(y, L) * L + x] != me;
        a += s[(uint64_t)wrap_up(z, L) * LL + yo + x] != me;
        a += s[(uint64_t)wrap_dn(z, L) * LL + yo + x] != me;
        acc += a;
        bool flip = a >= 4;
        if (a == 3) {
            const Words4 r = philox10((uint32_t)(j >> 7), t, p, 0u, k0, k1);
            flip = (r.w[(j >> 5) & 3] >> (j & 31)) & 1u;
        }
        if (flip) {
            s[i] = (int8_t)-me;
            ++flips;
        }
    }
    if (bond_acc != nullptr)
        block_add_u64(acc, bond_acc);
    if (flip_acc != nullptr)
        block_add_u64(flips, flip_acc);
}

// Per-axis unsatisfied bonds: [s_i != s_{i+e_x}], [.. e_y], [.. e_z].
__global__ void __launch_bounds__(kThreads) k_i8_bonds(uint32_t L, uint64_t N, const int8_t *s,
                                                       unsigned long long *acc3)
{
    unsigned long long bx = 0, by = 0, bz = 0;
    const uint64_t LL = (uint64_t)L * L;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * kThreads) {
        const uint32_t x = (uint32_t)(i % L), y = (uint32_t)((i / L) % L);
        const uint64_t z = i / LL;
        const int8_t me = s[i];
        bx += s[i - x + wrap_up(x, L)] != me;
        by += s[z * LL + (uint64_t)wrap_up(y, L) * L + x] != me;
        bz += s[(uint64_t)wrap_up((uint32_t)z, L) * LL + (uint64_t)y * L + x] != me;
    }
    block_add_u64(bx, acc3 + 0);
    block_add_u64(by, acc3 + 1);
    block_add_u64(bz, acc3 + 2);
}

// Correlation sums: blockIdx.y = a*(L/2+1) + r for the pair (axis a, shift r),
// and blockIdx.y = 3*(L/2+1) for the magnetisation.
__global__ void __launch_bounds__(kThreads) k_i8_corr(uint32_t L, uint64_t N, const int8_t *s,
                                                      unsigned long long *S)
{
    const uint32_t R = L / 2 + 1;
    const uint32_t q = blockIdx.y;
    const uint64_t LL = (uint64_t)L * L;
    long long acc = 0;
    if (q == 3 * R) {
        for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < N;
             i += (uint64_t)gridDim.x * kThreads)
            acc += s[i];
    } else {
        const uint32_t a = q / R, r = q % R;
        for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < N;
             i += (uint64_t)gridDim.x * kThreads) {
            uint32_t x = (uint32_t)(i % L), y = (uint32_t)((i / L) % L);
            uint32_t z = (uint32_t)(i / LL);
            if (a == 0) x = (x + r) % L;
            else if (a == 1) y = (y + r) % L;
            else z = (z + r) % L;
            acc += (int)s[i] * (int)s[(uint64_t)z * LL + (uint64_t)y * L + x];
        }
    }
    block_add_u64((unsigned long long)acc, S + q);
}

__global__ void __launch_bounds__(kThreads) k_i8_check(uint64_t n, const int8_t *s,
                                                       unsigned long long *bad)
{
    unsigned long long b = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kThreads)
        b += (s[i] != 1 && s[i] != -1);
    block_add_u64(b, bad);
}

__global__ void __launch_bounds__(kThreads)
    k_i8_window(uint32_t L, const int8_t *s, uint32_t ox, uint32_t oy, uint32_t oz, uint32_t W,
                uint32_t lz0, uint64_t n, int8_t *out)
{
    const uint64_t WW = (uint64_t)W * W;
    for (uint64_t k = (uint64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
         k += (uint64_t)gridDim.x * kThreads) {
        const uint32_t lx = (uint32_t)(k % W), ly = (uint32_t)((k / W) % W);
        const uint32_t lz = lz0 + (uint32_t)(k / WW);
        const uint64_t x = (ox + lx) % L, y = (oy + ly) % L, z = (oz + lz) % L;
        out[k] = s[(z * L + y) * L + x];
    }
}

__global__ void __launch_bounds__(kThreads) k_fill_u64(unsigned long long *p, uint64_t n,
                                                       unsigned long long v)
{
    for (uint64_t k = (uint64_t)blockIdx.x * kThreads + threadIdx.x; k < n;
         k += (uint64_t)gridDim.x * kThreads)
        p[k] = v;
}

uint32_t grid_for(uint64_t work, uint32_t cap)
{
    uint64_t g = (work + kThreads - 1) / kThreads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

}  // namespace

hipError_t i8_init(hipStream_t st, uint32_t L, uint64_t seed, int8_t *s)
{
    const uint64_t N = (uint64_t)L * L * L;
    const uint64_t blocks = (N + 128 - 1) / 128;
    const uint32_t g = (uint32_t)((blocks + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_i8_init, dim3(g), dim3(kThreads), 0, st, N, (uint32_t)seed,
                       (uint32_t)(seed >> 32), s);
    return hipGetLastError();
}

hipError_t i8_half_sweep(hipStream_t st, uint32_t L, uint64_t seed, uint32_t t, int which,
                         bool mixed, int8_t *s, unsigned long long *bond_acc,
                         unsigned long long *flip_acc)
{
    const uint64_t half_n = (uint64_t)L * L * L / 2;
    hipLaunchKernelGGL(k_i8_half, dim3(grid_for(half_n, 8192)), dim3(kThreads), 0, st, L, half_n,
                       (uint32_t)seed, (uint32_t)(seed >> 32), t, (uint32_t)which,
                       mixed ? 1u : 0u, s, bond_acc, flip_acc);
    return hipGetLastError();
}

hipError_t i8_bonds(hipStream_t st, uint32_t L, const int8_t *s, unsigned long long *acc3)
{
    const uint64_t N = (uint64_t)L * L * L;
    hipLaunchKernelGGL(k_i8_bonds, dim3(grid_for(N, 2048)), dim3(kThreads), 0, st, L, N, s, acc3);
    return hipGetLastError();
}

hipError_t i8_corr(hipStream_t st, uint32_t L, const int8_t *s, long long *S, long long *M)
{
    // S and M are contiguous: M sits at S[3*(L/2+1)].
    (void)M;
    const uint64_t N = (uint64_t)L * L * L;
    const uint32_t R = L / 2 + 1;
    hipLaunchKernelGGL(k_i8_corr, dim3(grid_for(N, 128), 3 * R + 1), dim3(kThreads), 0, st, L, N,
                       s, reinterpret_cast<unsigned long long *>(S));
    return hipGetLastError();
}

hipError_t i8_check_pm1(hipStream_t st, size_t n, const int8_t *s, unsigned long long *bad)
{
    hipLaunchKernelGGL(k_i8_check, dim3(grid_for(n, 2048)), dim3(kThreads), 0, st, (uint64_t)n, s,
                       bad);
    return hipGetLastError();
}

hipError_t i8_window(hipStream_t st, uint32_t L, const int8_t *s, uint32_t ox, uint32_t oy,
                     uint32_t oz, uint32_t W, uint32_t lz0, uint32_t nz, int8_t *out)
{
    const uint64_t n = (uint64_t)W * W * nz;
    hipLaunchKernelGGL(k_i8_window, dim3(grid_for(n, 8192)), dim3(kThreads), 0, st, L, s, ox, oy,
                       oz, W, lz0, n, out);
    return hipGetLastError();
}

hipError_t fill_u64(hipStream_t st, unsigned long long *p, size_t n, unsigned long long v)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 1024)), dim3(kThreads), 0, st, p, (uint64_t)n,
                       v);
    return hipGetLastError();
}

}  // namespace qz
