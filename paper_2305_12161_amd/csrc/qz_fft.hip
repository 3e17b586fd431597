// qz_fft.hip -- the paper's own correlation measurement (Methods, "Calculating
// the correlation function"): the mean of s_i s_{i+d} over i for EVERY
// displacement d through the correlation theorem,
//     sum_i s_i s_{i+d} = (1/N) [F^{-1} |F s|^2]_d        (eq:sisik),
// with real-to-complex transforms in double precision (as the paper's FFTW),
// in place, and then averaged over spherical shells (the paper's radial
// average) together with the structure factor S(k) = |F s(k)|^2 / N.
// Shells: a displacement d (minimum image, each component in [-L/2, L/2)) or
// a wavevector k (integer components, same range) belongs to shell
// round(|d|) or round(|k|).
#include <hipfft/hipfft.h>

#include "qz_device.hpp"
#include "qz_internal.hpp"

namespace qz {
namespace {

constexpr int kFftBlock = 256;

// spins -> doubles in the padded in-place layout X[(z*L + y)*pad + x]
__global__ void __launch_bounds__(kFftBlock) k_fft_unpack_bit(uint32_t L, uint32_t pad,
                                                              const uint32_t *P0, const uint32_t *P1,
                                                              double *X)
{
    const uint32_t W = L / 64;
    const uint64_t N = (uint64_t)L * L * L;
    for (uint64_t i = (uint64_t)blockIdx.x * kFftBlock + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * kFftBlock) {
        const uint32_t x = (uint32_t)(i % L);
        const uint64_t row = i / L;
        const uint32_t y = (uint32_t)(row % L), z = (uint32_t)(row / L);
        const uint32_t c = (x + y + z) & 1u;
        const uint32_t word = (c ? P1 : P0)[row * W + (x >> 6)];
        X[row * pad + x] = ((word >> ((x >> 1) & 31u)) & 1u) ? 1.0 : -1.0;
    }
}

__global__ void __launch_bounds__(kFftBlock) k_fft_unpack_i8(uint32_t L, uint32_t pad,
                                                             const int8_t *s, double *X)
{
    const uint64_t N = (uint64_t)L * L * L;
    for (uint64_t i = (uint64_t)blockIdx.x * kFftBlock + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * kFftBlock) {
        const uint64_t row = i / L;
        X[row * pad + (i % L)] = (double)s[i];
    }
}

__device__ __forceinline__ int signed_comp(uint32_t v, uint32_t L)
{
    return v < L / 2 ? (int)v : (int)v - (int)L;   // [-L/2, L/2)
}

// Power spectrum: F(k) -> (|F(k)|^2, 0) in place, with S(k) shell sums.  The
// half spectrum stores kx = 0..L/2; an entry with 0 < kx < L/2 stands for k
// and -k (weight 2).  F(0) (the magnetisation) is saved before it is replaced.
__global__ void __launch_bounds__(kFftBlock)
    k_fft_power(uint32_t L, double2 *F, uint32_t nb, double *sk_sum, unsigned long long *sk_cnt,
                double *M_out)
{
    extern __shared__ double sh[];
    double *bsum = sh;
    unsigned int *bcnt = reinterpret_cast<unsigned int *>(sh + nb);
    for (uint32_t b = threadIdx.x; b < nb; b += kFftBlock) {
        bsum[b] = 0.0;
        bcnt[b] = 0u;
    }
    __syncthreads();
    const uint32_t H = L / 2 + 1;
    const uint64_t n = (uint64_t)L * L * H;
    for (uint64_t i = (uint64_t)blockIdx.x * kFftBlock + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * kFftBlock) {
        const uint32_t kx = (uint32_t)(i % H);
        const uint64_t row = i / H;
        const int ky = signed_comp((uint32_t)(row % L), L), kz = signed_comp((uint32_t)(row / L), L);
        const double2 f = F[i];
        if (i == 0)
            *M_out = f.x;
        const double p = f.x * f.x + f.y * f.y;
        F[i] = make_double2(p, 0.0);
        const double kk = sqrt((double)kx * kx + (double)ky * ky + (double)kz * kz);
        const uint32_t bin = (uint32_t)rint(kk);
        const unsigned int w = (kx == 0 || kx == L / 2) ? 1u : 2u;
        if (bin < nb) {
            atomicAdd(bsum + bin, w * p);
            atomicAdd(bcnt + bin, w);
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += kFftBlock)
        if (bcnt[b]) {
            atomicAdd(sk_sum + b, bsum[b]);
            atomicAdd(sk_cnt + b, (unsigned long long)bcnt[b]);
        }
}

// Shell sums of the inverse transform R(d) = N * sum_i s_i s_{i+d}.
__global__ void __launch_bounds__(kFftBlock)
    k_fft_radial(uint32_t L, uint32_t pad, const double *R, uint32_t nb, double *c_sum,
                 unsigned long long *c_cnt)
{
    extern __shared__ double sh[];
    double *bsum = sh;
    unsigned int *bcnt = reinterpret_cast<unsigned int *>(sh + nb);
    for (uint32_t b = threadIdx.x; b < nb; b += kFftBlock) {
        bsum[b] = 0.0;
        bcnt[b] = 0u;
    }
    __syncthreads();
    // one wave per row (y, z); each lane walks 8 consecutive x, so a wave
    // reads 512 consecutive values per step, and merges equal shells along its
    // run before adding them to the block's sums
    const uint64_t rows = (uint64_t)L * L;
    const uint32_t lane = threadIdx.x & 63u, nwv = kFftBlock / 64u;
    for (uint64_t row = (uint64_t)blockIdx.x * nwv + (threadIdx.x >> 6); row < rows;
         row += (uint64_t)gridDim.x * nwv) {
        const int dy = signed_comp((uint32_t)(row % L), L), dz = signed_comp((uint32_t)(row / L), L);
        const double base = (double)dy * dy + (double)dz * dz;
        const double *r = R + row * pad;
        for (uint32_t x0 = 8u * lane; x0 < L; x0 += 512u) {
            const uint32_t xe = min(x0 + 8u, L);
            uint32_t cur = 0xFFFFFFFFu;
            double acc = 0.0;
            unsigned int cnt = 0u;
            for (uint32_t x = x0; x < xe; ++x) {
                const int dx = signed_comp(x, L);
                const uint32_t bin = (uint32_t)rint(sqrt(base + (double)dx * dx));
                if (bin != cur) {
                    if (cnt && cur < nb) {
                        atomicAdd(bsum + cur, acc);
                        atomicAdd(bcnt + cur, cnt);
                    }
                    cur = bin;
                    acc = 0.0;
                    cnt = 0u;
                }
                acc += r[x];
                ++cnt;
            }
            if (cnt && cur < nb) {
                atomicAdd(bsum + cur, acc);
                atomicAdd(bcnt + cur, cnt);
            }
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += kFftBlock)
        if (bcnt[b]) {
            atomicAdd(c_sum + b, bsum[b]);
            atomicAdd(c_cnt + b, (unsigned long long)bcnt[b]);
        }
}

__global__ void k_fft_zero(double *d, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        d[i] = 0.0;
}

}  // namespace

uint32_t fft_pad(uint32_t L) { return 2 * (L / 2 + 1); }

uint32_t fft_nbins(uint32_t L)
{
    // shells up to round(sqrt(3) L/2), the corner of the minimum-image cube
    return (uint32_t)(0.8660254037844386 * L + 0.5) + 2;
}

hipError_t fft_unpack(hipStream_t st, uint32_t L, int layout, const void *spins0,
                      const void *spins1, double *X)
{
    const uint64_t N = (uint64_t)L * L * L;
    const uint32_t g = (uint32_t)std::min<uint64_t>((N + kFftBlock - 1) / kFftBlock, 65536);
    if (layout == 1)
        hipLaunchKernelGGL(k_fft_unpack_bit, dim3(g), dim3(kFftBlock), 0, st, L, fft_pad(L),
                           (const uint32_t *)spins0, (const uint32_t *)spins1, X);
    else
        hipLaunchKernelGGL(k_fft_unpack_i8, dim3(g), dim3(kFftBlock), 0, st, L, fft_pad(L),
                           (const int8_t *)spins0, X);
    return hipGetLastError();
}

hipError_t fft_power(hipStream_t st, uint32_t L, double *X, uint32_t nb, double *sk_sum,
                     unsigned long long *sk_cnt, double *M_out)
{
    const uint64_t n = (uint64_t)L * L * (L / 2 + 1);
    const uint32_t g = (uint32_t)std::min<uint64_t>((n + kFftBlock - 1) / kFftBlock, 8192);
    const size_t lds = (size_t)nb * (8 + 4);
    hipLaunchKernelGGL(k_fft_power, dim3(g), dim3(kFftBlock), lds, st, L,
                       reinterpret_cast<double2 *>(X), nb, sk_sum, sk_cnt, M_out);
    return hipGetLastError();
}

hipError_t fft_radial(hipStream_t st, uint32_t L, const double *X, uint32_t nb, double *c_sum,
                      unsigned long long *c_cnt)
{
    const uint64_t rows = (uint64_t)L * L;
    const uint64_t rows_per_block = kFftBlock / 64;   // one wave per row
    const uint32_t g = (uint32_t)std::min<uint64_t>((rows + rows_per_block - 1) / rows_per_block, 16384);
    const size_t lds = (size_t)nb * (8 + 4);
    hipLaunchKernelGGL(k_fft_radial, dim3(g), dim3(kFftBlock), lds, st, L, fft_pad(L), X, nb,
                       c_sum, c_cnt);
    return hipGetLastError();
}

hipError_t fft_zero(hipStream_t st, double *d, size_t n)
{
    hipLaunchKernelGGL(k_fft_zero, dim3(64), dim3(256), 0, st, d, (uint64_t)n);
    return hipGetLastError();
}

}  // namespace qz
