#!/usr/bin/env python3
"""Benchmark of the zero-temperature checkerboard quench on one MI355X.

Workload: the L=2048 quench (1-bit layout, seed 3, infinite-temperature start,
1e5 MCS) with the unsatisfied-bond count fused into
the sweeps at the 40 log-spaced times (--trace-every N: every N MCS instead)
and the axis correlation sums taken at the same times.  A
"step" is one Monte Carlo sweep of that run, including the measurements that
fall on it; W untimed sweeps are followed by K timed ones (by default the timed
window runs to t = 1e5, i.e. the whole job after the first W sweeps).

Prints ONE JSON line.  `value` is spin-flip attempts per ns over the timed
window (N attempts per sweep).  `roofline` prices the sweep kernel against
HBM: N/4 algorithmic bytes per sweep (each 1-bit spin read once and written
once) over the kernel's average duration, timed with HIP events on the
library's stream.  `cpu_baseline` is the CPU oracle on a bounded sample of the
same lattice (a window replay), on this host's cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/ns + % HBM roofline at L=2048; batched vs plain flips/ns"
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch from rocprofv3 counters, per kernel (one or two sweeps per launch)
TRAFFIC_FILES = {1: os.path.join(ROOT, "profiles", "traffic_sweep_bit_L2048.json"),
                 2: os.path.join(ROOT, "profiles", "traffic_sweep2_bit_L2048.json")}
# VALU instructions per launch of the uncounted two-sweep kernel, from rocprofv3 counters
VALU_FILE = os.path.join(ROOT, "profiles", "valu_sweep2_bit_L2048.json")
# wave64 VALU issue limit: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction
# per SIMD every 4 cycles (16 lanes per SIMD; the same unit count gives the
# 78.6 TFLOP/s fp64 vector peak)
VALU_PEAK_WAVE_INSTR_PER_S = 256 * 4 * 2.4e9 / 4
KERNEL_SOURCES = ["paper_2305_12161_amd/csrc/qz_bit.hip", "paper_2305_12161_amd/csrc/qz_bit2.hip",
                  "paper_2305_12161_amd/csrc/qz_bitops.hpp", "paper_2305_12161_amd/csrc/qz_device.hpp"]


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed sweeps (default: to t=1e5)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--L", type=int, default=2048)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--tuning", type=str, default="", help="V,Ty,Tz for the one-sweep kernel")
    ap.add_argument("--pass", dest="sweeps_per_pass", type=int, default=0,
                    help="sweeps per pass over memory (1 or 2; 0 = the library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-corr", action="store_true", help="skip the correlation measurements")
    ap.add_argument("--trace-every", type=int, default=0,
                    help="trace B every N MCS; 0 (default): at the 40 "
                         "log-spaced times of the run, as the L=2048 configuration asks")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-replica workload")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-request workload")
    ap.add_argument("--no-int8", action="store_true", help="skip the int8 configurations")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the mixed-cycle, double-checkerboard and FFT measurements")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="arrivals per second (default: the configured literal)")
    return ap.parse_args()


def plain_rate(binding, torch, L, n):
    """Attempts/ns of the single-lattice kernel on one lattice of side L (1-bit)."""
    lat = binding.Lattice(L, 1234, "bit")
    lat.run(4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.run(n)
    torch.cuda.synchronize()
    return L ** 3 * n / ((time.perf_counter() - t0) * 1e9)


def batched_workload(binding, torch, workloads):
    """512 x L64 + 64 x L128 + 8 x L256 replicas, 1e4 MCS, B every 10 MCS each."""
    specs = [(r.L, r.seed) for r in workloads.batch_mix_584()]
    t_max = workloads.batch_mix_584()[0].t_max
    warm = binding.Batch(specs[:2] + specs[-1:], trace_every=10, trace_cap=1024)
    warm.run(64)
    warm.sync()
    del warm
    # the launch shape: the autotuner's stored winners, else the library's
    # own autotune at creation (reported below either way)
    b = binding.Batch(specs, trace_every=10, trace_cap=t_max // 10 + 8)
    tuning = b.tuning()
    b.sync()
    t0 = time.perf_counter()
    piece = 1000
    for t in range(0, t_max, piece):
        b.run(min(piece, t_max - t))
        b.sync()
        print(f"# batched t={t + piece} at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    wall = time.perf_counter() - t0
    sites = sum(L ** 3 for L, _ in specs)
    rate = sites * t_max / (wall * 1e9)
    # the batch's 2 x sites/8 bytes of spins fit in the last-level cache: price
    # it against a device copy of the same footprint rather than HBM
    foot = 2 * sites // 8
    src = torch.ones(foot // 2, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    reps = 200
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    copy_gbs = foot * reps / ((time.perf_counter() - c0) * 1e9)
    del src, dst
    # the plain single-lattice kernel on one lattice of each size, for comparison
    plain = {L: plain_rate(binding, torch, L, 400) for L in sorted({L for L, _ in specs})}
    plain_wall = sum(L ** 3 * t_max / (plain[L] * 1e9) for L, _ in specs)
    return {
        "workload": "512 x L64 + 64 x L128 + 8 x L256 replicas (seeds 0x40000000 + r), 1-bit, "
                    f"1e4 MCS each, B every 10 MCS per replica, graph replays of "
                    f"{tuning['graph_sweeps']} sweeps",
        "tuning": tuning,
        "value": round(rate, 2), "unit": "attempts/ns", "wall_s": round(wall, 4),
        "ms_per_mcs": round(wall * 1e3 / t_max, 5),
        "plain_one_lattice_attempts_per_ns": {str(L): round(v, 2) for L, v in plain.items()},
        "plain_sequential_wall_s": round(plain_wall, 3),
        "batched_over_plain": round(plain_wall / wall, 2),
        "alg_GBs": round(sites / 4 * t_max / (wall * 1e9), 1),
        "copy_same_footprint_GBs": round(copy_gbs, 1),
        "footprint_MiB": round(foot / 2 ** 20, 1),
        "trace_points_per_replica": t_max // 10,
    }


def served_workload(binding, torch, workloads, n_req, rate):
    from paper_2305_12161_amd import serve
    reqs = workloads.request_stream(n=n_req, rate_per_s=rate)
    every, chunk = 100, 100
    be = serve.GpuBackend(budget_bytes=workloads.SERVE_BUDGET_BYTES,
                          batch_slots=workloads.SERVE_BATCH_SLOTS, every=every, chunk=chunk)
    srv = serve.Server(be, chunk=chunk)
    def progress(done, total, secs):
        if done % 100 == 0 or done == total:
            print(f"# served {done}/{total} at {secs:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res = srv.serve(reqs, progress=progress)
    wall = time.perf_counter() - t0
    st = serve.summarize(res, wall)
    st.update({
        "workload": f"{n_req} requests, L uniform in {list(workloads.SERVE_SIZES)}, t_max uniform "
                    f"in {list(workloads.SERVE_TMAX)}, Poisson arrivals at {rate:g}/s (numpy "
                    f"PCG64 seed 5), HBM budget {workloads.SERVE_BUDGET_BYTES >> 20} MiB, "
                    f"chunks of {chunk} MCS",
        "unit": "attempts/ns",
    })
    for k in ("p50_latency_s", "p99_latency_s", "attempts_per_ns", "wall_s"):
        st[k] = round(st[k], 4)
    return st


def next_rows_workload(binding, torch, L, seed):
    """The rows beyond the plain path, on the L = 2048 start advanced 100 MCS:
    the mixed cycle (colour order drawn per sweep; one and two sweeps per
    pass), the
    double checkerboard (coarse cubes of side 8 and 16, both cycles), and the
    double-precision FFT correlation with shell averages (at L = 1024)."""
    st = torch.cuda.current_stream()

    def per_sweep_ms(lat, n):
        lat.run(2)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        lat.run(n)
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    def rates(ms):
        return {"ms_per_sweep": round(ms, 4),
                "attempts_per_ns": round(L ** 3 / (ms * 1e6), 1),
                # N/4 algorithmic bytes per sweep against the HBM peak
                "roofline_frac": round((L ** 3 // 4) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    out = {"L": L, "start": "seed %d, t = 100" % seed}
    lat = binding.Lattice(L, seed, "bit")
    lat.run(100)
    lat.set_pass(1)
    out["plain_01_one_sweep_pass"] = rates(per_sweep_ms(lat, 40))
    lat.set_cycle(True)
    out["mixed_cycle_one_sweep_pass"] = rates(per_sweep_ms(lat, 40))
    # two sweeps per pass where consecutive sweeps draw the same first colour
    lat.set_pass(2)
    out["mixed_cycle"] = rates(per_sweep_ms(lat, 80))
    for B in (8, 16):
        lat.set_double_checkerboard(B)
        for mixed in (False, True):
            lat.set_cycle(mixed)
            key = "double_checkerboard_B%d_%s" % (B, "mixed" if mixed else "01")
            # two sweeps per pass, the default at this size: a sweep in one
            # pass over memory (plus one in-place phase in the mixed cycle)
            lat.set_pass(2)
            out[key] = rates(per_sweep_ms(lat, 10))
            # the same sweeps as in-place phases only
            lat.set_pass(1)
            out[key + "_phases"] = rates(per_sweep_ms(lat, 10))
    del lat
    torch.cuda.empty_cache()
    Lf = 1024
    f = binding.Lattice(Lf, seed, "bit")
    f.run(100)
    f.fft_corr()                   # plan and scratch once
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f.fft_corr()
    out["fft_corr_L1024_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    del f
    torch.cuda.empty_cache()
    return out


def int8_workloads(binding, torch, workloads):
    """The two int8 configurations, run in full: L = 32 (seed 1, 1e3 MCS, B
    every 10 MCS) and L = 256 (seed 2, 1e4 MCS, B and the axis correlation at
    the 40 log-spaced times).  At L = 256 the sweep is two in-place launches
    of the 16-byte half-sweep kernel; at L = 32 the whole run is one launch
    holding the lattice in LDS.  The algorithmic bytes are 2N per sweep (each
    byte read once and written once), N per half-sweep.  Both lattices stay in the
    on-chip caches (32 KiB, 16 MiB), so a device copy of the same footprint is
    timed beside them."""
    st = torch.cuda.current_stream()
    out = {}

    def copy_probe(nbytes):
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        reps = 200
        a.record(st)
        for _ in range(reps):
            dst.copy_(src)
        b.record(st)
        torch.cuda.synchronize()
        return 2 * nbytes * reps / (a.elapsed_time(b) * 1e6)   # GB/s (read + write)

    def launch_ms(lat, n):
        lat.run(4)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        lat.run(n)
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / (2 * n)        # two half-sweep launches per sweep

    for cfg in (workloads.RUN_I8_L32, workloads.RUN_I8_L256):
        L, N = cfg.L, cfg.L ** 3
        lat = binding.Lattice(L, cfg.seed, "i8", stream=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        corr = 0.0
        if cfg.trace_every:
            lat.run(cfg.t_max, cfg.trace_every)
        else:
            for tc in cfg.corr_times:
                lat.run(tc - lat.t)
                torch.cuda.synchronize()
                c0 = time.perf_counter()
                lat.corr()
                lat.bonds()
                corr += time.perf_counter() - c0
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        assert lat.t == cfg.t_max
        half_ms = launch_ms(lat, 200)
        achieved = N / (half_ms * 1e6)              # GB/s: N bytes per half-sweep launch
        copy_gbs = copy_probe(N)
        out[cfg.name] = {
            "workload": (f"L={L} int8, seed {cfg.seed}, {cfg.t_max} MCS, " +
                         (f"B every {cfg.trace_every} MCS" if cfg.trace_every else
                          f"B and C(r) at the {len(cfg.corr_times)} log-spaced times")),
            "attempts_per_ns": round(N * cfg.t_max / (wall * 1e9), 2),
            "wall_s": round(wall, 4),
            "measurement_s": round(corr, 4),
            "sweep_attempts_per_ns": round(N / (2 * half_ms * 1e6), 2),
            "roofline": {"bound": "hbm", "kernel": ("k_i8_onchip (whole run in one launch, lattice in LDS; time per half-sweep)" if L in (16, 32) else "k_i8_half16 (one colour, in place)"),
                         "alg_bytes_per_launch": N, "avg_launch_ms": round(half_ms, 5),
                         "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "copy_same_footprint_GBs": round(copy_gbs, 1),
                         "frac_of_copy": round(achieved / copy_gbs, 4)},
        }
        del lat
    return out


def cpu_baseline(L, seed, budget_s=15.0):
    """Oracle window replay on a cube of the same lattice: attempts per ns on host cores."""
    import oracle
    cores = min(16, len(os.sched_getaffinity(0)))
    used = oracle.set_threads(cores)
    W = 256 if L >= 256 else L
    w = oracle.init_window(L, seed, (0, 0, 0), W)
    # run chunks of sweeps until about budget_s of CPU time has passed
    oracle.window_advance(L, seed, (0, 0, 0), w, 0, 1)   # warm up
    T, dt, chunk = 0, 0.0, 8
    while dt < budget_s:
        t0 = time.perf_counter()
        oracle.window_advance(L, seed, (0, 0, 0), w, 1 + T, chunk)
        dt += time.perf_counter() - t0
        T += chunk
        chunk = min(chunk * 2, 512)
    attempts = (W - 2) ** 3 * T
    # the same replay on one thread, for a shorter time
    oracle.set_threads(1)
    T1, dt1, chunk = 0, 0.0, 1
    while dt1 < budget_s / 4:
        t0 = time.perf_counter()
        oracle.window_advance(L, seed, (0, 0, 0), w, 1 + T + T1, chunk)
        dt1 += time.perf_counter() - t0
        T1 += chunk
        chunk = min(chunk * 2, 64)
    oracle.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": attempts / (dt * 1e9), "unit": "attempts/ns", "cores": used, "kind": "oracle",
            "value_1_thread": (W - 2) ** 3 * T1 / (dt1 * 1e9), "cpu_model": model,
            "sample": f"oracle window replay: {W}^3 cube of the L={L} seed-{seed} start, "
                      f"sweeps 1..{T}, {(W - 2) ** 3} sites updated per sweep, {dt:.1f} s on "
                      f"{used} threads; then {T1} more sweeps on 1 thread, {dt1:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the quench of one "
              "lattice is not sharded across GPUs; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2305_12161_amd import binding, workloads

    L, seed = args.L, args.seed
    t_max = workloads.RUN_BIT_L2048.t_max
    W = args.warmup
    K = args.steps if args.steps is not None else max(1, t_max - W)
    corr_times = [] if args.no_corr else [t for t in workloads.log_times(t_max) if W < t <= W + K]
    N = L ** 3
    every = args.trace_every
    # sweeps whose entering B is traced: the log-spaced
    # times, or every `every` MCS; the last sweep always (for the final lengths)
    if every > 0:
        trace_times = list(range(0, W + K, every))
    else:
        trace_times = [t for t in workloads.log_times(t_max) if t < W + K]
    trace_times = sorted(set(trace_times + [W + K - 1]))
    trace_index = {t: i for i, t in enumerate(trace_times)}

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    lat = binding.Lattice(L, seed, "bit", stream=stream)
    # tiles: given on the command line, else the autotuner's stored winners
    # for this L (tune.py), else the library's defaults
    tuning_source = "library defaults"
    if args.sweeps_per_pass:
        lat.set_pass(args.sweeps_per_pass)
    if args.tuning:
        lat.set_tuning(*[int(v) for v in args.tuning.split(",")])
        tuning_source = "command line"
    else:
        from paper_2305_12161_amd import tune as tuner
        stored1, stored2 = tuner.best_single(L), tuner.best_pass2(L)
        if stored1:
            lat.set_tuning(*stored1)
        if stored2 and lat.pass_config()[0] == 2:
            lat.set_pass(2, *stored2)
        if stored1 or stored2:
            tuning_source = "tuned.json"
    tune = lat.tuning()
    pcfg = lat.pass_config()
    per_launch = pcfg[0]   # sweeps carried by one launch of the dominant kernel
    trace = torch.zeros(len(trace_times), dtype=torch.int64, device="cuda")
    print(f"# L={L} seed={seed} tuning={tune} warmup={W} steps={K} corr_times={len(corr_times)}",
          file=sys.stderr, flush=True)

    def advance(t_from, t_to, timing):
        """Sweeps t_from..t_to-1: whole launches of the pass kernel first (two
        sweeps each by default), then at most one single sweep; the traced
        times among them are listed to the library, which counts B and the
        inside whichever launch runs that sweep."""
        n = t_to - t_from
        whole = n - n % per_launch
        for ta, m in ((t_from, whole), (t_from + whole, n - whole)):
            if m == 0:
                continue
            listed = [x for x in trace_times if ta <= x < ta + m]
            i0 = trace_index[listed[0]] if listed else 0
            if timing is not None:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
            lat.run_device_at(m, [x - ta for x in listed], trace[i0:i0 + len(listed)], None)
            if timing is not None:
                b.record(stream)
                timing.append((a, b, m, ta, m % per_launch == 0 and m >= per_launch))

    # warmup (untimed)
    advance(0, W, None)
    torch.cuda.synchronize()
    assert lat.t == W

    timing = []
    corr_ms = []
    ells = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = W
    for tc in sorted(set(corr_times + [W + K])):
        advance(t, tc, timing)
        t = tc
        if tc in corr_times:
            torch.cuda.synchronize()   # time the measurement alone, not the queued sweeps
            c0 = time.perf_counter()
            S, M = lat.corr()
            corr_ms.append((time.perf_counter() - c0) * 1e3)
            ells.append((tc, S, M))
            print(f"# t={tc} at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert lat.t == W + K

    # the accepted flips of one sweep right after the window (untimed): the
    # timed sweeps trace the bond count only, since counting the flips of a
    # pass's first sweep makes that pass about a fifth slower
    _, F_after = lat.run_at(2, [0])
    flips_after = int(F_after[0])
    sweep_ms = sum(a.elapsed_time(b) for a, b, _, _, _ in timing)
    n_timed = sum(n for _, _, n, _, _ in timing)
    avg_sweep_s = sweep_ms / 1e3 / max(1, n_timed)
    # the dominant kernel's launches: the parts made of whole passes
    whole = [(a.elapsed_time(b), n) for a, b, n, _, w in timing if w]
    launches = sum(n for _, n in whole) // per_launch
    launch_s = (sum(ms for ms, _ in whole) / 1e3 / launches if launches
                else per_launch * avg_sweep_s)

    # late times (t >= 1e4), where few sites tie: the window's own launches
    # there, else a second leg after it -- the lattice advanced untimed to
    # t = 1e4 and 40 sweeps timed
    late = [(a.elapsed_time(b), n) for a, b, n, t_start, w in timing if w and t_start >= 10_000]
    late_src = "timed window"
    if not late:
        late_src = "after the timed window: advanced untimed to t = 1e4, 40 sweeps timed"
        lat.run(max(0, 10_000 - lat.t))
        if lat.t % 2:
            lat.run(1)
        late = []
        for _ in range(4):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lat.run_device_at(10, [], None, None)
            b.record(stream)
            late.append((a, b))
        torch.cuda.synchronize()
        late = [(a.elapsed_time(b), 10) for a, b in late]
    late_launch_s = sum(ms for ms, _ in late) / 1e3 / (sum(n for _, n in late) // per_launch)
    # the correlation's cost per measurement: those in the window, else one
    # taken after it
    if not corr_ms and not args.no_corr:
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        lat.corr()
        corr_ms.append((time.perf_counter() - c0) * 1e3)
    corr_s = sum(corr_ms) / len(corr_ms) / 1e3 if corr_ms else 0.0
    # whole-job rate: a sweep as timed in the window (B fused at the
    # traced sweeps) plus the correlation at the job's own density, 40
    # measurements per t_max sweeps.  A short window near t = 0 holds far
    # more of the log-spaced times than its share; its raw wall-clock rate is
    # reported beside this as window_wall.
    n_corr_job = 0 if args.no_corr else len(workloads.log_times(t_max))
    job_sweep_s = avg_sweep_s + corr_s * n_corr_job / t_max
    value = N / (job_sweep_s * 1e9)
    # algorithmic bytes: N/4 per sweep (each 1-bit spin read once and written
    # once); a launch of the two-sweep kernel carries two sweeps
    alg_bytes = per_launch * (N // 4)
    achieved = alg_bytes / launch_s / 1e9

    traffic = None
    tfile = TRAFFIC_FILES.get(per_launch)
    if tfile and os.path.exists(tfile):
        with open(tfile) as f:
            tr = json.load(f)
        if tr.get("kernel_sha") == kernel_sha() and tr.get("L") == L:
            traffic = tr.get("bytes_per_launch")
    # the uncounted two-sweep kernel's VALU instructions per launch (counters),
    # against the issue limit over the same launch time: its real bound
    valu = None
    if per_launch == 2 and os.path.exists(VALU_FILE):
        with open(VALU_FILE) as f:
            vf = json.load(f)
        if vf.get("kernel_sha") == kernel_sha() and vf.get("L") == L:
            instr = vf["SQ_INSTS_VALU"]
            valu = {"wave_instr_per_launch": instr, "peak_wave_instr_per_s": VALU_PEAK_WAVE_INSTR_PER_S,
                    "frac_t_ge_1e4": round(instr / late_launch_s / VALU_PEAK_WAVE_INSTR_PER_S, 4),
                    "source": os.path.relpath(VALU_FILE, ROOT)}

    from paper_2305_12161_amd import measure
    B_last = int(trace[trace_index[W + K - 1]].item())
    window = [trace_index[x] for x in trace_times if W <= x < W + K]
    bond_cadence = (f"every {every} MCS" if every > 0 else
                    f"at the {len(window)} of 40 log-spaced times in the timed window and "
                    f"the last sweep")
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "attempts/ns",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(job_sweep_s * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"L{L}_bit_quench: periodic L={L} simple-cubic Ising, 1-bit colour-separated "
                        f"spins, seed {seed}, T=inf start, T=0 checkerboard dynamics to t={W + K} MCS, "
                        f"unsatisfied-bond count (fused) {bond_cadence}, axis C(r<=L/2) at the "
                        f"{len(corr_times)} of 40 log-spaced times in the timed window",
            "L": L, "layout": "bit", "seed": seed, "t_window": [W, W + K],
            "tuning_V_Ty_Tz": list(tune), "tuning_source": tuning_source, "sweeps_per_pass": pcfg[0],
            "pass2_tuning_V_Ty_Tz": list(pcfg[1:]), "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": ("k_bit_sweep2 (two fused two-colour sweeps per pass, bond count fused)"
                       if per_launch == 2 else
                       "k_bit_sweep (fused two-colour sweep, bond count fused)"),
            "sweeps_per_launch": per_launch,
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_ms": round(launch_s * 1e3, 5),
            "frac_t_ge_1e4": round(alg_bytes / late_launch_s / 1e9 / HBM_PEAK_GBS, 4),
            "avg_launch_ms_t_ge_1e4": round(late_launch_s * 1e3, 5),
            "t_ge_1e4_source": late_src,
            # the bytes the kernel really moves (counter-measured `traffic`) over
            # the same launch time: a two-sweep launch keeps the state between
            # its sweeps on chip, so `achieved` (algorithmic) can exceed the peak
            "traffic_GBs": round(traffic / launch_s / 1e9, 1) if traffic else None,
            "traffic_frac": (round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
                             if traffic else None),
            "traffic_frac_t_ge_1e4": (round(traffic / late_launch_s / 1e9 / HBM_PEAK_GBS, 4)
                                      if traffic else None),
            "valu": valu,
        },
        "value_basis": ("per sweep: the timed window's sweeps (bond count fused at "
                        "the traced sweeps) plus the axis correlation charged at the job's density "
                        f"of {n_corr_job} measurements per {t_max} MCS"),
        "window_wall": {"attempts_per_ns": round(N * K / (wall * 1e9), 2),
                        "ms_per_step": round(wall * 1e3 / K, 5),
                        "correlations_in_window": len(corr_times)},
        "sweep_only_attempts_per_ns": round(N / avg_sweep_s / 1e9, 2),
        "corr_ms_mean": round(sum(corr_ms) / len(corr_ms), 3) if corr_ms else None,
        "corr_count": len(corr_ms),          # in the window, or one after it
        "ell_E_final": round(measure.energy_length(B_last, N), 4),
        # accepted moves (a physics output, not the work unit): spins flipped
        # per site by the sweep right after the window, taken apart from it
        "accepted_flips_per_site_after_window": round(flips_after / N, 7),
        "ell_C_final": (round(measure.crossing_length(ells[-1][1], ells[-1][2], N), 4)
                        if ells else None),
    }
    del lat
    torch.cuda.empty_cache()
    # the secondary legs report their own failure instead of hiding the main line
    def leg(name, fn):
        print(f"# {name}", file=sys.stderr, flush=True)
        try:
            out[name] = fn()
        except Exception as e:  # noqa: BLE001
            out[name] = {"error": f"{type(e).__name__}: {e}"}
            print(f"# {name} failed: {e}", file=sys.stderr, flush=True)
    if not args.no_batch:
        leg("batched", lambda: batched_workload(binding, torch, workloads))
        if "value" in out.get("batched", {}):
            # the batch against the single-lattice kernel at its best size
            # (the L = 2048 sweeps above), beside the one-lattice-at-a-time
            # comparison at the batch's own sizes
            out["batched"]["batched_over_L2048_sweeps"] = round(
                out["batched"]["value"] / out["sweep_only_attempts_per_ns"], 4)
    if not args.no_serve:
        rate = args.serve_rate if args.serve_rate else workloads.SERVE_RATE_PER_S
        leg("served", lambda: served_workload(binding, torch, workloads, args.serve_requests, rate))
    if not args.no_int8:
        leg("int8", lambda: int8_workloads(binding, torch, workloads))
    if not args.no_next:
        leg("next_rows", lambda: next_rows_workload(binding, torch, L, seed))
    if not args.no_cpu_baseline:
        leg("cpu_baseline", lambda: cpu_baseline(L, seed))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
