"""Autotuner for the sweep kernels: times candidate tilings on the device and
keeps the fastest.  Results never depend on the tuning, only speed does.

    python -m paper_2305_12161_amd.tune --L 2048            # single lattice, both passes
    python -m paper_2305_12161_amd.tune --batch-mix-584     # batched replicas

Winners are written to tuned.json next to this file; `best_single(L)`,
`best_pass2(L)` and `best_batch(L)` read them back (None when a size was never
tuned).  The library's own defaults come from the same measurements and need
no cache.
"""
import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")


def _load():
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {"single": {}, "batch": {}}


def _save(d):
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def best_single(L: int):
    v = _load()["single"].get(str(L))
    return tuple(v["tuning"]) if v else None


def best_pass2(L: int):
    v = _load().get("pass2", {}).get(str(L))
    return tuple(v["tuning"]) if v else None


def best_batch(L: int):
    v = _load()["batch"].get(str(L))
    return (v["Tz"], v["graph_sweeps"]) if v else None


def batch_tuning_json(sizes):
    """The stored batch winners for every side in `sizes` as the library's
    tuning text, or None (the library then autotunes) if a side was never
    tuned."""
    d = _load()["batch"]
    if not sizes or any(str(L) not in d for L in sizes):
        return None
    graph = min(int(d[str(L)]["graph_sweeps"]) for L in sizes)
    out = {"graph_sweeps": graph, "tz": {str(L): int(d[str(L)]["Tz"]) for L in sizes}}
    if 64 in sizes and "onchip" in d["64"]:
        out["onchip"] = int(d["64"]["onchip"])
    return json.dumps(out)


def single_candidates(L: int):
    W = L // 64
    out = []
    for V in (4, 2, 1):
        if W % V:
            continue
        R = W // V
        rows = [L] if L * R <= 1024 else []
        E = 8
        while E * R <= 1024 and E <= L:
            if E - 4 >= 4:
                rows.append(E - 4)
            E *= 2
        for Ty in rows:
            for Tz in (4, 8, 16, 32, 64):
                if Tz <= L:
                    out.append((V, Ty, Tz))
    return out


def pass2_candidates(L: int):
    """(V, Ty, Tz) of the two-sweep pass: Ty + 8 rows held per tile."""
    W = L // 64
    out = []
    for V in (4, 2, 1):
        if W % V:
            continue
        for Ty in (8, 24, 56, 120):
            for Tz in (8, 16, 32, 64):
                if Ty <= L and Tz <= L:
                    out.append((V, Ty, Tz))
    return out


def tune_pass2(L: int, sweeps: int = 30, verbose: bool = True):
    import torch
    from . import binding
    st = torch.cuda.current_stream()
    best = None
    lat = binding.Lattice(L, 11, "bit")
    for cand in pass2_candidates(L):
        try:
            lat.set_pass(2, *cand)
        except binding.QuenchError:
            continue
        lat.run(4)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        lat.run(sweeps)
        b.record(st)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / sweeps
        if verbose:
            print(json.dumps({"L": L, "pass2": cand, "ms_per_sweep": round(ms, 5)}), flush=True)
        if best is None or ms < best[1]:
            best = (cand, ms)
    d = _load()
    d.setdefault("pass2", {})[str(L)] = {"tuning": list(best[0]), "ms_per_sweep": round(best[1], 5)}
    _save(d)
    return best


def tune_single(L: int, sweeps: int = 30, verbose: bool = True):
    import torch
    from . import binding
    st = torch.cuda.current_stream()
    best = None
    lat = binding.Lattice(L, 11, "bit")
    lat.set_pass(1)
    for cand in single_candidates(L):
        try:
            lat.set_tuning(*cand)
        except binding.QuenchError:
            continue
        lat.run(3)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        lat.run(sweeps)
        b.record(st)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / sweeps
        if verbose:
            print(json.dumps({"L": L, "tuning": cand, "ms_per_sweep": round(ms, 5)}), flush=True)
        if best is None or ms < best[1]:
            best = (cand, ms)
    d = _load()
    d["single"][str(L)] = {"tuning": list(best[0]), "ms_per_sweep": round(best[1], 5)}
    _save(d)
    return best


def tune_batch(specs, sweeps: int = 10000, verbose: bool = True):
    """The on-chip path for side 64, then planes per sub-tile for every side
    the sub-tile launch runs, then sweeps per graph.  Each candidate runs the whole
    job of `sweeps` MCS from the random start: the cost of a sweep falls as the
    domains grow (fewer spins flip), so timing only the first sweeps would
    weigh the early times the job barely spends any time in."""
    import torch
    from . import binding
    sizes = sorted({L for L, _ in specs})
    chosen = {L: None for L in sizes}
    results = {}
    # untimed first sweeps that capture the graphs: a multiple of every graph
    # length tried, when the job is long enough to leave most of it timed
    warm = 200 if sweeps >= 400 else 0
    if sweeps <= warm:
        raise ValueError("sweeps must be positive")

    def time_batch(tz, graph, onchip=0):
        b = binding.Batch(specs, tuning={"graph_sweeps": graph, "onchip": onchip,
                                         "tz": {str(L): v for L, v in tz.items() if v}})
        if warm:
            b.run(warm)
        b.sync()
        t0 = time.perf_counter()
        b.run(sweeps - warm)
        b.sync()
        ms = (time.perf_counter() - t0) * 1e3 / (sweeps - warm)
        del b
        torch.cuda.empty_cache()
        return ms

    # side-64 replicas on chip (all sweeps of a graph in one launch) or as
    # sub-tiles; decided first, since it changes how many sub-tiles the other
    # sides share the sweep launch with
    onchip = 0
    if 64 in sizes:
        t_sub, t_chip = time_batch(chosen, 50, 0), time_batch(chosen, 50, 1)
        if verbose:
            print(json.dumps({"onchip": {"0": round(t_sub, 5), "1": round(t_chip, 5)}}), flush=True)
        onchip = int(t_chip < t_sub)
    for L in sizes:
        if L == 64 and onchip:
            continue
        for Tz in (2, 4, 8, 16, 32):
            if Tz > L or L % Tz:
                continue
            ms = time_batch({**chosen, L: Tz}, 50, onchip)
            if verbose:
                print(json.dumps({"L": L, "Tz": Tz, "ms_per_sweep": round(ms, 5)}), flush=True)
            if L not in results or ms < results[L][1]:
                results[L] = (Tz, ms)
        chosen[L] = results[L][0]
    for L in sizes:
        if chosen[L] is None:            # side 64 on chip: its sub-tile shape stays the default
            chosen[L] = 8 if L % 8 == 0 else 1
    best_graph = None
    for gs in (10, 25, 50, 100, 200):
        ms = time_batch(chosen, gs, onchip)
        if verbose:
            print(json.dumps({"graph_sweeps": gs, "ms_per_sweep": round(ms, 5)}), flush=True)
        if best_graph is None or ms < best_graph[1]:
            best_graph = (gs, ms)
    d = _load()
    for L in sizes:
        d["batch"][str(L)] = {"Tz": chosen[L], "graph_sweeps": best_graph[0]}
        if L == 64:
            d["batch"][str(L)]["onchip"] = onchip
    _save(d)
    return chosen, best_graph


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, nargs="*", default=[])
    ap.add_argument("--batch-mix-584", action="store_true")
    ap.add_argument("--out", type=str, default="",
                    help="write the winners to this file instead of tuned.json next to tune.py")
    args = ap.parse_args()
    if args.out:
        global CACHE
        CACHE = os.path.abspath(args.out)
    for L in args.L:
        print(json.dumps({"L": L, "best_one_sweep": tune_single(L)}), flush=True)
        print(json.dumps({"L": L, "best_two_sweep": tune_pass2(L)}), flush=True)
    if args.batch_mix_584:
        from . import workloads
        specs = [(r.L, r.seed) for r in workloads.batch_mix_584()]
        print(json.dumps({"batch_best": tune_batch(specs)}), flush=True)


if __name__ == "__main__":
    main()
