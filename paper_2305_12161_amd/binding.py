"""ctypes binding of libquench.so (include/quench.h), argument marshalling only.

Device memory comes from torch tensors and work runs on torch's current HIP
stream; every step of the dynamics and of the measurements runs in the HIP
library.  There is no fallback: if the library is missing this module raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libquench.so")

QZ_OK, QZ_EINVAL, QZ_ENOMEM, QZ_EDEVICE, QZ_ESTATE, QZ_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
LAYOUTS = {"i8": 0, "bit": 1}


class QuenchError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"[{status}] {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    c = ctypes
    vp, u32, u64, sz, i32 = c.c_void_p, c.c_uint32, c.c_uint64, c.c_size_t, c.c_int
    sig = {
        "qz_abi_version": ([], i32),
        "qz_state_bytes": ([u32, i32], sz),
        "qz_create": ([u32, u64, i32, vp, sz, vp, c.POINTER(vp)], i32),
        "qz_destroy": ([vp], i32),
        "qz_run": ([vp, u64, u64, c.POINTER(u64)], i32),
        "qz_run_device": ([vp, u64, u64, vp], i32),
        "qz_run_traced": ([vp, u64, u64, c.POINTER(u64), c.POINTER(u64)], i32),
        "qz_run_device_traced": ([vp, u64, u64, vp, vp], i32),
        "qz_run_at": ([vp, u64, c.POINTER(u64), sz, c.POINTER(u64), c.POINTER(u64)], i32),
        "qz_run_device_at": ([vp, u64, c.POINTER(u64), sz, vp, vp], i32),
        "qz_bonds": ([vp, c.POINTER(u64)], i32),
        "qz_bonds_device": ([vp, vp], i32),
        "qz_corr": ([vp, c.POINTER(c.c_int64), c.POINTER(c.c_int64)], i32),
        "qz_corr_noalloc": ([vp, c.POINTER(c.c_int64), c.POINTER(c.c_int64)], i32),
        "qz_time": ([vp, c.POINTER(u64)], i32),
        "qz_download_spins": ([vp, c.POINTER(c.c_int8)], i32),
        "qz_upload_spins": ([vp, c.POINTER(c.c_int8), u64], i32),
        "qz_download_window": ([vp, c.POINTER(u32), u32, c.POINTER(c.c_int8)], i32),
        "qz_set_tuning": ([vp, i32, i32, i32], i32),
        "qz_set_cycle": ([vp, i32], i32),
        "qz_set_double_checkerboard": ([vp, u32], i32),
        "qz_fft_nbins": ([u32], u32),
        "qz_fft_prepare": ([vp, c.POINTER(sz)], i32),
        "qz_fft_corr": ([vp, vp, sz, c.POINTER(c.c_double), c.POINTER(c.c_double),
                         c.POINTER(u64), c.POINTER(u64), c.POINTER(c.c_double)], i32),
        "qz_get_tuning": ([vp, c.POINTER(i32)], i32),
        "qz_set_pass": ([vp, i32, i32, i32, i32], i32),
        "qz_get_pass": ([vp, c.POINTER(i32)], i32),
        "qz_status_string": ([i32], c.c_char_p),
        "qz_last_error": ([], c.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def _check(status):
    if status != QZ_OK:
        raise QuenchError(status, lib.qz_last_error().decode(errors="replace"))


def state_bytes(L: int, layout: str) -> int:
    return int(lib.qz_state_bytes(L, LAYOUTS[layout]))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream, ctypes.c_void_p(stream.cuda_stream)


def _counts(n, trace_every=0):
    """Sweep count and trace cadence as non-negative integers: a negative value
    would reach the library as a huge unsigned count."""
    n, trace_every = int(n), int(trace_every)
    if n < 0 or trace_every < 0:
        raise ValueError("sweep counts and trace cadences must be non-negative")
    return n, trace_every


def _dev_buf(t, need: int):
    """Device pointer of a torch tensor that receives `need` 64-bit values, or
    None.  Refuses tensors the library would write past or misread."""
    if t is None:
        return None
    if not t.is_cuda or t.element_size() != 8 or not t.is_contiguous():
        raise ValueError("trace buffers must be contiguous 64-bit device tensors")
    if t.numel() < need:
        raise ValueError(f"trace buffer holds {t.numel()} values, the run writes {need}")
    return ctypes.c_void_p(t.data_ptr())


class Lattice:
    """One quench lattice held on the device (torch-owned memory)."""

    def __init__(self, L: int, seed: int, layout: str = "bit", device=None, stream=None):
        import torch
        if layout not in LAYOUTS:
            raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
        self.L, self.seed, self.layout = int(L), int(seed), layout
        nbytes = state_bytes(L, layout)
        if nbytes == 0:
            code = QZ_EUNSUPPORTED if (L >= 4 and L % 2 == 0) else QZ_EINVAL
            raise QuenchError(code, f"L={L} is not valid for the {layout} layout")
        device = torch.device("cuda") if device is None else torch.device(device)
        self.stream, sh = _stream_handle(stream)
        # allocated from the pool of the stream that uses it: when the lattice
        # is dropped, the memory is reused only behind the work queued there
        with torch.cuda.stream(self.stream):
            self.mem = torch.empty(nbytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib.qz_create(self.L, self.seed & (2**64 - 1), LAYOUTS[layout],
                             ctypes.c_void_p(self.mem.data_ptr()), nbytes, sh, ctypes.byref(h)))
        self._h = h

    @property
    def N(self) -> int:
        return self.L ** 3

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.qz_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        v = ctypes.c_uint64()
        _check(lib.qz_time(self._h, ctypes.byref(v)))
        return int(v.value)

    def run(self, n: int, trace_every: int = 0) -> np.ndarray:
        n, trace_every = _counts(n, trace_every)
        if trace_every:
            out = np.zeros(n // trace_every, dtype=np.uint64)
            _check(lib.qz_run(self._h, n, trace_every,
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
            return out
        _check(lib.qz_run(self._h, n, 0, None))
        return np.zeros(0, dtype=np.uint64)

    def run_device(self, n: int, trace_every: int, dev_trace) -> None:
        """Asynchronous run; dev_trace is a torch int64/uint64 device tensor."""
        n, trace_every = _counts(n, trace_every)
        ptr = _dev_buf(dev_trace, n // trace_every if trace_every else 0)
        _check(lib.qz_run_device(self._h, n, trace_every, ptr))

    def run_traced(self, n: int, trace_every: int):
        """Run n sweeps; returns (B, flips) at every trace_every-th sweep: the bond
        count entering the sweep and the number of spins it flipped."""
        n, trace_every = _counts(n, trace_every)
        if trace_every <= 0:
            raise ValueError("trace_every must be positive")
        B = np.zeros(n // trace_every, dtype=np.uint64)
        F = np.zeros(n // trace_every, dtype=np.uint64)
        P = ctypes.POINTER(ctypes.c_uint64)
        _check(lib.qz_run_traced(self._h, n, trace_every, B.ctypes.data_as(P), F.ctypes.data_as(P)))
        return B.astype(np.int64), F.astype(np.int64)

    def run_device_traced(self, n: int, trace_every: int, dev_B, dev_flips) -> None:
        """Asynchronous run with device traces of B and of the accepted flips."""
        n, trace_every = _counts(n, trace_every)
        need = n // trace_every if trace_every else 0
        pb, pf = _dev_buf(dev_B, need), _dev_buf(dev_flips, need)
        _check(lib.qz_run_device_traced(self._h, n, trace_every, pb, pf))

    def run_at(self, n: int, at):
        """Run n sweeps; returns (B, flips) for the sweeps at the listed offsets
        (strictly increasing, each < n): the bond count entering the sweep and
        the number of spins it flipped."""
        n, _ = _counts(n)
        P = ctypes.POINTER(ctypes.c_uint64)
        lst = np.ascontiguousarray(at, dtype=np.uint64)
        B = np.zeros(lst.size, dtype=np.uint64)
        F = np.zeros(lst.size, dtype=np.uint64)
        _check(lib.qz_run_at(self._h, n, lst.ctypes.data_as(P), lst.size, B.ctypes.data_as(P),
                             F.ctypes.data_as(P)))
        return B.astype(np.int64), F.astype(np.int64)

    def run_device_at(self, n: int, at, dev_B, dev_flips) -> None:
        """Asynchronous run; device traces of B and of the flips at the listed sweeps."""
        n, _ = _counts(n)
        P = ctypes.POINTER(ctypes.c_uint64)
        lst = np.ascontiguousarray(at, dtype=np.uint64)
        pb, pf = _dev_buf(dev_B, lst.size), _dev_buf(dev_flips, lst.size)
        _check(lib.qz_run_device_at(self._h, n, lst.ctypes.data_as(P), lst.size, pb, pf))

    def bonds(self) -> np.ndarray:
        out = np.zeros(3, dtype=np.uint64)
        _check(lib.qz_bonds(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out.astype(np.int64)

    def bonds_device(self, dev_out) -> None:
        """Asynchronous bonds(): [B_x, B_y, B_z] into the first three values of
        a 64-bit device tensor, on the lattice's stream."""
        _check(lib.qz_bonds_device(self._h, _dev_buf(dev_out, 3)))

    def corr(self):
        R = self.L // 2 + 1
        S = np.zeros((3, R), dtype=np.int64)
        M = ctypes.c_int64()
        _check(lib.qz_corr(self._h, S.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           ctypes.byref(M)))
        return S, int(M.value)

    def corr_noalloc(self):
        """corr() through the entry point that allocates nothing (the library's
        static scratch; the idle copy is left alone)."""
        R = self.L // 2 + 1
        S = np.zeros((3, R), dtype=np.int64)
        M = ctypes.c_int64()
        _check(lib.qz_corr_noalloc(self._h, S.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   ctypes.byref(M)))
        return S, int(M.value)

    def download(self) -> np.ndarray:
        out = np.empty((self.L, self.L, self.L), dtype=np.int8)
        _check(lib.qz_download_spins(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))
        return out

    def upload(self, spins: np.ndarray, t: int) -> None:
        a = np.ascontiguousarray(spins, dtype=np.int8)
        if a.shape != (self.L,) * 3:
            raise ValueError("spins must have shape (L, L, L)")
        _check(lib.qz_upload_spins(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), t))

    def window(self, origin, W: int) -> np.ndarray:
        o = (ctypes.c_uint32 * 3)(*[int(v) % self.L for v in origin])
        out = np.empty((W, W, W), dtype=np.int8)
        _check(lib.qz_download_window(self._h, o, W,
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))
        return out

    def set_tuning(self, V: int, Ty: int, Tz: int) -> None:
        _check(lib.qz_set_tuning(self._h, V, Ty, Tz))

    def fft_corr(self):
        """Shell means of C(r) and S(k) by the double-precision FFT route.

        Returns (C, Sk, n_r, n_k, m); scratch device memory comes from torch.
        """
        import torch
        need = ctypes.c_size_t()
        _check(lib.qz_fft_prepare(self._h, ctypes.byref(need)))
        scratch = torch.empty(int(need.value), dtype=torch.uint8, device=self.mem.device)
        nb = int(lib.qz_fft_nbins(self.L))
        C = np.zeros(nb)
        Sk = np.zeros(nb)
        nr = np.zeros(nb, dtype=np.uint64)
        nk = np.zeros(nb, dtype=np.uint64)
        m = ctypes.c_double()
        dp = ctypes.POINTER(ctypes.c_double)
        up = ctypes.POINTER(ctypes.c_uint64)
        _check(lib.qz_fft_corr(self._h, ctypes.c_void_p(scratch.data_ptr()), int(need.value),
                               C.ctypes.data_as(dp), Sk.ctypes.data_as(dp), nr.ctypes.data_as(up),
                               nk.ctypes.data_as(up), ctypes.byref(m)))
        del scratch
        return C, Sk, nr.astype(np.int64), nk.astype(np.int64), float(m.value)

    def set_double_checkerboard(self, B: int) -> None:
        """Double checkerboard with coarse cubes of side B (0: plain checkerboard)."""
        _check(lib.qz_set_double_checkerboard(self._h, B))

    def set_cycle(self, mixed: bool) -> None:
        """Mixed cycle (colour order drawn per sweep) if True, else the 01 cycle."""
        _check(lib.qz_set_cycle(self._h, 1 if mixed else 0))

    def tuning(self):
        out = (ctypes.c_int * 3)()
        _check(lib.qz_get_tuning(self._h, out))
        return tuple(int(v) for v in out)

    def set_pass(self, sweeps: int, V: int = 0, Ty: int = 0, Tz: int = 0) -> None:
        """Sweeps per pass over memory: 1, or 2 (two sweeps kept on chip; V, Ty,
        Tz tune that kernel, all 0 = default).  Results do not change."""
        _check(lib.qz_set_pass(self._h, sweeps, V, Ty, Tz))

    def pass_config(self):
        """(sweeps per pass, V, Ty, Tz of the two-sweep kernel)."""
        out = (ctypes.c_int * 4)()
        _check(lib.qz_get_pass(self._h, out))
        return tuple(int(v) for v in out)


# --------------------------------------------------------------------------
# batched replicas
# --------------------------------------------------------------------------
class _ReplicaSpec(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("t_max", ctypes.c_uint64)]


def _batch_signatures():
    c = ctypes
    vp, u32, u64, sz, i32 = c.c_void_p, c.c_uint32, c.c_uint64, c.c_size_t, c.c_int
    spec_p = c.POINTER(_ReplicaSpec)
    sig = {
        "qz_batch_state_bytes": ([spec_p, sz, u32], sz),
        "qz_batch_create": ([spec_p, sz, u32, u32, vp, sz, vp, c.c_char_p, c.POINTER(vp)], i32),
        "qz_batch_destroy": ([vp], i32),
        "qz_batch_run": ([vp, u64, u64, c.POINTER(u64)], i32),
        "qz_batch_sync": ([vp], i32),
        "qz_batch_slot_replace": ([vp, sz, spec_p], i32),
        "qz_batch_slot_reset": ([vp, sz, u64], i32),
        "qz_batch_slot_active": ([vp, sz, i32], i32),
        "qz_batch_slot_time": ([vp, sz, c.POINTER(u64)], i32),
        "qz_batch_trace": ([vp, sz, u64, u64, c.POINTER(u64)], i32),
        "qz_batch_download": ([vp, sz, c.POINTER(c.c_int8)], i32),
        "qz_batch_bonds": ([vp, sz, c.POINTER(u64)], i32),
        "qz_batch_corr": ([vp, sz, c.POINTER(c.c_int64), c.POINTER(c.c_int64)], i32),
        "qz_batch_set_tuning": ([vp, u32, u32, u32], i32),
        "qz_batch_tuning_json": ([vp, c.c_char_p, sz], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res


_batch_signatures()


def _spec(s):
    """(L, seed) or (L, seed, t_max) -> the C struct (t_max 0: no limit)."""
    L, seed = int(s[0]), int(s[1])
    t_max = int(s[2]) if len(s) > 2 else 0
    return _ReplicaSpec(L, seed & (2**64 - 1), t_max)


def batch_state_bytes(specs, trace_cap: int) -> int:
    arr = (_ReplicaSpec * len(specs))(*[_spec(s) for s in specs])
    return int(lib.qz_batch_state_bytes(arr, len(specs), trace_cap))


class Batch:
    """Replica slots (L, seed[, t_max]) advanced together on the device.

    tuning: the launch shape handed to the library -- "tuned" (default) takes
    the autotuner's stored winners (tune.py) when every side of the batch has
    one, else lets the library autotune at creation; None always lets the
    library autotune; a dict or JSON text is passed as given."""

    def __init__(self, specs, trace_every: int = 0, trace_cap: int = 1024, device=None,
                 stream=None, tuning="tuned"):
        import json
        import torch
        self.specs = [(int(s[0]), int(s[1])) for s in specs]
        arr = (_ReplicaSpec * len(self.specs))(*[_spec(s) for s in specs])
        nbytes = int(lib.qz_batch_state_bytes(arr, len(self.specs), trace_cap))
        if nbytes == 0:
            raise QuenchError(QZ_EUNSUPPORTED, "unsupported replica size in the batch")
        if isinstance(tuning, str) and tuning == "tuned":
            from . import tune
            tuning = tune.batch_tuning_json(sorted({L for L, _ in self.specs}))
        if isinstance(tuning, dict):
            tuning = json.dumps(tuning)
        device = torch.device("cuda") if device is None else torch.device(device)
        self.stream, sh = _stream_handle(stream)
        with torch.cuda.stream(self.stream):
            self.mem = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.trace_every, self.trace_cap = int(trace_every), int(trace_cap)
        h = ctypes.c_void_p()
        _check(lib.qz_batch_create(arr, len(self.specs), self.trace_every, self.trace_cap,
                                   ctypes.c_void_p(self.mem.data_ptr()), nbytes, sh,
                                   tuning.encode() if tuning is not None else None,
                                   ctypes.byref(h)))
        self._h = h

    def __len__(self):
        return len(self.specs)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.qz_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, n: int, trace_every: int = 0):
        """Advance every active slot n sweeps.  trace_every > 0 (the batch's
        cadence) returns an int64 array [slot, i] of B at the traced times
        reached in this run (-1 where a slot did not reach that time) and
        synchronises; otherwise the call is asynchronous and returns None."""
        n, trace_every = _counts(n, trace_every)
        if trace_every:
            P = -(-n // trace_every)
            out = np.zeros(len(self.specs) * P, dtype=np.uint64)
            _check(lib.qz_batch_run(self._h, n, trace_every,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
            return out.view(np.int64).reshape(len(self.specs), P)
        _check(lib.qz_batch_run(self._h, n, 0, None))
        return None

    def replace(self, slot: int, L: int, seed: int, t_max: int = 0) -> None:
        """Put a new replica (side L up to the slot's original side) into a slot."""
        spec = _spec((L, seed, t_max))
        _check(lib.qz_batch_slot_replace(self._h, slot, ctypes.byref(spec)))
        self.specs[slot] = (int(L), int(seed))

    def tuning(self) -> dict:
        """The launch shape in use: {"source", "graph_sweeps", "tz": {L: Tz}}."""
        import json
        buf = ctypes.create_string_buffer(4096)
        _check(lib.qz_batch_tuning_json(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def sync(self) -> None:
        _check(lib.qz_batch_sync(self._h))

    def reset(self, slot: int, seed: int) -> None:
        _check(lib.qz_batch_slot_reset(self._h, slot, int(seed) & (2**64 - 1)))
        self.specs[slot] = (self.specs[slot][0], int(seed))

    def set_active(self, slot: int, active: bool) -> None:
        _check(lib.qz_batch_slot_active(self._h, slot, 1 if active else 0))

    def time(self, slot: int) -> int:
        v = ctypes.c_uint64()
        _check(lib.qz_batch_slot_time(self._h, slot, ctypes.byref(v)))
        return int(v.value)

    def trace(self, slot: int, t_from: int, count: int) -> np.ndarray:
        out = np.zeros(count, dtype=np.uint64)
        _check(lib.qz_batch_trace(self._h, slot, t_from, count,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out

    def download(self, slot: int) -> np.ndarray:
        L = self.specs[slot][0]
        out = np.empty((L, L, L), dtype=np.int8)
        _check(lib.qz_batch_download(self._h, slot,
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))))
        return out

    def bonds(self, slot: int) -> np.ndarray:
        out = np.zeros(3, dtype=np.uint64)
        _check(lib.qz_batch_bonds(self._h, slot, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out.astype(np.int64)

    def corr(self, slot: int):
        L = self.specs[slot][0]
        S = np.zeros((3, L // 2 + 1), dtype=np.int64)
        M = ctypes.c_int64()
        _check(lib.qz_batch_corr(self._h, slot, S.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 ctypes.byref(M)))
        return S, int(M.value)

    def set_tuning(self, L: int, Tz: int, graph_sweeps: int) -> None:
        _check(lib.qz_batch_set_tuning(self._h, L, Tz, graph_sweeps))
