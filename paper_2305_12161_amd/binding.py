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
        "qz_bonds": ([vp, c.POINTER(u64)], i32),
        "qz_corr": ([vp, c.POINTER(c.c_int64), c.POINTER(c.c_int64)], i32),
        "qz_time": ([vp, c.POINTER(u64)], i32),
        "qz_download_spins": ([vp, c.POINTER(c.c_int8)], i32),
        "qz_upload_spins": ([vp, c.POINTER(c.c_int8), u64], i32),
        "qz_download_window": ([vp, c.POINTER(u32), u32, c.POINTER(c.c_int8)], i32),
        "qz_set_tuning": ([vp, i32, i32, i32], i32),
        "qz_get_tuning": ([vp, c.POINTER(i32)], i32),
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
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream, sh = _stream_handle(stream)
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
        if trace_every:
            out = np.zeros(n // trace_every, dtype=np.uint64)
            _check(lib.qz_run(self._h, n, trace_every,
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
            return out
        _check(lib.qz_run(self._h, n, 0, None))
        return np.zeros(0, dtype=np.uint64)

    def run_device(self, n: int, trace_every: int, dev_trace) -> None:
        """Asynchronous run; dev_trace is a torch int64/uint64 device tensor."""
        ptr = ctypes.c_void_p(dev_trace.data_ptr()) if dev_trace is not None else None
        _check(lib.qz_run_device(self._h, n, trace_every, ptr))

    def bonds(self) -> np.ndarray:
        out = np.zeros(3, dtype=np.uint64)
        _check(lib.qz_bonds(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out.astype(np.int64)

    def corr(self):
        R = self.L // 2 + 1
        S = np.zeros((3, R), dtype=np.int64)
        M = ctypes.c_int64()
        _check(lib.qz_corr(self._h, S.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
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

    def tuning(self):
        out = (ctypes.c_int * 3)()
        _check(lib.qz_get_tuning(self._h, out))
        return tuple(int(v) for v in out)
