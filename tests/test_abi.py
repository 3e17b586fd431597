"""Host-only checks of the C ABI: the built library loads, exports every entry
point the header declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "quench.h")
LIB = os.path.join(ROOT, "paper_2305_12161_amd", "libquench.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qz_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_expected_calls():
    names = declared_functions()
    # the single-lattice and batch calls of the boundary
    for need in ("qz_create", "qz_run", "qz_bonds", "qz_corr", "qz_time", "qz_destroy",
                 "qz_state_bytes", "qz_download_spins", "qz_upload_spins", "qz_download_window",
                 "qz_status_string", "qz_last_error", "qz_batch_state_bytes", "qz_batch_create",
                 "qz_batch_run", "qz_batch_slot_replace", "qz_batch_destroy"):
        assert need in names


class _Spec(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("t_max", ctypes.c_uint64)]


def test_batch_rejects_bad_arguments_without_device(lib):
    """Batch creation checks sizes, memory and the tuning text before any
    device work: a well-formed text gets as far as the memory check."""
    lib.qz_batch_state_bytes.restype = ctypes.c_size_t
    lib.qz_batch_state_bytes.argtypes = [ctypes.POINTER(_Spec), ctypes.c_size_t, ctypes.c_uint32]
    lib.qz_batch_create.restype = ctypes.c_int
    lib.qz_batch_create.argtypes = [ctypes.POINTER(_Spec), ctypes.c_size_t, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p, ctypes.c_char_p,
                                    ctypes.POINTER(ctypes.c_void_p)]
    specs = (_Spec * 3)(_Spec(64, 1, 0), _Spec(128, 2, 1000), _Spec(256, 3, 0))
    need = lib.qz_batch_state_bytes(specs, 3, 16)
    assert need >= 2 * (64 ** 3 + 128 ** 3 + 256 ** 3) // 8
    bad = (_Spec * 1)(_Spec(96, 1, 0))
    assert lib.qz_batch_state_bytes(bad, 1, 16) == 0
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: every call below fails first
    args = (specs, 3, 4, 16, fake)
    assert lib.qz_batch_create(bad, 1, 4, 16, fake, 1 << 30, None, None, ctypes.byref(h)) == -5
    assert lib.qz_batch_create(specs, 3, 4, 0, fake, 1 << 30, None, None, ctypes.byref(h)) == -1
    for text in (b"", b"{", b'{"tz": {"64": 3}}', b'{"tz": {"96": 8}}', b'{"graph": 5}',
                 b'{"graph_sweeps": -1}', b'{"tz": {"64": 8}} x', b'{"tz": [8]}'):
        assert lib.qz_batch_create(*args, 1 << 30, None, text, ctypes.byref(h)) == -1, text
    for text in (None, b"{}", b'{"graph_sweeps": 100, "tz": {"64": 8, "128": 16, "256": 4}}',
                 b' { "tz" : { } , "graph_sweeps" : 0 } '):
        assert lib.qz_batch_create(*args, need - 1, None, text, ctypes.byref(h)) == -2, text


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_abi_version_and_sizes(lib):
    lib.qz_abi_version.restype = ctypes.c_int
    assert lib.qz_abi_version() == 2
    lib.qz_state_bytes.restype = ctypes.c_size_t
    lib.qz_state_bytes.argtypes = [ctypes.c_uint32, ctypes.c_int]
    # int8: N bytes of spins; bit: two copies of N/8 bytes
    assert lib.qz_state_bytes(32, 0) >= 32 ** 3
    assert lib.qz_state_bytes(2048, 1) >= 2 * 2048 ** 3 // 8
    assert lib.qz_state_bytes(2048, 1) < 2 * 2048 ** 3 // 8 + (64 << 20)
    assert lib.qz_state_bytes(7, 0) == 0          # odd L
    assert lib.qz_state_bytes(2, 0) == 0          # L < 4
    assert lib.qz_state_bytes(96, 1) == 0         # bit layout needs L % 64 == 0
    assert lib.qz_state_bytes(96, 0) > 0
    assert lib.qz_state_bytes(64, 5) == 0         # unknown layout


def test_create_rejects_bad_arguments_without_device(lib):
    lib.qz_create.restype = ctypes.c_int
    lib.qz_create.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.qz_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: every call below fails first
    assert lib.qz_create(7, 1, 0, fake, 1 << 30, None, ctypes.byref(h)) == -1
    assert lib.qz_create(96, 1, 1, fake, 1 << 30, None, ctypes.byref(h)) == -5
    assert lib.qz_create(64, 1, 3, fake, 1 << 30, None, ctypes.byref(h)) == -1
    assert lib.qz_create(64, 1, 1, None, 1 << 30, None, ctypes.byref(h)) == -1
    assert lib.qz_create(64, 1, 1, fake, 16, None, ctypes.byref(h)) == -2
    assert lib.qz_create(64, 1, 1, fake, 1 << 30, None, None) == -1
    assert b"" != lib.qz_last_error()


def test_status_strings(lib):
    lib.qz_status_string.restype = ctypes.c_char_p
    lib.qz_status_string.argtypes = [ctypes.c_int]
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.qz_status_string(code)
    assert lib.qz_status_string(-99) == b"unknown status"


def test_null_handle_calls(lib):
    lib.qz_run.restype = ctypes.c_int
    lib.qz_run.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
    assert lib.qz_run(None, 1, 0, None) == -1
    assert lib.qz_destroy(None) == -1


def test_binding_rejects_negative_counts():
    """A negative sweep count or cadence would reach the library as a huge
    unsigned count (a run that does not end): the binding refuses it."""
    from paper_2305_12161_amd import binding
    assert binding._counts(5, 2) == (5, 2)
    for bad in ((-1, 0), (10, -5), (-180, 0)):
        with pytest.raises(ValueError):
            binding._counts(*bad)
