"""The streaming-copy measurement hook (pdn_stream_copy): exact copies of
ragged sizes (not a multiple of the 16 KiB a workgroup moves), nothing
written past the end, and the documented rejections.  Device memory comes
from the HIP runtime directly."""
import ctypes as C
import sys

import numpy as np
import pytest

import paper_2301_05552_amd as pdn

pytestmark = pytest.mark.gpu


def _hip():
    h = C.CDLL("libamdhip64.so")
    h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    h.hipFree.argtypes = [C.c_void_p]
    h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    h.hipDeviceSynchronize.argtypes = []
    return h


def test_stream_copy_ragged_sizes_and_errors():
    print("[gpu case] stream copy ragged sizes", flush=True)
    sys.stdout.flush()
    h = _hip()
    n = (3 << 20) + 7 * 1024 + 48                      # bytes: 3 MiB + 7 KiB + 48
    cap = n + 64
    src, dst = C.c_void_p(), C.c_void_p()
    assert h.hipMalloc(C.byref(src), cap) == 0 and h.hipMalloc(C.byref(dst), cap) == 0
    try:
        a = np.random.default_rng(1).integers(1, 255, cap, dtype=np.uint8)
        zero = np.zeros(cap, np.uint8)
        assert h.hipMemcpy(src, a.ctypes.data_as(C.c_void_p), cap, 1) == 0          # host to device
        for nb in (0, 16, 4096, 16384 + 16, n):
            assert h.hipMemcpy(dst, zero.ctypes.data_as(C.c_void_p), cap, 1) == 0
            pdn.stream_copy(src.value, dst.value, nb)
            assert h.hipDeviceSynchronize() == 0
            out = np.empty(cap, np.uint8)
            assert h.hipMemcpy(out.ctypes.data_as(C.c_void_p), dst, cap, 2) == 0    # device to host
            assert np.array_equal(out[:nb], a[:nb])
            assert not out[nb:].any()                                               # nothing past the end
        with pytest.raises(pdn.PdnError):
            pdn.stream_copy(src.value, dst.value, 24)                # not a multiple of 16
        with pytest.raises(pdn.PdnError):
            pdn.stream_copy(src.value + 8, dst.value, 32)            # misaligned
    finally:
        h.hipFree(src)
        h.hipFree(dst)
