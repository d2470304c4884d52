"""scvt_refine_noalloc (static device scratch, no allocation) against
scvt_refine through the C ABI: bit-identical refined generators on two
calls in a row, the second with a smaller handle, and the size limit.

The output buffer is the caller's: it is allocated here with the HIP
runtime the library itself links (not torch's bundled one)."""
import ctypes

import numpy as np
import pytest

import paper_1709_06924_amd.inputs as I

pytestmark = pytest.mark.gpu


class DeviceBuffer:
    """A device allocation of the HIP runtime libscvt.so uses."""

    def __init__(self, nbytes):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.ptr = ctypes.c_void_p()
        assert self.hip.hipMalloc(ctypes.byref(self.ptr), ctypes.c_size_t(nbytes)) == 0
        self.nbytes = nbytes

    def fill_nan(self):
        # 0xFF bytes: a NaN in every double
        assert self.hip.hipMemset(self.ptr, ctypes.c_int(0xFF), ctypes.c_size_t(self.nbytes)) == 0

    def to_host(self, shape):
        out = np.empty(shape, dtype=np.float64)
        assert out.nbytes <= self.nbytes
        assert self.hip.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), self.ptr,
                                  ctypes.c_size_t(out.nbytes), ctypes.c_int(2)) == 0  # D2H
        return out

    def free(self):
        self.hip.hipFree(self.ptr)


def test_refine_noalloc_matches_refine():
    from paper_1709_06924_amd import scvt
    d = I.density_tanh(I.latlon(30, 90), 0.5, 0.2, 8)
    for n, seed in ((40962, 31), (5003, 32)):  # second call: smaller input
        print("refine_noalloc n", n, flush=True)
        S = scvt.Solver(I.uniform_sphere(n, seed), d, m_hist=5)
        S.step()
        want = S.refine()
        m = ctypes.c_int64(0)
        assert scvt._lib.scvt_refine_noalloc(S.h, None, ctypes.byref(m)) == 0
        assert m.value == want.shape[0] == 4 * n - 6
        buf = DeviceBuffer(3 * 8 * m.value)
        buf.fill_nan()
        m2 = ctypes.c_int64(0)
        assert scvt._lib.scvt_refine_noalloc(S.h, buf.ptr, ctypes.byref(m2)) == 0
        assert m2.value == m.value
        got = buf.to_host((m.value, 3))
        buf.free()
        assert np.array_equal(got, want)
        # the handle's state is unchanged by either call
        F = S.energy()[0]
        S.step()
        assert S.energy()[0] <= F
        S.close()


def test_refine_noalloc_rejects_sizes_beyond_its_scratch():
    from paper_1709_06924_amd import scvt
    n = scvt.REFINE_NOALLOC_MAX_N + 1
    print("refine_noalloc limit n", n, flush=True)
    S = scvt.Solver(I.uniform_sphere(n, 33), None, m_hist=0)
    m = ctypes.c_int64(0)
    assert scvt._lib.scvt_refine_noalloc(S.h, None, ctypes.byref(m)) == -2
    S.close()
