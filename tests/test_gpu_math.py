"""The device's refined special functions against their stated error bounds
(the host build of the kernels' code divides and takes square roots
exactly, so only the device can check these): the values come from
scvt_calib_math (libscvt_calib.so), which evaluates the very functions the
geometry and quadrature kernels call.  References: numpy's correctly
rounded FP64 division and square root (their own half-ulp rounding is
inside every bound checked)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ULP = 2.0 ** -52


@pytest.fixture(scope="module")
def device_math():
    from paper_1709_06924_amd import build
    import paper_1709_06924_amd.scvt  # noqa: F401  (fails loudly without libscvt)
    lib = ctypes.CDLL(build.CALIB_LIB)
    lib.scvt_calib_math.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    lib.scvt_calib_math.restype = ctypes.c_int

    def run(x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros((len(x), 9))
        assert lib.scvt_calib_math(len(x), x.ctypes.data, out.ctypes.data) == 0
        return out
    return run


def rel(a, b):
    return np.abs(a - b) / np.abs(b)


def test_fp64_refined_functions(device_math):
    rng = np.random.default_rng(41)
    x = np.exp(rng.uniform(np.log(1e-12), np.log(1e6), 200000))
    out = device_math(x)
    rs = 1.0 / np.sqrt(x)
    print("rsq_pos %.2e rcp_fast %.2e sqrt_fast %.2e rcp_nr %.2e sqrt_nr %.2e"
          % (rel(out[:, 0], rs).max(), rel(out[:, 1], 1 / x).max(), rel(out[:, 2], np.sqrt(x)).max(),
             rel(out[:, 3], 1 / x).max(), rel(out[:, 4], np.sqrt(x)).max()), flush=True)
    # one second-order correction of the estimate: about an ulp
    assert rel(out[:, 0], rs).max() <= 3 * ULP
    # two Newton steps: about an ulp; x times rsq_pos: two roundings more
    assert rel(out[:, 1], 1 / x).max() <= 3 * ULP
    assert rel(out[:, 2], np.sqrt(x)).max() <= 5 * ULP
    # one Newton step (stated 2^-46, for 1 <= x < 2^1010) and the first-order
    # square root (stated 2.2e-14)
    big = x >= 1.0
    assert rel(out[big, 3], 1 / x[big]).max() <= 2.0 ** -46
    assert rel(out[:, 4], np.sqrt(x)).max() <= 2.2e-14


def test_reciprocal_square_root_near_one(device_math):
    """|p|^-1 of the quadrature: the binomial series within 1e-4 of 1 (next
    term below 3e-17), else rsq_pos."""
    rng = np.random.default_rng(42)
    x = np.concatenate([1.0 - rng.uniform(0, 1e-4, 100000), 1.0 - rng.uniform(1e-4, 0.2, 100000),
                        1.0 + rng.uniform(0, 1e-4, 1000)])
    out = device_math(x)
    r = rel(out[:, 5], 1.0 / np.sqrt(x))
    print("rsq_near1 %.2e" % r.max(), flush=True)
    assert r.max() <= 3 * ULP


def test_fp32_hardware_functions(device_math):
    """The mixed path's FP32 rsqrt, reciprocal and 2^x: about one FP32 ulp
    (2^-23) on positive normal arguments (2^x over the range the split
    logistic uses)."""
    rng = np.random.default_rng(43)
    xf = np.exp(rng.uniform(np.log(1e-6), np.log(1e6), 100000)).astype(np.float32).astype(np.float64)
    out = device_math(xf)
    e32 = 2.0 ** -23
    r_rsq = rel(out[:, 6], 1.0 / np.sqrt(xf)).max()
    r_rcp = rel(out[:, 7], 1.0 / xf).max()
    u = rng.uniform(-60, 60, 100000).astype(np.float32).astype(np.float64)
    out2 = device_math(u)
    r_exp = rel(out2[:, 8], np.exp2(u)).max()
    print("rsqf %.2e rcpf %.2e exp2 %.2e (FP32 ulp %.2e)" % (r_rsq, r_rcp, r_exp, e32), flush=True)
    assert r_rsq <= 2 * e32 and r_rcp <= 2 * e32 and r_exp <= 2 * e32
