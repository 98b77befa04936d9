"""The entry point that allocates nothing (spock_apply_T_noalloc) against
spock_apply_T: the same kernels with their scratch in the library's static
device array, so every entry of T(z, eta) and both residual maxima must be
bitwise equal, in float64 and float32.  Two calls in a row on different
problems, the second smaller, so the second runs on what the first left in
the array."""
import numpy as np
import pytest

from paper_2505_12078_amd import spock as S
from paper_2505_12078_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need an MI355X; none is visible")
    S.load()


def _compare(prob, seed, precision):
    import torch
    dt = torch.float64 if precision == S.FP64 else torch.float32
    rng = np.random.default_rng(seed)
    with S.Problem(prob) as P:
        P.set_x0(prob["x0"])
        z = rng.standard_normal(P.nz) * 2
        e = rng.standard_normal(P.neta) * 2
        if precision == S.FP32:  # both paths then start from the same float32 values
            z = z.astype(np.float32).astype(np.float64)
            e = e.astype(np.float32).astype(np.float64)
        zr, er, xir = P.apply_T(z, e, precision)
        zt = torch.tensor(z, dtype=dt, device="cuda")
        et = torch.tensor(e, dtype=dt, device="cuda")
        # outputs start as a sentinel: every entry must be written by the step
        zo = torch.full((P.nz,), 12345.0, dtype=dt, device="cuda")
        eo = torch.full((P.neta,), 12345.0, dtype=dt, device="cuda")
        torch.cuda.synchronize()
        xi = P.apply_T_noalloc(zt.data_ptr(), et.data_ptr(), zo.data_ptr(), eo.data_ptr(), precision)
        zg = zo.cpu().double().numpy()
        eg = eo.cpu().double().numpy()
        # the inputs are read only
        assert np.array_equal(zt.cpu().double().numpy(), z) and np.array_equal(et.cpu().double().numpy(), e)
    print("n=%d precision=%d max|dz|=%.3g max|deta|=%.3g xi=%s ref=%s" % (
        prob["parent"].size, precision, np.abs(zg - zr).max(), np.abs(eg - er).max(), xi, xir))
    assert np.array_equal(zg, zr) and np.array_equal(eg, er)
    assert np.array_equal(xi, xir)


@pytest.mark.parametrize("precision", [S.FP64, S.FP32])
def test_noalloc_step_equals_apply_T_twice_second_smaller(precision):
    _compare(W.config_problem(1), 5, precision)   # 229 nodes, nx = 20, nu = 10
    _compare(W.config_problem(0), 6, precision)   # 15 nodes, nx = 2, nu = 1


@pytest.mark.parametrize("precision", [S.FP64, S.FP32])
def test_noalloc_step_with_general_formulation(precision):
    """The same with the node kernels built for the general formulation: a
    spectral risk given as conic data, then an l1 input penalty (smaller)."""
    _compare(W.spectral_risk(W.random_ragged_problem(4, N=3, nx=3, nu=2), weight=0.4), 7, precision)
    _compare(W.l1_input_penalty(W.random_ragged_problem(7, N=2, nx=3, nu=2, ball=False), 2.0), 8, precision)


def test_noalloc_rejects_aliasing_and_bad_precision():
    import torch
    prob = W.config_problem(0)
    with S.Problem(prob) as P:
        z = torch.zeros(P.nz, dtype=torch.float64, device="cuda")
        e = torch.zeros(P.neta, dtype=torch.float64, device="cuda")
        o = torch.zeros(P.neta, dtype=torch.float64, device="cuda")
        with pytest.raises(S.SpockError) as ex:
            P.apply_T_noalloc(z.data_ptr(), e.data_ptr(), z.data_ptr(), o.data_ptr())
        assert ex.value.code == S.SPOCK_E_INVALID
        with pytest.raises(S.SpockError) as ex:
            P.apply_T_noalloc(z.data_ptr(), e.data_ptr(), o.data_ptr(), o.data_ptr() + 8, S.MIXED)
        assert ex.value.code == S.SPOCK_E_INVALID
