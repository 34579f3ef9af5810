"""lbm_macros_noalloc (the moments entry point that allocates nothing: its
partial sums live in a file-scope device array) against lbm_macros, through the
C-ABI, on two calls in a row -- the second on a smaller domain -- and with a
non-finite population."""
import numpy as np
import pytest

from tests.gpu_cases import annulus_case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _compare(B, d):
    import torch
    rho_h, u_h, sums_h, unstable = d.macros()
    N, D = d.N, d.D
    rho = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    u = torch.full((N, D), float("nan"), dtype=torch.float64, device="cuda")
    sums = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    d.macros_noalloc(rho, u, sums)
    torch.cuda.synchronize()
    rho, u, sums = rho.cpu().numpy(), u.cpu().numpy(), sums.cpu().numpy()
    assert np.array_equal(rho, rho_h, equal_nan=True)      # the same per-node arithmetic
    assert np.array_equal(u, u_h, equal_nan=True)
    mom = list(sums_h[1:1 + D]) + [0.0] * (3 - D)
    np.testing.assert_allclose(sums[:4], [sums_h[0]] + mom, rtol=1e-12, atol=1e-15 * np.nan_to_num(abs(sums_h[0])))
    assert sums[4] == 0.0 and sums[7] == 0.0
    np.testing.assert_allclose(sums[5], (u_h ** 2).sum(), rtol=1e-12)
    return sums, unstable


def test_noalloc_matches_macros_twice_smaller_second(gpu_lib):
    B = gpu_lib
    for scale, steps in ((2.0, 120), (1.0, 60)):              # the second call on a smaller domain
        _say("case annulus scale", scale, "f64")
        d, _, _ = annulus_case(scale=scale).gpu(B, "f64", "FQ")
        d.step(steps)
        sums, unstable = _compare(B, d)
        assert not unstable and sums[6] == 0.0
        d.close()


def test_noalloc_packing_f32_and_non_finite_count(gpu_lib):
    from paper_2009_04604_amd import workloads as W
    B = gpu_lib
    _say("case packing 64^3 f32")
    d, mask, _ = W.packing_domain(64, "f32")
    d.step(30)
    _compare(B, d)
    f = d.get_state()
    n = int(np.flatnonzero(mask)[17])
    f[3, n] = np.nan
    d.set_state(f)
    sums, unstable = _compare(B, d)
    assert unstable and sums[6] == 1.0
    d.close()
