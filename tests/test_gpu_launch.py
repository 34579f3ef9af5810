"""Launch options change nothing but speed: both XCD deals of the step kernel's
workgroups (hardware round-robin, contiguous eighths) give bit-identical states
on both layouts; the FP64 sums of lbm_macros agree to rounding; values outside
the documented set are rejected."""
import numpy as np
import pytest

import synth
from tests.gpu_cases import Case, annulus_case

pytestmark = pytest.mark.gpu

DEALS = (0, 1)


def _say(*a):
    print(*a, flush=True)


def _packing():
    n = 40
    c, r = synth.sphere_packing(n=n, r_min=3.0, r_max=6.0, solid_fraction=0.4, seed=5)
    return Case("D3Q19", (n, n, n), spheres=[(cc, rr, True, None, None) for cc, rr in zip(c, r)],
                tau=0.9, force=(1e-4, 2e-5, 0.0))


@pytest.mark.parametrize("layout", ["compact", "dense"])
@pytest.mark.parametrize("which", ["annulus", "packing"])
def test_xcd_deal_changes_nothing(gpu_lib, which, layout):
    case = annulus_case() if which == "annulus" else _packing()
    states, sums = [], []
    for deal in DEALS:
        _say("case", which, layout, "xcd deal", deal)
        d, _, _ = case.gpu(gpu_lib, "f32", layout=layout)
        d.set_launch_option(0, deal)
        d.step(40)
        states.append(d.get_state())
        sums.append(d.macros(fields=False)[2])
        d.close()
    for s in states[1:]:
        assert np.array_equal(s, states[0])
    for s in sums[1:]:
        np.testing.assert_allclose(s[:-1], sums[0][:-1], rtol=1e-12, atol=1e-12)


def test_invalid_deal_rejected(gpu_lib):
    B = gpu_lib
    d, _, _ = annulus_case().gpu(B, "f32")
    for v in (-1, 2, 64):
        with pytest.raises(B.LBMError) as e:
            d.set_launch_option(0, v)
        assert e.value.code == B.LBM_EINVAL
    with pytest.raises(B.LBMError):
        d.set_launch_option(1, 0)
    d.close()
