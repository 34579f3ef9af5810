"""The FP64 sums of lbm_macros against values computed from the oracle's own
fields: mass and momentum (sum rho, sum rho u over the fluid) and the residual
||u(t) - u(t - k)|| / ||u(t)|| between two calls k steps apart (the relative L2
form of Sec. III.B's error metric), on a flow with a net momentum (the channel
with inlet and cylinder) and on the forced 3D packing."""
import numpy as np
import pytest

from tests.gpu_cases import Case, channel_case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _oracle_sums(sim, D):
    rho, u = sim.macros()
    fl = sim.fluid
    return rho[fl].sum(), (rho[fl][None, :] * u[:D, fl]).sum(axis=1), u[:D, fl]


@pytest.mark.parametrize("which", ["channel", "packing"])
def test_sums_and_residual_against_oracle(gpu_lib, which):
    if which == "channel":
        case = channel_case()
    else:
        import synth
        c, r = synth.sphere_packing(n=40, r_min=4.0, r_max=7.0, solid_fraction=0.35, seed=21)
        case = Case("D3Q19", (40, 40, 40), spheres=[(cc, rr, True, None, None) for cc, rr in zip(c, r)], tau=0.9,
                    force=(1e-5, 2e-6, 0.0))
    _say("case sums", which, "f64")
    d, _, _ = case.gpu(gpu_lib, "f64")
    sim = case.oracle()
    D = d.D
    d.step(100)
    sim.run(100)
    _, _, s1, _ = d.macros(fields=False)
    _, _, u1 = _oracle_sums(sim, D)
    # first call: the residual is taken against the initial field (u0 + F / (2 rho0))
    u_init = np.array(case.u0[:D])[:, None] + 0.5 * np.array(case.force[:D])[:, None] / case.rho0
    r1 = np.linalg.norm(u1 - u_init) / np.linalg.norm(u1)
    assert abs(s1[-1] / r1 - 1) < 1e-10
    for k in (40, 7):
        d.step(k)
        sim.run(k)
        _, _, s2, unstable = d.macros(fields=False)
        mass, mom, u2 = _oracle_sums(sim, D)
        res = np.linalg.norm(u2 - u1) / np.linalg.norm(u2)
        _say("lag", k, "mass", s2[0], mass, "momentum", s2[1:1 + D], mom, "residual", s2[-1], res)
        assert not unstable
        assert abs(s2[0] / mass - 1) < 1e-13
        np.testing.assert_allclose(s2[1:1 + D], mom, rtol=1e-10, atol=1e-12 * np.abs(mom).max())
        assert res > 0 and abs(s2[-1] / res - 1) < 1e-8
        u1 = u2
    d.close()
