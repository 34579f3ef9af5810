"""GPU parity at the edges of the wall distance q (Sec. II.D: the variants'
branches at q = 1/2, the cutoff q_min = 0.01 below which the quadratic variants
fall back to ELIBB-F, the limit q = 1, and the smallest q the builders give a
node on the wall, 1e-12): plane walls at distance q in a forced channel with a
sliding top wall, every variant, FP64 against the oracle."""
import numpy as np
import pytest

from tests.gpu_cases import Case, fluid_velocity_error

pytestmark = pytest.mark.gpu

QS = [1e-12, 0.005, 0.01, 0.5, 1.0]
VARIANTS = ["FQ", "F", "UQ", "U", "HWBB"]


def _case(q):
    return Case("D2Q9", (6, 12, 1), periodic=(True, False, True),
                faces=[(2, q, None, 0), (3, q, (0.02, 0.0, 0.0), 0)], tau=1.2, force=(2e-6, 0.0, 0.0), rho0=1.01)


@pytest.mark.parametrize("q", QS)
def test_plane_walls_at_edge_q_every_variant(gpu_lib, q):
    for v in VARIANTS:
        print("case plane walls q", q, "variant", v, flush=True)
        case = _case(q)
        d, _, links = case.gpu(gpu_lib, "f64", v)
        assert np.abs(links["q"] - q).max() <= 1e-15 + 1e-12 * q
        sim = case.oracle(v)
        d.step(200)
        sim.run(200)
        err, rho_g, rho_o, _, unstable = fluid_velocity_error(d, sim)
        d.close()
        assert not unstable
        assert err <= 1e-12, (q, v, err)
        np.testing.assert_allclose(rho_g, rho_o, rtol=1e-13)
