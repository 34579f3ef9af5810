"""Special-case pin: at q = 1/2 every fragmented and quadratic ELIBB variant
reduces to half-way bounce-back with Ladd's moving-wall term (Sec. II.B-E,
eq. ME-solid-to-fluid).  The expected result is a textbook half-way
bounce-back BGK step written here with plain loops over nodes and directions,
independently of the oracle's vectorised code."""
import numpy as np
import pytest

from tests import cases

C = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)]
W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
OPP = [C.index((-a, -b)) for a, b in C]


def textbook_step(f, nx, ny, tau, u_top):
    """f[i][y][x] -> one BGK step with half-way bounce-back at y = -1/2 (rest) and
    y = ny - 1/2 (moving at u_top); periodic in x."""
    fs = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
    rho = [[0.0] * nx for _ in range(ny)]
    for y in range(ny):
        for x in range(nx):
            r = sum(f[i][y][x] for i in range(9))
            ux = sum(f[i][y][x] * C[i][0] for i in range(9)) / r
            uy = sum(f[i][y][x] * C[i][1] for i in range(9)) / r
            rho[y][x] = r
            for i in range(9):
                cu = C[i][0] * ux + C[i][1] * uy
                feq = W[i] * r * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
                fs[i][y][x] = f[i][y][x] - (f[i][y][x] - feq) / tau
    out = [[[0.0] * nx for _ in range(ny)] for _ in range(9)]
    for y in range(ny):
        for x in range(nx):
            for i in range(9):
                sx, sy = (x - C[i][0]) % nx, y - C[i][1]
                if 0 <= sy < ny:
                    out[i][y][x] = fs[i][sy][sx]
                else:
                    uw = u_top if sy >= ny else (0.0, 0.0)
                    cu = C[i][0] * uw[0] + C[i][1] * uw[1]
                    out[i][y][x] = fs[OPP[i]][y][x] + 6.0 * W[i] * rho[y][x] * cu
    return out


@pytest.mark.parametrize("variant", ["FQ", "F", "UQ", "HWBB"])
def test_half_way_step_matches_textbook(variant):
    nx, ny, tau, U = 5, 4, 0.7, (0.02, 0.0)
    sim = cases.channel(nx, ny, q=0.5, u_top=(U[0], U[1], 0.0), tau=tau, variant=variant)
    rng = np.random.default_rng(11)
    sim.f = sim.f * (1.0 + 0.05 * rng.standard_normal(sim.f.shape))
    f_list = [[[float(sim.f[i, x + nx * y]) for x in range(nx)] for y in range(ny)] for i in range(9)]
    for _ in range(3):
        f_list = textbook_step(f_list, nx, ny, tau, U)
        sim.step()
    expect = np.array([[f_list[i][y][x] for y in range(ny) for x in range(nx)] for i in range(9)])
    np.testing.assert_allclose(sim.f, expect, rtol=1e-14, atol=1e-16)
