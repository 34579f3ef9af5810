"""Pins of the oracle's velocity sets and equilibrium (Sec. II.A, eq. Eq2ndOrder).

The expected values are the defining moment identities of a Gauss-Hermite
lattice with c_s^2 = 1/3, evaluated in exact rational arithmetic for the
weights, and the moments the second-order equilibrium must reproduce.
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest

from oracle import lattice, solver

LATS = [lattice.D2Q9, lattice.D3Q19, lattice.D3Q27]


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_moment_identities_exact(lat):
    w = lat.w_exact
    c = lat.c
    d = lat.d
    assert sum(w) == 1
    for a in range(3):
        assert sum(wi * int(ci[a]) for wi, ci in zip(w, c)) == 0
    for a, b in itertools.product(range(d), repeat=2):
        m2 = sum(wi * int(ci[a]) * int(ci[b]) for wi, ci in zip(w, c))
        assert m2 == (Fraction(1, 3) if a == b else 0)
    for a, b, g in itertools.product(range(d), repeat=3):
        assert sum(wi * int(ci[a] * ci[b] * ci[g]) for wi, ci in zip(w, c)) == 0
    # fourth-order isotropy: sum w c_a c_b c_g c_d = cs^4 (d_ab d_gd + d_ag d_bd + d_ad d_bg)
    cs4 = Fraction(1, 9)
    for a, b, g, e in itertools.product(range(d), repeat=4):
        m4 = sum(wi * int(ci[a] * ci[b] * ci[g] * ci[e]) for wi, ci in zip(w, c))
        iso = cs4 * ((a == b) * (g == e) + (a == g) * (b == e) + (a == e) * (b == g))
        assert m4 == iso


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_direction_table(lat):
    assert lat.q == {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}[lat.name]
    assert (lat.c[0] == 0).all()
    assert len({tuple(v) for v in lat.c}) == lat.q
    for i in range(lat.q):
        assert (lat.c[lat.opp[i]] == -lat.c[i]).all()
        assert lat.w[lat.opp[i]] == lat.w[i]
    if lat.name == "D2Q9":
        assert [tuple(v[:2]) for v in lat.c] == [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1)]
    else:
        assert [tuple(v) for v in lat.c[1:7]] == [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
        assert [tuple(v) for v in lat.c[7:11]] == [(1, 1, 0), (1, -1, 0), (-1, 1, 0), (-1, -1, 0)]
        assert [tuple(v) for v in lat.c[11:15]] == [(1, 0, 1), (1, 0, -1), (-1, 0, 1), (-1, 0, -1)]
        assert [tuple(v) for v in lat.c[15:19]] == [(0, 1, 1), (0, 1, -1), (0, -1, 1), (0, -1, -1)]
        if lat.name == "D3Q27":
            assert [tuple(v) for v in lat.c[19:]] == [(1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1),
                                                     (-1, 1, 1), (-1, 1, -1), (-1, -1, 1), (-1, -1, -1)]


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_equilibrium_moments(lat):
    rng = np.random.default_rng(0)
    n = 50
    rho = 0.8 + 0.4 * rng.random(n)
    u = 0.1 * (rng.random((3, n)) - 0.5)
    if lat.d == 2:
        u[2] = 0
    feq = solver.equilibrium(lat, rho, u)
    c = lat.c.astype(float)
    np.testing.assert_allclose(feq.sum(0), rho, rtol=1e-14)
    np.testing.assert_allclose(c.T @ feq, rho * u, atol=1e-15)
    for a in range(lat.d):
        for b in range(lat.d):
            m = (c[:, a] * c[:, b]) @ feq
            np.testing.assert_allclose(m, rho * ((a == b) / 3.0 + u[a] * u[b]), rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_guo_source_moments(lat):
    rng = np.random.default_rng(1)
    u = 0.05 * rng.standard_normal((3, 7))
    F = np.array([1e-3, -2e-3, 5e-4]) if lat.d == 3 else np.array([1e-3, -2e-3, 0.0])
    if lat.d == 2:
        u[2] = 0
    S = solver.guo_source(lat, u, F)
    c = lat.c.astype(float)
    np.testing.assert_allclose(S.sum(0), 0.0, atol=1e-18)
    np.testing.assert_allclose(c.T @ S, np.repeat(F[:, None], 7, 1), rtol=1e-12, atol=1e-18)
    # second moment of Guo's term: sum c_a c_b S = u_a F_b + u_b F_a
    for a in range(lat.d):
        for b in range(lat.d):
            np.testing.assert_allclose((c[:, a] * c[:, b]) @ S, u[a] * F[b] + u[b] * F[a], atol=1e-17)
