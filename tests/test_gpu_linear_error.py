"""The paper's linear-error comparison along the x-axis (Sec. III.B, eq. LE and
eq. rRMSErotatingCylinders: cylindrical Couette, beta = 1/2, TRT with Lambda =
3/16, Re = 10) at r2 - r1 = 40 lu: the ELIBB variants on the GPU path (FP64)
against the oracle-only BFL comparator stored by tests/golden/make_fixtures.py
(e3); r2 - r1 = 10 is covered on the CPU (tests/test_oracle_bfl.py)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "e3_bfl_linear_error.npz")


def _gpu_axis(B, width, variant, tau=0.8, magic=3.0 / 16.0, Re=10.0):
    r1, r2 = float(width), 2.0 * width
    L = int(2 * r2 + 8)
    c = (L / 2.0, L / 2.0, 0.0)
    nu = (tau - 0.5) / 3
    om1 = Re * nu / (r2 - r1) / r1
    g = B.Geometry("D2Q9", L, L, 1)
    g.add_sphere(c, r1, True, Omega=(0, 0, om1))
    g.add_sphere(c, r2, False)
    mask, links = g.build()
    g.close()
    d = B.Domain("D2Q9", L, L, 1, mask, tau, storage="f64", collision="TRT", magic=magic)
    d.set_boundary_links(links, variant=variant)
    d.step(int(2.0 * (r2 - r1) ** 2 / nu))
    _, u, _, unstable = d.macros()
    d.close()
    assert not unstable
    return u, L, int(c[1])


def test_linear_error_high_resolution_against_bfl(gpu_lib):
    if not os.path.exists(GOLD):
        pytest.skip("e3 fixture not written (tests/golden/make_fixtures.py e3)")
    z = np.load(GOLD, allow_pickle=False)
    assert json.loads(str(z["meta"]))["variant"] == "BFL"
    x, uy_th = z["w40_x"].astype(int), z["w40_uy_th"]
    rr = {"BFL": float(z["w40_rrse_axis"])}
    le = {"BFL": float(z["w40_le"].mean())}
    for v in ("F", "FQ", "U", "HWBB"):
        print("case linear error r2 - r1 = 40,", v, flush=True)
        u, L, yc = _gpu_axis(gpu_lib, 40, v)
        uy = u[x + L * yc, 1]
        rr[v] = float(np.sqrt(((uy - uy_th) ** 2).sum() / (uy_th ** 2).sum()))
        le[v] = float((np.abs(uy - uy_th) / np.abs(uy_th)).mean())
    print("rRSE along the axis", rr, "mean LE", le, flush=True)
    # the paper's findings: fragmented schemes ahead of the unified ELIBB-U,
    # ELIBB-F and ELIBB-FQ close to BFL, half-way bounce-back worst
    for v in ("BFL", "F", "FQ"):
        assert rr[v] < rr["U"] and rr[v] < rr["HWBB"]
    for v in ("F", "FQ"):
        assert rr[v] < 2.0 * rr["BFL"]
    assert rr["HWBB"] == max(rr.values())
