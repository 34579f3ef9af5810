"""Pins of the s-rule and the Lagrange weights (Sec. II.C-D, eq. s, eq.
x_to_s_helper, eq. poli_coeff).

Golden values: the closed-form coefficients the paper prints (eq. bfl for BFL,
the ELIBB-U pair, the ELIBB-F a5 for q >= 1/2), stored with citations in
tests/golden/printed_coefficients.json.  Mathematical pins: polynomial
exactness of the Lagrange weights, partition of unity, q = 1/2 reducing the
fragmented and quadratic variants to half-way bounce-back.
"""
import json
import os
import re

import numpy as np
import pytest

from oracle import boundary

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "printed_coefficients.json")))
QS = np.array([0.011, 0.05, 0.1, 0.25, 0.3333, 0.49, 0.5, 0.51, 0.6, 0.75, 0.9, 0.999, 1.0])
IDX = {p: k for k, p in enumerate(boundary.POINTS)}


def _eval(expr, q):
    """Evaluate a printed formula such as "(2q-1)/(2q)" (implicit products)."""
    return eval(re.sub(r"(\d)q", r"\1*q", expr), {"q": q})


def test_bfl_printed_coefficients_from_s_rule():
    g = GOLD["bfl"]
    a = boundary.bfl_coefficients(QS)
    lo, hi = QS < 0.5, QS >= 0.5
    np.testing.assert_allclose(a["P2"][lo], _eval(g["q_lt_half"]["f_ibar_star_F"], QS[lo]), rtol=1e-14)
    np.testing.assert_allclose(a["PFF"][lo], _eval(g["q_lt_half"]["f_ibar_star_FF"], QS[lo]), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(a["P2"][hi], _eval(g["q_ge_half"]["f_ibar_star_F"], QS[hi]), rtol=1e-14)
    np.testing.assert_allclose(a["P3"][hi], _eval(g["q_ge_half"]["f_i_star_F"], QS[hi]), rtol=1e-13, atol=1e-15)


def test_elibb_u_printed():
    a = boundary.coefficients("U", QS)
    np.testing.assert_allclose(a[:, IDX["P0"]], _eval(GOLD["elibb_u"]["a4"], QS), rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(a[:, IDX["P1"]], _eval(GOLD["elibb_u"]["a5"], QS), rtol=1e-14)
    assert np.all(a[:, IDX["P2"]] == 0) and np.all(a[:, IDX["P3"]] == 0)


def test_elibb_f_printed_a5():
    hi = QS >= 0.5
    a = boundary.coefficients("F", QS[hi])
    np.testing.assert_allclose(a[:, IDX["P1"]], _eval(GOLD["elibb_f_q_ge_half_a5"]["a5"], QS[hi]), rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("variant", boundary.VARIANTS)
def test_partition_of_unity_and_exactness(variant):
    a = boundary.coefficients(variant, QS, GOLD["q_cutoff"]["value"])
    np.testing.assert_allclose(a.sum(axis=1), 1.0, rtol=0, atol=2e-15)
    # Lagrange weights reproduce polynomials up to the interpolation degree
    s = np.stack([boundary.S_OF_POINT[p](QS) for p in boundary.POINTS], axis=1)
    for k, q in enumerate(QS):
        pts = boundary.point_set(variant, q)
        if variant == "UQ" and q == 1.0:
            continue   # coincident nodes: the limit value, checked below
        for m in range(len(pts)):
            assert abs((a[k] * s[k] ** m).sum() - q ** m) < 1e-13


@pytest.mark.parametrize("variant", ["F", "UQ", "FQ", "HWBB"])
def test_half_way_reduces_to_bounce_back(variant):
    a = boundary.coefficients(variant, np.array([0.5]))[0]
    np.testing.assert_allclose(a, [0, 0, 1, 0], atol=1e-15)


def test_cutoff_switches_quadratic_to_linear():
    qc = GOLD["q_cutoff"]["value"]
    q = np.array([0.5 * qc, 0.999 * qc])
    for v in ("UQ", "FQ"):
        np.testing.assert_array_equal(boundary.coefficients(v, q, qc), boundary.coefficients("F", q, qc))
    q = np.array([qc, 2 * qc])
    assert not np.allclose(boundary.coefficients("FQ", q, qc), boundary.coefficients("F", q, qc))


def test_uq_limit_at_q_one_is_continuous():
    a1 = boundary.coefficients("UQ", np.array([1.0]))[0]
    a0 = boundary.coefficients("UQ", np.array([1.0 - 1e-7]))[0]
    np.testing.assert_allclose(a1, a0, atol=1e-6)


def test_fragmented_tends_to_wall_population_as_q_to_zero():
    a = boundary.coefficients("F", np.array([1e-9]))[0]
    np.testing.assert_allclose(a, [1, 0, 0, 0], atol=1e-8)


def test_variant_point_sets_match_paper_description():
    # UQ and FQ share the point set below 1/2 (Sec. III.A observation 2)
    q = np.linspace(0.02, 0.49, 17)
    np.testing.assert_array_equal(boundary.coefficients("UQ", q), boundary.coefficients("FQ", q))
    # the unified variants do not depend on which side of 1/2 q falls
    assert boundary.point_set("U", 0.2) == boundary.point_set("U", 0.8)
    assert boundary.point_set("UQ", 0.2) == boundary.point_set("UQ", 0.8)
    assert boundary.point_set("F", 0.2) != boundary.point_set("F", 0.8)
