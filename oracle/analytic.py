"""Closed-form reference flows (Sec. III).

Status: pinned -- each is checked in tests against an independent property
(boundary values, the PDE residual by finite differences, the t -> infinity
limit).
"""
import numpy as np

from . import precision as prec


def circular_couette(r, r1, r2, omega1):
    """Steady azimuthal velocity between an inner cylinder of radius r1 turning at
    angular speed omega1 and a resting outer cylinder of radius r2 (Sec. III.B):
    u_theta = (r1^2 - beta^2 r^2) omega1 / ((1 - beta^2) r),  beta = r1 / r2."""
    beta = r1 / r2
    r = np.asarray(r, dtype=prec.REAL)
    return (r1 * r1 - beta * beta * r * r) * omega1 / ((1.0 - beta * beta) * r)


def impulsive_couette(y, h, U, nu, t, nterms=100):
    """Impulsively started plane Couette flow (eq. solution-couette): wall at y = 0 at
    rest, wall at y = h moving at U from t = 0; series truncated at nterms (the
    paper uses 100 terms)."""
    y = np.asarray(y, dtype=prec.REAL)
    s = y / h
    for n in range(1, nterms + 1):
        s = s + (2.0 / np.pi) * ((-1.0) ** n / n) * np.exp(-n * n * np.pi * np.pi * nu * t / (h * h)) * np.sin(n * np.pi * y / h)
    return U * s


def poiseuille(n, H, F, rho, nu):
    """Force-driven plane Poiseuille profile u(n) = F n (H - n) / (2 rho nu), n the
    distance from one wall, H the channel width (textbook)."""
    n = np.asarray(n, dtype=prec.REAL)
    return F * n * (H - n) / (2.0 * rho * nu)
