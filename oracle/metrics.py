"""Error norms (Sec. III).

Status: pinned by elementary cases in tests (identical fields give 0, a uniform
relative perturbation eps gives eps).
"""
import numpy as np

from . import precision as prec


def rrse(u, u_th):
    """Relative root squared error (eq. rRMSE): sqrt(sum (u - u_th)^2 / sum u_th^2)."""
    u = np.asarray(u, dtype=prec.REAL)
    u_th = np.asarray(u_th, dtype=prec.REAL)
    return float(np.sqrt(((u - u_th) ** 2).sum() / (u_th ** 2).sum()))


def rel_l2(a, ref):
    """||a - ref||_2 / ||ref||_2 over all given entries (parity metric)."""
    a = np.asarray(a, dtype=prec.REAL).reshape(-1)
    ref = np.asarray(ref, dtype=prec.REAL).reshape(-1)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def mean_density_fluctuation(rho, rho0=1.0):
    """|sum_i (rho_i - rho0) / N| over the given nodes (Sec. III.B, mass conservation)."""
    rho = np.asarray(rho, dtype=prec.REAL).reshape(-1)
    return float(abs((rho - rho0).sum() / rho.size))
