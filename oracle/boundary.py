"""ELIBB boundary reconstruction (Sec. II.C-E of the paper).

For a cut link (x_F, i) -- i is the population that is missing at the boundary
node F after streaming, so x_F - c_i lies in the solid -- the ELIBB general form
(eq. ELIBB-general) rebuilds f_i(x_F, t+1) as a weighted sum of up to four
quantities, each placed at a signed link coordinate s (eq. s, eq. x_to_s_helper):

  name  quantity                                              s
  P0    wall population at t+1,  ~f_i^{t+1}(x_W)              0
  P1    post-collision wall population, ~f_i^*(x_W)           1
  P2    post-collision bounced population f_ibar^*(x_F)       1 - q
  P3    post-collision population f_i^*(x_F)                  1 + q

and the target f_i^{t+1}(x_F) sits at s = q.  The weights are the Lagrange
basis (eq. poli_coeff) over the variant's point set evaluated at s_ref = q.

Readings taken where the paper is ambiguous (all listed in the design notes):
* s uses |c_i|^2 in the denominator so that the helper values of eq.
  x_to_s_helper hold (eq. s prints |c_i|); this reproduces the printed BFL
  (eq. bfl) and ELIBB-U coefficients.
* the post-collision wall population sits at s = 1 (the resting-wall value of
  eq. x_to_s_helper); wall motion enters only through the momentum correction
  (eq. ME-solid-to-fluid) and the wall equilibria.
* the wall equilibria use rho_F(t) and u_w(t+1) for P0, u_w(t) for P1
  (eq. ELIBB-approximation-eq1/eq2); the wall non-equilibria use the bounced
  non-equilibrium of node F at time t (eq. neqbb-s): pre-collision for P0,
  post-collision for P1.
* the moving-wall correction (eq. ME-solid-to-fluid) is added to nodal
  populations with s < 1, i.e. to P2 only, with rho = rho_F(t), u_w = u_w(t).
* the ELIBB-F coefficients printed in Sec. II.D are garbled (they do not sum to
  one); the Lagrange rule is used instead.  UQ and FQ fall back to F below the
  cutoff q_min (0.01 in the paper).

Status: the s-rule and Lagrange weights are pinned against the printed BFL and
ELIBB-U coefficients and against polynomial exactness; the assembly is pinned by
exact invariants (rest state, co-moving uniform flow) and by the q = 1/2
reduction to textbook half-way bounce-back with Ladd's correction.
"""
import numpy as np

from . import precision as prec

VARIANTS = ("FQ", "F", "UQ", "U", "HWBB")

# s-coordinate of each interpolation point as a function of q (eq. x_to_s_helper)
S_OF_POINT = {
    "P0": lambda q: np.zeros_like(q),
    "P1": lambda q: np.ones_like(q),
    "P2": lambda q: 1.0 - q,
    "P3": lambda q: 1.0 + q,
    # f_ibar^*(x_FF), the non-local population of the BFL scheme (not used by ELIBB)
    "PFF": lambda q: -q,
}
POINTS = ("P0", "P1", "P2", "P3")


def bfl_coefficients(q):
    """Linear BFL weights from the same s-rule (oracle-only comparator, Sec. II.B).

    q < 1/2: points {PFF (s=-q), P2 (s=1-q)};  q >= 1/2: points {P2, P3 (s=1+q)}.
    Returns dict point -> weight array.
    """
    q = np.asarray(q, dtype=prec.REAL)
    out = {"PFF": np.zeros_like(q), "P2": np.zeros_like(q), "P3": np.zeros_like(q)}
    for sel, key in ((q < 0.5, ("PFF", "P2")), (q >= 0.5, ("P2", "P3"))):
        if sel.any():
            qs = q[sel]
            for p, a in zip(key, lagrange_weights([S_OF_POINT[k](qs) for k in key], qs)):
                out[p][sel] = a
    return out


def point_set(variant, q, q_cut=0.01):
    """Interpolation points used by a variant for one value of q (Sec. II.D)."""
    if variant == "HWBB":
        return ("P2",)
    if variant == "U":
        return ("P0", "P1")
    if variant == "F" or (variant in ("UQ", "FQ") and q < q_cut):
        return ("P0", "P2") if q < 0.5 else ("P2", "P1")
    if variant == "UQ":
        return ("P0", "P2", "P1")
    if variant == "FQ":
        return ("P0", "P2", "P1") if q < 0.5 else ("P2", "P1", "P3")
    raise ValueError(f"unknown variant {variant!r}")


def lagrange_weights(s_nodes, s_ref):
    """Lagrange basis polynomials at s_ref (eq. poli_coeff).

    s_nodes: list of arrays (one per interpolation point); s_ref: array.
    Returns a list of arrays a_j with sum_j a_j s_j^m = s_ref^m for m <= n.
    """
    out = []
    for j, sj in enumerate(s_nodes):
        a = np.ones_like(s_ref)
        for k, sk in enumerate(s_nodes):
            if k != j:
                a = a * (s_ref - sk) / (sj - sk)
        out.append(a)
    return out


def point_set_groups(variant, q, q_cut=0.01):
    """Vectorised form of point_set: list of (mask, point set) covering all q."""
    q = np.asarray(q, dtype=prec.REAL)
    lo, hi = q < 0.5, q >= 0.5
    f_sets = [(lo, ("P0", "P2")), (hi, ("P2", "P1"))]
    if variant == "HWBB":
        return [(np.ones(q.shape, bool), ("P2",))]
    if variant == "U":
        return [(np.ones(q.shape, bool), ("P0", "P1"))]
    if variant == "F":
        return f_sets
    cut = q < q_cut
    fallback = [(m & cut, key) for m, key in f_sets]
    if variant == "UQ":
        return fallback + [(~cut, ("P0", "P2", "P1"))]
    if variant == "FQ":
        return fallback + [(~cut & lo, ("P0", "P2", "P1")), (~cut & hi, ("P2", "P1", "P3"))]
    raise ValueError(f"unknown variant {variant!r}")


def coefficients(variant, q, q_cut=0.01):
    """Coefficient matrix (n_links x 4) on (P0, P1, P2, P3) for an array of q.

    Links are grouped by point set; within a group the generic Lagrange product
    is evaluated with s_ref = q.
    """
    q = np.asarray(q, dtype=prec.REAL).reshape(-1)
    out = np.zeros((q.size, 4), dtype=prec.REAL)
    for sel, key in point_set_groups(variant, q, q_cut):
        if not sel.any():
            continue
        qs = q[sel]
        s_nodes = [S_OF_POINT[p](qs) for p in key]
        with np.errstate(divide="ignore", invalid="ignore"):
            weights = lagrange_weights(s_nodes, qs)
        for p, a in zip(key, weights):
            out[sel, POINTS.index(p)] = a
    # The unified quadratic point set {P0 (s=0), P2 (s=1-q), P1 (s=1)} has two
    # coincident nodes at q = 1 exactly (the node next to a wall point lying on
    # a lattice node).  The Lagrange weights are continuous there; take their
    # limit q -> 1: a(P0) -> -1, a(P2) -> 1, a(P1) -> 1.
    if variant == "UQ":
        at_one = q == 1.0
        out[at_one] = (-1.0, 1.0, 1.0, 0.0)
    return out


def equilibrium_dir(lat, i, rho, u):
    """Second-order equilibrium of direction(s) i (eq. Eq2ndOrder) for given rho, u.

    i: int array (n,), rho: (n,), u: (3, n).
    """
    c = lat.c[i].T.astype(prec.REAL)          # (3, n)
    w = lat.w[i]
    cu = (c * u).sum(axis=0)
    uu = (u * u).sum(axis=0)
    cs2 = lat.cs2
    return w * rho * (1.0 + cu / cs2 + (cu * cu - cs2 * uu) / (2.0 * cs2 * cs2))


WALL_NEQ = ("bounceback", "regularized")


def _hermite2_of(lat):
    """H_ab = c_a c_b - cs2 delta_ab of every direction, over the lattice's D axes: (Q, D, D)."""
    D = lat.d
    c = lat.c[:, :D].astype(prec.REAL)
    return np.einsum("na,nb->nab", c, c) - lat.cs2 * np.eye(D)[None]


def _hermite3_of(lat):
    """H_abg = c_a c_b c_g - cs2 (delta_ab c_g + delta_ag c_b + delta_bg c_a) of
    every direction: (Q, D, D, D)."""
    D = lat.d
    c = lat.c[:, :D].astype(prec.REAL)
    I = np.eye(D)
    ccc = np.einsum("na,nb,ng->nabg", c, c, c)
    dc = (np.einsum("ab,ng->nabg", I, c) + np.einsum("ag,nb->nabg", I, c) + np.einsum("bg,na->nabg", I, c))
    return ccc - lat.cs2 * dc


_TABLES = {}


def _tables(lat):
    """Per-lattice tables: H2, H3 and c c of every direction (computed once)."""
    if lat.name not in _TABLES:
        c = lat.c[:, :lat.d].astype(prec.REAL)
        _TABLES[lat.name] = (_hermite2_of(lat), _hermite3_of(lat), np.einsum("ja,jb->jab", c, c))
    return _TABLES[lat.name]


def hermite2(lat, i):
    """Second-order Hermite polynomial of directions i (App. Hermite), (n, D, D)."""
    return _tables(lat)[0][i]


def hermite3(lat, i):
    """Third-order Hermite polynomial of directions i (App. Hermite), (n, D, D, D)."""
    return _tables(lat)[1][i]


def neq_stress(lat, f, feq):
    """Non-equilibrium second moment Pi_ab = sum_j c_ja c_jb (f_j - f^eq_j) over
    the lattice's D axes.  f, feq: (Q, n).  Returns (n, D, D)."""
    return np.tensordot(f - feq, _tables(lat)[2], axes=(0, 0))


def regularized_neq(lat, i, Pi, u):
    """Non-equilibrium of directions i rebuilt from its Hermite expansion truncated
    at third order (eq. fi_neq, App. C):
        f_i^neq = w_i [ H_i2 : a2 / (2 cs2^2) + H_i3 : a3 / (6 cs2^3) ]
    with a2 = Pi, the non-equilibrium stress, and a3 from the recursion of
    eq. malaspinas at n = 3 (divided by rho):
        a3_abg = u_a Pi_bg + u_b Pi_ag + u_g Pi_ab.
    Reading: Pi stands for the first-order Hermite coefficient a^(1)_2; the stress
    Lambda of eq. fi_neq is replaced through a^(1)_2 = -cs2 tau rho Lambda, the
    relation under which the rebuilt non-equilibrium has second moment Pi (the
    printed constants of eq. fi_neq and eq. a12Eqlambda disagree in sign and in a
    factor cs2).  rho and tau then drop out.

    i: (n,) directions; Pi: (n, D, D); u: (3, n) velocity.  Returns (n,).
    """
    D = lat.d
    cs2 = lat.cs2
    uD = np.asarray(u, dtype=prec.REAL)[:D].T                   # (n, D)
    a3 = (np.einsum("na,nbg->nabg", uD, Pi) + np.einsum("nb,nag->nabg", uD, Pi)
          + np.einsum("ng,nab->nabg", uD, Pi))
    t2 = np.einsum("nab,nab->n", hermite2(lat, i), Pi) / (2.0 * cs2 ** 2)
    t3 = np.einsum("nabg,nabg->n", hermite3(lat, i), a3) / (6.0 * cs2 ** 3)
    return lat.w[i] * (t2 + t3)


def link_points(lat, i, rho_F, feq_F, f_F, fstar_F, uw_t, uw_t1, wall_neq="bounceback"):
    """The four interpolation quantities P0..P3 for links with missing direction i.

    i: (n,) missing directions; rho_F: (n,) density of node F at t;
    feq_F, f_F, fstar_F: (Q, n) equilibrium, pre- and post-collision populations
    of node F at time t; uw_t, uw_t1: (3, n) wall velocity at x_W at t and t+1.
    wall_neq: how the wall non-equilibrium is estimated (Sec. II, "Approximation
    of the wall populations"): "bounceback", the bounced non-equilibrium of F
    (eq. neqbb-s), or "regularized", eq. fi_neq with the wall velocity and the
    non-equilibrium stress of F (Lambda(x_W) ~ Lambda(x_F)): pre-collision for
    P0 (with u_w(t+1)), post-collision for P1 (with u_w(t)).
    Returns P (4, n).
    """
    ib = lat.opp[i]
    n = np.arange(i.size)
    if wall_neq == "bounceback":
        n_pre = f_F[ib, n] - feq_F[ib, n]          # bounced pre-collision non-equilibrium (eq. neqbb-s)
        n_post = fstar_F[ib, n] - feq_F[ib, n]     # bounced post-collision non-equilibrium
    elif wall_neq == "regularized":
        n_pre = regularized_neq(lat, i, neq_stress(lat, f_F, feq_F), uw_t1)
        n_post = regularized_neq(lat, i, neq_stress(lat, fstar_F, feq_F), uw_t)
    else:
        raise ValueError(f"unknown wall non-equilibrium {wall_neq!r}")
    P0 = equilibrium_dir(lat, i, rho_F, uw_t1) + n_pre
    P1 = equilibrium_dir(lat, i, rho_F, uw_t) + n_post
    cu_w = (lat.c[i].T.astype(prec.REAL) * uw_t).sum(axis=0)
    P2 = fstar_F[ib, n] + 2.0 * lat.w[i] * rho_F * cu_w / lat.cs2   # eq. ME-solid-to-fluid
    P3 = fstar_F[i, n]
    return np.stack([P0, P1, P2, P3])


def bfl_value(lat, i, q, rho_F, fstar_F, fstar_FF, ff_ok, uw_t):
    """Linear BFL (eq. bfl), the two-node interpolated bounce-back the paper
    compares the ELIBB with: for the cut link (x_F, i), with x_FF = x_F + c_i the
    next node along the link, away from the wall,
        q <  1/2:  f_i(x_F, t+1) = 2q f*_ibar(x_F) + (1 - 2q) f*_ibar(x_FF) + m,
        q >= 1/2:  f_i(x_F, t+1) = f*_ibar(x_F) / (2q) + (2q - 1)/(2q) f*_i(x_F) + m / (2q),
    (weights from bfl_coefficients, i.e. the paper's printed ones), m = 2 w_i rho_F
    c_i.u_w / c_s^2 the moving-wall term of eq. ME-solid-to-fluid, added where the
    bounce happens (in full before the bounce-back streaming when q < 1/2, carried
    with the bounced population's weight 1/(2q) when q >= 1/2; the paper states BFL
    for resting walls).  Where x_FF is not a fluid node (ff_ok false; a gap one
    node wide) the link falls back to half-way bounce-back, f*_ibar(x_F) + m.

    i: (n,); q: (n,); rho_F: (n,); fstar_F, fstar_FF: (Q, n); ff_ok: (n,) bool;
    uw_t: (3, n).  Returns (n,)."""
    ib = lat.opp[i]
    n = np.arange(i.size)
    c = lat.c[i].T.astype(prec.REAL)
    m = 2.0 * lat.w[i] * rho_F * (c * uw_t).sum(axis=0) / lat.cs2
    w = bfl_coefficients(q)
    lo = q < 0.5
    f_lo = w["P2"] * fstar_F[ib, n] + w["PFF"] * np.where(ff_ok, fstar_FF[ib, n], 0.0) + m
    f_hi = w["P2"] * (fstar_F[ib, n] + m) + w["P3"] * fstar_F[i, n]
    hw = fstar_F[ib, n] + m
    return np.where(lo, np.where(ff_ok, f_lo, hw), f_hi)


def reconstruct(coef, P):
    """f_i(x_F, t+1) = sum_k a_k P_k  (eq. interpolated_bb_equation)."""
    return (coef.T * P).sum(axis=0)


def momentum_exchange(lat, i, fstar_F, f_new, uw_t, group, n_groups, arm=None):
    """Force exerted by the fluid on the walls during one step, per link group
    (Sec. II "Force computation", the Galilean-invariant momentum exchange of
    Wen et al.).  For a cut link (x_F, i) the population f*_ibar(x_F, t) leaves
    towards the wall and comes back as f_i(x_F, t+1):
        F_link = (c_ibar - u_w) f*_ibar(x_F, t) - (c_i - u_w) f_i(x_F, t+1).
    (The printed formula writes the outgoing post-collision population with the
    index i; it is read as ibar, the direction pointing into the wall.)
    The torque is T = sum over the group's links of r x F_link with the lever
    arm r given per link (the paper names the torque without fixing the arm;
    the caller passes the wall point's offset from the group's reference).

    i: (n,) missing directions; fstar_F: (Q, n) post-collision populations of the
    links' nodes at t; f_new: (n,) rebuilt f_i(x_F, t+1); uw_t: (3, n) wall
    velocity at x_W; group: (n,) group ids; arm: (3, n) or None.  Returns
    (n_groups, 3) forces, and with an arm also (n_groups, 3) torques.
    """
    ib = lat.opp[i]
    n = np.arange(i.size)
    c = lat.c.astype(prec.REAL)
    out_ = fstar_F[ib, n]
    contrib = (c[ib].T - uw_t) * out_[None, :] - (c[i].T - uw_t) * f_new[None, :]   # (3, n)
    F = np.zeros((n_groups, 3), dtype=prec.REAL)
    T = np.zeros((n_groups, 3), dtype=prec.REAL)
    tq = None if arm is None else np.cross(arm.T, contrib.T).T
    for g in range(n_groups):
        sel = group == g
        F[g] = contrib[:, sel].sum(axis=1)
        if tq is not None:
            T[g] = tq[:, sel].sum(axis=1)
    return F if arm is None else (F, T)
