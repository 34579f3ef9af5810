"""One lattice-Boltzmann time step with ELIBB boundaries, plain FP64 NumPy.

State: the pre-collision populations f_i(x, t) of every fluid node (NaN on solid
nodes, so that a read of solid data poisons the result).  One step t -> t+1
(Sec. II.A, eq. LBE; Sec. II.B-E):

1. moments at every fluid node: rho = sum_i f_i, rho u = sum_i c_i f_i + F/2
   (the F/2 shift belongs to Guo's forcing, a textbook addition: the paper has no
   body force);
2. collision: f*_i = f_i - omega (f_i - f^eq_i(rho, u)) + (1 - omega/2) S_i with
   omega = 1/tau (eq. LB-BGK, tau = taubar + 1/2) and the second-order
   equilibrium (eq. Eq2ndOrder); S_i is Guo's source term; or the TRT model
   (see collide);
3. streaming: f_i(x, t+1) = f*_i(x - c_i, t) for every pair that is not a cut
   link, wrapping on periodic axes (eq. LBE);
4. zero-gradient outlet (a reading: open boundaries are outside the paper);
5. every cut link is rebuilt by the ELIBB (eq. ELIBB-general) from node F's own
   time-t data (see oracle.boundary).

Fresh-node refill for moving bodies (Sec. III.C and the LIR appendix, which is
run before collide-and-stream; the LIR algorithm itself is only in a missing
figure) is replaced by an equilibrium refill: a node that became fluid takes
f^eq(rho_bar, u_body(x)), rho_bar the mean density of its neighbours that hold
valid populations (rho0 if there are none).

Status: pinned -- exact invariants (rest, co-moving uniform flow, periodic mass
and momentum, momentum growth by F per node and step under Guo forcing), the
textbook half-way bounce-back reduction, and closed-form flows (circular
Couette, impulsively started Couette, force-driven Poiseuille); the refill against hand-listed
neighbour sets on tiny grids (tests/test_oracle_refill.py: fluid at both times,
fresh and newly solid neighbours excluded, rho0 when none is left, faces); the
zero-gradient outlet only as far as its mass growth under a velocity inlet.
"""
import numpy as np

from . import boundary
from . import precision as prec


def equilibrium(lat, rho, u):
    """f^eq_i(rho, u) for all i (eq. Eq2ndOrder).  rho (n,), u (3, n) -> (Q, n)."""
    cs2 = lat.cs2
    c = lat.c.astype(prec.REAL)                 # (Q, 3)
    cu = c @ u                                   # (Q, n)
    uu = (u * u).sum(axis=0)                     # (n,)
    return lat.w[:, None] * rho[None, :] * (1.0 + cu / cs2 + (cu * cu - cs2 * uu[None, :]) / (2.0 * cs2 * cs2))


def moments(lat, f, force):
    """rho and u of populations f (Q, n); u includes the F/2 shift of Guo's scheme."""
    rho = f.sum(axis=0)
    j = lat.c.astype(prec.REAL).T @ f           # (3, n)
    u = (j + 0.5 * np.asarray(force, dtype=prec.REAL)[:, None]) / rho[None, :]
    return rho, u


def guo_source(lat, u, force):
    """S_i = w_i [ (c_i - u)/cs2 + (c_i . u) c_i / cs2^2 ] . F   (Guo, Zheng & Shi 2002)."""
    cs2 = lat.cs2
    F = np.asarray(force, dtype=prec.REAL)
    c = lat.c.astype(prec.REAL)
    cF = c @ F                                   # (Q,)
    uF = F @ u                                   # (n,)
    cu = c @ u                                   # (Q, n)
    return lat.w[:, None] * ((cF[:, None] - uF[None, :]) / cs2 + cu * cF[:, None] / (cs2 * cs2))


def trt_omega_minus(tau, magic):
    """omega^- of the TRT model from the magic parameter (eq. magic-parameter):
    Lambda = (1/omega^+ - 1/2)(1/omega^- - 1/2) with omega^+ = 1/tau."""
    return prec.scalar(1) / (prec.scalar(magic) / (prec.scalar(tau) - prec.scalar(0.5)) + prec.scalar(0.5))


def collide(lat, f, tau, force, magic=None):
    """Collision with Guo forcing. Returns f*, rho, u, f^eq (all on the given nodes).

    magic None: BGK (eq. LB-BGK), f* = f - omega (f - f^eq) + (1 - omega/2) S.
    magic = Lambda: TRT (Sec. II.A, TRT models): the symmetric parts
    g^+ = (g_i + g_ibar)/2 relax with omega^+ = 1/tau, the antisymmetric parts
    g^- = (g_i - g_ibar)/2 with omega^- (eq. magic-parameter),
      f* = f - omega^+ (f^+ - f^eq+) - omega^- (f^- - f^eq-)
             + (1 - omega^+/2) S^+ + (1 - omega^-/2) S^-,
    Guo's source split the same way (the paper has no body force).
    """
    omega = prec.scalar(1) / prec.scalar(tau)
    rho, u = moments(lat, f, force)
    feq = equilibrium(lat, rho, u)
    has_force = np.any(np.asarray(force) != 0.0)
    if magic is None:
        fstar = f - omega * (f - feq)
        if has_force:
            fstar = fstar + (1.0 - 0.5 * omega) * guo_source(lat, u, force)
        return fstar, rho, u, feq
    om_m = trt_omega_minus(tau, magic)
    o = lat.opp
    sym = lambda g: 0.5 * (g + g[o])
    asym = lambda g: 0.5 * (g - g[o])
    fstar = f - omega * (sym(f) - sym(feq)) - om_m * (asym(f) - asym(feq))
    if has_force:
        S = guo_source(lat, u, force)
        fstar = fstar + (1.0 - 0.5 * omega) * sym(S) + (1.0 - 0.5 * om_m) * asym(S)
    return fstar, rho, u, feq


class Simulation:
    """A lattice with a fixed (or externally updated) geometry and link list."""

    def __init__(self, dom, tau, force=(0.0, 0.0, 0.0), rho0=1.0, u0=(0.0, 0.0, 0.0), magic=None):
        self.dom = dom
        self.lat = dom.lat
        self.tau = float(tau)
        self.magic = None if magic is None else float(magic)   # TRT magic parameter, None = BGK
        self.force = np.asarray(force, dtype=prec.REAL).reshape(3)
        self.rho0 = float(rho0)
        self.u0 = np.asarray(u0, dtype=prec.REAL).reshape(3)
        self.f = None
        self.fluid = None
        self.t = 0
        self.last_force = None     # (n_groups, 3): wall forces of the last step
        self.last_torque = None    # (n_groups, 3): wall torques of the last step about the group centres
        self.link_group = None
        self.n_groups = 1
        self.centres = np.zeros((1, 3))

    # -- geometry -----------------------------------------------------------------
    def set_geometry(self, fluid, links, variant="FQ", q_cut=0.01, wall_neq="bounceback"):
        """Install a fluid mask and a cut-link list (dict from oracle.geometry.cut_links).
        wall_neq: the wall non-equilibrium estimator (see boundary.link_points)."""
        dom, lat = self.dom, self.lat
        fl = np.asarray(fluid, dtype=bool).reshape(-1)
        if wall_neq not in boundary.WALL_NEQ:
            raise ValueError(f"unknown wall non-equilibrium {wall_neq!r}")
        self.fluid = fl
        self.variant, self.q_cut, self.wall_neq = variant, float(q_cut), wall_neq
        L = {k: np.asarray(v) for k, v in links.items()}
        self.links = L
        # BFL (oracle-only comparator, eq. bfl) also reads the next node along the
        # link, x_FF = x_F + c_i; the ELIBB variants use their Lagrange weights
        if variant == "BFL":
            self.coef = None
            if L["node"].size:
                from .geometry import _index
                xs = dom.coords(L["node"]) + lat.c[L["dir"]].T
                ok = np.ones(xs.shape[1], dtype=bool)
                for a in range(3):
                    if dom.periodic[a]:
                        xs[a] = np.mod(xs[a], dom.n[a])
                    else:
                        ok &= (xs[a] >= 0) & (xs[a] < dom.n[a])
                self.ff = np.where(ok, _index(dom, np.where(ok, xs, 0)), 0)
                self.ff_ok = ok & fl[self.ff]
        else:
            self.coef = boundary.coefficients(variant, L["q"], q_cut)
        cut = np.zeros((lat.q, dom.N), dtype=bool)
        if L["node"].size:
            if not fl[L["node"]].all():
                raise ValueError("a link starts on a non-fluid node")
            if (L["dir"] == 0).any():
                raise ValueError("direction 0 cannot be cut")
            if np.any(cut[L["dir"], L["node"]]):
                raise ValueError("duplicate link")
            cut[L["dir"], L["node"]] = True
            if np.unique(L["dir"] * dom.N + L["node"]).size != L["node"].size:
                raise ValueError("duplicate link")
        X = dom.coords()
        nodes = np.flatnonzero(fl)
        self.stream, self.outlet = [], []
        from .geometry import _source, _index, beyond_outlet, outlet_producer
        for i in range(lat.q):
            xs = X[:, nodes]
            src, inside = _source(dom, xs.copy(), lat.c[i])
            sidx = np.where(inside, _index(dom, np.where(inside, src, 0)), 0)
            ok = inside & fl[sidx] & ~cut[i, nodes]
            if (inside & fl[sidx] & cut[i, nodes]).any():
                raise ValueError(f"direction {i}: a link whose source node is fluid")
            self.stream.append((nodes[ok], sidx[ok]))
            rest = ~ok & ~cut[i, nodes]
            od, osrc = np.zeros(0, np.int64), np.zeros(0, np.int64)
            if rest.any() and dom.outlet_face is not None:
                bo = beyond_outlet(dom, src[:, rest])
                prod = outlet_producer(dom, fl, xs[:, rest], lat.c[i])
                good = bo & (prod >= 0)
                od, osrc = nodes[rest][good], prod[good]
                rest_idx = np.flatnonzero(rest)[good]
                rest[rest_idx] = False
            if rest.any():
                bad = nodes[np.flatnonzero(rest)[0]]
                raise ValueError(f"population (node={bad}, dir={i}) is neither streamed nor covered by a link")
            self.outlet.append((od, osrc))

    # -- state --------------------------------------------------------------------
    def init_equilibrium(self, rho=None, u=None):
        lat, N = self.lat, self.dom.N
        rho = np.full(N, self.rho0, dtype=prec.REAL) if rho is None else np.asarray(rho, dtype=prec.REAL).reshape(N)
        u = np.repeat(self.u0.reshape(3, 1), N, axis=1) if u is None else np.asarray(u, dtype=prec.REAL).reshape(3, N)
        self.f = np.full((lat.q, N), np.nan, dtype=prec.REAL)
        fl = self.fluid
        self.f[:, fl] = equilibrium(lat, rho[fl], u[:, fl])
        self.t = 0

    def step(self):
        lat = self.lat
        fl = self.fluid
        nodes = np.flatnonzero(fl)
        f = self.f
        fstar = np.full_like(f, np.nan)
        feq = np.full_like(f, np.nan)
        rho = np.full(f.shape[1], np.nan, dtype=f.dtype)
        u = np.full((3, f.shape[1]), np.nan, dtype=f.dtype)
        fs, r, uu, fe = collide(lat, f[:, nodes], self.tau, self.force, self.magic)
        fstar[:, nodes], rho[nodes], u[:, nodes], feq[:, nodes] = fs, r, uu, fe
        fnew = np.full_like(f, np.nan)
        for i in range(lat.q):
            dst, src = self.stream[i]
            fnew[i, dst] = fstar[i, src]
            od, osrc = self.outlet[i]
            fnew[i, od] = fstar[i, osrc]
        L = self.links
        if L["node"].size:
            n, d = L["node"], L["dir"]
            if self.variant == "BFL":
                fnew[d, n] = boundary.bfl_value(lat, d, L["q"], rho[n], fstar[:, n], fstar[:, self.ff], self.ff_ok,
                                                L["uw_t"])
            else:
                P = boundary.link_points(lat, d, rho[n], feq[:, n], f[:, n], fstar[:, n], L["uw_t"], L["uw_t1"],
                                         self.wall_neq)
                fnew[d, n] = boundary.reconstruct(self.coef, P)
            grp = np.zeros(n.size, np.int64) if self.link_group is None else self.link_group
            # lever arm: wall point x_W = x_F - q c_i relative to the group's centre (minimum image)
            xw = self.dom.coords(n).astype(prec.REAL) - L["q"][None, :] * lat.c[d].T
            arm = self.dom.min_image(xw - self.centres[grp].T)
            if lat.d == 2:
                arm[2] = 0.0
            self.last_force, self.last_torque = boundary.momentum_exchange(
                lat, d, fstar[:, n], fnew[d, n], L["uw_t"], grp, self.n_groups, arm)
        self.f = fnew
        self.t += 1

    def set_link_groups(self, group, n_groups, centres=None):
        """Group ids (one per link, in the link list's order) for the forces, and
        the reference point of each group's torque (default: the origin)."""
        g = np.asarray(group, dtype=np.int64).reshape(-1)
        if g.size != self.links["node"].size or (g.size and (g.min() < 0 or g.max() >= n_groups)):
            raise ValueError("bad link groups")
        self.link_group, self.n_groups = g, int(n_groups)
        self.centres = np.zeros((self.n_groups, 3)) if centres is None else \
            np.asarray(centres, dtype=prec.REAL).reshape(self.n_groups, 3)

    def run(self, n):
        for _ in range(int(n)):
            self.step()

    def macros(self):
        """rho (N,) and u (3, N) of the current state; NaN on solid nodes."""
        rho, u = moments(self.lat, self.f, self.force)
        return rho, u

    # -- moving geometry ----------------------------------------------------------
    def refill(self, new_fluid, u_body):
        """Equilibrium refill of nodes that become fluid (old solid -> new fluid).

        u_body: (3, N) body velocity used at the fresh nodes.  Must be called with
        the new geometry before the step that first uses it.
        """
        lat, dom = self.lat, self.dom
        new_fl = np.asarray(new_fluid, dtype=bool).reshape(-1)
        old_fl = self.fluid
        fresh = new_fl & ~old_fl
        valid = new_fl & old_fl
        rho_all = np.where(valid, np.nan_to_num(self.f).sum(axis=0), 0.0)
        X = dom.coords()
        idx = np.flatnonzero(fresh)
        f = self.f.copy()
        f[:, ~new_fl] = np.nan
        if idx.size:
            tot = np.zeros(idx.size, dtype=prec.REAL)
            cnt = np.zeros(idx.size, dtype=prec.REAL)
            from .geometry import _source, _index
            for j in range(1, lat.q):
                nb, inside = _source(dom, X[:, idx].copy(), -lat.c[j])     # x + c_j
                nidx = np.where(inside, _index(dom, np.where(inside, nb, 0)), 0)
                ok = inside & valid[nidx]
                tot += np.where(ok, rho_all[nidx], 0.0)
                cnt += ok
            rho_bar = np.where(cnt > 0, tot / np.maximum(cnt, 1), self.rho0)
            f[:, idx] = equilibrium(lat, rho_bar, np.asarray(u_body)[:, idx])
        self.f = f
        return idx


def step_at(dom, f, fluid, links, nodes, tau, force=(0.0, 0.0, 0.0), variant="FQ", q_cut=0.01, magic=None,
            wall_neq="bounceback"):
    """f(x, t+1) at the given fluid nodes only, from the full state f (Q, N) at t.

    The same step as Simulation.step, evaluated node by node: every pulled
    population is the post-collision value of its source node (collided here),
    or the outlet producer's, or the ELIBB value of the node's own cut link.
    ``links`` must contain every cut link of the requested nodes (other links
    are ignored).  Returns (Q, len(nodes)).
    """
    from .geometry import _source, _index, beyond_outlet, outlet_producer
    lat = dom.lat
    fl = np.asarray(fluid, dtype=bool).reshape(-1)
    nodes = np.asarray(nodes, dtype=np.int64)
    X = dom.coords()
    xs = X[:, nodes]
    out = np.full((lat.q, nodes.size), np.nan, dtype=prec.REAL)
    force = np.asarray(force, dtype=prec.REAL)
    # the nodes' own collision (needed by their links)
    fs_self, rho_s, u_s, feq_s = collide(lat, f[:, nodes], tau, force, magic)
    L = {k: np.asarray(v) for k, v in links.items()}
    key = L["node"] * lat.q + L["dir"]
    order = np.argsort(key)
    for i in range(lat.q):
        src, inside = _source(dom, xs.copy(), lat.c[i])
        sidx = np.where(inside, _index(dom, np.where(inside, src, 0)), 0)
        k = np.searchsorted(key[order], nodes * lat.q + i)
        k = np.minimum(k, key.size - 1) if key.size else k
        is_cut = (key.size > 0) & (key[order][k] == nodes * lat.q + i) if key.size else np.zeros(nodes.size, bool)
        stream = inside & fl[sidx] & ~is_cut
        if stream.any():
            fs_src, _, _, _ = collide(lat, f[:, sidx[stream]], tau, force, magic)
            out[i, stream] = fs_src[i]
        rest = ~stream & ~is_cut
        if rest.any() and dom.outlet_face is not None:
            bo = beyond_outlet(dom, src[:, rest])
            prod = outlet_producer(dom, fl, xs[:, rest], lat.c[i])
            good = bo & (prod >= 0)
            if good.any():
                fs_p, _, _, _ = collide(lat, f[:, prod[good]], tau, force, magic)
                idx = np.flatnonzero(rest)[good]
                out[i, idx] = fs_p[i]
        if is_cut.any():
            sel = np.flatnonzero(is_cut)
            li = order[k[sel]]
            coef = boundary.coefficients(variant, L["q"][li], q_cut)
            P = boundary.link_points(lat, np.full(sel.size, i), rho_s[sel], feq_s[:, sel], f[:, nodes[sel]],
                                     fs_self[:, sel], L["uw_t"][:, li], L["uw_t1"][:, li], wall_neq)
            out[i, sel] = boundary.reconstruct(coef, P)
    return out
