"""Fluid classification and cut links for the oracle (Sec. II.B, figure of the 2D
boundary nodes; the link distance q is |x_W - x_F| / |c_i|, eq. bfl).

A node is fluid iff it lies strictly inside the fluid region.  A pair
(x_F, i), x_F fluid, is a cut link iff x_F - c_i is not fluid or lies outside a
non-periodic face that is not covered by the zero-gradient outlet.  q is the
first wall crossing along the segment p(lam) = x_F - lam c_i, lam in (0, 1], so
0 < q <= 1 (a wall point on a lattice node makes that node solid and gives
q = 1 to its neighbour).

Shapes:
* ``Sphere``    ball (3D) or disk (2D, centre z = 0), solid inside or outside,
                rigid-body wall velocity u_w = V + Omega x (x_W - centre).
* ``Cylinder``  circular cylinder along z through the centre (3D lattices): the
                sphere's formulas in the xy-plane.
* ``FaceWall``  a plane parallel to a non-periodic domain face at distance q_f
                from the first node layer, with a wall velocity given as a
                function of x_W (constant, or the parabolic inlet profile).
The zero-gradient outlet (a reading; the paper has no open boundaries): on the
outlet face, a population whose pull source lies beyond the face is copied from
the post-collision value of the face-layer node one step back along the face
(the "producer"), if that node is fluid; otherwise the pair must be a cut link.

Status: pinned -- the q of straight walls (exact closed values) and of circles
with lattice points on them (q = 1 exactly) in tests; circle/sphere/cylinder q
values are pinned against a bisection of the signed distance, and a cylinder's
layers against the 2D disk.
"""
import numpy as np

FACES = ("-x", "+x", "-y", "+y", "-z", "+z")
LAM_MIN = 1e-12      # smallest q given to a link whose node lies on the wall within rounding


class Domain:
    def __init__(self, lat, nx, ny, nz=1, periodic=(True, True, True), outlet_face=None):
        self.lat = lat
        self.shape = (nz, ny, nx)            # array order (z, y, x)
        self.n = (nx, ny, nz)                # axis order (x, y, z)
        self.periodic = tuple(bool(p) for p in periodic)
        if lat.d == 2:
            assert nz == 1
            self.periodic = (self.periodic[0], self.periodic[1], True)
        self.outlet_face = outlet_face
        if outlet_face is not None:
            assert not self.periodic[outlet_face // 2], "outlet face must be on a non-periodic axis"
        self.N = nx * ny * nz

    def coords(self, idx=None):
        """Integer coordinates (3, n) of the given nodes (all by default), node index
        n = x + nx (y + ny z)."""
        nx, ny, nz = self.n
        idx = np.arange(self.N) if idx is None else np.asarray(idx, dtype=np.int64)
        return np.stack([idx % nx, (idx // nx) % ny, idx // (nx * ny)])

    def min_image(self, d):
        """Minimum-image displacement on periodic axes; d has shape (3, ...)."""
        d = np.array(d, dtype=np.float64)
        for a in range(3):
            if self.periodic[a]:
                L = self.n[a]
                d[a] = d[a] - L * np.round(d[a] / L)
        return d


class Sphere:
    # axes the distance is measured along (a cylinder drops z)
    AXES = np.array([1.0, 1.0, 1.0])

    def __init__(self, centre, radius, solid_inside=True, V=(0.0, 0.0, 0.0), Omega=(0.0, 0.0, 0.0)):
        self.centre = np.asarray(centre, dtype=np.float64).reshape(3)
        self.radius = float(radius)
        self.solid_inside = bool(solid_inside)
        self.V = np.asarray(V, dtype=np.float64).reshape(3)
        self.Omega = np.asarray(Omega, dtype=np.float64).reshape(3)

    def _rel(self, dom, pts):
        return dom.min_image(pts - self.centre[:, None]) * self.AXES[:, None]

    def solid(self, dom, pts):
        d = self._rel(dom, pts)
        r2 = (d * d).sum(axis=0)
        R2 = self.radius ** 2
        return r2 < R2 if self.solid_inside else r2 > R2

    def on_or_solid(self, dom, pts):
        d = self._rel(dom, pts)
        r2 = (d * d).sum(axis=0)
        R2 = self.radius ** 2
        return r2 <= R2 if self.solid_inside else r2 >= R2

    def crossing(self, dom, xf, c):
        """First crossing lam in (0, 1] of the segment xf - lam c with the surface, NaN if none."""
        d = self._rel(dom, xf)
        c = c * self.AXES[:, None]
        a = (c * c).sum(axis=0)
        b = (d * c).sum(axis=0)
        c0 = (d * d).sum(axis=0) - self.radius ** 2
        disc = b * b - a * c0
        ok = (disc >= 0.0) & (a > 0.0)
        sq = np.sqrt(np.where(ok, disc, 0.0))
        aa = np.where(a > 0.0, a, 1.0)
        # |d - lam c|^2 = R^2  <=>  a lam^2 - 2 b lam + c0 = 0
        lam = (b - sq) / aa if self.solid_inside else (b + sq) / aa
        # a fluid node lying on the surface to within rounding gives a root at
        # lam ~ 0 (possibly -1e-16): it is accepted and clamped to LAM_MIN
        good = ok & (lam > -1e-12) & (lam <= 1.0 + 1e-12)
        return np.where(good, np.clip(lam, LAM_MIN, 1.0), np.nan)

    def velocity(self, dom, xw):
        r = self._rel(dom, xw)
        return self.V[:, None] + np.cross(self.Omega, r.T).T


class Cylinder(Sphere):
    """Circular cylinder of infinite extent along z whose axis passes through
    ``centre`` (the cylindrical Couette geometry of Sec. III.B on a 3D lattice):
    the sphere's distance, crossing and rigid-body velocity taken in the
    xy-plane.  A direction along the axis never crosses it."""
    AXES = np.array([1.0, 1.0, 0.0])


class FaceWall:
    def __init__(self, face, q=0.5, velocity=None):
        self.face = int(face)
        self.q = float(q)
        self._vel = velocity

    def plane(self, dom):
        a = self.face // 2
        return -self.q if self.face % 2 == 0 else dom.n[a] - 1 + self.q

    def crossing(self, dom, xf, c):
        a = self.face // 2
        ca = c[a].astype(np.float64)
        with np.errstate(divide="ignore", invalid="ignore"):
            lam = (xf[a] - self.plane(dom)) / ca
        good = (ca != 0) & (lam > 0.0) & (lam <= 1.0 + 1e-12)
        return np.where(good, np.minimum(lam, 1.0), np.nan)

    def velocity(self, dom, xw):
        if self._vel is None:
            return np.zeros_like(xw, dtype=np.float64)
        if callable(self._vel):
            return np.asarray(self._vel(xw), dtype=np.float64)
        return np.repeat(np.asarray(self._vel, dtype=np.float64).reshape(3, 1), xw.shape[1], axis=1)


class TiltedBand:
    """Periodic family of straight channels in a 2D periodic box (oracle-only test
    geometry): with g(x, y) = (y - slope x - b) mod period, a node is fluid iff
    0 < g < width.  The walls are the lines g = 0 and g = width, at rest."""

    def __init__(self, slope, b, period, width):
        self.slope, self.b, self.period, self.width = float(slope), float(b), float(period), float(width)

    def g(self, pts):
        return np.mod(pts[1] - self.slope * pts[0] - self.b, self.period)

    def on_or_solid(self, dom, pts):
        g = self.g(pts)
        return ~((g > 0.0) & (g < self.width))

    def crossing(self, dom, xf, c):
        g0 = self.g(xf)                              # in (0, width) for a fluid node
        dg = c[1] - self.slope * c[0]                # g(xf - lam c) = g0 - lam dg
        with np.errstate(divide="ignore", invalid="ignore"):
            lam_lo = g0 / dg                         # reaches g = 0 (dg > 0)
            lam_hi = (g0 - self.width) / dg          # reaches g = width (dg < 0)
        lam = np.where(dg > 0, lam_lo, np.where(dg < 0, lam_hi, np.nan))
        good = (lam > 0.0) & (lam <= 1.0 + 1e-12)
        return np.where(good, np.minimum(lam, 1.0), np.nan)

    def velocity(self, dom, xw):
        return np.zeros_like(xw, dtype=np.float64)


def parabolic_inlet(ny, u_max):
    """u_x at the -x wall: 4 u_max (y+1/2)(ny-1/2-y)/ny^2 (channel walls at y=-1/2, ny-1/2)."""
    def vel(xw):
        y = xw[1]
        ux = 4.0 * u_max * (y + 0.5) * (ny - 0.5 - y) / float(ny * ny)
        return np.stack([ux, np.zeros_like(ux), np.zeros_like(ux)])
    return vel


def _bbox_nodes(dom, sph, pad):
    """Node indices of the (wrapped / clipped) integer box around a sphere."""
    rng = []
    for a in range(3):
        if dom.lat.d == 2 and a == 2:
            rng.append(np.array([0]))
            continue
        if sph.AXES[a] == 0.0:                   # unbounded along this axis (cylinder)
            rng.append(np.arange(dom.n[a]))
            continue
        lo = int(np.floor(sph.centre[a] - sph.radius)) - pad
        hi = int(np.ceil(sph.centre[a] + sph.radius)) + pad
        r = np.arange(lo, hi + 1)
        L = dom.n[a]
        if dom.periodic[a]:
            r = np.unique(np.mod(r, L))
        else:
            r = r[(r >= 0) & (r < L)]
        rng.append(r)
    z, y, x = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
    return (x + dom.n[0] * (y + dom.n[1] * z)).reshape(-1)


def classify(dom, spheres):
    """Boolean fluid mask (nz, ny, nx): strictly outside every solid region."""
    X = dom.coords().astype(np.float64)
    fluid = np.ones(dom.N, dtype=bool)
    for s in spheres:
        if isinstance(s, Sphere) and s.solid_inside:
            idx = _bbox_nodes(dom, s, 1)
            fluid[idx] &= ~s.on_or_solid(dom, X[:, idx])
        else:
            fluid &= ~s.on_or_solid(dom, X)
    return fluid.reshape(dom.shape)


def _source(dom, x, c):
    """Pull source x - c with wrap on periodic axes; returns (src coords, inside flag)."""
    src = x - c[:, None]
    inside = np.ones(x.shape[1], dtype=bool)
    for a in range(3):
        L = dom.n[a]
        if dom.periodic[a]:
            src[a] = np.mod(src[a], L)
        else:
            inside &= (src[a] >= 0) & (src[a] < L)
    return src, inside


def _index(dom, p):
    nx, ny, _ = dom.n
    return p[0] + nx * (p[1] + ny * p[2])


def outlet_producer(dom, fluid_flat, x, c):
    """For pairs whose source lies beyond the outlet face: the producer node index
    (source pulled back onto the face layer) if that node exists and is fluid, else -1."""
    f = dom.outlet_face
    a = f // 2
    prod = x - c[:, None]
    prod[a] = 0 if f % 2 == 0 else dom.n[a] - 1
    ok = np.ones(x.shape[1], dtype=bool)
    for b in range(3):
        L = dom.n[b]
        if dom.periodic[b]:
            prod[b] = np.mod(prod[b], L)
        else:
            ok &= (prod[b] >= 0) & (prod[b] < L)
    idx = np.where(ok, _index(dom, np.where(ok, prod, 0)), 0)
    ok &= fluid_flat[idx]
    return np.where(ok, idx, -1)


def beyond_outlet(dom, src):
    f = dom.outlet_face
    if f is None:
        return np.zeros(src.shape[1], dtype=bool)
    a = f // 2
    return src[a] < 0 if f % 2 == 0 else src[a] >= dom.n[a]


def cut_links(dom, fluid, spheres=(), faces=(), uw_t1_fn=None, nodes=None):
    """All cut links of a fluid mask.

    Returns a dict of arrays: node (n,), dir (n,), q (n,), uw_t (3, n), uw_t1 (3, n).
    Links are ordered by node index, then direction.  ``uw_t1_fn(shape, xw)``
    optionally gives the wall velocity at t+1 (moving bodies); by default the wall
    velocity does not change over the step.  ``nodes`` restricts the search to the
    given fluid nodes (sorted ascending).
    """
    lat = dom.lat
    fl = fluid.reshape(-1)
    if nodes is None:
        nodes = np.flatnonzero(fl)
    else:
        nodes = np.asarray(nodes, dtype=np.int64)
        assert fl[nodes].all() and np.all(np.diff(nodes) > 0)
    X = dom.coords(nodes)
    xs = X
    out = {"node": [], "dir": [], "q": [], "uw_t": [], "uw_t1": [], "shape": []}
    for i in range(1, lat.q):
        c = lat.c[i]
        src, inside = _source(dom, xs.copy(), c)
        src_idx = np.where(inside, _index(dom, np.where(inside, src, 0)), 0)
        src_fluid = inside & fl[src_idx]
        need = ~src_fluid
        if dom.outlet_face is not None:
            bo = beyond_outlet(dom, src) & need
            if bo.any():
                prod = outlet_producer(dom, fl, xs[:, bo], c)
                covered = np.zeros_like(need)
                covered[np.flatnonzero(bo)[prod >= 0]] = True
                need &= ~covered
        if not need.any():
            continue
        xf = xs[:, need].astype(np.float64)
        cc = np.repeat(c.reshape(3, 1).astype(np.float64), xf.shape[1], axis=1)
        best = np.full(xf.shape[1], np.inf)
        owner = np.full(xf.shape[1], -1)
        shapes = list(spheres) + list(faces)
        link_nodes = nodes[need]                      # sorted ascending
        for k, shp in enumerate(shapes):
            if isinstance(shp, Sphere) and shp.solid_inside:
                # only links whose node lies in the sphere's box padded by 2 can cross it
                cand = _bbox_nodes(dom, shp, 2)
                pos = np.searchsorted(link_nodes, cand)
                keep = pos < link_nodes.size
                pos, cand = pos[keep], cand[keep]
                sel = pos[link_nodes[pos] == cand]        # one link per node per direction
            else:
                sel = np.arange(link_nodes.size)
            if sel.size == 0:
                continue
            lam = shp.crossing(dom, xf[:, sel], cc[:, sel])
            better = np.isfinite(lam) & (lam < best[sel])
            best[sel] = np.where(better, lam, best[sel])
            owner[sel] = np.where(better, k, owner[sel])
        if (owner < 0).any():
            bad = np.flatnonzero(owner < 0)[0]
            raise ValueError(f"no wall crossing for link node={link_nodes[bad]} dir={i}")
        xw = xf - best * cc
        uw = np.zeros_like(xw)
        uw1 = np.zeros_like(xw)
        for k, shp in enumerate(shapes):
            sel = owner == k
            if sel.any():
                uw[:, sel] = shp.velocity(dom, xw[:, sel])
                uw1[:, sel] = uw[:, sel] if uw_t1_fn is None else uw_t1_fn(shp, xw[:, sel])
        out["node"].append(nodes[need])
        out["dir"].append(np.full(need.sum(), i))
        out["q"].append(best)
        out["uw_t"].append(uw)
        out["uw_t1"].append(uw1)
        out["shape"].append(owner)
    if not out["node"]:
        return {"node": np.zeros(0, np.int64), "dir": np.zeros(0, np.int64), "q": np.zeros(0),
                "uw_t": np.zeros((3, 0)), "uw_t1": np.zeros((3, 0)), "shape": np.zeros(0, np.int64)}
    node = np.concatenate(out["node"])
    d = np.concatenate(out["dir"])
    order = np.lexsort((d, node))
    return {
        "node": node[order].astype(np.int64),
        "dir": d[order].astype(np.int64),
        "q": np.concatenate(out["q"])[order],
        "uw_t": np.concatenate(out["uw_t"], axis=1)[:, order],
        "uw_t1": np.concatenate(out["uw_t1"], axis=1)[:, order],
        "shape": np.concatenate(out["shape"])[order].astype(np.int64),   # spheres first, then faces
    }
