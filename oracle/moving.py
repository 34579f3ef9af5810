"""Moving rigid sphere with prescribed motion (Sec. II.E moving boundaries; the
Jeffery-orbit study of Sec. III.C uses moving objects with refilled fresh nodes).

Kinematics (prescribed, not computed from forces): centre
x_c(t) = x_0 + A sin(2 pi t / T) e, translational velocity
V(t) = A (2 pi / T) cos(2 pi t / T) e, constant angular velocity Omega; or a
path of any form given by samples of x_c, V and optionally Omega per step
(SampledKinematics).

One step t -> t+1 (readings, listed in the design notes):
1. geometry(t): fluid nodes and cut links of the sphere at x_c(t);
   u_w(t) = V(t) + Omega(t) x (x_W - x_c(t)) and
   u_w(t+1) = V(t+1) + Omega(t+1) x (x_W - x_c(t)) at each link's wall point;
2. nodes fluid at t but solid at t-1 are refilled with
   f^eq(rho_bar, V(t) + Omega(t) x (x - x_c(t))) before the step;
3. the ordinary step with that geometry.

Status: pinned -- V(t) against central differences of x_c(t) over a period and
its closed values at t = 0 and T/4; a sampled path against the sinusoid it
samples and against the co-moving invariant on a straight path; a sampled spin
against the constant spin it repeats, its time index (an impulsive spin-up
moves the walls at t+1 only) and the mirror symmetry of a reversed spin;
several spheres by the co-moving invariant with two spheres, the independence
of their order (flow, and each sphere's force and torque) and hand-placed
refill points; the per-sphere force and torque (links grouped by the sphere
they cross, torques about each centre) by two mirror-image spheres; the refill
rule against hand-listed
neighbour sets (tests/test_oracle_refill.py); the co-moving invariant (a sphere
moving at the velocity of a uniform flow leaves it unchanged, refills
included).
"""
import numpy as np

from . import geometry as G
from .solver import Simulation


class Kinematics:
    def __init__(self, x0, amplitude, period, direction, omega):
        self.x0 = np.asarray(x0, dtype=np.float64)
        self.A = float(amplitude)
        self.T = float(period)
        self.e = np.asarray(direction, dtype=np.float64)
        self.Omega = np.asarray(omega, dtype=np.float64)

    def centre(self, t):
        return self.x0 + self.A * np.sin(2.0 * np.pi * t / self.T) * self.e

    def velocity(self, t):
        return self.A * (2.0 * np.pi / self.T) * np.cos(2.0 * np.pi * t / self.T) * self.e

    def omega(self, t):
        return self.Omega.copy()


class SampledKinematics:
    """A prescribed path given by samples: x_c(t) = centre[t], V(t) =
    velocity[t] at integer steps t (arrays [n][3]); the angular velocity is
    constant (omega of 3 values) or sampled too (omega [n][3]).  The step of
    MovingSphereSim asks for x_c(t), V(t), V(t+1), Omega(t) and Omega(t+1)
    only, so n samples drive n - 2 steps."""

    def __init__(self, centre, velocity, omega):
        self.C = np.asarray(centre, dtype=np.float64).reshape(-1, 3)
        self.V = np.asarray(velocity, dtype=np.float64).reshape(-1, 3)
        assert self.C.shape == self.V.shape and self.C.shape[0] >= 2
        om = np.asarray(omega, dtype=np.float64)
        if om.size == 3:
            self.W = None
            self.Omega = om.reshape(3)
        else:
            self.W = om.reshape(-1, 3)
            assert self.W.shape == self.C.shape
            self.Omega = None

    def centre(self, t):
        return self.C[int(t)].copy()

    def velocity(self, t):
        return self.V[int(t)].copy()

    def omega(self, t):
        return self.Omega.copy() if self.W is None else self.W[int(t)].copy()


class MovingSpheresSim:
    """Several rigid spheres in prescribed motion (kins[s] with radii[s]).

    Readings for more than one sphere: a node is solid when it lies in or on
    any sphere; a cut link takes the first crossing over the spheres (the first
    in the list wins a tie, the host builder's rule) and that sphere's wall
    velocities; a fresh node takes the rigid-body velocity of the sphere whose
    surface is nearest (|x - x_c| - R smallest, the first on a tie).  Forces and
    torques are kept for one sphere (about its centre)."""

    def __init__(self, dom, radii, kins, tau, variant="FQ", q_cut=0.01, rho0=1.0, u0=(0.0, 0.0, 0.0), magic=None,
                 wall_neq="bounceback"):
        self.dom = dom
        self.radii = [float(r) for r in radii]
        self.kins = list(kins)
        assert len(self.radii) == len(self.kins) >= 1
        self.variant, self.q_cut, self.wall_neq = variant, q_cut, wall_neq
        self.sim = Simulation(dom, tau, rho0=rho0, u0=u0, magic=magic)
        self.t = 0
        self._install(first=True)
        self.sim.init_equilibrium()

    def geometry(self, t):
        return self._geometry(t)

    def _geometry(self, t):
        sphs = [G.Sphere(k.centre(t), r, True, V=k.velocity(t), Omega=k.omega(t))
                for r, k in zip(self.radii, self.kins)]
        fluid = G.classify(self.dom, sphs)
        at1 = {id(s): (k.centre(t), k.velocity(t + 1), k.omega(t + 1)) for s, k in zip(sphs, self.kins)}

        def uw1(shape, xw):
            c_t, V1, Om1 = at1[id(shape)]
            r = self.dom.min_image(xw - c_t[:, None])
            return V1[:, None] + np.cross(Om1, r.T).T
        links = G.cut_links(self.dom, fluid, sphs, uw_t1_fn=uw1)
        return fluid, links, sphs

    def body_velocity(self, sphs, X):
        """Rigid-body velocity at the points X (3, N) of the sphere whose surface is nearest."""
        u = sphs[0].velocity(self.dom, X)
        if len(sphs) > 1:
            gap = np.stack([np.sqrt((s._rel(self.dom, X) ** 2).sum(axis=0)) - s.radius for s in sphs])
            near = np.argmin(gap, axis=0)
            for j, s in enumerate(sphs[1:], start=1):
                sel = near == j
                if sel.any():
                    u[:, sel] = s.velocity(self.dom, X[:, sel])
        return u

    def _install(self, first=False):
        fluid, links, sphs = self._geometry(self.t)
        if not first:
            X = self.dom.coords().astype(np.float64)
            self.sim.refill(fluid, self.body_velocity(sphs, X))
        self.sim.set_geometry(fluid, links, self.variant, self.q_cut, wall_neq=self.wall_neq)

    def step(self):
        # one force group per sphere (the sphere each link crosses), torques about
        # the sphere centres at the geometry's time t
        self.sim.set_link_groups(self.sim.links["shape"], len(self.kins),
                                 np.array([k.centre(self.t) for k in self.kins]))
        self.sim.step()
        self.t += 1
        self._install()

    def run(self, n):
        for _ in range(int(n)):
            self.step()


class MovingSphereSim(MovingSpheresSim):
    """One rigid sphere of radius `radius` moving with `kin`."""

    def __init__(self, dom, radius, kin, tau, **kw):
        super().__init__(dom, [radius], [kin], tau, **kw)

    @property
    def radius(self):
        return self.radii[0]

    @property
    def kin(self):
        return self.kins[0]

    def geometry(self, t):
        fluid, links, sphs = self._geometry(t)
        return fluid, links, sphs[0]
