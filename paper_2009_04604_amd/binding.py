"""ctypes binding of liblbm (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch supplies the device memory arena for the population buffers and the
stream (torch.cuda.current_stream()), nothing else.  The functions keep the
C names (lbm_init_domain, lbm_set_boundary_links, lbm_step, lbm_macros, ...);
``Domain`` and ``Geometry`` are thin object wrappers over them.

The library must have been built (``python -m paper_2009_04604_amd.build``);
loading fails loudly otherwise -- there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LATTICES = {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2}
LAYOUTS = {"compact": 0, "dense": 1}
COLLISIONS = {"BGK": 0, "TRT": 1}
STORAGE = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3, "f16s-sr": 2, "bf16s-sr": 3}
# storage names with stochastic rounding of the 16-bit stores (LBM_ROUND_STOCHASTIC)
STOCHASTIC = {"f16s-sr", "bf16s-sr"}
VARIANTS = {"FQ": 0, "F": 1, "UQ": 2, "U": 3, "HWBB": 4}
WALL_NEQ = {"bounceback": 0, "regularized": 1}
FACES = {"-x": 0, "+x": 1, "-y": 2, "+y": 3, "-z": 4, "+z": 5}
Q_OF = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27}
D_OF = {"D2Q9": 2, "D3Q19": 3, "D3Q27": 3}

EXPORTED = [
    "lbm_arena_bytes", "lbm_init_domain", "lbm_set_boundary_links", "lbm_step", "lbm_macros",
    "lbm_get_state", "lbm_set_state", "lbm_set_stream", "lbm_set_launch_option", "lbm_get_info", "lbm_free_domain",
    "lbm_last_error", "lbm_set_moving_sphere", "lbm_geometry_create", "lbm_geometry_add_sphere", "lbm_geometry_add_spheres",
    "lbm_geometry_add_face_wall", "lbm_geometry_build", "lbm_geometry_get", "lbm_geometry_free",
    "lbm_batch_create", "lbm_batch_step", "lbm_batch_set_option", "lbm_batch_autotune", "lbm_batch_get_choice",
    "lbm_batch_free", "lbm_step_batch", "lbm_set_link_groups", "lbm_momentum_exchange", "lbm_geometry_get_shapes",
    "lbm_set_wall_neq", "lbm_geometry_add_cylinder", "lbm_force_torque", "lbm_set_force_tracking",
    "lbm_moving_force", "lbm_moving_forces", "lbm_macros_noalloc", "lbm_stream_probe", "lbm_set_moving_sphere_path",
    "lbm_set_moving_sphere_motion", "lbm_set_moving_spheres",
]
BATCH_OPTIONS = {"graph": 0, "grid": 1, "order": 2, "autotune": 3}


class LBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblbm error {code}: {msg}")
        self.code = code


class DomainDesc(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("periodic", ctypes.c_int32), ("storage", ctypes.c_int32), ("tau", ctypes.c_double),
        ("force", ctypes.c_double * 3), ("rho0", ctypes.c_double), ("u0", ctypes.c_double * 3),
        ("outlet_face", ctypes.c_int32), ("stream", ctypes.c_void_p), ("arena", ctypes.c_void_p),
        ("arena_bytes", ctypes.c_size_t), ("layout", ctypes.c_int32), ("collision", ctypes.c_int32),
        ("magic", ctypes.c_double), ("rounding", ctypes.c_int32),
    ]


class DomainInfo(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int64), ("n_fluid", ctypes.c_int64), ("n_boundary_nodes", ctypes.c_int64),
        ("n_links", ctypes.c_int64), ("population_bytes", ctypes.c_int64), ("link_bytes", ctypes.c_int64),
        ("steps_done", ctypes.c_int64), ("q", ctypes.c_int32), ("storage", ctypes.c_int32),
    ]


_lib = None
P = ctypes.c_void_p
I32, I64, DBL = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


def lib():
    """Load liblbm.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2009_04604_amd.build`")
    # torch first: liblbm then binds to the HIP runtime torch has loaded, so torch's
    # streams and device memory are valid in the library (loaded first, the library
    # would pull in the system runtime and torch would bring a second one)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "lbm_arena_bytes": (ctypes.c_size_t, [P, P]),
        "lbm_set_launch_option": (I32, [P, I32, I32]),
        "lbm_init_domain": (I32, [P, P, P]),
        "lbm_set_boundary_links": (I32, [P, I64, P, P, P, P, P, I32, DBL]),
        "lbm_step": (I32, [P, I32]),
        "lbm_set_moving_sphere": (I32, [P, P, DBL, DBL, DBL, P, P, I32, DBL]),
        "lbm_set_moving_sphere_path": (I32, [P, DBL, P, I64, P, P, I32, DBL]),
        "lbm_set_moving_sphere_motion": (I32, [P, DBL, I64, P, P, P, I32, DBL]),
        "lbm_set_moving_spheres": (I32, [P, I32, P, I64, P, P, P, I32, DBL]),
        "lbm_macros": (I32, [P, P, P, P]),
        "lbm_get_state": (I32, [P, P]),
        "lbm_set_state": (I32, [P, P]),
        "lbm_set_stream": (I32, [P, P]),
        "lbm_get_info": (I32, [P, P]),
        "lbm_free_domain": (I32, [P]),
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_geometry_create": (I32, [I32, I32, I32, I32, I32, I32, P]),
        "lbm_geometry_add_sphere": (I32, [P, P, DBL, I32, P, P]),
        "lbm_geometry_add_spheres": (I32, [P, I64, P, P]),
        "lbm_geometry_add_face_wall": (I32, [P, I32, DBL, P, I32]),
        "lbm_geometry_build": (I32, [P, P, P]),
        "lbm_geometry_get": (I32, [P, P, P, P, P, P, P]),
        "lbm_geometry_free": (I32, [P]),
        "lbm_batch_create": (I32, [P, P]),
        "lbm_batch_step": (I32, [P, P, I32, I32]),
        "lbm_batch_set_option": (I32, [P, I32, I32]),
        "lbm_batch_autotune": (I32, [P, P, I32, I32]),
        "lbm_batch_get_choice": (I32, [P, P, P, P]),
        "lbm_batch_free": (I32, [P]),
        "lbm_step_batch": (I32, [P, I32, I32]),
        "lbm_set_link_groups": (I32, [P, P, I32]),
        "lbm_momentum_exchange": (I32, [P, P]),
        "lbm_geometry_get_shapes": (I32, [P, P]),
        "lbm_set_wall_neq": (I32, [P, I32]),
        "lbm_geometry_add_cylinder": (I32, [P, P, DBL, I32, P, P]),
        "lbm_force_torque": (I32, [P, P, P, P]),
        "lbm_set_force_tracking": (I32, [P, I32]),
        "lbm_moving_force": (I32, [P, P, P]),
        "lbm_moving_forces": (I32, [P, I32, P, P]),
        "lbm_macros_noalloc": (I32, [P, P, P, P]),
        "lbm_stream_probe": (I32, [P, P, I64, I64, I32, I32, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(code):
    if code != LBM_OK:
        raise LBMError(code, lib().lbm_last_error().decode())
    return code


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


def make_desc(lattice, nx, ny, nz, tau, storage="f32", periodic=(True, True, True), force=(0, 0, 0),
              rho0=1.0, u0=(0, 0, 0), outlet_face=None, stream=None, arena=None, arena_bytes=0, layout="compact",
              collision="BGK", magic=3.0 / 16.0):
    d = DomainDesc()
    d.lattice = LATTICES[lattice]
    d.nx, d.ny, d.nz = int(nx), int(ny), int(nz)
    d.periodic = sum(int(bool(p)) << a for a, p in enumerate(periodic))
    d.storage = STORAGE[storage]
    d.rounding = 1 if storage in STOCHASTIC else 0
    d.tau = float(tau)
    for a in range(3):
        d.force[a] = float(force[a])
        d.u0[a] = float(u0[a])
    d.rho0 = float(rho0)
    d.outlet_face = -1 if outlet_face is None else (FACES[outlet_face] if isinstance(outlet_face, str) else int(outlet_face))
    d.stream = stream
    d.arena = arena
    d.arena_bytes = int(arena_bytes)
    d.layout = LAYOUTS[layout]
    d.collision = COLLISIONS[collision] if isinstance(collision, str) else int(collision)
    d.magic = float(magic)
    return d


# ---- C names ------------------------------------------------------------------
def lbm_arena_bytes(desc, fluid_mask=None):
    m = None if fluid_mask is None else np.ascontiguousarray(np.asarray(fluid_mask).reshape(-1), dtype=np.uint8)
    return lib().lbm_arena_bytes(ctypes.byref(desc), _ptr(m))


def lbm_set_launch_option(h, option, value):
    _check(lib().lbm_set_launch_option(h, int(option), int(value)))


def lbm_init_domain(desc, fluid_mask):
    m = np.ascontiguousarray(np.asarray(fluid_mask).reshape(-1), dtype=np.uint8)
    h = ctypes.c_void_p()
    _check(lib().lbm_init_domain(ctypes.byref(desc), _ptr(m), ctypes.byref(h)))
    return h


def lbm_set_boundary_links(h, node, dir, q, uw_t=None, uw_t1=None, variant="FQ", q_cutoff=0.01):
    node = np.ascontiguousarray(node, dtype=np.int64)
    dir = np.ascontiguousarray(dir, dtype=np.int8)
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = node.size

    def vel(u):
        if u is None:
            return None
        u = np.asarray(u, dtype=np.float64)
        if u.shape == (3, n):
            u = u.T
        return np.ascontiguousarray(u.reshape(n, 3))
    uw_t, uw_t1 = vel(uw_t), vel(uw_t1)
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    _check(lib().lbm_set_boundary_links(h, n, _ptr(node), _ptr(dir), _ptr(q), _ptr(uw_t), _ptr(uw_t1), v, float(q_cutoff)))


def lbm_set_moving_sphere(h, x0, radius, amplitude, period, direction, omega, variant="FQ", q_cutoff=0.01):
    x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(3)
    e = np.ascontiguousarray(direction, dtype=np.float64).reshape(3)
    om = np.ascontiguousarray(omega, dtype=np.float64).reshape(3)
    v = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    _check(lib().lbm_set_moving_sphere(h, _ptr(x0), float(radius), float(amplitude), float(period), _ptr(e), _ptr(om),
                                       v, float(q_cutoff)))


def lbm_set_moving_sphere_path(h, radius, omega, centre, velocity, variant="FQ", q_cutoff=0.01):
    c = np.ascontiguousarray(centre, dtype=np.float64).reshape(-1, 3)
    v = np.ascontiguousarray(velocity, dtype=np.float64).reshape(-1, 3)
    if c.shape != v.shape:
        raise ValueError("centre and velocity need the same number of samples")
    om = np.ascontiguousarray(omega, dtype=np.float64).reshape(3)
    var = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    _check(lib().lbm_set_moving_sphere_path(h, float(radius), _ptr(om), c.shape[0], _ptr(c), _ptr(v), var,
                                            float(q_cutoff)))


def lbm_set_moving_sphere_motion(h, radius, centre, velocity, omega, variant="FQ", q_cutoff=0.01):
    c = np.ascontiguousarray(centre, dtype=np.float64).reshape(-1, 3)
    v = np.ascontiguousarray(velocity, dtype=np.float64).reshape(-1, 3)
    om = np.ascontiguousarray(omega, dtype=np.float64).reshape(-1, 3)
    if c.shape != v.shape or c.shape != om.shape:
        raise ValueError("centre, velocity and omega need the same number of samples")
    var = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    _check(lib().lbm_set_moving_sphere_motion(h, float(radius), c.shape[0], _ptr(c), _ptr(v), _ptr(om), var,
                                              float(q_cutoff)))


def lbm_set_moving_spheres(h, radius, centre, velocity, omega, variant="FQ", q_cutoff=0.01):
    r = np.ascontiguousarray(radius, dtype=np.float64).reshape(-1)
    ns = r.size
    c = np.ascontiguousarray(centre, dtype=np.float64).reshape(-1, ns, 3)
    v = np.ascontiguousarray(velocity, dtype=np.float64).reshape(-1, ns, 3)
    om = np.ascontiguousarray(omega, dtype=np.float64).reshape(-1, ns, 3)
    if c.shape != v.shape or c.shape != om.shape:
        raise ValueError("centre, velocity and omega need the same [n_samples, n_spheres, 3] shape")
    var = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    _check(lib().lbm_set_moving_spheres(h, ns, _ptr(r), c.shape[0], _ptr(c), _ptr(v), _ptr(om), var,
                                        float(q_cutoff)))


def lbm_step(h, n_steps):
    _check(lib().lbm_step(h, int(n_steps)))


def lbm_macros(h, N, D, fields=True):
    rho = np.empty(N) if fields else None
    u = np.empty(N * D) if fields else None
    sums = np.empty(D + 2)
    code = lib().lbm_macros(h, _ptr(rho), _ptr(u), _ptr(sums))
    if code not in (LBM_OK, LBM_EUNSTABLE):
        _check(code)
    return rho, (u.reshape(N, D) if fields else None), sums, code == LBM_EUNSTABLE


def lbm_get_state(h, Q, N):
    f = np.empty((Q, N))
    _check(lib().lbm_get_state(h, _ptr(f)))
    return f


def lbm_set_state(h, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(lib().lbm_set_state(h, _ptr(f)))


def lbm_get_info(h):
    info = DomainInfo()
    _check(lib().lbm_get_info(h, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in DomainInfo._fields_}


def lbm_free_domain(h):
    _check(lib().lbm_free_domain(h))


def lbm_stream_probe(src, dst, n, stride, arrays, shift, stream=None):
    """Bandwidth calibration copy (see include/lbm.h); src, dst torch float32 CUDA tensors."""
    need = int(arrays) * int(stride)
    if src.dtype != dst.dtype or str(src.dtype) != "torch.float32" or src.numel() < need or dst.numel() < need:
        raise ValueError(f"lbm_stream_probe: src and dst must be float32 with at least arrays * stride = {need} elements")
    if stream is None:
        stream = _torch_stream()
    _check(lib().lbm_stream_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), int(n),
                                  int(stride), int(arrays), int(shift), stream))


# ---- object wrappers ----------------------------------------------------------
class Domain:
    """One lattice resident on the GPU.

    fluid_mask: (nz, ny, nx) or flat bool array.  The population buffers live in
    a torch uint8 tensor (the arena) kept alive by this object; work goes to the
    current torch stream unless ``stream`` is given.
    """

    def __init__(self, lattice, nx, ny, nz, fluid_mask, tau, storage="f32", periodic=(True, True, True),
                 force=(0, 0, 0), rho0=1.0, u0=(0, 0, 0), outlet_face=None, stream=None, torch_arena=True,
                 layout="compact", collision="BGK", magic=3.0 / 16.0):
        self.lattice, self.storage = lattice, storage
        self.n = (int(nx), int(ny), int(nz))
        self.N = int(nx) * int(ny) * int(nz)
        self.Q, self.D = Q_OF[lattice], D_OF[lattice]
        if stream is None:
            stream = _torch_stream()
        desc = make_desc(lattice, nx, ny, nz, tau, storage, periodic, force, rho0, u0, outlet_face, stream,
                         layout=layout, collision=collision, magic=magic)
        self._arena = None
        if torch_arena:
            import torch
            nbytes = lbm_arena_bytes(desc, fluid_mask)
            self._arena = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            base = self._arena.data_ptr()
            desc.arena = (base + 255) // 256 * 256
            desc.arena_bytes = nbytes
        self.desc = desc
        self.h = lbm_init_domain(desc, fluid_mask)

    def set_boundary_links(self, links=None, variant="FQ", q_cutoff=0.01, **kw):
        if links is not None:
            kw = {"node": links["node"], "dir": links["dir"], "q": links["q"],
                  "uw_t": links.get("uw_t"), "uw_t1": links.get("uw_t1"), **kw}
        lbm_set_boundary_links(self.h, variant=variant, q_cutoff=q_cutoff, **kw)

    def set_moving_sphere(self, x0, radius, amplitude, period, direction, omega, variant="FQ", q_cutoff=0.01):
        lbm_set_moving_sphere(self.h, x0, radius, amplitude, period, direction, omega, variant, q_cutoff)

    def set_moving_sphere_path(self, radius, omega, centre, velocity, variant="FQ", q_cutoff=0.01):
        """centre, velocity: [n_samples, 3] per step (see lbm_set_moving_sphere_path)."""
        lbm_set_moving_sphere_path(self.h, radius, omega, centre, velocity, variant, q_cutoff)

    def set_moving_spheres(self, radius, centre, velocity, omega, variant="FQ", q_cutoff=0.01):
        """radius [n_spheres]; centre, velocity, omega: [n_samples, n_spheres, 3] (see lbm_set_moving_spheres)."""
        lbm_set_moving_spheres(self.h, radius, centre, velocity, omega, variant, q_cutoff)

    def set_moving_sphere_motion(self, radius, centre, velocity, omega, variant="FQ", q_cutoff=0.01):
        """centre, velocity, omega: [n_samples, 3] per step (see lbm_set_moving_sphere_motion)."""
        lbm_set_moving_sphere_motion(self.h, radius, centre, velocity, omega, variant, q_cutoff)

    def step(self, n=1):
        lbm_step(self.h, n)

    def macros(self, fields=True):
        """(rho [N], u [N, D], sums, unstable) -- synchronises the stream."""
        return lbm_macros(self.h, self.N, self.D, fields)

    def get_state(self):
        return lbm_get_state(self.h, self.Q, self.N)

    def set_state(self, f):
        lbm_set_state(self.h, f)

    def set_stream(self, stream):
        _check(lib().lbm_set_stream(self.h, stream))

    def set_link_groups(self, group=None, n_groups=1):
        g = None if group is None else np.ascontiguousarray(group, dtype=np.int32)
        _check(lib().lbm_set_link_groups(self.h, _ptr(g), int(n_groups)))
        self._n_groups = int(n_groups)

    def set_wall_neq(self, mode):
        """Wall non-equilibrium estimator: "bounceback" (eq. neqbb-s) or
        "regularized" (eq. fi_neq)."""
        m = WALL_NEQ[mode] if isinstance(mode, str) else int(mode)
        _check(lib().lbm_set_wall_neq(self.h, m))

    def force(self):
        """(n_groups, 3) momentum-exchange force of the last step (FP64)."""
        out = np.zeros((getattr(self, "_n_groups", 1), 3))
        _check(lib().lbm_momentum_exchange(self.h, _ptr(out)))
        return out

    def force_torque(self, centres=None):
        """(force, torque), each (n_groups, 3), of the last step; torque about
        centres (n_groups, 3) (None: the origin)."""
        n = getattr(self, "_n_groups", 1)
        c = None if centres is None else np.ascontiguousarray(centres, dtype=np.float64).reshape(n, 3)
        f, t = np.zeros((n, 3)), np.zeros((n, 3))
        _check(lib().lbm_force_torque(self.h, _ptr(c), _ptr(f), _ptr(t)))
        return f, t

    def macros_noalloc(self, rho, u, sums):
        """lbm_macros_noalloc into caller-owned device tensors (float64, CUDA):
        rho (N,) or None, u (N, D) or None, sums (8,); asynchronous on the
        domain's stream."""
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        _check(lib().lbm_macros_noalloc(self.h, ptr(rho), ptr(u), ptr(sums)))

    def set_force_tracking(self, on=True):
        """Moving sphere: evaluate the force and torque of the last step of every
        step() call (before its links are rebuilt)."""
        _check(lib().lbm_set_force_tracking(self.h, 1 if on else 0))

    def moving_force(self):
        """(force (3,), torque (3,)) on the moving sphere during the last step."""
        f, t = np.zeros(3), np.zeros(3)
        _check(lib().lbm_moving_force(self.h, _ptr(f), _ptr(t)))
        return f, t

    def moving_forces(self, n_spheres):
        """(force (n, 3), torque (n, 3)) on each of the domain's n moving spheres
        during the last step, torques about each sphere's own centre."""
        f, t = np.zeros((n_spheres, 3)), np.zeros((n_spheres, 3))
        _check(lib().lbm_moving_forces(self.h, int(n_spheres), _ptr(f), _ptr(t)))
        return f, t

    def set_launch_option(self, option, value):
        lbm_set_launch_option(self.h, option, value)

    def info(self):
        return lbm_get_info(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm_free_domain(self.h)
            self.h = None
            self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _handles(domains):
    hs = [d.h if isinstance(d, Domain) else d for d in domains]
    return (ctypes.c_void_p * max(1, len(hs)))(*hs), len(hs)


def lbm_batch_create(stream=None):
    h = ctypes.c_void_p()
    _check(lib().lbm_batch_create(stream, ctypes.byref(h)))
    return h.value


def lbm_batch_step(b, domains, n_steps):
    arr, n = _handles(domains)
    _check(lib().lbm_batch_step(b, arr, n, int(n_steps)))


def lbm_batch_set_option(b, option, value):
    _check(lib().lbm_batch_set_option(b, BATCH_OPTIONS.get(option, option), int(value)))


def lbm_batch_autotune(b, domains, steps_per_candidate):
    arr, n = _handles(domains)
    _check(lib().lbm_batch_autotune(b, arr, n, int(steps_per_candidate)))


def lbm_batch_get_choice(b):
    g, o, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(lib().lbm_batch_get_choice(b, ctypes.byref(g), ctypes.byref(o), ctypes.byref(us)))
    return {"grid": g.value, "order": o.value, "us_per_step": us.value}


def lbm_batch_free(b):
    _check(lib().lbm_batch_free(b))


def lbm_step_batch(domains, n_steps):
    arr, n = _handles(domains)
    _check(lib().lbm_step_batch(arr, n, int(n_steps)))


class Batch:
    """Many domains stepped together (lbm_batch_*); all on one stream."""

    def __init__(self, stream=None):
        if stream is None:
            stream = _torch_stream()
        self.h = lbm_batch_create(stream)

    def step(self, domains, n_steps):
        lbm_batch_step(self.h, domains, n_steps)

    def set_option(self, option, value):
        lbm_batch_set_option(self.h, option, value)

    def autotune(self, domains, steps_per_candidate=4):
        lbm_batch_autotune(self.h, domains, steps_per_candidate)
        return lbm_batch_get_choice(self.h)

    def choice(self):
        return lbm_batch_get_choice(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Geometry:
    """Host geometry builder (lbm_geometry_*): fluid mask and cut links."""

    def __init__(self, lattice, nx, ny, nz=1, periodic=(True, True, True), outlet_face=None):
        self.lattice = lattice
        self.n = (int(nx), int(ny), int(nz))
        self.N = int(nx) * int(ny) * int(nz)
        per = sum(int(bool(p)) << a for a, p in enumerate(periodic))
        of = -1 if outlet_face is None else (FACES[outlet_face] if isinstance(outlet_face, str) else int(outlet_face))
        h = ctypes.c_void_p()
        _check(lib().lbm_geometry_create(LATTICES[lattice], int(nx), int(ny), int(nz), per, of, ctypes.byref(h)))
        self.h = h

    def add_sphere(self, centre, radius, solid_inside=True, V=None, Omega=None):
        c = np.ascontiguousarray(centre, dtype=np.float64).reshape(3)
        Vv = None if V is None else np.ascontiguousarray(V, dtype=np.float64).reshape(3)
        Om = None if Omega is None else np.ascontiguousarray(Omega, dtype=np.float64).reshape(3)
        _check(lib().lbm_geometry_add_sphere(self.h, _ptr(c), float(radius), int(bool(solid_inside)), _ptr(Vv), _ptr(Om)))

    def add_cylinder(self, centre, radius, solid_inside=True, V=None, Omega=None):
        """Circular cylinder along z through ``centre``."""
        c = np.ascontiguousarray(centre, dtype=np.float64).reshape(3)
        Vv = None if V is None else np.ascontiguousarray(V, dtype=np.float64).reshape(3)
        Om = None if Omega is None else np.ascontiguousarray(Omega, dtype=np.float64).reshape(3)
        _check(lib().lbm_geometry_add_cylinder(self.h, _ptr(c), float(radius), int(bool(solid_inside)), _ptr(Vv),
                                               _ptr(Om)))

    def add_spheres(self, centres, radii):
        c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
        r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
        _check(lib().lbm_geometry_add_spheres(self.h, r.size, _ptr(c), _ptr(r)))

    def add_face_wall(self, face, q_face=0.5, uw=None, profile=0):
        f = FACES[face] if isinstance(face, str) else int(face)
        u = None if uw is None else np.ascontiguousarray(uw, dtype=np.float64).reshape(3)
        _check(lib().lbm_geometry_add_face_wall(self.h, f, float(q_face), _ptr(u), int(profile)))

    def build(self):
        nf, nl = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().lbm_geometry_build(self.h, ctypes.byref(nf), ctypes.byref(nl)))
        n = nl.value
        mask = np.empty(self.N, dtype=np.uint8)
        node = np.empty(n, dtype=np.int64)
        d = np.empty(n, dtype=np.int8)
        q = np.empty(n)
        uw = np.empty((n, 3))
        uw1 = np.empty((n, 3))
        shape = np.empty(n, dtype=np.int32)
        _check(lib().lbm_geometry_get(self.h, _ptr(mask), _ptr(node), _ptr(d), _ptr(q), _ptr(uw), _ptr(uw1)))
        _check(lib().lbm_geometry_get_shapes(self.h, _ptr(shape)))
        return mask, {"node": node, "dir": d.astype(np.int64), "q": q, "uw_t": uw, "uw_t1": uw1,
                      "shape": shape.astype(np.int64)}

    def close(self):
        if getattr(self, "h", None) is not None:
            lib().lbm_geometry_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
