"""Workload set-ups on the product path: geometry from the library's host
builder (lbm_geometry_*), domains on the GPU (lbm_init_domain,
lbm_set_boundary_links).  Inputs are the seeded recipes of ``synth``.
"""
import numpy as np

import synth

from . import binding as B


def annulus_geometry(p):
    """Circular Couette annulus: inner cylinder turning at u_inner, outer at rest."""
    g = B.Geometry("D2Q9", p["nx"], p["ny"], 1)
    om1 = p["u_inner"] / p["r1"]
    g.add_sphere(p["centre"], p["r1"], True, Omega=(0, 0, om1))
    g.add_sphere(p["centre"], p["r2"], False)
    mask, links = g.build()
    g.close()
    return mask, links


def annulus3d_geometry(p, lattice="D3Q19", nz=4):
    """The circular Couette annulus on a 3D lattice: coaxial cylinders along z
    (inner turning at u_inner, outer at rest), periodic in z."""
    g = B.Geometry(lattice, p["nx"], p["ny"], nz)
    om1 = p["u_inner"] / p["r1"]
    g.add_cylinder(p["centre"], p["r1"], True, Omega=(0, 0, om1))
    g.add_cylinder(p["centre"], p["r2"], False)
    mask, links = g.build()
    g.close()
    return mask, links


def couette3d_domain(p, lattice="D3Q19", nz=4, storage="f64", variant="FQ", collision="BGK", magic=3.0 / 16.0,
                     wall_neq="bounceback"):
    mask, links = annulus3d_geometry(p, lattice, nz)
    d = B.Domain(lattice, p["nx"], p["ny"], nz, mask, p["tau"], storage=storage, collision=collision, magic=magic)
    d.set_boundary_links(links, variant=variant)
    d.set_wall_neq(wall_neq)
    return d, mask, links


def channel_geometry(p):
    """Channel with a cylinder: parabolic inlet at x = -1/2, walls at y = -1/2 and
    ny - 1/2, zero-gradient outlet at +x."""
    nx, ny = p["nx"], p["ny"]
    g = B.Geometry("D2Q9", nx, ny, 1, periodic=(False, False, True), outlet_face="+x")
    g.add_sphere(p["centre"], p["radius"], True)
    g.add_face_wall("-x", 0.5, uw=(p["u_max"], 0, 0), profile=1)
    g.add_face_wall("-y", 0.5)
    g.add_face_wall("+y", 0.5)
    mask, links = g.build()
    g.close()
    return mask, links


def packing_geometry(n, centres, radii, lattice="D3Q19"):
    g = B.Geometry(lattice, n, n, n)
    g.add_spheres(centres, radii)
    mask, links = g.build()
    g.close()
    return mask, links


def couette_domain(p, storage="f64", variant="FQ", layout="compact", collision="BGK", magic=3.0 / 16.0,
                   wall_neq="bounceback"):
    mask, links = annulus_geometry(p)
    d = B.Domain("D2Q9", p["nx"], p["ny"], 1, mask, p["tau"], storage=storage, rho0=p.get("rho0", 1.0), layout=layout,
                 collision=collision, magic=magic)
    d.set_boundary_links(links, variant=variant)
    d.set_wall_neq(wall_neq)
    return d, mask, links


def channel_domain(p, storage="f32", variant="FQ", layout="compact", wall_neq="bounceback"):
    mask, links = channel_geometry(p)
    d = B.Domain("D2Q9", p["nx"], p["ny"], 1, mask, p["tau"], storage=storage,
                 periodic=(False, False, True), outlet_face="+x", layout=layout)
    d.set_boundary_links(links, variant=variant)
    d.set_wall_neq(wall_neq)
    return d, mask, links


def packing_domain(n=256, storage="f32", tau=0.9, force=(1e-6, 0.0, 0.0), variant="FQ", spheres=None,
                   layout="compact", lattice="D3Q19", collision="BGK", magic=3.0 / 16.0, wall_neq="bounceback"):
    centres, radii = synth.sphere_packing(n=n) if spheres is None else spheres
    mask, links = packing_geometry(n, centres, radii, lattice)
    d = B.Domain(lattice, n, n, n, mask, tau, storage=storage, force=force, layout=layout, collision=collision,
                 magic=magic)
    d.set_boundary_links(links, variant=variant)
    d.set_wall_neq(wall_neq)
    return d, mask, links


def request_domain(req, storage="f16s", variant="FQ", layout="compact"):
    """One served request (``synth.request_stream``): circular Couette L x L or
    cylinder channel 2L x L."""
    if req["kind"] == "couette":
        return couette_domain(req, storage=storage, variant=variant, layout=layout)
    return channel_domain(req, storage=storage, variant=variant, layout=layout)


def moving_box_domain(box, storage="bf16s", variant="FQ", wall_neq="bounceback"):
    """One periodic box with a sphere in prescribed motion (``synth.moving_boxes``)."""
    n = (box["nx"], box["ny"], box["nz"])
    d = B.Domain("D3Q19", *n, np.ones(n[0] * n[1] * n[2], np.uint8), box["tau"], storage=storage,
                 rho0=box.get("rho0", 1.0), layout="dense")
    d.set_wall_neq(wall_neq)
    d.set_moving_sphere(box["x0"], box["radius"], box["amplitude"], box["period"], box["direction"], box["omega"],
                        variant=variant)
    return d
