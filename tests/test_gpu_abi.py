"""C-ABI argument validation on a live domain (needs the device to create one)."""
import numpy as np
import pytest

from tests.gpu_cases import annulus_case

pytestmark = pytest.mark.gpu


def _domain(B):
    case = annulus_case()
    nx, ny, nz = case.n
    g = B.Geometry("D2Q9", nx, ny, nz)
    for c, r, ins, V, Om in case.spheres:
        g.add_sphere(c, r, ins, V=V, Omega=Om)
    mask, links = g.build()
    d = B.Domain("D2Q9", nx, ny, nz, mask, case.tau, storage="f32")
    return d, mask, links


def test_step_before_links_is_state_error(gpu_lib):
    B = gpu_lib
    d, mask, links = _domain(B)
    with pytest.raises(B.LBMError) as e:
        d.step(1)
    assert e.value.code == B.LBM_ESTATE
    d.set_boundary_links(links)
    d.step(2)
    d.close()


@pytest.mark.parametrize("mutate", ["duplicate", "fluid_source", "solid_node", "dir0", "q0", "q_big", "missing", "variant"])
def test_invalid_links_rejected(gpu_lib, mutate):
    B = gpu_lib
    d, mask, links = _domain(B)
    L = {k: np.array(v, copy=True) for k, v in links.items()}
    variant = "FQ"
    if mutate == "duplicate":
        for k in L:
            L[k] = np.concatenate([L[k], L[k][:1]]) if L[k].ndim == 1 else np.concatenate([L[k], L[k][:1]], 0)
    elif mutate == "fluid_source":
        # x = (24 + 14, 24): mid-annulus, every neighbour fluid
        L["node"][0] = 38 + 48 * 24
    elif mutate == "solid_node":
        L["node"][0] = 0
    elif mutate == "dir0":
        L["dir"][0] = 0
    elif mutate == "q0":
        L["q"][0] = 0.0
    elif mutate == "q_big":
        L["q"][0] = 1.5
    elif mutate == "missing":
        for k in L:
            L[k] = L[k][1:]
    elif mutate == "variant":
        variant = 9
    with pytest.raises(B.LBMError) as e:
        d.set_boundary_links(L, variant=variant)
    assert e.value.code == B.LBM_EINVAL
    assert "link" in str(e.value) or "variant" in str(e.value) or "population" in str(e.value)
    d.close()


def test_non_finite_population_reports_unstable_through_the_abi(gpu_lib):
    """A NaN put into one population through lbm_set_state spreads to its
    neighbours in a step; lbm_macros then returns LBM_EUNSTABLE (not LBM_OK)
    and its message counts the non-finite nodes, which the moments it wrote
    show."""
    import ctypes
    B = gpu_lib
    d, mask, links = _domain(B)
    d.set_boundary_links(links)
    d.step(5)
    f = d.get_state()
    n = int(np.flatnonzero(mask)[len(np.flatnonzero(mask)) // 2])
    f[1, n] = np.nan
    d.set_state(f)
    d.step(1)
    rho = np.empty(d.N)
    u = np.empty(d.N * d.D)
    sums = np.empty(d.D + 2)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    code = B.lib().lbm_macros(d.h, p(rho), p(u), p(sums))
    assert code == B.LBM_EUNSTABLE
    msg = B.lib().lbm_last_error().decode()
    bad = int(msg.split(" at ")[1].split()[0])
    assert "non-finite" in msg and 1 <= bad <= 9          # the node and the neighbours it streamed to
    fl = mask.astype(bool)
    assert int((~(np.isfinite(rho[fl]) & np.isfinite(u.reshape(-1, d.D)[fl]).all(1))).sum()) == bad
    d.close()
