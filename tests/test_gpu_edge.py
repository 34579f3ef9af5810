"""Degenerate inputs through the C-ABI: zero and negative step counts, an empty
batch, a domain without a single fluid node, and lattices smaller than one
segment (every pull wraps onto the same few nodes) against the FP64 oracle."""
import numpy as np
import pytest

from tests.gpu_cases import Case, annulus_case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def test_zero_steps_leave_the_state_unchanged(gpu_lib):
    B = gpu_lib
    _say("case zero steps")
    d, _, _ = annulus_case().gpu(B, "f32")
    d.step(3)
    f0 = d.get_state()
    d.step(0)
    f1 = d.get_state()
    assert np.array_equal(f0, f1, equal_nan=True)
    with pytest.raises(B.LBMError) as e:
        d.step(-1)
    assert e.value.code == B.LBM_EINVAL
    d.close()


def test_empty_batch_is_a_no_op(gpu_lib):
    B = gpu_lib
    _say("case empty batch")
    b = B.Batch()
    b.step([], 5)
    b.close()


@pytest.mark.parametrize("layout", ["compact", "dense"])
def test_domain_without_fluid(gpu_lib, layout):
    """A sphere covering the whole periodic box: no fluid node, no link."""
    B = gpu_lib
    _say("case all solid", layout)
    n = (70, 9, 5)
    g = B.Geometry("D3Q19", *n)
    g.add_sphere((35.0, 4.0, 2.0), 100.0, True)
    mask, links = g.build()
    g.close()
    assert not mask.any() and len(links["q"]) == 0
    d = B.Domain("D3Q19", *n, mask, 0.8, storage="f32", force=(1e-5, 0.0, 0.0), layout=layout)
    d.set_boundary_links(links)
    d.step(4)
    rho, u, sums, unstable = d.macros()
    assert d.info()["n_fluid"] == 0
    assert sums[0] == 0.0 and not unstable
    d.close()


@pytest.mark.parametrize("n", [(1, 1, 1), (65, 3, 1), (1, 2, 3)], ids=["1x1", "65x3", "1x2x3"])
@pytest.mark.parametrize("layout", ["compact", "dense"])
def test_smaller_than_a_segment(gpu_lib, n, layout):
    """Periodic boxes whose rows are shorter than (or one node longer than) a
    64-lane segment, with a body force and a perturbed start, FP64 against the oracle."""
    B = gpu_lib
    lat = "D2Q9" if n[2] == 1 else "D3Q19"
    _say("case tiny box", lat, n, layout)
    case = Case(lat, n, tau=0.7, force=(2e-5, -1e-5, 0.0))
    d, _, _ = case.gpu(B, "f64", layout=layout)
    sim = case.oracle()
    rng = np.random.default_rng(7)
    sim.f = sim.f * (1.0 + 0.01 * rng.standard_normal(sim.f.shape))
    d.set_state(sim.f)
    d.step(25)
    sim.run(25)
    assert np.abs(d.get_state() - sim.f).max() < 1e-14
    d.close()
