"""Batched stepping (lbm_batch_*): every domain of a batch must end in exactly
the state it reaches when stepped alone with lbm_step -- bit for bit, since the
per-node arithmetic is shared -- for every launch choice (graph or eager
launches, grid, tile order), across calls whose step counts change the buffer
parity, across membership changes, and for moving spheres across the
kinematics upload chunks.  With stochastic rounding the random words depend
only on a domain's own slots and step count, so the same holds."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _static_set(B, W):
    """Uneven static domains of several kinds (compact and dense, D2Q9 and D3Q19)."""
    reqs = synth.request_stream(n_requests=6, l_min=64, l_max=160, seed=7)
    out = []
    kinds = ("f16s", "f32", "f16s-sr", "bf16s-sr")   # with both rounding modes of the 16-bit stores
    for k, r in enumerate(reqs):
        storage = kinds[k % len(kinds)]
        out.append(lambda r=r, storage=storage: W.request_domain(r, storage=storage)[0])
    c, rad = synth.sphere_packing(n=48, seed=11)
    out.append(lambda: W.packing_domain(48, "f32", spheres=(c, rad))[0])
    out.append(lambda: W.packing_domain(48, "f32", spheres=(c, rad), layout="dense")[0])
    out.append(lambda: W.couette_domain(synth.couette_annulus(scale=2.0), storage="f64")[0])
    return out


def _moving_set(B, W, storage):
    boxes = synth.moving_boxes(n_boxes=3, side_min=40, side_max=56, r_min=5.0, r_max=7.0, amplitude=4.0,
                               period=120.0, seed=5)
    return [lambda b=b: W.moving_box_domain(b, storage=storage) for b in boxes]


def _twins(makers):
    return [m() for m in makers], [m() for m in makers]


def _same_state(alone, batched):
    for k, (a, b) in enumerate(zip(alone, batched)):
        fa, fb = a.get_state(), b.get_state()
        assert np.array_equal(fa, fb), f"domain {k}: max |diff| {np.abs(fa - fb).max()}"
        assert a.info()["steps_done"] == b.info()["steps_done"]


@pytest.mark.parametrize("graph,grid,order", [(1, 0, 1), (0, 0, 0), (1, 2, 2), (1, 4, 0), (0, 6, 1)])
def test_static_batch_bit_identical(gpu_lib, graph, grid, order):
    from paper_2009_04604_amd import workloads as W
    B = gpu_lib
    _say("case static batch graph", graph, "grid", grid, "order", order)
    alone, batched = _twins(_static_set(B, W))
    b = B.Batch()
    b.set_option("graph", graph)
    b.set_option("grid", grid)
    b.set_option("order", order)
    for n in (7, 10, 1, 4):          # odd counts flip the buffer parity between calls
        for d in alone:
            d.step(n)
        b.step(batched, n)
    _same_state(alone, batched)
    # membership change: drop two domains, keep stepping the rest
    keep = [0, 2, 3, 5, 6]
    for d in [alone[k] for k in keep]:
        d.step(9)
    b.step([batched[k] for k in keep], 9)
    _same_state([alone[k] for k in keep], [batched[k] for k in keep])
    b.close()
    for d in alone + batched:
        d.close()


@pytest.mark.parametrize("storage", ["f32", "bf16s", "bf16s-sr"])
def test_moving_batch_bit_identical(gpu_lib, storage):
    from paper_2009_04604_amd import workloads as W
    B = gpu_lib
    _say("case moving batch", storage)
    alone, batched = _twins(_moving_set(B, W, storage))
    # a static domain of the same kind in the same group
    alone.append(W.packing_domain(40, storage, spheres=synth.sphere_packing(n=40, seed=3), layout="dense")[0])
    batched.append(W.packing_domain(40, storage, spheres=synth.sphere_packing(n=40, seed=3), layout="dense")[0])
    b = B.Batch()
    for n in (3, 300):               # 300 crosses a kinematics upload chunk
        for d in alone:
            d.step(n)
        b.step(batched, n)
        _same_state(alone, batched)
        for a, c in zip(alone, batched):
            ia, ic = a.info(), c.info()
            assert (ia["n_fluid"], ia["n_links"]) == (ic["n_fluid"], ic["n_links"])
    b.close()
    for d in alone + batched:
        d.close()


def test_autotune_keeps_results(gpu_lib):
    from paper_2009_04604_amd import workloads as W
    B = gpu_lib
    _say("case autotune")
    makers = _static_set(B, W)[:4]
    alone, batched = _twins(makers)
    b = B.Batch()
    ch = b.autotune(batched, steps_per_candidate=2)
    assert ch["grid"] in (0, 2, 4, 6) and ch["order"] in (0, 1, 2) and ch["us_per_step"] > 0
    for d in alone:
        d.step(1 + 12 * 2)
    _same_state(alone, batched)
    b.set_option("autotune", 1)
    b.step(batched, 20)
    for d in alone:
        d.step(20)
    _same_state(alone, batched)
    B.lbm_step_batch(batched, 5)     # one-shot form
    for d in alone:
        d.step(5)
    _same_state(alone, batched)
    b.close()
    for d in alone + batched:
        d.close()


def test_batch_validation(gpu_lib):
    import torch
    from paper_2009_04604_amd import workloads as W
    B = gpu_lib
    _say("case batch validation")
    d1 = W.couette_domain(synth.couette_annulus(), storage="f32")[0]
    d2 = W.couette_domain(synth.couette_annulus(), storage="f32")[0]
    b = B.Batch()
    with pytest.raises(B.LBMError) as e:
        b.step([d1, d1], 1)
    assert e.value.code == B.LBM_EINVAL
    with pytest.raises(B.LBMError) as e:
        b.step([d1], -1)
    assert e.value.code == B.LBM_EINVAL
    nolinks = B.Domain("D2Q9", 32, 32, 1, np.ones(32 * 32, np.uint8), 0.8, periodic=(True, False, True))
    with pytest.raises(B.LBMError) as e:
        b.step([d1, nolinks], 1)
    assert e.value.code == B.LBM_ESTATE
    s = torch.cuda.Stream()
    d2.set_stream(s.cuda_stream)
    with pytest.raises(B.LBMError) as e:
        b.step([d1, d2], 1)
    assert e.value.code == B.LBM_EINVAL
    with pytest.raises(B.LBMError) as e:
        b.set_option("grid", 1000)
    assert e.value.code == B.LBM_EINVAL
    torch.cuda.synchronize()
    b.close()
    for d in (d1, d2, nolinks):
        d.close()


def test_member_replaced_by_new_domain(gpu_lib):
    """A batch whose member is freed and replaced by a new domain (which the
    allocator may place at the freed one's address) must rebuild its tables."""
    from paper_2009_04604_amd import workloads as W
    B = gpu_lib
    _say("case batch member replaced")
    reqs = synth.request_stream(n_requests=4, l_min=64, l_max=96, seed=21)
    mk = [lambda r=r: W.request_domain(r, storage="f32")[0] for r in reqs]
    b = B.Batch()
    a0 = mk[0]()
    b.step([a0], 6)
    a0.close()
    a1 = mk[1]()                 # alone after a lone member was freed
    t1 = mk[1]()
    b.step([a1], 6)
    t1.step(6)
    _same_state([t1], [a1])
    x = mk[2]()
    tx = mk[2]()
    b.step([x, a1], 4)
    tx.step(4)
    t1.step(4)
    a1.close()
    a3 = mk[3]()                 # same position, possibly the same address
    t3 = mk[3]()
    b.step([x, a3], 5)
    tx.step(5)
    t3.step(5)
    _same_state([tx, t3], [x, a3])
    b.close()
    for d in (t1, x, tx, a3, t3):
        d.close()
