"""The seeded input generators are deterministic and meet their recipes."""
import numpy as np

import synth


def test_packing_non_overlapping_and_dense():
    c, r = synth.sphere_packing(n=64, r_min=4.0, r_max=8.0, solid_fraction=0.3, seed=7)
    c2, r2 = synth.sphere_packing(n=64, r_min=4.0, r_max=8.0, solid_fraction=0.3, seed=7)
    np.testing.assert_array_equal(c, c2)
    np.testing.assert_array_equal(r, r2)
    assert np.all(np.diff(r) <= 0)                      # largest first
    assert (4.0 / 3.0 * np.pi * r ** 3).sum() / 64 ** 3 >= 0.3
    d = c[:, None, :] - c[None, :, :]
    d -= 64 * np.round(d / 64)
    dist = np.sqrt((d * d).sum(-1))
    iu = np.triu_indices(len(r), 1)
    assert np.all(dist[iu] > (r[:, None] + r[None, :])[iu])


def test_generators_deterministic():
    a = synth.cylinder_channel()
    b = synth.cylinder_channel()
    assert a == b
    assert 400 <= a["centre"][0] < 401 and 512 <= a["centre"][1] < 513
    assert abs(a["tau"] - 0.56) < 1e-12
    r1 = synth.request_stream(16, rate=10.0)
    r2 = synth.request_stream(16, rate=10.0)
    assert r1 == r2
    assert all(64 <= q["L"] <= 1024 for q in r1)
    assert np.all(np.diff([q["arrival"] for q in r1]) > 0)
    bx = synth.moving_boxes(4)
    assert all(96 <= b["nx"] <= 192 and 10 <= b["radius"] <= 16 for b in bx)
    for b in bx:
        assert abs(np.linalg.norm(b["omega"]) * b["radius"] - 0.02) < 1e-12
