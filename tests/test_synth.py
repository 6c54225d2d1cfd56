"""Input generator checks: determinism and the geometry/parameter recipe."""
import numpy as np
import pytest

from paper_1906_01211_amd import synth


def _min_image(d, box):
    return d - box * np.rint(d / box)


@pytest.mark.parametrize("name", ["water216", "water7853"])
def test_deterministic(name):
    a = synth.make(name)
    b = synth.make(name)
    assert np.array_equal(a.xyz, b.xyz)
    assert np.array_equal(a.mpole, b.mpole)
    assert a.n == 3 * synth.CONFIGS[name]["n_w"]


def test_water_geometry_and_parameters():
    w = synth.make("water216")
    xyz = w.xyz.reshape(-1, 3, 3)
    oh1 = _min_image(xyz[:, 1] - xyz[:, 0], w.box)
    oh2 = _min_image(xyz[:, 2] - xyz[:, 0], w.box)
    assert np.allclose(np.linalg.norm(oh1, axis=1), 0.9572, atol=1e-12)
    assert np.allclose(np.linalg.norm(oh2, axis=1), 0.9572, atol=1e-12)
    cosang = np.sum(oh1 * oh2, axis=1) / 0.9572 ** 2
    assert np.allclose(np.degrees(np.arccos(cosang)), 104.52, atol=1e-9)
    assert (w.xyz >= 0).all() and (w.xyz < w.box).all()
    assert abs(w.mpole[:, 0].sum()) < 1e-12                    # neutral
    tr = w.mpole[:, 4] + w.mpole[:, 7] + w.mpole[:, 9]
    assert np.abs(tr).max() < 1e-15                            # traceless
    assert abs(w.n / w.box ** 3 - 0.1001) < 5e-4               # liquid density
    assert np.array_equal(w.molid, np.arange(w.n) // 3)


def test_lattice_subset_and_density():
    w = synth.make("water7853")
    assert w.n == 23559
    assert abs(w.n / w.box ** 3 - 0.0978) < 5e-4
    c = synth.make("water32000_charge_lj")
    assert c.n == 96000 and abs(c.mpole[:, 0].sum()) < 1e-9
    assert np.all(c.mpole[:, 1:] == 0)


def test_serving_stream():
    reqs = synth.serving_requests(512, rate=100.0)
    n = np.array([3 * r["n_w"] for r in reqs])
    assert n.min() >= 297 and n.max() <= 30003
    assert all(r["seed"] == 20000 + r["k"] for r in reqs)
    arr = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(arr) > 0)
