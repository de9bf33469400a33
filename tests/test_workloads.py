"""The seeded input generators: sizes, determinism, mesh validity."""
import numpy as np
import pytest

import workloads as w


def tri_area2(xy, tri):
    v = xy[tri]
    return ((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1])
            - (v[:, 2, 0] - v[:, 0, 0]) * (v[:, 1, 1] - v[:, 0, 1]))


def test_config0_shape_and_loading():
    p = w.config0()
    assert (p.n_nodes, p.n_elems) == (2145, 4096)
    assert np.all(tri_area2(p.xy, p.tri) > 0)
    assert int(p.fixed[:, 1].sum()) == 2 * 65 and int(p.fixed[:, 0].sum()) == 0
    assert p.d0.sum() == 33
    assert set(np.unique(p.v0[p.fixed.astype(bool)])) == {-0.5, 0.5}


def test_generators_are_deterministic():
    a, b = w.config0(), w.config0()
    assert np.array_equal(a.xy, b.xy) and np.array_equal(a.tri, b.tri)
    m1 = w.plate_mesh(60, 40, 1e-3, 0.25, 9, random_diag=True, n_holes=1, hole_radius_cells=3)
    m2 = w.plate_mesh(60, 40, 1e-3, 0.25, 9, random_diag=True, n_holes=1, hole_radius_cells=3)
    assert np.array_equal(m1["xy"], m2["xy"]) and np.array_equal(m1["tri"], m2["tri"])


def test_boundary_nodes_slide_along_the_boundary():
    p = w.small_plate(10, 6, jitter=0.3, seed=1)
    ij = p.meta["ij"]
    h = p.meta["h"]
    left = ij[:, 0] == 0
    bottom = ij[:, 1] == 0
    assert np.all(p.xy[left, 0] == 0.0) and np.all(p.xy[bottom, 1] == 0.0)
    corners = (ij[:, 0] % 10 == 0) & (ij[:, 1] % 6 == 0)
    assert np.allclose(p.xy[corners], ij[corners] * h, rtol=0, atol=0)


def test_perforated_plate():
    m = w.plate_mesh(80, 40, 1e-3, 0.25, 2, random_diag=True, n_holes=2, hole_radius_cells=4)
    xy, tri = m["xy"], m["tri"]
    assert np.all(tri_area2(xy, tri) > 0)
    assert tri.max() == len(xy) - 1 and len(np.unique(tri)) == len(xy)   # no orphans
    cen = xy[tri].mean(1)
    for c in m["hole_centres"]:
        assert np.all(np.hypot(*(cen - c).T) >= m["hole_radius"])


def test_batched_draws():
    nx, gc = w.config4_draws()
    assert len(nx) == 64 and nx.min() >= 128 and nx.max() <= 512 and np.all(nx % 8 == 0)
    assert gc.min() >= 1.0 and gc.max() <= 10.0
