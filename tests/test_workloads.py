"""The synthetic input recipes: shapes, ranges and seeds of the named workloads."""
import numpy as np

import workloads as W


def test_grid_is_the_cell_centred_lattice():
    P = W.grid_points(4, 100.0)
    assert P.shape == (16, 2)
    np.testing.assert_array_equal(np.unique(P[:, 0]), [12.5, 37.5, 62.5, 87.5])
    np.testing.assert_array_equal(np.unique(P[:, 1]), [12.5, 37.5, 62.5, 87.5])
    # every lattice point once
    assert len({tuple(p) for p in P}) == 16


def test_named_workloads_shapes_and_ranges():
    G = W.workload_points("g1_matern32aniso_grid256")
    assert G.shape == (65536, 2) and G.min() > 0.0 and G.max() < 100.0
    assert len(np.unique(G[:, 0])) == 256
    G2 = W.workload_points("g1_matern32aniso_grid256", 64 * 64)
    assert G2.shape == (4096, 2)
    M = W.workload_points("m1_matern32aniso_scattered65536")
    np.testing.assert_array_equal(M, 100.0 * W.uniform_points(65536, 71))
    U = W.workload_points("c3_matern32_n65536")
    assert U.shape == (65536, 2) and U.min() >= 0.0 and U.max() < 1.0
    np.testing.assert_array_equal(U, W.workload_points("c3_matern32_n65536"))  # seeded


def test_batch_instances_recipe():
    inst = W.batch_instances(8, 41)
    assert len(inst) == 8
    for P, th in inst:
        assert 2048 <= len(P) <= 32768
        w, h = P[:, 0].max(), P[:, 1].max()
        assert w * h <= 1.0 + 1e-12  # inside a unit-area rectangle
        assert 0.02 <= th[0] <= 0.2 and th[1:] == (1.0, 1e-4)
