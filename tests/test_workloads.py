"""Seeded input generator: determinism, shapes, node ordering."""
import numpy as np

from oracle import fe_space
from paper_1411_0519_amd import workloads


def test_deterministic_and_shapes():
    w, f, u0 = workloads.workload(1)
    w2, f2, u02 = workloads.workload(1)
    assert f.shape == (1, 16, 31) and u0.shape == (1, 31)
    assert np.array_equal(f, f2) and np.array_equal(u0, u02)
    assert f.min() >= -1 and f.max() <= 1


def test_node_ordering_matches_x_fastest():
    for d, n in ((1, 7), (2, 5), (3, 3)):
        xs = workloads.coordinates(d, n)
        ref = fe_space.node_coordinates(d, n)
        for i in range(d):
            assert np.allclose(xs[i], ref[:, i])


def test_reduced_workload_overrides():
    w, f, u0 = workloads.workload(2, n=15, N=8)
    assert f.shape == (1, 8, 225)
    # bumps are time-constant
    assert np.array_equal(f[0, 0], f[0, 7])
    w, f, u0 = workloads.workload(4, n=7, N=4, batch=3)
    assert f.shape == (3, 4, 49) and u0.shape == (3, 49)
    assert not np.allclose(u0[0], u0[1])


def test_streamed_batch_equals_make():
    w = dict(workloads.WORKLOADS[4])
    w.update(n=15, N=8, batch=5)
    _, f, u0 = workloads.workload(4, n=15, N=8, batch=5)
    it, u0_fn = workloads.make_streamed(**w)
    fs = np.stack(list(it))
    assert np.array_equal(fs, f)
    assert np.array_equal(u0_fn(), u0)
