import numpy as np

import cqm_workloads as W


def test_icosphere_counts_and_topology():
    for k in range(5):
        V, T = W.icosphere(k)
        M = len(T)
        assert M == 20 * 4 ** k
        edges = {tuple(sorted(e)) for t in T for e in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))}
        assert len(V) - len(edges) + M == 2  # Euler characteristic of a sphere
        assert np.allclose(np.linalg.norm(V, axis=1), 1.0)
        P = V[T]
        n = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
        assert np.all(np.einsum("ij,ij->i", n, P.mean(1)) > 0)  # outward


def test_area_converges_to_sphere():
    prev = None
    for k in range(1, 5):
        V, T = W.icosphere(k)
        P = V[T]
        A = 0.5 * np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1).sum()
        err = abs(A - 4 * np.pi)
        if prev is not None:
            assert 3.5 < prev / err < 4.5  # O(h^2)
        prev = err


def test_problem_mix_is_seeded():
    a = W.problem_mix(48)
    b = W.problem_mix(48)
    assert [x.name for x in a] == [x.name for x in b]
    assert {x.N for x in a} <= {16, 32, 64, 128}
    assert all(0.2 <= x.wave.sigma <= 0.4 for x in a)
    arr = W.poisson_arrivals(20.0, 60.0)
    assert 1000 < len(arr) < 1400 and np.all(np.diff(arr) > 0)
