"""Pins of the oracle's compressed operator (H2 x MACA)."""
import numpy as np
import pytest

import cqm_workloads as W
import oracle as O


@pytest.fixture(scope="module")
def sphere2():
    return W.icosphere(2)


def test_cluster_tree_is_a_partition(sphere2):
    V, T = sphere2
    cl = O.cluster_tree(V, T, 8)
    assert sorted(cl[0]["idx"].tolist()) == list(range(len(T)))
    for c in cl:
        if c["sons"]:
            assert len(c["sons"]) == 2
            a, b = (set(cl[s]["idx"].tolist()) for s in c["sons"])
            assert a and b and not (a & b) and (a | b) == set(c["idx"].tolist())
        else:
            assert len(c["idx"]) <= 8


def test_block_partition_covers_once_and_is_admissible(sphere2):
    V, T = sphere2
    cl = O.cluster_tree(V, T, 8)
    far, near = O.block_tree(cl, 1.0)
    cover = np.zeros((len(T), len(T)), dtype=int)
    for r, c in far + near:
        cover[np.ix_(cl[r]["idx"], cl[c]["idx"])] += 1
    assert np.all(cover == 1)
    for r, c in far:
        dr = np.linalg.norm(cl[r]["hi"] - cl[r]["lo"])
        dc = np.linalg.norm(cl[c]["hi"] - cl[c]["lo"])
        gap = np.maximum(0, np.maximum(cl[r]["lo"] - cl[c]["hi"], cl[c]["lo"] - cl[r]["hi"]))
        assert max(dr, dc) <= np.linalg.norm(gap) + 1e-15
    for r, c in near:
        assert not cl[r]["sons"] and not cl[c]["sons"]
    assert len(far) > 0


def test_chebyshev_interpolation_exact_for_low_degree(sphere2):
    V, T = sphere2
    cl = O.cluster_tree(V, T, 8)
    m = 4
    nodes = O.cheb_nodes(cl[3], m)
    g = np.stack(np.meshgrid(*nodes, indexing="ij"), -1).reshape(-1, 3)
    f = lambda X: 1 + X[:, 0] ** 3 * X[:, 1] ** 2 - 2 * X[:, 2] ** 3 * X[:, 0]  # degree < m per axis
    X = np.random.default_rng(0).uniform(cl[3]["lo"], cl[3]["hi"], size=(50, 3))
    L = O.compress._lagrange_3d(nodes, X)
    assert np.max(np.abs(L @ f(g) - f(X))) < 1e-12
    # and not for degree m on an axis
    f2 = lambda X: X[:, 0] ** 4
    assert np.max(np.abs(L @ f2(g) - f2(X))) > 1e-8


def test_cluster_bases_are_nested(sphere2):
    V, T = sphere2
    cl = O.cluster_tree(V, T, 8)
    m = 3
    for cid, c in enumerate(cl):
        if not c["sons"]:
            continue
        nd = O.cheb_nodes(c, m)
        Up = O.cluster_basis(V, T, c, nd)
        pos = {int(t): k for k, t in enumerate(c["idx"])}
        for s in c["sons"]:
            ns = O.cheb_nodes(cl[s], m)
            Us = O.cluster_basis(V, T, cl[s], ns)
            E = O.transfer_matrix(ns, nd)
            rows = [pos[int(t)] for t in cl[s]["idx"]]
            assert np.max(np.abs(Up[rows] - Us @ E)) < 1e-12 * np.max(np.abs(Up))


def test_maca_recovers_low_rank_and_zero_tensors():
    rng = np.random.default_rng(1)
    A = [rng.standard_normal((7, 5)) + 1j * rng.standard_normal((7, 5)) for _ in range(3)]
    B = [rng.standard_normal(11) + 1j * rng.standard_normal(11) for _ in range(3)]
    G = sum(np.einsum("ij,k->ijk", a, b) for a, b in zip(A, B))
    C, d, info = O.maca(G, 1e-14)
    assert info["rank"] <= 4
    R = G - np.einsum("lij,lk->ijk", np.asarray(C), np.asarray(d))
    assert np.max(np.abs(R)) < 1e-12 * np.max(np.abs(G))
    C0, d0, info0 = O.maca(np.zeros((4, 4, 6)), 1e-6)
    assert info0["rank"] == 0


def test_maca_gram_identity_and_vanishing_crosses():
    rng = np.random.default_rng(2)
    x = np.linspace(0, 1, 9)
    s = 1.0 + 0.5j * np.arange(13)
    G = np.exp(-s[None, None, :] * (1 + x[:, None, None] + 2 * x[None, :, None])) \
        + 1e-3 * rng.standard_normal((9, 9, 13))
    C, d, info = O.maca(G, 1e-4)
    assert abs(info["norm2"] - O.maca_norm2(C, d)) < 1e-12 * info["norm2"]
    R = G - np.einsum("lij,lk->ijk", np.asarray(C), np.asarray(d))
    # the residual vanishes on every pivot slice and pivot fibre
    for (k, i, j), dl in zip(info["pivots"], d):
        assert abs(dl[k] - 1.0) < 1e-15
        assert np.max(np.abs(R[:, :, k])) < 1e-12 * np.max(np.abs(G))
        assert np.max(np.abs(R[i, j, :])) < 1e-12 * np.max(np.abs(G))
    assert len({k for k, _, _ in info["pivots"]}) == info["rank"]  # frequencies not reused


@pytest.fixture(scope="module")
def small_problem():
    V, T = W.icosphere(2)
    N, Tend = 16, 2.0
    s, _, _ = O.frequencies(N, Tend)
    dense = O.dense_tensor(V, T, s)
    return V, T, s, dense


def test_compressed_operator_error_decays_with_eps_and_m(small_problem):
    V, T, s, dense = small_problem
    x = W.random_complex((len(s), len(T)), seed=3)
    ref = np.stack([dense[:, :, l] @ x[l] for l in range(len(s))])
    errs_eps = []
    for eps in (1e-3, 1e-6):
        op = O.build_compressed(V, T, s, 8, 1.0, 4, eps, dense=dense)
        y = O.compressed_matvec(op, x)
        errs_eps.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs_eps[1] < errs_eps[0]
    errs_m = []
    for m in (2, 3, 4):
        op = O.build_compressed(V, T, s, 8, 1.0, m, 1e-12, dense=dense)
        y = O.compressed_matvec(op, x)
        errs_m.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs_m[0] > errs_m[1] > errs_m[2]
    assert errs_m[2] < 1e-4


def test_compressed_dense_matches_matvec(small_problem):
    V, T, s, dense = small_problem
    op = O.build_compressed(V, T, s, 8, 1.0, 3, 1e-8, dense=dense)
    A = O.compressed_dense(op, len(T))
    x = W.random_complex((len(s), len(T)), seed=4)
    y = O.compressed_matvec(op, x)
    for l in range(len(s)):
        assert np.linalg.norm(A[:, :, l] @ x[l] - y[l]) < 1e-13 * np.linalg.norm(y[l])


def test_on_demand_near_blocks_equal_the_dense_tensor_slices():
    # Algorithm 3 forms only the entries of the block it compresses; the
    # oracle's on-demand block tensors equal the slices of the fully
    # assembled tensor (to rounding: sums may be formed in another order),
    # so both builds approximate the same tensor to the MACA tolerance
    V, T = W.icosphere(1)
    s, _, _ = O.frequencies(6, 2.0)
    dense = O.dense_tensor(V, T, s)
    a = O.build_compressed(V, T, s, 4, 1.0, 3, 1e-8, dense=dense)
    assert len(a["near"]) > 0 and len(a["far"]) > 0
    cl = a["clusters"]
    lookup = O.compress._near_lookup(V, T)
    for (r, c) in a["near"]:
        ir, ic = cl[r]["idx"], cl[c]["idx"]
        G = O.block_tensor(V, T, ir, ic, s, lookup)
        ref = dense[np.ix_(ir, ic)]
        assert np.max(np.abs(G - ref)) <= 1e-14 * np.max(np.abs(ref))
    b = O.build_compressed(V, T, s, 4, 1.0, 3, 1e-8)
    x = W.random_complex((len(s), len(T)), seed=4)
    ya, yb = O.compressed_matvec(a, x), O.compressed_matvec(b, x)
    assert np.linalg.norm(ya - yb) <= 1e-7 * np.linalg.norm(ya)


def test_sampled_rows_equal_the_whole_operator_rows(small_problem):
    # compressing only the blocks whose row cluster holds a sampled triangle
    # leaves those rows of the product unchanged: every other block adds
    # nothing to them, and the kept blocks are compressed the same way
    V, T, s, dense = small_problem
    x = W.random_complex((len(s), len(T)), seed=6)
    full = O.build_compressed(V, T, s, 8, 1.0, 3, 1e-8, dense=dense)
    rows = np.asarray(sorted(set(full["clusters"][5]["idx"].tolist()) | {0, 17, 250}))
    part = O.build_compressed(V, T, s, 8, 1.0, 3, 1e-8, dense=dense, rows=rows)
    assert 0 < len(part["blocks"]) < len(full["blocks"])
    yf = O.compressed_matvec(full, x)[:, rows]
    yp = O.compressed_matvec(part, x)[:, rows]
    assert np.array_equal(yf, yp)
