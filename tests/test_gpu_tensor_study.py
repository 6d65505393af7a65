"""The tensor-approximation study of Section 7.1 (bench.py --part study) at a
size the oracle covers: the relative Frobenius error e = ||V - V~|| / ||V||
of the GPU's compressed tensor, measured through the C ABI by products with
every unit vector, against the same quantity of the oracle's compressed
tensor (Algorithm 3, written out densely), and the trends the paper reports:
e falls with eps until the H2 interpolation error dominates (Corollary
combierr), and falls with the order m (Theorem h2err)."""
import sys

import numpy as np
import pytest

import cqm_workloads as W
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import bench  # noqa: E402
from paper_2006_05186_amd import cqm as C  # noqa: E402

N, TEND, NMIN, ETA = 16, 2.0, 8, 1.0


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = C.cqm_ctx_create(0)
    yield c
    C.cqm_ctx_destroy(c)


@pytest.fixture(scope="module")
def case():
    V, T = W.icosphere(2)
    s, _, _ = O.frequencies(N, TEND)
    say("oracle: dense tensor of the 320-triangle sphere, N = 16")
    dense = O.dense_tensor(V, T, s)
    return V, T, s, dense


def test_study_error_matches_oracle_and_follows_the_paper(ctx, case):
    V, T, s, dense = case
    nrm = np.linalg.norm(dense)
    res = {}
    for m in (2, 3):
        for eps in (1e-2, 1e-4, 1e-8):
            op = O.build_compressed(V, T, s, NMIN, ETA, m, eps, dense=dense)
            e_or = np.linalg.norm(O.compressed_dense(op, len(T)) - dense) / nrm
            g = bench.tensor_error(C, torch, ctx, V, T, N, TEND, NMIN, ETA, m, eps)
            res[(m, eps)] = g["e"]
            say(f"m={m} eps={eps:.0e}: e GPU {g['e']:.3e} oracle {e_or:.3e}, max rank "
                f"{g['max_rank']}, storage {g['storage_vs_dense']:.3f} of dense, "
                f"{g['storage_vs_plain_h2']:.3f} of plain H2")
            # the same approximant up to pivots flipped by rounding near-ties
            assert abs(g["e"] - e_or) <= 0.1 * e_or + 1e-12, (m, eps)
            assert g["far_blocks"] == len(op["far"]) and g["near_blocks"] == len(op["near"])
            assert 0 < g["storage_vs_plain_h2"] < 1
    for m in (2, 3):
        assert res[(m, 1e-4)] <= res[(m, 1e-2)]
        assert res[(m, 1e-8)] <= res[(m, 1e-4)] * 1.01
    assert res[(3, 1e-8)] < res[(2, 1e-8)]
