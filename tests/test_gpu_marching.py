"""Time-marching solve on the GPU (cqm_solve_marching) against the marching
oracle (oracle/marching.py: the same weights of eq. dft and the same step
recursion, LU of What_0) and against the all-at-once solve, which it equals
up to terms of order rho^(N+1)."""
import os
import sys

import numpy as np
import pytest

import cqm_workloads as W
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2006_05186_amd import cqm as C  # noqa: E402
from paper_2006_05186_amd.solver import Problem  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = C.cqm_ctx_create(0)
    yield c
    C.cqm_ctx_destroy(c)


@pytest.fixture(scope="module")
def c1():
    wl = W.C1
    V, T = wl.mesh()
    say("oracle: marching and all-at-once solves of the 320-triangle workload")
    qm = O.solve_marching(V, T, wl.N, wl.T)
    qa = O.solve(V, T, wl.N, wl.T)
    _, _, area = O.triangle_quadrature(V, T)
    return wl, V, T, qm, qa, area


@pytest.mark.parametrize("mode", [C.CQM_FP64_PLAIN, C.CQM_MIXED_PLAIN])
def test_marching_matches_oracle_marching(ctx, c1, mode):
    wl, V, T, qm, qa, area = c1
    p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, marching=1)
    p.set_plane_wave()
    q, rc, d = p.solve_marching()
    q = q.cpu().numpy()
    e_m = O.rel_error(q, qm, area)
    e_a = O.rel_error(q, qa, area)
    s, rho, dt = O.frequencies(wl.N, wl.T)
    say(f"marching M=320 N=32 mode={mode}: rc={rc} err vs oracle marching {e_m:.2e}, vs "
        f"all-at-once {e_a:.2e} (rho^F {rho ** (wl.N + 1):.1e}); CG iterations {d.total_iters} "
        f"(max {d.max_iters} per step), residual {d.max_rel_residual:.1e}")
    assert rc == C.CQM_OK and d.converged == 1 and d.n_systems == wl.N + 1
    assert e_m < 1e-8
    assert e_a < 10 * rho ** (wl.N + 1)
    p.close()


def test_marching_C2_against_stored_all_at_once(ctx):
    wl = W.C2
    V, T = wl.mesh()
    g = np.load(os.path.join(GOLDEN, f"{wl.name}.npz"))
    _, _, area = O.triangle_quadrature(V, T)
    s, rho, dt = O.frequencies(wl.N, wl.T)
    p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_FP64_PLAIN, marching=1)
    p.set_plane_wave()
    q, rc, d = p.solve_marching()
    err = O.rel_error(q.cpu().numpy(), g["q"], area)
    say(f"marching M=1280 N=64: rc={rc} err vs oracle all-at-once {err:.2e} "
        f"(rho^F {rho ** (wl.N + 1):.1e}), CG iterations {d.total_iters}, setup {d.t_setup_ms:.1f} "
        f"ms, steps {d.t_solve_ms:.1f} ms")
    assert rc == C.CQM_OK and err < 10 * rho ** (wl.N + 1)
    p.close()


@pytest.mark.parametrize("mode", [C.CQM_FP64_H2ACA, C.CQM_MIXED_H2ACA])
def test_compressed_marching_matches_oracle(ctx, mode):
    """Weights from the transformed MACA fibres (eq. fastdft) on the
    80-triangle sphere with admissible blocks (leaf size 4, eta 1, m = 3)
    against the oracle's compressed marching (same partition, order and
    tolerance); pivots of near-ties may differ, so the bar is that of the
    compressed all-at-once comparison."""
    wl = W.C0_TINY
    V, T = wl.mesh()
    kw = dict(n_min=4, eta=1.0, cheb_m=3, eps_aca=1e-10)
    say("oracle: compressed marching of the 80-triangle sphere")
    qref = O.solve_marching_compressed(V, T, wl.N, wl.T, 4, 1.0, 3, 1e-10)
    qplain = O.solve_marching(V, T, wl.N, wl.T)
    _, _, area = O.triangle_quadrature(V, T)
    p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, marching=1, **kw)
    p.set_plane_wave()
    q, rc, d = p.solve_marching()
    q = q.cpu().numpy()
    e = O.rel_error(q, qref, area)
    e_plain = O.rel_error(q, qplain, area)
    say(f"compressed marching mode={mode}: rc={rc} err vs oracle compressed marching {e:.2e}, "
        f"vs plain marching {e_plain:.2e} (oracle's own {O.rel_error(qref, qplain, area):.2e}); "
        f"far/near blocks {d.n_far_blocks}/{d.n_near_blocks}, CG iterations {d.total_iters}")
    assert rc == C.CQM_OK and d.converged == 1 and d.n_far_blocks > 0
    assert e < (1e-6 if mode == C.CQM_FP64_H2ACA else 1e-4)
    p.close()


def test_compressed_marching_C1_against_plain(ctx, c1):
    """320 triangles, N = 32, the configured compressed form with a tight MACA
    tolerance: the compressed weights give the plain marching solution to
    the approximation level."""
    wl, V, T, qm, qa, area = c1
    p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_FP64_H2ACA, marching=1, eps_aca=1e-10)
    p.set_plane_wave()
    q, rc, d = p.solve_marching()
    e = O.rel_error(q.cpu().numpy(), qm, area)
    say(f"compressed marching M=320 N=32: rc={rc} err vs oracle marching {e:.2e}, CG iterations "
        f"{d.total_iters}, setup {d.t_setup_ms:.1f} ms, steps {d.t_solve_ms:.1f} ms")
    assert rc == C.CQM_OK and e < 1e-6
    p.close()


@pytest.mark.parametrize("m", [4, 6])
def test_compressed_marching_with_cores_matches_oracle(ctx, m):
    """Two 320-triangle spheres six radii apart (their clusters form 320 x 320
    admissible blocks kept as Tucker cores, so the fast right-hand side
    convolves cluster coefficients and the lag-0 collapse covers cores),
    N = 16, leaf size 16, eta = 1, m = 4 and 6, tolerance 1e-10, against the
    oracle's compressed marching (tests/golden/two_spheres640_N16_T2_h2march.npz,
    make_golden.py --h2march)."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "two_spheres640_N16_T2_h2march.npz"))
    V, T = W.two_spheres(2)
    N, Tend = 16, 2.0
    _, _, area = O.triangle_quadrature(V, T)
    for mode, tol in ((C.CQM_FP64_H2ACA, 1e-6), (C.CQM_MIXED_H2ACA, 1e-4)):
        p = Problem(ctx, V, T, N, Tend, mode=mode, marching=1, n_min=16, eta=1.0, cheb_m=m,
                    eps_aca=1e-10)
        p.set_plane_wave()
        q, rc, d = p.solve_marching()
        q = q.cpu().numpy()
        e = O.rel_error(q, g[f"q_m{m}"], area)
        e_plain = O.rel_error(q, g["q_plain"], area)
        say(f"compressed marching, two spheres, m={m} mode={mode}: rc={rc} err vs oracle "
            f"{e:.2e}, vs plain marching {e_plain:.2e}; far/near blocks "
            f"{d.n_far_blocks}/{d.n_near_blocks}, CG iterations {d.total_iters}")
        assert rc == C.CQM_OK and d.converged == 1 and e < tol
        p.close()


def test_marching_argument_checks(ctx):
    wl = W.C0_TINY
    V, T = wl.mesh()
    for kw in ({"marching": 0}, {"marching": 1, "form": C.CQM_FORM_MATRIX_FREE},
               {"marching": 1, "mode": C.CQM_MIXED_H2ACA, "aca_band": C.CQM_BAND_HALF},
               {"marching": 1, "mode": C.CQM_MIXED_H2ACA, "precond": C.CQM_PRECOND_NONE}):
        p = Problem(ctx, V, T, wl.N, wl.T, **kw)
        p.set_plane_wave()
        with pytest.raises(C.CqmError) as e:
            p.solve_marching()
        assert e.value.code == C.CQM_EINVAL
        p.close()
