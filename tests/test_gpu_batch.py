"""Uneven batch: problems of different meshes, step counts and pulses solved
in shared launches match the same problems solved alone and the oracle."""
import sys

import numpy as np
import pytest

import cqm_workloads as W
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2006_05186_amd import cqm as C  # noqa: E402
from paper_2006_05186_amd.solver import Problem, solve_batch  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = C.cqm_ctx_create(0)
    yield c
    C.cqm_ctx_destroy(c)


@pytest.mark.parametrize("layout", [C.CQM_ARNOLDI_AUTO, C.CQM_ARNOLDI_GROUP])
def test_uneven_batch_matches_alone_and_oracle(ctx, layout):
    """Systems of different lengths share the launches (split Arnoldi with
    different slice counts per system under AUTO here, one workgroup per
    system under GROUP)."""
    mix = W.problem_mix(6, seed=7, levels=(1, 2), steps=(8, 16), T=2.0)
    say("batch of " + ", ".join(f"{w.name}(M={w.M},N={w.N})" for w in mix))
    probs, alone = [], []
    for w in mix:
        V, T = w.mesh()
        for store in (probs, alone):
            p = Problem(ctx, V, T, w.N, w.T, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE,
                        arnoldi_layout=layout)
            p.set_plane_wave(w.wave.direction, w.wave.sigma, w.wave.t0)
            store.append(p)
    res, rc = solve_batch(probs)
    assert rc == C.CQM_OK
    for w, (q, d), p in zip(mix, res, alone):
        qa, rca, _ = p.solve()
        V, T = w.mesh()
        _, _, area = O.triangle_quadrature(V, T)
        ref = O.solve(V, T, w.N, w.T, direction=w.wave.direction, sigma=w.wave.sigma, t0=w.wave.t0)
        e_alone = O.rel_error(q.cpu().numpy(), qa.cpu().numpy(), area)
        e_or = O.rel_error(q.cpu().numpy(), ref, area)
        say(f"  {w.name}: vs alone {e_alone:.2e} vs oracle {e_or:.2e} iters {d.total_iters}")
        assert rca == C.CQM_OK and e_alone < 1e-9 and e_or < 1e-8
    for p in probs + alone:
        p.close()


def test_batch_mixing_forms_and_precisions(ctx):
    """Dense, matrix-free and FP64 problems in one call (grouped by precision)."""
    V1, T1 = W.icosphere(1)
    V2, T2 = W.ellipsoid(1, (1.2, 0.8, 1.0))
    specs = [(V1, T1, 8, C.CQM_MIXED_PLAIN, C.CQM_FORM_MATRIX_FREE),
             (V2, T2, 10, C.CQM_FP64_PLAIN, C.CQM_FORM_DENSE),
             (V1, T1, 6, C.CQM_MIXED_PLAIN, C.CQM_FORM_DENSE)]
    probs = []
    for V, T, N, mode, form in specs:
        p = Problem(ctx, V, T, N, 2.0, mode=mode, form=form)
        p.set_plane_wave()
        probs.append(p)
    res, rc = solve_batch(probs)
    assert rc == C.CQM_OK
    for (V, T, N, _, _), (q, d) in zip(specs, res):
        _, _, area = O.triangle_quadrature(V, T)
        ref = O.solve(V, T, N, 2.0)
        assert O.rel_error(q.cpu().numpy(), ref, area) < 1e-8
    for p in probs:
        p.close()


def test_batch_rejects_mixed_preconditioning(ctx):
    """Stored-operator problems batched together share one Krylov layout: a
    batch mixing preconditioned and plain ones is refused, not half-solved."""
    V1, T1 = W.icosphere(1)
    say("batch precond mismatch M=80")
    a = Problem(ctx, V1, T1, 6, 2.0, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE,
                precond=C.CQM_PRECOND_BLOCK_JACOBI)
    b = Problem(ctx, V1, T1, 6, 2.0, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE,
                precond=C.CQM_PRECOND_NONE)
    for p in (a, b):
        p.set_plane_wave()
    with pytest.raises(C.CqmError) as e:
        solve_batch([a, b])
    assert e.value.code == C.CQM_EINVAL
    # each alone still solves
    for p in (a, b):
        _, rc, d = p.solve()
        assert rc == C.CQM_OK and d.converged == 1
    a.close()
    b.close()


def test_batch_work_queue_assembly_equals_single_assembly(ctx):
    # a batch assembles its stored operators in one work-queue launch
    # (workgroups claim (problem, tile pair, frequency tile) items); the
    # entries must be exactly those of each problem's own assembly
    say("work-queue assembly vs single assembly")
    specs = [(W.icosphere(2), 16, 2.0), (W.ellipsoid(1, (1.3, 0.7, 1.0)), 8, 2.0),
             (W.icosphere(3), 32, 4.0)]
    probs = []
    for (V, T), N, Tend in specs:
        p = Problem(ctx, V, T, N, Tend, mode=C.CQM_FP64_PLAIN, form=C.CQM_FORM_DENSE)
        p.set_plane_wave()
        probs.append(p)
    res, rc = solve_batch(probs)
    assert rc == C.CQM_OK
    for ((V, T), N, Tend), p in zip(specs, probs):
        H = N // 2 + 1
        x = torch.as_tensor(W.random_complex((H, len(T)), seed=17), device="cuda")
        y_batch = p.apply(x, 0, 64).cpu().numpy()
        q = Problem(ctx, V, T, N, Tend, mode=C.CQM_FP64_PLAIN, form=C.CQM_FORM_DENSE)
        y_alone = q.apply(x, 0, 64).cpu().numpy()
        assert np.array_equal(y_batch, y_alone), (len(T), N)
        q.close()
        p.close()
