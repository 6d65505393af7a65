"""GPU parity: the HIP library against the FP64 oracle, through the C ABI."""
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
    assert torch.cuda.is_available()
    c = C.cqm_ctx_create(0)
    yield c
    C.cqm_ctx_destroy(c)


@pytest.fixture(scope="module")
def c1():
    wl = W.C1
    V, T = wl.mesh()
    r = O.solve(V, T, wl.N, wl.T, return_all=True)
    _, _, area = O.triangle_quadrature(V, T)
    return wl, V, T, r, area


def test_near_static_entries_match_oracle(ctx, c1):
    wl, V, T, r, _ = c1
    say("near static M=320")
    p = Problem(ctx, V, T, wl.N, wl.T)
    rp, col, sv = C.cqm_near_entries(p.handle)
    pairs = r["pairs"]
    assert len(col) == len(pairs)
    got = {(i, int(col[k])): sv[k] for i in range(len(T)) for k in range(rp[i], rp[i + 1])}
    for (i, j, _), ref in zip(pairs, r["static"]):
        assert abs(got[(i, j)] - ref) <= 1e-13 * abs(ref)
    p.close()


@pytest.mark.parametrize("form", [C.CQM_FORM_DENSE, C.CQM_FORM_MATRIX_FREE])
@pytest.mark.parametrize("mode", [C.CQM_FP64_PLAIN, C.CQM_MIXED_PLAIN])
def test_apply_V_matches_oracle(ctx, c1, form, mode):
    wl, V, T, r, _ = c1
    say(f"apply_V M=320 form={form} mode={mode}")
    p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=form)
    H = O.num_frequencies_half(wl.N + 1)
    x = W.random_complex((H, len(T)), seed=7)
    xt = torch.as_tensor(x, device="cuda")
    precs = (64, 32) if mode == C.CQM_MIXED_PLAIN or form == C.CQM_FORM_MATRIX_FREE else (64,)
    for prec in precs:
        y = p.apply(xt, 0, prec).cpu().numpy().astype(np.complex128)
        for l in range(H):
            A = O.assemble_V(V, T, r["s"][l], pairs=r["pairs"], static=r["static"])
            ref = A @ x[l]
            err = np.linalg.norm(y[l] - ref) / np.linalg.norm(ref)
            tol = 1e-13 if prec == 64 else 2e-6
            assert err < tol, (l, prec, err)
    # a sub-range of frequencies
    y2 = p.apply(xt[3:5], 3, 64).cpu().numpy()
    A = O.assemble_V(V, T, r["s"][4], pairs=r["pairs"], static=r["static"])
    assert np.linalg.norm(y2[1] - A @ x[4]) < 1e-13 * np.linalg.norm(A @ x[4])
    p.close()


def test_gpu_operator_symmetric(ctx, c1):
    wl, V, T, r, _ = c1
    p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_FP64_PLAIN, form=C.CQM_FORM_MATRIX_FREE)
    H = O.num_frequencies_half(wl.N + 1)
    x = torch.as_tensor(W.random_complex((H, len(T)), seed=1), device="cuda")
    z = torch.as_tensor(W.random_complex((H, len(T)), seed=2), device="cuda")
    Vx, Vz = p.apply(x).cpu().numpy(), p.apply(z).cpu().numpy()
    xn, zn = x.cpu().numpy(), z.cpu().numpy()
    for l in range(H):
        a, b = zn[l] @ Vx[l], xn[l] @ Vz[l]
        scale = np.abs(zn[l]) @ np.abs(Vx[l])
        assert abs(a - b) < 1e-13 * scale, (l, abs(a - b), scale)
    p.close()


@pytest.mark.parametrize("form", [C.CQM_FORM_DENSE, C.CQM_FORM_MATRIX_FREE])
@pytest.mark.parametrize("mode", [C.CQM_FP64_PLAIN, C.CQM_MIXED_PLAIN])
def test_solve_C1_matches_oracle(ctx, c1, form, mode):
    wl, V, T, r, area = c1
    say(f"solve C1 form={form} mode={mode}")
    p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=form)
    p.set_plane_wave()
    q, rc, diag = p.solve()
    q = q.cpu().numpy()
    err = O.rel_error(q, r["q"], area)
    say(f"  rc={rc} err={err:.3e} iters={diag.total_iters} cycles={diag.cycles} "
        f"resid={diag.max_rel_residual:.2e}")
    assert rc == C.CQM_OK
    assert diag.max_rel_residual <= 1e-13
    assert diag.converged == 1
    assert err < 1e-8
    p.close()


@pytest.mark.parametrize("form", [C.CQM_FORM_DENSE, C.CQM_FORM_MATRIX_FREE])
@pytest.mark.parametrize("mode", [C.CQM_FP64_PLAIN, C.CQM_MIXED_PLAIN])
def test_block_jacobi_keeps_the_answer_and_cuts_steps(ctx, c1, mode, form):
    """Right preconditioning by the inverses of the 64 x 64 diagonal blocks
    changes the Krylov space, not the system: both runs meet the oracle's
    answer, the preconditioned one in fewer Arnoldi steps (stored form: the
    blocks are tiles of the operator; matrix-free form: assembled on their
    own)."""
    wl, V, T, r, area = c1
    runs = {}
    for pc in (C.CQM_PRECOND_NONE, C.CQM_PRECOND_BLOCK_JACOBI):
        say(f"block-Jacobi C1 mode={mode} form={form} precond={pc}")
        p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=form, precond=pc)
        p.set_plane_wave()
        q, rc, d = p.solve()
        q = q.cpu().numpy()
        err = O.rel_error(q, r["q"], area)
        say(f"  rc={rc} err={err:.3e} iters={d.total_iters} max={d.max_iters} cycles={d.cycles}")
        assert rc == C.CQM_OK and d.converged == 1
        assert d.max_rel_residual <= 1e-13
        assert err < 1e-8
        runs[pc] = (q, d.total_iters)
        p.close()
    q0, it0 = runs[C.CQM_PRECOND_NONE]
    q1, it1 = runs[C.CQM_PRECOND_BLOCK_JACOBI]
    assert it1 < it0
    assert O.rel_error(q1, q0, area) < 1e-8


@pytest.mark.parametrize("restart", [2, 3, 5])
@pytest.mark.parametrize("form", [C.CQM_FORM_DENSE, C.CQM_FORM_MATRIX_FREE])
def test_short_restarts_match_oracle(ctx, c1, form, restart):
    """Restart lengths of a few steps: cycles end on the basis being full
    (the block product of the next step is then formed by the first step of
    the next cycle), many refinement cycles; both precisions."""
    wl, V, T, r, area = c1
    for mode in (C.CQM_FP64_PLAIN, C.CQM_MIXED_PLAIN):
        say(f"short restart m={restart} form={form} mode={mode}")
        p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=form, gmres_restart=restart,
                    max_cycles=400)
        p.set_plane_wave()
        q, rc, d = p.solve()
        err = O.rel_error(q.cpu().numpy(), r["q"], area)
        say(f"  rc={rc} err={err:.3e} iters={d.total_iters} cycles={d.cycles}")
        assert rc == C.CQM_OK and d.converged == 1 and err < 1e-8
        p.close()


def test_kernel_work_counters(ctx, c1):
    """The per-class work the kernels count for the roofline matches what the
    solve did: every far pair of the symmetric assembly once per frequency,
    one operator triangle per Arnoldi step, one far field per product."""
    wl, V, T, r, _ = c1
    M = len(T)
    nnz = len(r["pairs"])
    k = {n: i for i, n in enumerate(C.KERNEL_CLASSES)}
    say("kernel work counters M=320 dense/matrix-free mixed")
    p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_DENSE, profile=1)
    p.set_plane_wave()
    _, rc, d = p.solve()
    assert rc == C.CQM_OK
    w = list(d.kernel_work)
    assert w[k["assemble"]] == (M * M - nnz) // 2 * 36 * d.n_systems
    # stored operator: the upper triangle of V(s) (complex symmetric) once,
    # input and result vectors once
    per_product = M * (M + 1) // 2 + 2 * M
    assert w[k["gemv32"]] == d.total_iters * per_product * 8
    assert w[k["gemv64"]] % (per_product * 16) == 0 and w[k["gemv64"]] > 0
    assert w[k["arnoldi"]] >= sum(7 * M * 8 for _ in range(d.total_iters))
    assert d.kernel_calls[k["arnoldi"]] > 0 and d.kernel_ms[k["arnoldi"]] > 0
    p.close()
    p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_MATRIX_FREE,
                profile=1)
    p.set_plane_wave()
    _, rc, d = p.solve()
    assert rc == C.CQM_OK
    w = list(d.kernel_work)
    per = (M * M - nnz) * 36
    assert w[k["far32"]] == d.total_iters * per
    assert w[k["far64"]] % per == 0 and w[k["far64"]] >= d.n_systems * per
    p.close()


@pytest.mark.parametrize("layout", [C.CQM_ARNOLDI_GROUP, C.CQM_ARNOLDI_SPLIT])
@pytest.mark.parametrize("mode", [C.CQM_FP64_PLAIN, C.CQM_MIXED_PLAIN])
def test_arnoldi_layouts_match_oracle(ctx, c1, layout, mode):
    """Both Arnoldi layouts (one workgroup per system; split over row slices)
    reach the oracle's density, in both inner precisions."""
    wl, V, T, r, area = c1
    say(f"arnoldi layout={layout} mode={mode} M=320")
    p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=C.CQM_FORM_DENSE, arnoldi_layout=layout)
    p.set_plane_wave()
    q, rc, diag = p.solve()
    err = O.rel_error(q.cpu().numpy(), r["q"], area)
    say(f"  rc={rc} err={err:.3e} iters={diag.total_iters} cycles={diag.cycles}")
    assert rc == C.CQM_OK and diag.max_rel_residual <= 1e-13 and err < 1e-8
    p.close()


def test_autotuned_shapes_give_the_same_product(ctx, c1):
    """The far-product launch shape picked by timing (per context and shape)
    changes only the summation order: the product matches the fixed-shape one
    and the oracle; the chosen shape is reported."""
    wl, V, T, r, _ = c1
    H = O.num_frequencies_half(wl.N + 1)
    x = torch.as_tensor(W.random_complex((H, len(T)), seed=11), device="cuda")
    ys = {}
    for tune in (0, 1):
        c = C.cqm_ctx_create(0)
        p = Problem(c, V, T, wl.N, wl.T, mode=C.CQM_MIXED_PLAIN, form=C.CQM_FORM_MATRIX_FREE,
                    autotune=tune)
        ys[tune] = {prec: p.apply(x, 0, prec).cpu().numpy() for prec in (32, 64)}
        p.set_plane_wave()
        _, rc, d = p.solve()
        assert rc == C.CQM_OK
        assert d.far_tile in (17, 16, 13, 11, 9) and d.far_waves in (2048, 4096, 8192)
        say(f"  autotune={tune}: far tile {d.far_tile}, waves {d.far_waves}")
        p.close()
        C.cqm_ctx_destroy(c)
    for l in range(H):
        A = O.assemble_V(V, T, r["s"][l], pairs=r["pairs"], static=r["static"])
        ref = A @ x.cpu().numpy()[l]
        for tune in (0, 1):
            assert np.linalg.norm(ys[tune][64][l] - ref) < 1e-13 * np.linalg.norm(ref)
            assert np.linalg.norm(ys[tune][32][l] - ref) < 2e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("mode", [C.CQM_MIXED_PLAIN, C.CQM_FP64_PLAIN])
def test_graph_replayed_steps_equal_launched_ones(ctx, c1, mode):
    """Arnoldi steps replayed from captured HIP graphs (kept across solves of
    the same problem) give bit-identical densities to directly launched ones,
    on the first solve (capture) and on later ones (replay), with eager work
    and host synchronisations between replays."""
    wl, V, T, r, area = c1
    qs = {}
    for graphs in (0, 1):
        p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=C.CQM_FORM_DENSE, graphs=graphs)
        p.set_plane_wave()
        qs[graphs] = []
        for rep in range(3):
            q, rc, d = p.solve()
            assert rc == C.CQM_OK
            qs[graphs].append(q.cpu().numpy())
        p.close()
    say(f"graphs mode={mode}: err vs oracle {O.rel_error(qs[1][2], r['q'], area):.2e}")
    for q in qs[0] + qs[1]:
        assert np.array_equal(q, qs[0][0])
    assert O.rel_error(qs[1][2], r["q"], area) < 1e-8


def test_solve_C2_against_stored_oracle(ctx):
    wl = W.C2
    path = os.path.join(GOLDEN, f"{wl.name}.npz")
    g = np.load(path)
    V, T = wl.mesh()
    _, _, area = O.triangle_quadrature(V, T)
    for mode in (C.CQM_FP64_PLAIN, C.CQM_MIXED_PLAIN):
        say(f"solve C2 mode={mode}")
        p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=C.CQM_FORM_DENSE)
        p.set_plane_wave()
        q, rc, diag = p.solve()
        err = O.rel_error(q.cpu().numpy(), g["q"], area)
        steps = O.step_errors(q.cpu().numpy(), g["q"], area)
        say(f"  rc={rc} err={err:.3e} max step err={steps.max():.2e} iters={diag.total_iters} "
            f"t_setup={diag.t_setup_ms:.1f}ms t_solve={diag.t_solve_ms:.1f}ms")
        assert rc == C.CQM_OK and err < 1e-8
        p.close()


# N = 2 puts rho = 1e-4 per step: rounding of the three frequency solutions
# (~1e-16 times the condition number, ~10) is amplified by rho^-N = 1e8 with no
# averaging over steps, so its floor is ~1e-7 rather than the 1e-8 of N >= 7.
@pytest.mark.parametrize("level,N,T,axes,tol", [(1, 7, 2.0, (1.0, 1.0, 1.0), 1e-8),
                                                (1, 2, 0.5, (1.0, 1.0, 1.0), 2e-7),
                                                (1, 10, 3.0, (1.3, 0.7, 0.9), 1e-8)])
def test_small_and_ragged_cases(ctx, level, N, T, axes, tol):
    """Odd N (even F: a real middle frequency), the smallest N, an ellipsoid."""
    V, Tr = W.ellipsoid(level, axes)
    say(f"ragged level={level} N={N} axes={axes}")
    d = (0.3, -0.5, 0.8)
    ref = O.solve(V, Tr, N, T, direction=np.asarray(d) / np.linalg.norm(d), sigma=0.3, t0=1.2)
    _, _, area = O.triangle_quadrature(V, Tr)
    for form in (C.CQM_FORM_DENSE, C.CQM_FORM_MATRIX_FREE):
        p = Problem(ctx, V, Tr, N, T, mode=C.CQM_MIXED_PLAIN, form=form)
        p.set_plane_wave(d, 0.3, 1.2)
        q, rc, diag = p.solve()
        err = O.rel_error(q.cpu().numpy(), ref, area)
        assert rc == C.CQM_OK and err < tol, err
        p.close()


def test_dirichlet_samples_path(ctx):
    """Caller-provided samples at the quadrature points (random data)."""
    wl = W.C0_TINY
    V, T = wl.mesh()
    g = np.random.default_rng(4).standard_normal((wl.N + 1, len(T), 6))
    ref = O.solve(V, T, wl.N, wl.T, samples=g)
    _, _, area = O.triangle_quadrature(V, T)
    p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_FP64_PLAIN)
    p.set_samples(g)
    q, rc, _ = p.solve()
    assert rc == C.CQM_OK and O.rel_error(q.cpu().numpy(), ref, area) < 1e-8
    p.close()


def test_error_paths(ctx):
    wl = W.C0_TINY
    V, T = wl.mesh()
    # no workspace
    h = C.cqm_problem_create(ctx, V, T, wl.N, wl.T)
    out = torch.empty((wl.N + 1, len(T)), dtype=torch.float64, device="cuda")
    with pytest.raises(C.CqmError) as e:
        C.cqm_solve(h, out.data_ptr())
    assert e.value.code == C.CQM_ENOMEM
    C.cqm_problem_destroy(h)
    # bad meshes
    bad = T.copy()
    bad[0, 0] = len(V) + 5
    with pytest.raises(C.CqmError) as e:
        C.cqm_problem_create(ctx, V, bad, wl.N, wl.T)
    assert e.value.code == C.CQM_EINVAL
    deg = T.copy()
    deg[0] = [deg[0, 0], deg[0, 0], deg[0, 1]]
    with pytest.raises(C.CqmError):
        C.cqm_problem_create(ctx, V, deg, wl.N, wl.T)
    # no incident data
    p = Problem(ctx, V, T, wl.N, wl.T)
    with pytest.raises(C.CqmError) as e:
        p.solve()
    assert e.value.code == C.CQM_EINVAL
    # non-finite data -> CQM_ENAN, output still written
    g = np.zeros((wl.N + 1, len(T), 6))
    g[3, 5, 2] = np.nan
    p.set_samples(g)
    with pytest.raises(C.CqmError) as e:
        p.solve()
    assert e.value.code == C.CQM_ENAN
    # one cycle, tiny restart: not converged, diagnostics still filled
    p2 = Problem(ctx, V, T, wl.N, wl.T, gmres_restart=2, max_cycles=1)
    p2.set_plane_wave()
    q, rc, diag = p2.solve()
    assert rc == C.CQM_ENOCONV and diag.converged == 0 and diag.cycles == 1
    p.close()
    p2.close()
