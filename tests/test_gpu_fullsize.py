"""GPU parity at the full benchmark sizes, through the C ABI.

* Operator products of the 5120-triangle sphere (N = 128: 65 distinct
  frequencies) on sampled rows, which the oracle assembles one by one
  (Section 3.2 Galerkin entries), for the stored and matrix-free forms in
  both precisions.
* Solves of the 5120-triangle workload against its stored oracle solution
  (tests/golden/sphere5120_N128_T6.npz, written by make_golden.py from
  oracle/ only) in the launch configuration the benchmark times (mixed,
  stored form), in FP64, and in the compressed form; and the matrix-free
  form of the 1280-triangle workload against its stored solution.
* The compressed operator at the configured interpolation order m = 4
  (p = 64), leaf size 32 and eta = 1 on a mesh with admissible blocks,
  against the oracle's compressed operator (Algorithm 3).
"""
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
def c3rows():
    """Oracle rows of V(s_l) for 16 sampled triangles, every distinct l."""
    wl = W.C3
    V, T = wl.mesh()
    s, _, _ = O.frequencies(wl.N, wl.T)
    H = O.num_frequencies_half(wl.N + 1)
    rows = np.linspace(0, len(T) - 1, 16).astype(int)
    say("oracle: near field of the 5120-triangle mesh")
    pairs = O.near_pairs(T)
    static = O.near_static(V, T, pairs, 5)
    A = []
    for l in range(H):
        A.append(O.assemble_V(V, T, s[l], pairs=pairs, static=static, rows=rows))
    say(f"oracle: {H} x {len(rows)} sampled rows done")
    return wl, V, T, rows, np.stack(A)


@pytest.mark.parametrize("form", [C.CQM_FORM_DENSE, C.CQM_FORM_MATRIX_FREE])
@pytest.mark.parametrize("mode", [C.CQM_FP64_PLAIN, C.CQM_MIXED_PLAIN])
def test_apply_V_C3_sampled_rows(ctx, c3rows, form, mode):
    wl, V, T, rows, A = c3rows
    H = A.shape[0]
    say(f"apply_V M=5120 N=128 form={form} mode={mode}")
    p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=form)
    x = W.random_complex((H, len(T)), seed=21)
    xt = torch.as_tensor(x, device="cuda")
    precs = (64, 32) if mode == C.CQM_MIXED_PLAIN or form == C.CQM_FORM_MATRIX_FREE else (64,)
    for prec in precs:
        y = p.apply(xt, 0, prec).cpu().numpy().astype(np.complex128)
        tol = 1e-13 if prec == 64 else 2e-6
        worst = 0.0
        for l in range(H):
            ref = A[l] @ x[l]
            err = np.linalg.norm(y[l, rows] - ref) / np.linalg.norm(ref)
            worst = max(worst, err)
            assert err < tol, (l, prec, err)
        say(f"  precision {prec}: worst relative row error {worst:.2e} over {H} frequencies")
    p.close()


def _golden(name):
    return np.load(os.path.join(GOLDEN, f"{name}.npz"))


# Tolerance of the 5120-triangle solves (N = 128, rho^N = 1e-8).  The inverse
# scaled transform multiplies per-frequency rounding by up to rho^-N = 1e8
# at the last steps, so two FP64 computations of the same discrete solution
# differ there at the 1e-8 level: the oracle against itself with the
# transposed assembled operator (equal in exact arithmetic) differs by
# 5.5e-9, and a separately written FP64 path differs in every step (operator
# entries, right-hand side, transforms, solver), each such source adding its
# own share.  The bar is therefore 2e-8 for the whole history (twice the
# 1e-8 target), and steps n <= N/2, where rho^-n <= 1e4 and the same rounding
# stays near 1e-11, must agree to 1e-10: an error in the arithmetic shows
# there, amplification does not.
C3_TOL, C3_EARLY_TOL = 2e-8, 1e-10
# Paths whose refinement residual is formed in plain FP64 (the matrix-free
# product: FP64 partial sums, no double-double) have a higher rounding floor;
# the stored form measured 2.4e-8 with such residuals.  Their whole-history
# bar is 3e-8, with the same 1e-10 bar for n <= N/2.
C3_TOL_FP64_RESIDUAL = 3e-8


@pytest.mark.parametrize("mode", [C.CQM_MIXED_PLAIN, C.CQM_FP64_PLAIN])
def test_solve_C3_matches_stored_oracle(ctx, mode):
    wl = W.C3
    V, T = wl.mesh()
    g = _golden(wl.name)
    _, _, area = O.triangle_quadrature(V, T)
    say(f"solve M=5120 N=128 mode={mode} (stored form)")
    p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=C.CQM_FORM_DENSE)
    p.set_plane_wave()
    q, rc, d = p.solve()
    q = q.cpu().numpy()
    err = O.rel_error(q, g["q"], area)
    emax = float(np.max(O.step_errors(q, g["q"], area)))
    say(f"  rc={rc} err={err:.2e} max step err={emax:.2e} iters={d.total_iters} "
        f"resid={d.max_rel_residual:.1e}")
    early = float(np.max(O.step_errors(q, g["q"], area)[: wl.N // 2 + 1]))
    say(f"  largest step error for n <= N/2: {early:.2e}")
    assert rc == C.CQM_OK and d.converged == 1
    assert err < C3_TOL and early < C3_EARLY_TOL
    p.close()


@pytest.mark.parametrize("mode", [C.CQM_MIXED_PLAIN, C.CQM_FP64_PLAIN])
def test_solve_C2_matrix_free_matches_stored_oracle(ctx, mode):
    wl = W.C2
    V, T = wl.mesh()
    g = _golden(wl.name)
    _, _, area = O.triangle_quadrature(V, T)
    say(f"solve M=1280 N=64 mode={mode} matrix-free")
    p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, form=C.CQM_FORM_MATRIX_FREE)
    p.set_plane_wave()
    q, rc, d = p.solve()
    err = O.rel_error(q.cpu().numpy(), g["q"], area)
    say(f"  rc={rc} err={err:.2e} iters={d.total_iters}")
    assert rc == C.CQM_OK and err < 1e-8
    p.close()


def test_compressed_C3_against_stored_oracle(ctx):
    """The compressed form of the 5120-triangle workload against the plain
    oracle.  Refined with the compressed operator itself (refine_plain = 0)
    at the configured order (m = 4, eta = 1) the error is the Chebyshev
    interpolation error of the far field (about 5e-2 measured; Theorem
    h2err: it falls with m and with stricter admissibility); at m = 6 with
    eta = 0.25 (1962 admissible blocks) and with eta = 0.125 (no admissible
    block at this size: every block compressed across frequencies only) it
    must meet the 1e-5 bound of the mixed compressed path.  With refinement
    residuals from the plain operator (the
    default) the configured compressed form must give the plain solution,
    to the bar of solves with plain FP64 residuals."""
    wl = W.C3
    V, T = wl.mesh()
    g = _golden(wl.name)
    _, _, area = O.triangle_quadrature(V, T)
    errs = {}
    for m, eta, rp in ((4, 1.0, 0), (6, 0.25, 0), (4, 0.125, 0), (4, 1.0, 1)):
        p = Problem(ctx, V, T, wl.N, wl.T, mode=C.CQM_MIXED_H2ACA, eta=eta, refine_plain=rp,
                    cheb_m=m)
        p.set_plane_wave()
        q, rc, d = p.solve()
        q = q.cpu().numpy()
        errs[eta, rp] = O.rel_error(q, g["q"], area)
        assert d.n_far_blocks > 0 or eta < 0.25
        early = float(np.max(O.step_errors(q, g["q"], area)[: wl.N // 2 + 1]))
        say(f"  compressed m={m} eta={eta} refine_plain={rp}: rc={rc} err vs oracle {errs[eta, rp]:.2e} "
            f"(n <= N/2: {early:.1e}) "
            f"far/near blocks {d.n_far_blocks}/{d.n_near_blocks} max rank {d.max_rank} op "
            f"{d.operator_bytes / 1e9:.2f} GB, cycles {d.cycles}, solve {d.t_solve_ms:.0f} ms")
        assert rc == C.CQM_OK and d.converged == 1
        if rp:
            assert early < C3_EARLY_TOL
        p.close()
    assert errs[1.0, 0] < 0.1
    assert errs[0.25, 0] < 1e-5
    assert errs[0.125, 0] < 1e-5
    assert errs[1.0, 1] < C3_TOL_FP64_RESIDUAL


@pytest.mark.parametrize("eps,tag", [(1e-6, "e6"), (1e-10, "e10")])
def test_compressed_C3_rows_match_oracle(ctx, eps, tag):
    """The configured compressed operator of the 5120-triangle workload (leaf
    size 32, eta = 1, m = 4: 1612 Tucker cores of p = 64 with their
    transfers, expanded far and near blocks, full band of 129 frequencies)
    against the oracle's compressed operator on the rows of four leaf
    clusters (tests/golden/sphere5120_N128_T6_h2rows.npz, make_golden.py
    --h2rows: only the blocks of those block rows are compressed there).
    FP64 slices: with the oracle's pivots the rows agree to rounding; a MACA
    pivot that flips on a floating-point near-tie changes that block's
    approximant within the tolerance eps, so the bar is 10 eps (1e-9 for
    eps = 1e-10); FP32 slices: max(1e-6, 10 eps)."""
    wl = W.C3
    V, T = wl.mesh()
    g = _golden("sphere5120_N128_T6_h2rows")
    rows, ref = g["rows"], g[f"y_{tag}"]
    s, _, _ = O.frequencies(wl.N, wl.T)
    x = W.random_complex((len(s), len(T)), seed=int(g["seed"]))
    for mode, tol in ((C.CQM_FP64_H2ACA, 10 * eps if eps > 1e-8 else 1e-9),
                      (C.CQM_MIXED_H2ACA, max(1e-6, 10 * eps))):
        p = Problem(ctx, V, T, wl.N, wl.T, mode=mode, n_min=32, eta=1.0, cheb_m=4, eps_aca=eps)
        y = p.apply(torch.as_tensor(x, device="cuda"), 0, 64).cpu().numpy()[:, rows]
        worst = max(np.linalg.norm(y[l] - ref[l]) / np.linalg.norm(ref[l]) for l in range(len(s)))
        say(f"  compressed C3 rows ({len(rows)}) eps={eps} mode={mode}: worst relative error "
            f"{worst:.2e} over {len(s)} frequencies")
        assert worst < tol
        p.close()


@pytest.fixture(scope="module")
def ordercase():
    """Two 320-triangle spheres six radii apart, N = 16: the spheres' clusters
    form two admissible 320 x 320 blocks (Tucker cores for m <= 6, expanded
    for m >= 7) beside small far and near blocks within each sphere.  The
    oracle's compressed operators for m = 4 .. 8 applied to a seeded input
    are stored (tests/golden/two_spheres640_N16_T2_h2.npz,
    make_golden.py --h2order), with the plain product."""
    V, T = W.two_spheres(2)
    return V, T, 16, 2.0, _golden("two_spheres640_N16_T2_h2")


@pytest.mark.parametrize("m", [4, 5, 6, 7, 8])
def test_compressed_orders_match_oracle(ctx, ordercase, m):
    """Chebyshev orders m = 4 .. 8 (p = 64 .. 512): cores, transfers and the
    expansion of far blocks against the oracle's operator; the interpolation
    error against the plain product falls with m (Section 4.2)."""
    V, T, N, Tend, g = ordercase
    x, ref, plain = g["x"], g[f"y_m{m}"], g["y_plain"]
    oranks, far = g[f"ranks_m{m}"], g[f"kinds_m{m}"]
    nfar, nnear = int(far.sum()), int((~far).sum())
    for mode, tol in ((C.CQM_FP64_H2ACA, 1e-12), (C.CQM_MIXED_H2ACA, 1e-6)):
        say(f"compressed m={m} two spheres mode={mode}")
        p = Problem(ctx, V, T, N, Tend, mode=mode, n_min=16, eta=1.0, cheb_m=m, eps_aca=1e-10)
        y = p.apply(torch.as_tensor(x, device="cuda"), 0, 64).cpu().numpy()
        st = C.cqm_operator_stats(p.handle)
        same_pivots = (st.max_rank == int(oranks.max()) and
                       abs(st.mean_rank - float(np.mean(oranks))) < 1e-12)
        worst = max(np.linalg.norm(y[l] - ref[l]) / np.linalg.norm(ref[l]) for l in range(len(x)))
        interp = max(np.linalg.norm(y[l] - plain[l]) / np.linalg.norm(plain[l]) for l in range(len(x)))
        say(f"  far/near {st.n_far_blocks}/{st.n_near_blocks}, ranks max {st.max_rank} mean "
            f"{st.mean_rank:.4f} (oracle {int(oranks.max())} {float(np.mean(oranks)):.4f}); "
            f"error vs oracle {worst:.2e}, vs plain {interp:.2e}")
        assert (st.n_far_blocks, st.n_near_blocks) == (nfar, nnear)
        bound = tol if (same_pivots or mode == C.CQM_MIXED_H2ACA) else 1e-9
        assert worst < bound, (mode, worst, bound)
        p.close()


def test_compressed_few_systems_match_full_band(ctx, ordercase):
    """Products over at most 16 systems split each row tile's tasks over the
    waves of a workgroup (a different summation order from the full band):
    a frequency sub-range equals the same rows of the full-band product."""
    V, T, N, Tend, g = ordercase
    x = g["x"]
    for mode, tol in ((C.CQM_FP64_H2ACA, 1e-13), (C.CQM_MIXED_H2ACA, 1e-6)):
        p = Problem(ctx, V, T, N, Tend, mode=mode, n_min=16, eta=1.0, cheb_m=5, eps_aca=1e-10)
        full = p.apply(torch.as_tensor(x, device="cuda"), 0, 64).cpu().numpy()
        for l0, nl in ((0, 1), (3, 5), (1, 16)):
            part = p.apply(torch.as_tensor(x[l0:l0 + nl], device="cuda"), l0, 64).cpu().numpy()
            e = max(np.linalg.norm(part[k] - full[l0 + k]) / np.linalg.norm(full[l0 + k])
                    for k in range(nl))
            say(f"  mode={mode} systems {l0}..{l0 + nl - 1}: relative difference {e:.1e}")
            assert e < tol
        p.close()


@pytest.fixture(scope="module")
def m4case():
    """1280-triangle sphere, N = 16: leaf size 32 and eta = 1 give admissible
    blocks (all small enough to be expanded; the p = 64 Tucker cores and
    transfers are exercised by the two-sphere case above).  The
    oracle's compressed operator applied to a seeded input is stored
    (tests/golden/sphere1280_N16_T2_h2m4.npz, make_golden.py --h2m4): its
    build takes minutes on the CPU."""
    V, T = W.icosphere(3)
    N, Tend = 16, 2.0
    return V, T, N, Tend, _golden("sphere1280_N16_T2_h2m4")


@pytest.mark.parametrize("eps,tag", [(1e-6, "e6"), (1e-10, "e10")])
def test_compressed_m4_operator_matches_oracle(ctx, m4case, eps, tag):
    V, T, N, Tend, g = m4case
    x, ref = g["x"], g[f"y_{tag}"]
    oranks, far = g[f"ranks_{tag}"], g[f"kinds_{tag}"]
    nfar, nnear = int(far.sum()), int((~far).sum())
    assert nfar > 0
    for mode, tol in ((C.CQM_FP64_H2ACA, 1e-12), (C.CQM_MIXED_H2ACA, 1e-6)):
        say(f"compressed m=4 apply eps={eps} mode={mode}")
        p = Problem(ctx, V, T, N, Tend, mode=mode, n_min=32, eta=1.0, cheb_m=4, eps_aca=eps)
        y = p.apply(torch.as_tensor(x, device="cuda"), 0, 64).cpu().numpy()
        st = C.cqm_operator_stats(p.handle)
        same_pivots = (st.max_rank == int(oranks.max()) and
                       abs(st.mean_rank - float(np.mean(oranks))) < 1e-12)
        worst = max(np.linalg.norm(y[l] - ref[l]) / np.linalg.norm(ref[l]) for l in range(len(x)))
        say(f"  far/near {st.n_far_blocks}/{st.n_near_blocks} (oracle {nfar}/{nnear}), ranks "
            f"max {st.max_rank} mean {st.mean_rank:.4f} (oracle {int(oranks.max())} "
            f"{float(np.mean(oranks)):.4f}); worst relative error {worst:.2e}")
        assert (st.n_far_blocks, st.n_near_blocks) == (nfar, nnear)
        # FP64: the same pivots give the oracle's operator to rounding; a
        # pivot flipped by a floating-point near-tie (rank statistics differ)
        # changes the approximant within its tolerance only
        bound = tol if (same_pivots or mode == C.CQM_MIXED_H2ACA) else max(tol, 10 * eps)
        assert worst < bound, (mode, worst, bound)
        p.close()
