"""Pins of the time-marching oracle (oracle/marching.py) by facts the paper and
the mathematics fix, not by retyping its formulas."""
import numpy as np
import pytest

import cqm_workloads as W
import oracle as O


@pytest.fixture(scope="module")
def tiny():
    wl = W.C0_TINY
    V, T = wl.mesh()
    qm, Wt, ratio = O.solve_marching(V, T, wl.N, wl.T, return_weights=True)
    s, rho, dt = O.frequencies(wl.N, wl.T)
    _, _, area = O.triangle_quadrature(V, T)
    return wl, V, T, qm, Wt, ratio, rho, dt, area


def test_weights_are_real_and_the_first_is_spd(tiny):
    # V(conj s) = conj V(s) and s_{F-l} = conj s_l make every weight real (up to
    # rounding amplified by rho^-N = 1e8); the paper factorises What_0 as a real
    # symmetric positive definite matrix (Section 3.2)
    wl, V, T, qm, Wt, ratio, rho, dt, area = tiny
    assert ratio < 1e-7
    W0 = Wt[0]
    assert np.linalg.norm(W0 - W0.T) <= 1e-14 * np.linalg.norm(W0)
    assert np.linalg.eigvalsh(0.5 * (W0 + W0.T)).min() > 0


def test_first_weight_is_the_operator_at_three_halves_over_dt(tiny):
    # the zeroth coefficient of the generating function sum_n W_n xi^n is its
    # value at xi = 0: W_0 = V(delta(0)/dt) = V(3/(2 dt)) exactly; the F-point
    # transform adds aliased terms of order rho^F
    wl, V, T, qm, Wt, ratio, rho, dt, area = tiny
    A = O.assemble_V(V, T, 1.5 / dt)
    assert np.abs(A.imag).max() == 0.0
    assert np.linalg.norm(Wt[0] - A.real) <= 10 * rho ** (wl.N + 1) * np.linalg.norm(A.real)
    # and the second: W_1 = d/dxi V(delta(xi)/dt) at 0 = -(2/dt) dV/ds at 3/(2 dt),
    # checked by a centred difference of the oracle's own V(s) in s
    h = 1e-4 / dt
    dV = (O.assemble_V(V, T, 1.5 / dt + h) - O.assemble_V(V, T, 1.5 / dt - h)).real / (2 * h)
    assert np.linalg.norm(Wt[1] - (-2.0 / dt) * dV) <= 1e-6 * np.linalg.norm(Wt[1])


def test_marching_equals_the_all_at_once_solve(tiny):
    # both solve the same CQM convolution system; the all-at-once form wraps
    # it around a circle of F points (terms of order rho^F) and the marching
    # weights carry the same aliasing
    wl, V, T, qm, Wt, ratio, rho, dt, area = tiny
    qa = O.solve(V, T, wl.N, wl.T)
    assert O.rel_error(qm, qa, area) <= 10 * rho ** (wl.N + 1)


def test_march_recovers_a_known_history_for_scalar_weights():
    # K(s) = 1/s (time integration) has the BDF2 weights dt (1 - 3^-(n+1));
    # feeding the discrete convolution of a known sequence back must return
    # that sequence: pins the history sum's indices and the first-weight solve
    dt, N = 0.1, 40
    w = dt * (1.0 - 3.0 ** -(np.arange(N + 1) + 1.0))
    rng = np.random.default_rng(3)
    qs = rng.standard_normal((N + 1, 1))
    b = np.array([sum(w[n - k] * qs[k] for k in range(n + 1)) for n in range(N + 1)])
    q = O.march(w[:, None, None], b)
    assert np.max(np.abs(q - qs)) < 1e-11
    # a dropped history term (k = n - 1) would not return it
    bad = b.copy()
    bad[5] -= w[1] * qs[4]
    assert np.max(np.abs(O.march(w[:, None, None], bad) - qs)) > 1e-3


def test_compressed_weights_reduce_to_the_plain_ones(tiny):
    # no admissible block (eta = 0) and MACA to full rank (eps = 0): the
    # compressed tensor is the plain one, so the fibre transform of eq.
    # fastdft must give the plain weights of eq. dft
    wl, V, T, qm, Wt, ratio, rho, dt, area = tiny
    s, _, _ = O.frequencies(wl.N, wl.T)
    op = O.build_compressed(V, T, s, 8, 0.0, 2, 0.0)
    Wc, r = O.compressed_weights(op, rho, len(T))
    assert np.linalg.norm(Wc - Wt) <= 1e-7 * np.linalg.norm(Wt)


def test_fibre_transform_equals_the_transform_of_the_tensor(tiny):
    # the slices do not depend on frequency, so transforming the fibres and
    # transforming the expanded tensor give the same weights (with far blocks)
    wl, V, T, qm, Wt, ratio, rho, dt, area = tiny
    s, _, _ = O.frequencies(wl.N, wl.T)
    op = O.build_compressed(V, T, s, 4, 1.0, 2, 1e-6)
    assert len(op["far"]) > 0
    Wc, r = O.compressed_weights(op, rho, len(T))
    A = O.compressed_dense(op, len(T))  # (M, M, F)
    F = wl.N + 1
    direct = np.stack([(rho ** -n / F) * sum(A[:, :, l] * np.exp(2j * np.pi * n * l / F)
                                              for l in range(F)) for n in range(F)])
    # equal up to rounding, which rho^-n (up to 1e8) amplifies: 4e-8 measured
    assert np.linalg.norm(Wc - direct.real) <= 1e-6 * np.linalg.norm(direct.real)


def test_compressed_marching_approaches_the_plain_one(tiny):
    # the error against the plain marching solve falls with the MACA
    # tolerance until the interpolation error of the far field is left
    # (Corollary combierr), which falls with the order m (Theorem h2err)
    wl, V, T, qm, Wt, ratio, rho, dt, area = tiny
    err = lambda m, eps: O.rel_error(O.solve_marching_compressed(V, T, wl.N, wl.T, 4, 1.0, m, eps),
                                     qm, area)
    e_eps = [err(3, eps) for eps in (1e-2, 1e-4, 1e-6)]
    assert e_eps[0] > e_eps[1] > e_eps[2]
    e_m = [err(m, 1e-12) for m in (2, 3, 4)]
    assert e_m[0] > e_m[1] > e_m[2] and e_m[2] < 1e-5
