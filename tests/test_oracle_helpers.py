"""Pins of the oracle's smaller helpers: the 1-D rules, the interpolation
polynomials, the right-hand side, the error measures and the full-band
compressed solve.  Each is checked against a closed form, an exactness
property or a limit in which it must reduce to another, separately pinned,
oracle function.
"""
import math

import numpy as np
import pytest

import cqm_workloads as W
import oracle as O


@pytest.mark.parametrize("q", range(1, 9))
def test_gauss_legendre_exact_to_degree_2q_minus_1(q):
    x, w = O.gauss_legendre01(q)
    assert np.all((x > 0) & (x < 1)) and np.all(w > 0)
    for k in range(2 * q):
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 1e-15
    # a q-point rule cannot integrate x^(2q) exactly: it is a genuine q-point rule
    assert abs(np.dot(w, x ** (2 * q)) - 1.0 / (2 * q + 1)) > 1e-14


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8])
def test_lagrange_on_chebyshev_nodes_is_cardinal_and_reproduces_polynomials(m):
    box = dict(lo=np.array([-0.3, 0.1, 2.0]), hi=np.array([0.7, 0.4, 2.5]))
    nodes = O.cheb_nodes(box, m)
    t = np.linspace(-0.3, 0.7, 23)
    assert np.allclose(O.lagrange_1d(nodes[0], nodes[0]), np.eye(m), atol=1e-14)
    L = O.lagrange_1d(nodes[0], t)
    assert np.allclose(L.sum(axis=1), 1.0, atol=1e-13)
    for p in range(m):
        assert np.allclose(L @ nodes[0] ** p, t ** p, atol=1e-12)


def test_tensor_interpolation_index_matches_the_coupling_grid():
    # The cluster bases index mu = (a0 m + a1) m + a2; the coupling tensors of
    # far blocks lay their node grids out by meshgrid(..., indexing="ij").  The
    # two must agree, or U S U^T pairs the wrong nodes: interpolating
    # f = x y^2 + 3 z - x z (degree < m on each axis) through the grid values
    # must reproduce f off the grid.
    m = 3
    box = dict(lo=np.array([0.0, -1.0, 0.5]), hi=np.array([1.0, 0.0, 1.5]))
    nodes = O.cheb_nodes(box, m)
    grid = np.stack(np.meshgrid(*nodes, indexing="ij"), -1).reshape(-1, 3)
    f = lambda X: X[:, 0] * X[:, 1] ** 2 + 3.0 * X[:, 2] - X[:, 0] * X[:, 2]
    X = np.random.default_rng(5).uniform(box["lo"], box["hi"], size=(40, 3))
    from oracle.compress import _lagrange_3d
    assert np.allclose(_lagrange_3d(nodes, X) @ f(grid), f(X), atol=1e-12)


def flat_triangle(x0):
    V = np.array([[x0, 0.0, 0.0], [x0, 1.3, 0.2], [x0, 0.4, 0.9]])
    return V, np.array([[0, 1, 2]])


def test_rhs_on_a_wave_front_parallel_triangle_is_area_times_trace():
    # For d = e_x every point of a triangle in the plane x = x0 sees the same
    # value of the plane wave, so b_n = |tau| g_D(x0, t_n) with the
    # sound-soft data g_D = -A exp(-((t - x0 - t0) / sigma)^2).
    x0, N, Tend, sigma, t0, A = 0.35, 12, 3.0, 0.4, 1.1, 2.5
    V, T = flat_triangle(x0)
    area = 0.5 * np.linalg.norm(np.cross(V[1] - V[0], V[2] - V[0]))
    b = O.rhs(V, T, N, Tend, direction=(1.0, 0.0, 0.0), sigma=sigma, t0=t0, amplitude=A)
    t = np.arange(N + 1) * Tend / N
    expect = -A * area * np.exp(-(((t - x0 - t0) / sigma) ** 2))
    assert b.shape == (N + 1, 1)
    assert np.allclose(b[:, 0], expect, rtol=1e-14, atol=1e-300)


def test_rhs_samples_integrate_low_degree_data_exactly():
    # Replacing g_D by sampled values of a quadratic in space (exact for the
    # degree-4 rule) gives the closed-form integrals over each triangle.
    V, T = W.icosphere(1)
    X, Wq, area = O.triangle_quadrature(V, T)
    P = V[T]
    cen = P.mean(axis=1)
    N = 3
    samples = np.stack([(n + 1.0) * X[:, :, 0] for n in range(N + 1)])
    b = O.rhs(V, T, N, 1.0, samples=samples)
    for n in range(N + 1):
        assert np.allclose(b[n], (n + 1.0) * area * cen[:, 0], rtol=1e-13, atol=1e-15)
    # integral of x^2 over a triangle: |tau|/6 (sum of squares + sum of pairwise products)
    xs = P[:, :, 0]
    exact = area / 6.0 * (np.sum(xs ** 2, axis=1) + xs[:, 0] * xs[:, 1]
                          + xs[:, 1] * xs[:, 2] + xs[:, 0] * xs[:, 2])
    b2 = O.rhs(V, T, 1, 1.0, samples=np.stack([X[:, :, 0] ** 2, -X[:, :, 0] ** 2]))
    assert np.allclose(b2[0], exact, rtol=1e-13, atol=1e-15)
    assert np.allclose(b2[1], -exact, rtol=1e-13, atol=1e-15)


def test_error_measures_on_known_perturbations():
    rng = np.random.default_rng(11)
    F, M = 7, 30
    area = rng.uniform(0.5, 2.0, M)
    q_ref = rng.standard_normal((F, M))
    e = np.linspace(-0.3, 0.4, F)
    q = q_ref * (1.0 + e[:, None])
    assert np.allclose(O.step_errors(q, q_ref, area), np.abs(e), rtol=1e-13)
    # rel_error is the area-weighted aggregate over all steps
    w = np.sum(area[None, :] * q_ref ** 2, axis=1)
    assert math.isclose(O.rel_error(q, q_ref, area),
                        math.sqrt(np.sum(e ** 2 * w) / np.sum(w)), rel_tol=1e-13)
    assert O.rel_error(q_ref, q_ref, area) == 0.0
    # one element off by delta with q_ref = 1: sqrt(a_i F delta^2 / (F sum a))
    ones = np.ones((F, M))
    bump = ones.copy()
    bump[:, 4] += 0.1
    assert math.isclose(O.rel_error(bump, ones, area),
                        math.sqrt(area[4] * 0.01 / area.sum()), rel_tol=1e-13)


@pytest.mark.parametrize("N", [8, 9])
def test_compressed_solve_without_approximation_is_the_plain_solve(N):
    # eta = 0 admits no far block and eps = 0 runs every MACA to full frequency
    # rank, where cross approximation interpolates each pivot slice exactly:
    # the full-band solve with the compressed operator must then reproduce the
    # half-band plain solve.  rho^-N = 1e8 amplifies rounding in the inverse
    # transform, hence the bound.
    V, T = W.icosphere(1)
    _, _, area = O.triangle_quadrature(V, T)
    q = O.solve(V, T, N, 2.0)
    qc, im, op = O.solve_compressed(V, T, N, 2.0, 4, 0.0, 2, 0.0)
    assert not op["far"]
    assert O.rel_error(qc, q, area) < 1e-9
    assert im < 1e-9


def test_compressed_solve_converges_to_the_plain_solve():
    V, T = W.icosphere(1)
    _, _, area = O.triangle_quadrature(V, T)
    q = O.solve(V, T, 8, 2.0)
    errs = []
    for m, eps in ((2, 1e-3), (3, 1e-6), (4, 1e-10)):
        qc, _, op = O.solve_compressed(V, T, 8, 2.0, 4, 1.0, m, eps)
        assert op["far"]
        errs.append(O.rel_error(qc, q, area))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4


def test_gauss_legendre_five_points_match_the_closed_form_to_rounding():
    # the five-point Gauss-Legendre rule has the closed form
    #   t = 0, +-(1/3) sqrt(5 -+ 2 sqrt(10/7)),  w = 128/225, (322 +- 13 sqrt 70)/900
    # on [-1, 1]; the oracle's nodes and weights on [0, 1] must be these values
    # correctly rounded (a 1e-15 weight error becomes 1e-8 in the time domain)
    from decimal import Decimal as Dc, localcontext
    x, w = O.gauss_legendre01(5)
    with localcontext() as ctx:
        ctx.prec = 40
        s70, s107 = Dc(70).sqrt(), (Dc(10) / Dc(7)).sqrt()
        t = [-(5 + 2 * s107).sqrt() / 3, -(5 - 2 * s107).sqrt() / 3, Dc(0),
             (5 - 2 * s107).sqrt() / 3, (5 + 2 * s107).sqrt() / 3]
        wt = [(322 - 13 * s70) / 900, (322 + 13 * s70) / 900, Dc(128) / 225,
              (322 + 13 * s70) / 900, (322 - 13 * s70) / 900]
        for k in range(5):
            assert x[k] == float((t[k] + 1) / 2)
            assert abs(Dc(w[k]) - wt[k] / 2) <= Dc(2) ** -53 * (wt[k] / 2)
