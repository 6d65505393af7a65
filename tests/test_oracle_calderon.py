"""Pins of the double-layer oracle (oracle/calderon.py) by facts the paper and
the mathematics fix: the solid angle of a flat triangle (an independent
closed form for the static part), the double-layer eigenvalue of the sphere,
Gauss's integral, the exterior Calderon identity of Section 2.2 on a
non-spherical surface, and the direct solve's manufactured solution."""

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

import cqm_workloads as W
import oracle as O
import oracle.calderon as K
from static_reference import double_layer_reference


def _unit(v):
    return v / np.linalg.norm(v)


def test_static_rules_against_solid_angle():
    """Folded edge pair and vertex pair: the Duffy rules against the outer
    integral of the triangle's solid angle (no Duffy map involved)."""
    A, B, C = np.array([0., 0, 0]), np.array([1., 0, 0]), np.array([0.4, 0.9, 0.0])
    D = np.array([0.5, 0.0, 0.8])
    nj = _unit(np.cross(B - A, D - A))
    ref = double_layer_reference((A, B, C), (A, B, D))
    assert abs(K.static_K_edge(A, B, C, D, nj, 12) - ref) < 1e-10 * abs(ref)
    assert abs(K.static_K_edge(A, B, C, D, nj, 5) - ref) < 1e-4 * abs(ref)
    B1, B2 = np.array([-0.8, 0.1, 0.2]), np.array([-0.3, -0.9, 0.1])
    nj = _unit(np.cross(B1 - A, B2 - A))
    ref = double_layer_reference((A, B, C), (A, B1, B2))
    assert abs(K.static_K_vertex(A, B, C, B1, B2, nj, 12) - ref) < 1e-10 * abs(ref)
    assert abs(K.static_K_vertex(A, B, C, B1, B2, nj, 5) - ref) < 1e-5 * abs(ref)


def test_static_part_of_mesh_pairs_against_solid_angle():
    """Every class of near pair of a coarse ellipsoid, through near_static_K
    (pair classification, source normal, orientation): identical pairs are
    zero, the others match the solid-angle reference."""
    V, T = W.ellipsoid(1, (1.3, 0.8, 1.0))
    pairs = O.near_pairs(T)
    S = K.near_static_K(V, T, pairs, 12)
    ident, edge, vert = O.classify_pairs(T, pairs)
    assert np.all(S[ident[:, 0]] == 0.0)
    for k in (edge[0, 0], edge[7, 0], vert[0, 0], vert[11, 0]):
        i, j, _ = pairs[k]
        ref = double_layer_reference(tuple(V[T[i]]), tuple(V[T[j]]))
        assert abs(S[k] - ref) < 1e-9 * abs(ref) + 1e-15, (k, S[k], ref)


def test_remainder_against_extended_precision():
    mpmath.mp.dps = 40
    for z in (1e-6 + 2e-6j, 3e-3 - 1e-3j, 0.2 + 0.3j, 0.49j, 0.7 - 0.1j, 4.0 + 9.0j):
        zz = mpmath.mpc(z.real, z.imag)
        ref = complex(mpmath.exp(-zz) * (1 + zz) - 1)
        got = complex(K.remainder_K(np.asarray(z)))
        assert abs(got - ref) <= 1e-15 * abs(ref), z


def _kappa(s):
    """Double-layer eigenvalue of constants on the unit sphere:
    K(s)1 = s^2/2 (i0'(s) k0(s) + i0(s) k0'(s)), i0 = sinh z/z, k0 = e^-z/z
    (the kernel's expansion in modified spherical Bessel functions; the
    boundary value is the mean of the two one-sided limits)."""
    i0 = np.sinh(s) / s
    di0 = np.cosh(s) / s - np.sinh(s) / s ** 2
    k0 = np.exp(-s) / s
    dk0 = -np.exp(-s) / s - np.exp(-s) / s ** 2
    return 0.5 * s * s * (di0 * k0 + i0 * dk0)


def test_kappa_limits():
    # Laplace limit: Gauss's integral, -1/2 on the surface
    assert abs(_kappa(1e-4) + 0.5) < 1e-4


@pytest.mark.parametrize("s", [1.0, 2.0 + 3.0j])
def test_sphere_row_sums_converge_to_closed_form(s):
    exact = _kappa(s)
    errs = []
    for level in (1, 2, 3):
        V, T = W.icosphere(level)
        _, _, area = O.triangle_quadrature(V, T)
        A = K.assemble_K(V, T, s)
        errs.append(np.sqrt(np.sum(area * np.abs(A.sum(1) / area - exact) ** 2) / np.sum(area))
                    / abs(exact))
    assert errs[2] < 0.01
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 2.5


def test_gauss_integral_row_sums():
    """At s = 0 (Laplace) every row sums to -|tau_i|/2 on a closed surface;
    what is left is the quadrature error of the far pairs."""
    V, T = W.ellipsoid(2, (1.3, 0.8, 1.0))
    _, _, area = O.triangle_quadrature(V, T)
    A = K.assemble_K(V, T, 0.0)
    assert np.max(np.abs(A.imag)) == 0.0
    dev = np.abs(A.real.sum(1) / area + 0.5)
    assert dev.max() < 5e-3


def test_conjugate_symmetry():
    V, T = W.icosphere(1)
    s = 1.5 + 2.5j
    assert np.allclose(K.assemble_K(V, T, np.conj(s)), np.conj(K.assemble_K(V, T, s)),
                       rtol=0, atol=1e-15)


def _point_source(X, n, x0, s):
    """u = exp(-s r)/(4 pi r), r = |x - x0|, and its normal derivative."""
    d = X - x0
    r = np.linalg.norm(d, axis=-1)
    u = np.exp(-s * r) / (4 * np.pi * r)
    du = -(1 + s * r) * np.exp(-s * r) / (4 * np.pi * r ** 3) * np.einsum("...k,...k->...", d, n)
    return u, du


def test_exterior_calderon_identity():
    """An exterior solution of the Laplace-domain wave equation (a point
    source inside an ellipsoid): its Cauchy data satisfy V q = (-1/2 + K) g
    (the first row of eq. wavebie for the exterior problem, the direct
    formulation of Section 2.2); the Galerkin residual falls with h."""
    s = 0.8 + 2.0j
    x0 = np.array([0.15, -0.1, 0.2])
    res = []
    for level in (1, 2, 3):
        V, T = W.ellipsoid(level, (1.3, 0.8, 1.0))
        X, Wt, area = O.triangle_quadrature(V, T)
        n = K.normals(V, T)
        u, du = _point_source(X, n[:, None, :], x0, s)
        g = (Wt * u).sum(1) / area  # L2 projections onto piecewise constants
        q = (Wt * du).sum(1) / area
        lhs = O.assemble_V(V, T, s) @ q
        Ks = K.assemble_K(V, T, s)
        rhs = -0.5 * area * g + Ks @ g
        res.append(np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs))
    assert res[2] < 0.02
    assert res[0] / res[1] > 1.7 and res[1] / res[2] > 1.7
    # the adjoint's normal (n_x instead of n_y) breaks the identity
    wrong = -0.5 * area * g + Ks.T @ g
    assert np.linalg.norm(lhs - wrong) / np.linalg.norm(wrong) > 5 * res[2]


def test_direct_solve_recovers_the_point_source_flux():
    """One frequency of the direct solve: with g the trace of a point source
    inside the ellipsoid, V q = (-1/2 I + K) g returns its normal derivative."""
    s = 1.0 + 1.5j
    x0 = np.array([0.1, 0.05, -0.1])
    errs = []
    for level in (2, 3):
        V, T = W.ellipsoid(level, (1.3, 0.8, 1.0))
        X, Wt, area = O.triangle_quadrature(V, T)
        n = K.normals(V, T)
        u, du = _point_source(X, n[:, None, :], x0, s)
        g, qex = (Wt * u).sum(1) / area, (Wt * du).sum(1) / area
        q = sla.solve(O.assemble_V(V, T, s), -0.5 * area * g + K.assemble_K(V, T, s) @ g)
        errs.append(np.sqrt(np.sum(area * np.abs(q - qex) ** 2) / np.sum(area * np.abs(qex) ** 2)))
    assert errs[1] < 0.05 and errs[0] / errs[1] > 1.7


def _profile(t, ts=0.3):
    z = t - ts
    return np.where(z > -0.2, np.cos(5 * z + 1) - 1, 0.0)


def test_direct_solve_radial_data_gives_sphere_transfer_function():
    """Uniform Dirichlet data gamma(t) on the unit sphere: the Neumann datum is
    constant with Laplace transform gamma_hat (-1/2 + kappa(s)) 2s/(1 - e^-2s);
    the mesh solution's area mean approaches this scalar CQM solution."""
    N, Tend = 16, 4.0
    s, rho, dt = O.frequencies(N, Tend)
    F = N + 1
    gam = _profile(np.arange(F) * dt)
    ghat = O.forward_dft(gam[:, None], rho, F)
    H = (-0.5 + _kappa(s)) * 2 * s / (1 - np.exp(-2 * s))
    scalar, _ = O.inverse_dft(ghat * H[:, None], rho, F, conjugate_fill=False)
    errs = []
    for level in (1, 2):
        V, Tr = W.icosphere(level)
        _, _, area = O.triangle_quadrature(V, Tr)
        samples = np.broadcast_to(gam[:, None, None], (F, len(Tr), 6)).copy()
        q = K.solve_direct(V, Tr, N, Tend, samples=samples)
        mean = (q * area).sum(1) / area.sum()
        errs.append(np.linalg.norm(mean - scalar[:, 0]) / np.linalg.norm(scalar))
    assert errs[1] < 0.03 and errs[0] / errs[1] > 2.5


def test_adjoint_static_rules_against_solid_angle():
    """K'[tau, t] is K[t, tau]: the adjoint rules (target normal) against the
    solid-angle reference with the roles of the triangles exchanged."""
    A, B, C = np.array([0., 0, 0]), np.array([1., 0, 0]), np.array([0.4, 0.9, 0.0])
    D = np.array([0.5, 0.0, 0.8])
    ni = _unit(np.cross(B - A, C - A))
    ref = double_layer_reference((A, B, D), (A, B, C))
    assert abs(K.static_Kp_edge(A, B, C, D, ni, 12) - ref) < 1e-10 * abs(ref)
    B1, B2 = np.array([-0.8, 0.1, 0.2]), np.array([-0.3, -0.9, 0.1])
    ref = double_layer_reference((A, B1, B2), (A, B, C))
    assert abs(K.static_Kp_vertex(A, B, C, B1, B2, ni, 12) - ref) < 1e-10 * abs(ref)


@pytest.mark.parametrize("s", [0.0, 1.0 + 2.0j])
def test_adjoint_is_the_transpose(s):
    """For piecewise constants on both sides the Galerkin matrix of K' (normal
    derivative at the target) is the transpose of K's; the two are coded
    separately (other normal, other sign, other Duffy rules)."""
    V, T = W.ellipsoid(1, (1.3, 0.8, 1.0))
    A, B = K.assemble_K(V, T, s), K.assemble_Kp(V, T, s)
    assert np.linalg.norm(B - A.T) <= 1e-13 * np.linalg.norm(A)


def test_neumann_trace_of_the_single_layer_potential():
    """Exterior jump relation (eq. wavebio): the single-layer potential of the
    indirect density phi (V phi = g) has the Neumann trace (-1/2 + K') phi,
    which the direct formulation computes as q from the same g; the two
    Galerkin answers approach each other as h falls."""
    s = 1.0 + 1.5j
    x0 = np.array([0.1, 0.05, -0.1])
    errs = []
    for level in (1, 2, 3):
        V, T = W.ellipsoid(level, (1.3, 0.8, 1.0))
        X, Wt, area = O.triangle_quadrature(V, T)
        u, _ = _point_source(X, K.normals(V, T)[:, None, :], x0, s)
        g = (Wt * u).sum(1) / area
        A = O.assemble_V(V, T, s)
        phi = sla.solve(A, area * g)
        q = sla.solve(A, -0.5 * area * g + K.assemble_K(V, T, s) @ g)
        lhs = -0.5 * area * phi + K.assemble_Kp(V, T, s) @ phi
        errs.append(np.linalg.norm(lhs - area * q) / np.linalg.norm(area * q))
    assert errs[2] < 0.05 and errs[0] / errs[1] > 1.5 and errs[1] / errs[2] > 1.5
