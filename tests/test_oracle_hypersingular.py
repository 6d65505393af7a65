"""Pins of the hypersingular oracle (oracle/hypersingular.py) by facts that do
not come from the oracle itself: the Sauter-Schwab transformations against the
single layer's independent Duffy rules (unit weights) and against a closed-form
inner potential with linear weights; the sphere's hypersingular eigenvalues
(spherical Bessel functions), which the assembled P1 Galerkin matrix must
approach at second order; the symmetry of the Galerkin form; constants in the
kernel of the Laplace limit."""

import numpy as np
import pytest
import scipy.special as sp

import cqm_workloads as W
import oracle.cqm as C
import oracle.hypersingular as H
from static_reference import weighted_static_reference

A, B, CC = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.4, 0.9, 0.0])
D = np.array([0.5, 0.0, 0.8])
B1, B2 = np.array([-0.8, 0.1, 0.2]), np.array([-0.3, -0.9, 0.1])


def test_unit_weights_reduce_to_single_layer_rules():
    """Summed over both weights the transformations give the piecewise-constant
    static integrals, which the single layer computes by other rules."""
    cases = (("identical", (A, B, CC), (A, B, CC), C.static_identical(A, B, CC, 14)),
             ("edge", (A, B, CC), (A, B, D), C.static_edge(A, B, CC, D, 14)),
             ("vertex", (A, B, CC), (A, B1, B2), C.static_vertex(A, B, CC, B1, B2, 14)))
    for kind, Ti, Tj, ref in cases:
        v = H.ss_static_weighted(kind, [Ti], [Tj], 10)[0]
        assert abs(v.sum() / ref - 1) < 1e-9, kind


@pytest.mark.parametrize("kind,Tj", [("edge", (A, B, D)), ("vertex", (A, B1, B2))])
def test_weighted_static_against_closed_form(kind, Tj):
    """All nine weights of a folded edge pair and of a vertex pair against the
    closed-form weighted potential (no transformation involved)."""
    Ti = (A, B, CC)
    v = H.ss_static_weighted(kind, [Ti], [Tj], 10)[0]
    ref = np.array([[weighted_static_reference(Ti, Tj, a, b, 1e-10) for b in range(3)]
                    for a in range(3)])
    assert np.abs(v - ref).max() < 1e-9 * np.abs(ref).max()


def test_weighted_static_identical_against_closed_form():
    Ti = (A, B, CC)
    v = H.ss_static_weighted("identical", [Ti], [Ti], 10)[0]
    for a, b in ((0, 0), (1, 2)):
        ref = weighted_static_reference(Ti, Ti, a, b, 1e-7)
        assert abs(v[a, b] / ref - 1) < 1e-6
    assert np.abs(v - v.T).max() < 1e-14 * np.abs(v).max()


def test_mesh_pairs_use_local_vertex_order():
    """near_static_weighted maps each class to the triangles' own vertex order:
    on a mesh the weighted values of (i, j) and (j, i) are transposes (the
    classes evaluate the mirrored pair by different transformations), and an
    edge pair and a vertex pair of the mesh match the closed form."""
    V, T = W.ellipsoid(1, (1.0, 0.8, 0.6))
    pairs = C.near_pairs(T)
    w = H.near_static_weighted(V, T, pairs, 8)
    index = {(i, j): k for k, (i, j, _) in enumerate(pairs)}
    worst = 0.0
    for k, (i, j, _) in enumerate(pairs):
        worst = max(worst, np.abs(w[k] - w[index[(j, i)]].T).max() / np.abs(w[k]).max())
    assert worst < 1e-6  # quadrature error at q = 8; a wrong vertex map is O(1)
    # one edge pair and one vertex pair fully against the closed form
    for want in (2, 1):
        k = next(k for k, (i, j, ns) in enumerate(pairs) if ns == want)
        i, j, _ = pairs[k]
        ref = np.array([[weighted_static_reference(V[T[i]], V[T[j]], a, b, 1e-9) for b in range(3)]
                        for a in range(3)])
        assert np.abs(w[k] - ref).max() < 1e-7 * np.abs(ref).max()


def _sphere_eigenvalue(n, s, R=1.0):
    """Hypersingular eigenvalue of degree n on the sphere of radius R for the
    kernel exp(-s r)/(4 pi r): -s^3 R^2 i_n'(sR) k_n'(sR), with the modified
    spherical Bessel functions normalised so that k_0(z) = exp(-z)/z."""
    kd = (2.0 / np.pi) * sp.spherical_kn(n, s * R, derivative=True)
    return -s ** 3 * R ** 2 * sp.spherical_in(n, s * R, derivative=True) * kd


def test_sphere_eigenvalues_second_order():
    """Rayleigh quotients of the P1 interpolants of spherical harmonics of
    degrees 0, 1, 2 (constants, z, xy) on icospheres: the error against the
    exact eigenvalue falls by about four per refinement (flat triangles and
    linear elements are both second order)."""
    s = 1.0 + 1.5j
    errs = []
    for lev in (2, 3):
        V, T = W.icosphere(lev)
        Dm = H.assemble_D(V, T, s)
        Mm = H.mass_P1(V, T)
        x, y, z = V.T
        e = []
        for n, f in ((0, np.ones(len(V))), (1, z), (2, x * y)):
            e.append(abs((f @ Dm @ f) / (f @ Mm @ f) / _sphere_eigenvalue(n, s) - 1))
        errs.append(np.array(e))
        # complex-symmetric Galerkin form, up to the near rules' quadrature
        assert np.abs(Dm - Dm.T).max() < 1e-8 * np.abs(Dm).max()
    assert (errs[0] < 1.5e-2).all() and (errs[1] < 4e-3).all(), errs
    assert (errs[0] / errs[1] > 3.0).all(), errs


def test_laplace_limit_annihilates_constants():
    """At s -> 0 only the curl term remains, and curls of a constant vanish."""
    V, T = W.icosphere(1)
    Dm = H.assemble_D(V, T, 1e-9)
    assert np.abs(Dm @ np.ones(len(V))).max() < 1e-12 * np.abs(Dm).max()
    Ds = H.assemble_D(V, T, 0.8)
    assert np.abs(Ds @ np.ones(len(V))).max() > 1e-3 * np.abs(Ds).max()


def test_sampled_rows_match_full_matrix():
    V, T = W.icosphere(2)
    full = H.assemble_D(V, T, 0.7 + 0.3j)
    rows = np.array([0, 5, 40, 161])
    part = H.assemble_D(V, T, 0.7 + 0.3j, rows=rows)
    assert np.abs(part - full[rows]).max() < 1e-13 * np.abs(full).max()
