"""The hypersingular operator D(s) on the piecewise-linear space (cqm_apply_D)
against the oracle (oracle/hypersingular.py): products with D(s_l) entry for
entry on small meshes (all quadrature classes, several frequency tiles, a
ragged tail of vertices), sampled rows at 5120 triangles, and properties that
hold at any size (the Galerkin form's symmetry, the sphere's eigenvalues)."""
import sys

import numpy as np
import pytest
import scipy.special as sp

import cqm_workloads as W
import oracle as O
import oracle.hypersingular as H

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2006_05186_amd import cqm as C  # noqa: E402
from paper_2006_05186_amd.solver import Problem  # noqa: E402

DIRECT = C.CQM_FORMULATION_DIRECT


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = C.cqm_ctx_create(0)
    yield c
    C.cqm_ctx_destroy(c)


def _check_rows(V, T, s, x, y, rows=None, pairs=None):
    ref = H.assemble_D(V, T, s, rows=rows, pairs=pairs) @ x
    got = y if rows is None else y[rows]
    return np.linalg.norm(got - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("full", [False, True])
def test_apply_D_matches_oracle(ctx, full):
    """A 320-triangle ellipsoid (162 vertices), N = 16: every frequency the
    problem solves, in the plain and the compressed mode's band."""
    V, T = W.ellipsoid(2, (1.3, 0.8, 1.0))
    N, Tend = 16, 2.0
    kw = {"mode": C.CQM_MIXED_H2ACA} if full else {}
    p = Problem(ctx, V, T, N, Tend, formulation=DIRECT, **kw)
    s, _, _ = O.frequencies(N, Tend)
    nl = len(s) if full else N // 2 + 1
    x = W.random_complex((nl, len(V)), seed=31)
    say(f"apply_D M={len(T)} nv={len(V)} frequencies {nl}")
    y = p.apply_D(torch.as_tensor(x, device="cuda")).cpu().numpy()
    ls = (0, 1, nl // 2, nl - 1)
    pairs = O.near_pairs(T)
    worst = max(_check_rows(V, T, s[l], x[l], y[l], pairs=pairs) for l in ls)
    say(f"  worst relative error {worst:.1e}")
    assert worst < 1e-12
    # a frequency sub-range addresses the same matrices; one frequency alone
    y2 = p.apply_D(torch.as_tensor(x[3:6], device="cuda"), l0=3).cpu().numpy()
    assert np.abs(y2 - y[3:6]).max() <= 1e-14 * np.abs(y).max()
    y3 = p.apply_D(torch.as_tensor(x[nl - 1:], device="cuda"), l0=nl - 1).cpu().numpy()
    assert np.abs(y3 - y[nl - 1:]).max() <= 1e-14 * np.abs(y).max()
    p.close()


def test_apply_D_two_components(ctx):
    """Two spheres (640 triangles, 324 vertices): far pairs across the gap."""
    V, T = W.two_spheres(2, distance=3.0)
    N, Tend = 8, 2.0
    p = Problem(ctx, V, T, N, Tend, formulation=DIRECT)
    s, _, _ = O.frequencies(N, Tend)
    nl = N // 2 + 1
    x = W.random_complex((nl, len(V)), seed=32)
    y = p.apply_D(torch.as_tensor(x, device="cuda")).cpu().numpy()
    worst = max(_check_rows(V, T, s[l], x[l], y[l]) for l in (0, nl - 1))
    say(f"apply_D two spheres M={len(T)}: worst relative error {worst:.1e}")
    assert worst < 1e-12
    p.close()


def test_apply_D_sampled_rows_full_size(ctx):
    """5120 triangles (2562 vertices), N = 128, T = 6 (the headline mesh and
    time grid), every frequency of the band in one call: sampled vertex rows
    against the oracle, the symmetry y2.(D y1) = y1.(D y2) of the Galerkin
    form (bilinear; near pairs are integrated from either side, so equal to
    quadrature accuracy, which improves with q_duffy)."""
    V, T = W.icosphere(4)
    N, Tend = 128, 6.0
    p = Problem(ctx, V, T, N, Tend, formulation=DIRECT)
    s, _, _ = O.frequencies(N, Tend)
    nl = N // 2 + 1
    x1 = W.random_complex((nl, len(V)), seed=33)
    x2 = W.random_complex((nl, len(V)), seed=34)
    say(f"apply_D M={len(T)} nv={len(V)} frequencies {nl}")
    y1 = p.apply_D(torch.as_tensor(x1, device="cuda")).cpu().numpy()
    y2 = p.apply_D(torch.as_tensor(x2, device="cuda")).cpu().numpy()
    rows = np.array([0, 1, 700, 1500, 2561])
    tri = set(np.nonzero(np.isin(T, rows).any(axis=1))[0].tolist())
    pairs = [q for q in O.near_pairs(T) if q[0] in tri]
    worst = max(_check_rows(V, T, s[l], x1[l], y1[l], rows=rows, pairs=pairs) for l in (0, 40, nl - 1))
    say(f"  sampled rows: worst relative error {worst:.1e}")
    assert worst < 1e-12

    def asym(y1, y2):
        return max(abs(np.dot(x2[l], y1[l]) - np.dot(x1[l], y2[l])) / abs(np.dot(x2[l], y1[l]))
                   for l in range(nl))

    sym5 = asym(y1, y2)
    p.close()
    # the asymmetry is the near rules' quadrature error (a pair and its mirror
    # go through different transformations), magnified by s^2 at the largest
    # |s_l| (about 85 here): it falls with more Gauss points per axis
    p = Problem(ctx, V, T, N, Tend, formulation=DIRECT, q_duffy=8)
    z1 = p.apply_D(torch.as_tensor(x1, device="cuda")).cpu().numpy()
    z2 = p.apply_D(torch.as_tensor(x2, device="cuda")).cpu().numpy()
    sym8 = asym(z1, z2)
    say(f"  symmetry: worst {sym5:.1e} (q = 5), {sym8:.1e} (q = 8)")
    assert sym5 < 1e-5 and sym8 < 0.1 * sym5
    p.close()


def test_apply_D_sphere_eigenvalue(ctx):
    """The degree-1 harmonic z on a 1280-triangle icosphere: the GPU product's
    Rayleigh quotient against the closed form -s^3 i_1'(s) k_1'(s) (unit
    radius), within the second-order discretisation error."""
    V, T = W.icosphere(3)
    N, Tend = 8, 2.0
    p = Problem(ctx, V, T, N, Tend, formulation=DIRECT)
    s, _, _ = O.frequencies(N, Tend)
    nl = N // 2 + 1
    z = np.tile(V[:, 2].astype(np.complex128), (nl, 1))
    y = p.apply_D(torch.as_tensor(z, device="cuda")).cpu().numpy()
    Mm = H.mass_P1(V, T)
    worst = 0.0
    for l in range(nl):
        kd = (2.0 / np.pi) * sp.spherical_kn(1, s[l], derivative=True)
        lam = -s[l] ** 3 * sp.spherical_in(1, s[l], derivative=True) * kd
        rq = np.dot(z[l], y[l]) / np.dot(z[l].real, Mm @ z[l].real)
        worst = max(worst, abs(rq / lam - 1))
    say(f"apply_D sphere eigenvalue n=1: worst relative error {worst:.1e}")
    assert worst < 5e-3
    p.close()


def test_apply_D_needs_direct_formulation(ctx):
    V, T = W.icosphere(1)
    p = Problem(ctx, V, T, 4, 1.0)
    x = torch.zeros((1, len(V)), dtype=torch.complex128, device="cuda")
    with pytest.raises(C.CqmError):
        p.apply_D(x)
    p.close()
