"""Oracle of the time-marching solve: the CQM integration weights and the
step-by-step solution of the convolution system.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For the Dirichlet problem in the indirect single-layer form the Galerkin
system of Section 3.2 (eq. cqmgalapx with only the V block, right-hand side
eq. cqmrhs with only its single-layer history term) reads

    sum_{k=0}^{n} What_{n-k} q_k = b_n,    n = 0..N,

with the integration weights of eq. dft, taken over the F = N + 1 contour
points of the all-at-once form (the readings of cqm.py: F points, BDF2,
zeta = exp(2 pi i / F)):

    What_n = rho^-n / F  sum_{l=0}^{F-1} V(s_l) zeta^(n l mod F),   n = 0..N.

The weights are real (V(conj s) = conj V(s) and s_{F-l} = conj s_l), and
What_0 is real symmetric positive definite (it is V at the real frequency
delta(0)/dt = 3/(2 dt) up to the aliasing terms of order rho^F), so one
factorisation serves every step: What_0 q_n = b_n - sum_{k<n} What_{n-k} q_k,
solved progressively in time (Section 3.2, after eq. cqmrhs).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .cqm import (assemble_V, frequencies, near_pairs, near_static, num_frequencies_half, rhs,
                  twiddles)

__all__ = ["cqm_weights", "march", "solve_marching", "compressed_weights", "solve_marching_compressed"]


def cqm_weights(V, T, N, Tend, rho=None, q=5):
    """Integration weights What_n, n = 0..N, of eq. dft (F = N + 1 points).

    Assembles V(s_l) for the distinct frequencies l = 0..F/2 and takes the
    others as V(s_{F-l}) = conj V(s_l).  Returns (W real (N+1, M, M), the
    ratio ||Im W|| / ||Re W|| before the real part is taken, rho).
    """
    s, rho, dt = frequencies(N, Tend, rho)
    F = N + 1
    H = num_frequencies_half(F)
    pairs = near_pairs(T)
    static = near_static(V, T, pairs, q)
    half = [assemble_V(V, T, s[l], q, pairs, static) for l in range(H)]
    full = half + [np.conj(half[F - l]) for l in range(H, F)]
    tw = twiddles(F, +1)
    W = np.empty((F,) + half[0].shape, dtype=np.complex128)
    for n in range(F):
        acc = np.zeros_like(half[0])
        for l in range(F):
            acc += full[l] * tw[(n * l) % F]
        W[n] = acc * (rho ** (-n)) / F
    ratio = np.linalg.norm(W.imag) / max(np.linalg.norm(W.real), 1e-300)
    return W.real.copy(), ratio, rho


def march(W, b):
    """Solve sum_{k<=n} W[n-k] q_k = b_n for n = 0..len(b)-1 step by step:
    one LU factorisation of W[0], then per step the history sum and a
    forward/backward substitution."""
    lu = sla.lu_factor(W[0])
    q = np.zeros((len(b),) + np.shape(b[0]))
    for n in range(len(b)):
        r = np.array(b[n], dtype=np.float64, copy=True)
        for k in range(n):
            r -= W[n - k] @ q[k]
        q[n] = sla.lu_solve(lu, r)
    return q


def solve_marching(V, T, N, Tend, rho=None, q=5, direction=(1.0, 0.0, 0.0), sigma=0.25, t0=1.5,
                   amplitude=1.0, samples=None, return_weights=False):
    """Time-marching CQM solve of V * phi = g_D (the same discrete system as
    cqm.solve up to the aliasing of the weights, of order rho^F)."""
    W, ratio, rho = cqm_weights(V, T, N, Tend, rho, q)
    b = rhs(V, T, N, Tend, direction, sigma, t0, amplitude, samples)
    qn = march(W, b)
    if return_weights:
        return qn, W, ratio
    return qn


def compressed_weights(op, rho, M):
    """Integration weights of the compressed tensor (Section 6.2, eq. fastdft):
    the slices C_t of every block are frequency-independent, so the scaled
    DFT of eq. dft acts on the fibres alone,
        dhat_t[n] = rho^-n / F sum_l d_t[l] zeta^(n l mod F),
    and What_n = sum_blocks sum_t dhat_t[n] C_t (far blocks expanded with
    their cluster bases).  Returns (W real (F, M, M), ||Im W|| / ||Re W||)."""
    from .compress import compressed_dense
    F = op["F"]
    tw = twiddles(F, +1)
    scale = np.array([rho ** (-n) / F for n in range(F)])
    blocks = []
    for b in op["blocks"]:
        bb = dict(b)
        if b["C"]:
            D = np.asarray(b["d"])  # (rank, F)
            Dh = np.zeros_like(D)
            for n in range(F):
                acc = np.zeros(D.shape[0], dtype=np.complex128)
                for l in range(F):
                    acc += D[:, l] * tw[(n * l) % F]
                Dh[:, n] = acc * scale[n]
            bb["d"] = list(Dh)
        blocks.append(bb)
    Wc = compressed_dense(dict(op, blocks=blocks), M)  # (M, M, F)
    W = np.moveaxis(Wc, 2, 0)
    ratio = np.linalg.norm(W.imag) / max(np.linalg.norm(W.real), 1e-300)
    return W.real.copy(), ratio


def solve_marching_compressed(V, T, N, Tend, n_min, eta, m, eps, rho=None,
                              direction=(1.0, 0.0, 0.0), sigma=0.25, t0=1.5, amplitude=1.0,
                              return_weights=False):
    """Time-marching solve with the weights of the compressed tensor (the
    H2 x MACA operator of Algorithm 3 over all F = N + 1 frequencies)."""
    from .compress import build_compressed
    s, rho, dt = frequencies(N, Tend, rho)
    op = build_compressed(V, T, s, n_min, eta, m, eps)
    W, ratio = compressed_weights(op, rho, len(T))
    b = rhs(V, T, N, Tend, direction, sigma, t0, amplitude)
    qn = march(W, b)
    if return_weights:
        return qn, W, ratio
    return qn
