"""Convenience wrapper: one problem with a torch-allocated device workspace.

Marshalling only -- every step of the computation runs in libcqm.so.
"""
from __future__ import annotations

import numpy as np

from . import cqm as C


class Problem:
    def __init__(self, ctx, vertices, tris, N, T, device="cuda", **opts):
        import torch
        self.torch = torch
        self.M = int(np.asarray(tris).shape[0])
        self.nv = int(np.asarray(vertices).shape[0])
        self.N = int(N)
        self.options = C.cqm_default_options(**opts)
        self.handle = C.cqm_problem_create(ctx, vertices, tris, N, T, self.options)
        nbytes = C.cqm_workspace_size(self.handle)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        aligned = (base + 255) & ~255
        C.cqm_set_workspace(self.handle, aligned, nbytes)
        self.workspace_bytes = nbytes
        self.device = device

    def set_plane_wave(self, direction=(1.0, 0.0, 0.0), sigma=0.25, t0=1.5, amplitude=1.0):
        C.cqm_set_plane_wave(self.handle, direction, sigma, t0, amplitude)

    def set_samples(self, samples):
        t = self.torch.as_tensor(np.ascontiguousarray(samples), dtype=self.torch.float64,
                                 device=self.device)
        self._samples = t
        C.cqm_set_dirichlet_samples(self.handle, t.data_ptr())

    def solve(self, out=None):
        torch = self.torch
        if out is None:
            out = torch.empty((self.N + 1, self.M), dtype=torch.float64, device=self.device)
        rc, diag = C.cqm_solve(self.handle, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        return out, rc, diag

    def solve_marching(self, out=None):
        """Time-marching solve (needs marching=1 at construction)."""
        torch = self.torch
        if out is None:
            out = torch.empty((self.N + 1, self.M), dtype=torch.float64, device=self.device)
        rc, diag = C.cqm_solve_marching(self.handle, out.data_ptr(),
                                        torch.cuda.current_stream().cuda_stream)
        return out, rc, diag

    def apply(self, x, l0=0, precision=64):
        """x: complex torch tensor (nl, M) on device; returns V(s_l) x_l."""
        torch = self.torch
        dt = torch.complex128 if precision == 64 else torch.complex64
        x = x.to(dt).contiguous()
        y = torch.empty_like(x)
        C.cqm_apply_V(self.handle, l0, x.shape[0], precision, x.data_ptr(), y.data_ptr(),
                      torch.cuda.current_stream().cuda_stream)
        return y

    def apply_K(self, x, l0=0, adjoint=False):
        """x: complex torch tensor (nl, M) on device; returns K(s_l) x_l, or
        K'(s_l) x_l with adjoint (FP64; needs formulation=CQM_FORMULATION_DIRECT
        at construction)."""
        torch = self.torch
        x = x.to(torch.complex128).contiguous()
        y = torch.empty_like(x)
        C.cqm_apply_K(self.handle, l0, x.shape[0], x.data_ptr(), y.data_ptr(),
                      torch.cuda.current_stream().cuda_stream, adjoint)
        return y

    def apply_D(self, x, l0=0):
        """x: complex torch tensor (nl, nv) of vertex coefficients on device;
        returns D(s_l) x_l, the hypersingular operator on the piecewise-linear
        space (FP64; needs formulation=CQM_FORMULATION_DIRECT at
        construction)."""
        torch = self.torch
        x = x.to(torch.complex128).contiguous()
        y = torch.empty_like(x)
        C.cqm_apply_D(self.handle, l0, x.shape[0], x.data_ptr(), y.data_ptr(),
                      torch.cuda.current_stream().cuda_stream)
        return y

    def close(self):
        if self.handle is not None:
            C.cqm_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(problems, stream=None):
    """Solve several Problem objects together (cqm_solve_batch).  Returns the
    list of (q, diag) and the aggregate return code."""
    import torch
    outs = [torch.empty((p.N + 1, p.M), dtype=torch.float64, device=p.device) for p in problems]
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    rc, diags = C.cqm_solve_batch([p.handle for p in problems], [o.data_ptr() for o in outs], st)
    return list(zip(outs, diags)), rc


class Server:
    """Serving loop on one GPU (cqm_server_*): submit requests as they arrive,
    poll for results.  Marshalling only."""

    def __init__(self, ctx, hbm_budget, max_active=16, cache_operators=1, large_lane=0,
                 large_bytes=0, **solver):
        self.opts = C.cqm_server_default_options(max_active=max_active,
                                                 cache_operators=cache_operators,
                                                 large_lane=large_lane, large_bytes=large_bytes,
                                                 **solver)
        self.handle = C.cqm_server_create(ctx, hbm_budget, self.opts)
        self.shapes = {}

    def submit(self, vertices, tris, N, T, direction=(1.0, 0.0, 0.0), sigma=0.25, t0=1.5,
               amplitude=1.0):
        t = C.cqm_server_submit(self.handle, vertices, tris, N, T, direction, sigma, t0, amplitude)
        self.shapes[t] = (int(N) + 1, int(np.asarray(tris).shape[0]))
        return t

    def poll(self, ticket):
        """(done, rc, q or None, diag, latency_ms)."""
        out = np.empty(self.shapes[ticket])
        done, rc, d, lat = C.cqm_server_poll(self.handle, ticket, out)
        return done, rc, (out if done == 1 else None), d, lat

    def drain(self):
        C.cqm_server_drain(self.handle)

    def stats(self):
        return C.cqm_server_stats(self.handle).as_dict()

    def close(self):
        if self.handle is not None:
            C.cqm_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
