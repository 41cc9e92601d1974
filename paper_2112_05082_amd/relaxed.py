"""Differentiable objective of a relaxed codebook (argument marshalling only).

Forward: blended excitation U_k(w) (r3m_relaxed_rhs), relaxed solve
Z_k(w) I = U_k(w) (r3m_gmres_solve with relaxed weights), objective J = mean
bistatic RCS of the blended current over a direction set
(r3m_relaxed_objective).  Backward: adjoint solve with the transposed
operator Z_k(w)^T (transposed retrieval and Z^T) on P(w)^T dJ/dI~, then
r3m_relaxed_gradient.  Every step runs in the library; this module orders the
calls and holds the device buffers.
"""
from __future__ import annotations

import numpy as np
import torch

from . import r3m


class RelaxedRcs:
    """J(w) for a batch of relaxed codebooks sharing one complex128 spectral store.

    weights: float64 device tensor [total units][n_states] (e.g. a softmax of
    logits taken in torch); inc: [B][3] incidences (theta, phi, e0); dirs:
    [n_dir][2] observation directions.  The solves run GMRES on complex128
    spectra to `tol`, right-preconditioned by the inverses of the blended self
    blocks (precond=r3m.PRECOND_BLOCK_JACOBI; their transposes for the adjoint)
    or by the block ILU(0) of the blended near field (precond=
    r3m.PRECOND_BLOCK_ILU with ilu_radius <= the store's near radius; that of
    the transposed operator for the adjoint).
    """

    def __init__(self, ctx, geom, store, batch, inc, dirs, tol=1e-10, restart=60, max_iter=20000, e0=1.0,
                 precond=r3m.PRECOND_BLOCK_JACOBI, ilu_radius=1):
        self.ctx, self.geom, self.store, self.batch = ctx, geom, store, batch
        self.inc = np.asarray(inc, dtype=np.float64).reshape(-1, 3)
        self.dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 2)
        self.tol, self.restart, self.max_iter, self.e0, self.precond = tol, restart, max_iter, e0, precond
        self.ilu_radius = ilu_radius
        dev = batch.states.device
        n_a = store.n // store.n_states
        self.N = batch.total_units * n_a
        self.M = batch.total_units * store.n
        self.work = torch.empty(r3m.gmres_work_bytes(ctx, store, batch, restart, relaxed=True, precond=precond,
                                                     ilu_radius=ilu_radius), dtype=torch.uint8, device=dev)
        self.gwork = torch.empty(r3m.relaxed_gradient_work_bytes(ctx, store, batch), dtype=torch.uint8, device=dev)
        self.last_reports = None

    def _solve(self, w, b, transpose):
        x = torch.zeros_like(b)
        _, rep = r3m.r3m_gmres_solve(self.ctx, self.store, None, self.batch, b, x, self.tol, self.restart,
                                     self.max_iter, self.work, relaxed_weights=w, transpose=transpose,
                                     precond=self.precond, ilu_radius=self.ilu_radius)
        self.last_reports = rep
        return x

    def forward_parts(self, w):
        """J [B], sigma [B][n_dir], I, G, adjoint right-hand side."""
        w = w.detach().contiguous()
        dev = w.device
        b = torch.zeros(self.N, dtype=torch.complex128, device=dev)
        r3m.r3m_relaxed_rhs(self.ctx, self.geom, self.batch, w, self.inc, b)
        I = self._solve(w, b, False)
        B, nd = self.batch.B, len(self.dirs)
        J = torch.zeros(B, dtype=torch.float64, device=dev)
        sigma = torch.zeros(B * nd, dtype=torch.float64, device=dev)
        G = torch.zeros(self.M, dtype=torch.complex128, device=dev)
        adj = torch.zeros(self.N, dtype=torch.complex128, device=dev)
        r3m.r3m_relaxed_objective(self.ctx, self.geom, self.batch, w, I, self.dirs, self.e0, J, sigma, G, adj)
        return J, sigma.view(B, nd), I, G, adj

    def gradient(self, w, I, G, adj, dJ=None):
        w = w.detach().contiguous()
        lam = self._solve(w, adj, True)
        U = torch.zeros(self.M, dtype=torch.complex128, device=w.device)
        r3m.r3m_relaxed_rhs(self.ctx, self.geom, self.batch, w, self.inc, U, macro=True)
        grad = torch.zeros_like(w)
        r3m.r3m_relaxed_gradient(self.ctx, self.store, self.batch, w, I, lam, G, U,
                                 None if dJ is None else dJ.contiguous(), grad, self.gwork)
        return grad

    def __call__(self, w):
        return _RelaxedRcsFn.apply(w, self)


class _RelaxedRcsFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, w, obj):
        J, _, I, G, adj = obj.forward_parts(w)
        fctx.obj = obj
        fctx.save_for_backward(w, I, G, adj)
        return J

    @staticmethod
    def backward(fctx, dJ):
        w, I, G, adj = fctx.saved_tensors
        return fctx.obj.gradient(w, I, G, adj, dJ.to(torch.float64)), None
