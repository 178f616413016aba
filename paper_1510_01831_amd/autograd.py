"""torch.autograd.Function for the least-squares misfit of the Helmholtz
solution with respect to the squared slowness m (argument marshalling only;
forward solves, misfit, adjoint solves and the gradient run in libhz.so).

    J(m) = 1/2 sum_s || P u_s(m) - d_s ||^2,   H(m) u_s = f_s,

P samples every physical node of one depth row (the receivers).  The
backward pass reuses the forward factors: H is complex symmetric, so the
adjoint solve H^H lam = P^T r is conj(H^{-1} conj(P^T r)), and the gradient
kernel folds the PML copies of m onto the edge nodes they replicate.
"""
from __future__ import annotations

import torch

from . import hz


class HelmholtzMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, m, f, d_obs, rec_row: int, omega: float, n_pml: int, layers: int,
                cells: int, tol: float = 1e-13, max_iter: int = 200):
        B = f.shape[0]
        solver = hz.Solver(m.detach().to(torch.float64), omega, n_pml, layers, cells,
                           model_kind=hz.HZ_MODEL_SLOWNESS2, max_batch=B)
        u = solver.solve(f, tol=tol, max_iter=max_iter, ext=True)
        J, adj = solver.misfit(u, d_obs, rec_row)
        if ctx.needs_input_grad[0]:
            # the factors serve the adjoint solve; the context lives as long as
            # the graph node (a second backward with retain_graph=True reuses it)
            ctx.solver = solver
            ctx.tol, ctx.max_iter = tol, max_iter
            ctx.save_for_backward(u, adj)
        else:
            solver.close()                 # forward only: free the device memory now
            ctx.solver = None
        return torch.tensor(J, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(ctx, gJ):
        u, adj = ctx.saved_tensors
        lam = ctx.solver.adjoint(adj, tol=ctx.tol, max_iter=ctx.max_iter, ext=True)
        g = ctx.solver.misfit_gradient(u, lam)
        return (gJ * g.to(gJ.device), None, None, None, None, None, None, None, None, None)


def misfit(m, f, d_obs, rec_row, omega, n_pml, layers, cells, tol=1e-13, max_iter=200):
    """J(m) with autograd support (gradient through the adjoint-state method)."""
    return HelmholtzMisfit.apply(m, f, d_obs, rec_row, omega, n_pml, layers, cells, tol,
                                 max_iter)
