"""The definition u = H^{-1} f by a sparse direct solve, for grids where the
default column ordering of SuperLU runs out of time or memory.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The method reaches the discrete solution of the PML-truncated system of
App. A exactly (up to its Krylov tolerance); the reference for it is that
solution.  For the large grids (W^2 of several million unknowns) the sparse
LU is taken on the symmetrically permuted matrix P H P^T, with P a geometric
nested-dissection order of the grid (separator rows / columns last,
recursively), pivots on the diagonal (H is complex symmetric, and the
permutation keeps that), and the solve is followed by classical iterative
refinement with the residual of the assembled H in complex128:
    x_{k+1} = x_k + (LU)^{-1} (f - H x_k),
stopped when the relative residual no longer falls or reaches ``rtol``.
Only library primitives (SuperLU, sparse products) and the assembled H are
used; the ordering changes how the LU is computed, not what it computes.

Pins (tests/test_oracle_direct.py): the order is a permutation and its
separators split the grid; on small grids the solution equals SuperLU with
its default ordering and the DST-I closed form.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


def nested_dissection(nz: int, nx: int, leaf: int = 32) -> np.ndarray:
    """Nested-dissection order of the nz x nx grid (row-major node index
    z * nx + x): the longer side is cut by a middle separator line, both
    halves are ordered recursively, the separator follows them; blocks with
    at most ``leaf``^2 / 4 nodes (or a side of at most 2) keep row-major
    order.  Returns the permutation as an index array (new -> old)."""
    out = []

    def rec(z0, z1, x0, x1):                    # half-open ranges
        hz, hx = z1 - z0, x1 - x0
        if hz <= 0 or hx <= 0:
            return
        if hz * hx <= leaf * leaf // 4 or min(hz, hx) <= 2:
            zz, xx = np.meshgrid(np.arange(z0, z1), np.arange(x0, x1), indexing="ij")
            out.append((zz * nx + xx).ravel())
            return
        if hz >= hx:
            m = (z0 + z1) // 2
            rec(z0, m, x0, x1)
            rec(m + 1, z1, x0, x1)
            out.append(m * nx + np.arange(x0, x1))
        else:
            m = (x0 + x1) // 2
            rec(z0, z1, x0, m)
            rec(z0, z1, m + 1, x1)
            out.append(np.arange(z0, z1) * nx + m)

    rec(0, nz, 0, nx)
    return np.concatenate(out).astype(np.int64)


class DirectSolver:
    """u = H^{-1} f for the global operator of a Problem (App. A) by a
    nested-dissection sparse LU with iterative refinement."""

    def __init__(self, prob, leaf: int = 32):
        self.prob = prob
        W = prob.W
        H = prob.H.tocsc()
        self.H = prob.H.tocsr()
        self.perm = nested_dissection(W, W, leaf)
        self.iperm = np.empty_like(self.perm)
        self.iperm[self.perm] = np.arange(self.perm.size)
        Hp = H[self.perm][:, self.perm].tocsc()
        self.lu = spla.splu(Hp, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))

    def _lu_solve(self, R: np.ndarray) -> np.ndarray:
        return self.lu.solve(np.ascontiguousarray(R[self.perm]))[self.iperm]

    def solve(self, F: np.ndarray, rtol: float = 1e-15, max_refine: int = 8):
        """F: [N] or [N, B] right-hand sides on the extended grid (flattened
        row by row).  Returns (U, relative residuals per column)."""
        single = F.ndim == 1
        F2 = F[:, None] if single else F
        nf = np.linalg.norm(F2, axis=0)
        nf[nf == 0] = 1.0
        X = self._lu_solve(F2)
        R = F2 - self.H @ X
        res = np.linalg.norm(R, axis=0) / nf
        for _ in range(max_refine):
            if np.all(res <= rtol):
                break
            Xn = X + self._lu_solve(R)
            Rn = F2 - self.H @ Xn
            rn = np.linalg.norm(Rn, axis=0) / nf
            better = rn < res
            if not np.any(better):
                break
            X[:, better] = Xn[:, better]
            R[:, better] = Rn[:, better]
            res = np.where(better, rn, res)
        return (X[:, 0] if single else X), res
