"""The two added forms: mixed-precision refinement and the adjoint gradient.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Mixed precision.  The paper suggests applying the preconditioner with lower
accuracy than the SIE matrix (Sec. 5, footnote on compressed operators).  The
oracle's form: an approximate inverse Hhat^{-1} = the nested solver built on
complex64 local factors and operators (GMRES vectors and orthogonalisation in
complex128), wrapped in FP64 iterative refinement on the volume,
    u_{j+1} = u_j + Hhat^{-1}(f - H u_j),
until the relative update falls below a target.  Parity unpinned for the
intermediate iterates (they depend on rounding); pinned by the error of the
refined result against the FP64 direct solve.

Adjoint-state gradient.  With u_s = H(m)^{-1} f_s, r_s = P u_s - d_s and
J = 1/2 sum_s ||r_s||^2, differentiating the symmetric-form operator (its
m-dependence is the diagonal term -omega^2 m_ext / (alpha_x alpha_z), and m_ext
copies each edge value of m into the PML) gives
    dJ/dm_k = omega^2 Re sum_s sum_{e -> k} w_e mu_s[e] u_s[e],
    mu_s = H^{-T} P^T conj(r_s) = H^{-1} P^T conj(r_s)   (H = H^T),
    w_e = 1 / (alpha_x alpha_z)(e),
where e runs over the extended-grid nodes whose m is copied from physical
node k.  Pinned by central finite differences and the dot-product test.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .discretization import Problem
from .polarized import LayeredSolver


def refine_mixed(prob: Problem, layers: int, cells: int | None, f_ext: np.ndarray,
                 inner_tol: float = 1e-6, target: float = 1e-10, max_steps: int = 20):
    """FP64 iterative refinement around a complex64 nested solver.
    Returns (u_ext, history of relative updates)."""
    approx = LayeredSolver(prob, layers, cells, dtype=np.complex64)
    u = np.zeros_like(f_ext, dtype=complex)
    hist = []
    for _ in range(max_steps):
        r = f_ext - prob.apply(u)
        du, _ = approx.solve(r, tol=inner_tol)
        u = u + du
        rel = np.linalg.norm(du) / max(np.linalg.norm(u), 1e-300)
        hist.append(rel)
        if rel <= target:
            break
    return u, hist


def weight_ext(prob: Problem) -> np.ndarray:
    """w = 1/(alpha_x alpha_z) on the extended grid."""
    return 1.0 / (prob.az_n[:, None] * prob.ax_n[None, :])


def fold_to_physical(prob: Problem, g_ext: np.ndarray) -> np.ndarray:
    """Adjoint of the clamp extension m -> m_ext: sum every extended node onto
    the physical node it copies."""
    n, p = prob.n, prob.p
    zq = np.clip(np.arange(-p + 1, n + p + 1), 1, n) - 1
    out = np.zeros((n, n))
    np.add.at(out, (zq[:, None], zq[None, :]), g_ext)
    return out


class Misfit:
    """J(m) = 1/2 sum_s ||P u_s(m) - d_s||^2 with direct (splu) solves."""

    def __init__(self, omega: float, n_pml: int, f_phys: np.ndarray, rec_row: int,
                 d_obs: np.ndarray | None = None, beta: float = 2.0):
        self.omega, self.p, self.beta = omega, n_pml, beta
        self.f_phys = f_phys                      # [S, n, n]
        self.rec_row = rec_row                    # receivers: every node of this row
        self.d_obs = d_obs

    def forward(self, m: np.ndarray):
        prob = Problem(1.0 / np.sqrt(m), self.omega, self.p, self.beta)
        lu = spla.splu(prob.H.tocsc())
        F = prob.extend(self.f_phys).reshape(len(self.f_phys), -1).T
        U = lu.solve(np.ascontiguousarray(F)).T.reshape(-1, prob.W, prob.W)
        return prob, lu, U

    def record(self, prob: Problem, U: np.ndarray) -> np.ndarray:
        """P u: samples on the receiver row, physical columns."""
        return prob.restrict(U)[:, self.rec_row - 1, :]

    def value(self, m: np.ndarray) -> float:
        prob, lu, U = self.forward(m)
        r = self.record(prob, U) - self.d_obs
        return 0.5 * float(np.sum(np.abs(r) ** 2))

    def value_and_grad(self, m: np.ndarray):
        prob, lu, U = self.forward(m)
        r = self.record(prob, U) - self.d_obs
        J = 0.5 * float(np.sum(np.abs(r) ** 2))
        S = U.shape[0]
        adj_src = np.zeros((S, prob.n, prob.n), dtype=complex)
        adj_src[:, self.rec_row - 1, :] = np.conj(r)          # P^T conj(r)
        A = prob.extend(adj_src).reshape(S, -1).T
        MU = lu.solve(np.ascontiguousarray(A)).T.reshape(S, prob.W, prob.W)
        g_ext = prob.omega ** 2 * np.real(weight_ext(prob)[None] * MU * U).sum(axis=0)
        return J, fold_to_physical(prob, g_ext)
