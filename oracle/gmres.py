"""Left-preconditioned GMRES (the Krylov driver of Alg. 6).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Alg. 6 solves (P M) x = P f with x0 = 0.  The paper does not fix restart,
orthogonalisation or the residual used in the stopping test; this oracle takes
no restart, modified Gram-Schmidt with one full re-orthogonalisation pass,
complex Givens rotations, and stops once the preconditioned residual satisfies
||P(f - M x)|| <= tol ||P f||.  The iteration path is therefore the textbook
GMRES one (Saad & Schultz); it is pinned in tests against a dense solve.
"""
from __future__ import annotations

import numpy as np


def _givens(a: complex, b: complex):
    """(c, s) with [c, s; -conj(s), c] [a; b] = [r; 0], c real >= 0."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    t = np.hypot(abs(a), abs(b))
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s


def gmres(apply_A, b: np.ndarray, apply_P=None, tol: float = 1e-10, maxit: int = 200):
    """Solve A x = b, left-preconditioned by P.  Returns (x, info) where info
    holds the iteration count, the preconditioned residual history (relative)
    and whether ``tol`` was met."""
    P = apply_P if apply_P is not None else (lambda v: v)
    r0 = P(b)
    beta = np.linalg.norm(r0)
    n = b.size
    x = np.zeros_like(b, dtype=complex)
    info = {"iters": 0, "history": [1.0], "converged": beta == 0.0}
    if beta == 0.0:
        return x, info
    V = np.zeros((maxit + 1, n), dtype=complex)
    Hs = np.zeros((maxit + 1, maxit), dtype=complex)
    cs = np.zeros(maxit)
    sn = np.zeros(maxit, dtype=complex)
    g = np.zeros(maxit + 1, dtype=complex)
    g[0] = beta
    V[0] = r0.ravel() / beta
    k = 0
    for j in range(maxit):
        w = P(apply_A(V[j].reshape(b.shape))).ravel().astype(complex)
        for _ in range(2):                     # MGS + one re-orthogonalisation
            for i in range(j + 1):
                hij = np.vdot(V[i], w)
                Hs[i, j] += hij
                w = w - hij * V[i]
        Hs[j + 1, j] = np.linalg.norm(w)
        if Hs[j + 1, j] != 0:
            V[j + 1] = w / Hs[j + 1, j]
        for i in range(j):                     # previous rotations
            a, bb = Hs[i, j], Hs[i + 1, j]
            Hs[i, j] = cs[i] * a + sn[i] * bb
            Hs[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * bb
        cs[j], sn[j] = _givens(Hs[j, j], Hs[j + 1, j])
        a, bb = Hs[j, j], Hs[j + 1, j]
        Hs[j, j] = cs[j] * a + sn[j] * bb
        Hs[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        rel = abs(g[j + 1]) / beta
        info["history"].append(rel)
        if rel <= tol:
            info["converged"] = True
            break
    y = np.zeros(k, dtype=complex)
    for i in range(k - 1, -1, -1):             # back substitution
        y[i] = (g[i] - Hs[i, i + 1:k] @ y[i + 1:k]) / Hs[i, i]
    x = (V[:k].T @ y).reshape(b.shape)
    info["iters"] = k
    return x, info
