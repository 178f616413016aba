"""Preconditioned Bi-CGstab, the alternative Krylov driver of the paper's
iteration-count comparison (Table 3: GMRES and Bi-CGstab, each with the
Gauss-Seidel and the Jacobi preconditioner).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper names the method (van der Vorst's Bi-CGSTAB) without fixing its
variant; this oracle takes the right-preconditioned form with x0 = 0 and the
shadow residual equal to the initial residual: every iteration applies the
preconditioner and the matrix twice, and the residual it carries is the
unpreconditioned one, ||b - A x|| / ||b|| (checked at the half step s and at
the full step r).  Pinned in tests against dense solves.
"""
from __future__ import annotations

import numpy as np


def bicgstab(apply_A, b: np.ndarray, apply_P=None, tol: float = 1e-10, maxit: int = 200):
    """Solve A x = b with the right preconditioner P.  Returns (x, info):
    info["iters"] counts iterations (a convergence at the half step counts
    as its iteration), info["history"] the relative residual after each one,
    info["converged"] whether tol was met, info["breakdown"] a breakdown."""
    P = apply_P if apply_P is not None else (lambda v: v)
    shape = b.shape
    bf = np.asarray(b, dtype=complex).ravel()
    nb = np.linalg.norm(bf)
    x = np.zeros_like(bf)
    info = {"iters": 0, "history": [1.0], "converged": nb == 0.0, "breakdown": False}
    if nb == 0.0:
        return x.reshape(shape), info
    A = lambda v: np.asarray(apply_A(v.reshape(shape)), dtype=complex).ravel()
    K = lambda v: np.asarray(P(v.reshape(shape)), dtype=complex).ravel()
    r = bf.copy()
    rhat = r.copy()
    rho_prev = alpha = omega = 1.0 + 0j
    v = np.zeros_like(bf)
    p = np.zeros_like(bf)
    for it in range(1, maxit + 1):
        rho = np.vdot(rhat, r)
        if rho == 0:
            info["breakdown"] = True
            break
        beta = (rho / rho_prev) * (alpha / omega)
        p = r + beta * (p - omega * v)
        y = K(p)
        v = A(y)
        den = np.vdot(rhat, v)
        if den == 0:
            info["breakdown"] = True
            break
        alpha = rho / den
        s = r - alpha * v
        rel_s = np.linalg.norm(s) / nb
        if rel_s <= tol:                       # converged at the half step
            x = x + alpha * y
            info["iters"] = it
            info["history"].append(rel_s)
            info["converged"] = True
            return x.reshape(shape), info
        z = K(s)
        t = A(z)
        tt = np.vdot(t, t)
        if tt == 0:
            info["breakdown"] = True
            break
        omega = np.vdot(t, s) / tt
        x = x + alpha * y + omega * z
        r = s - omega * t
        rel = np.linalg.norm(r) / nb
        info["iters"] = it
        info["history"].append(rel)
        if rel <= tol:
            info["converged"] = True
            break
        if omega == 0:
            info["breakdown"] = True
            break
        rho_prev = rho
    return x.reshape(shape), info
