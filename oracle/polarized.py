"""Layered decomposition, SIE and polarized traces (Sec. 2.2, 3, 4.1; App. C).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Notation.  Layer l (0-based here) owns a block of physical rows.  Interface k
(k = 0..L-2) lies between layer k and layer k+1; its two trace rows are
``a`` (last row of layer k, local row n of layer k, local row 0 of layer k+1)
and ``b`` (first row of layer k+1: local row n+1 of layer k, local row 1 of
layer k+1).  A "pair" is the array [2, W] = (trace on row a, trace on row b).

Green's integrals (App. C, eq. pde_GRF_real): with C_{j,k} the diagonal
coupling block of H^l from row k to row j, the equivalent sources of a top
pair (x_a, x_b) and of a bottom pair (y_a, y_b) are
    T_l(x_a, x_b) = -E_1 C_{1,0} x_a + E_0 C_{0,1} x_b,
    B_l(y_a, y_b) =  E_{n+1} C_{n+1,n} y_a - E_n C_{n,n+1} y_b,
and G_down^l = (H^l)^{-1} T_l, G_up^l = (H^l)^{-1} B_l, N^l f = (H^l)^{-1} f^l.
The paper's sweeps (Algs. 3-4) print the opposite signs; the oracle follows
App. C everywhere (the sweeps are pinned against dense triangular solves).

Polarized system (eqs. jump_1..jump_4), unknowns d_k (down-going) and q_k
(up-going) pairs on interface k, with s = d + q:
  down rows (layer k):   d_k + E_a q_k - R_bot^k[G_down^k(s_{k-1}) + G_up^k(q_k)]
                         = R_bot^k N^k f
  up rows (layer k+1):   q_k + E_b d_k - R_top^{k+1}[G_up^{k+1}(s_{k+1}) + G_down^{k+1}(d_k)]
                         = R_top^{k+1} N^{k+1} f
where R_bot samples rows (n, n+1), R_top rows (0, 1), E_a keeps the a row of a
pair and E_b the b row; terms with a missing neighbour are absent.  Ordering
the unknowns (d_0..d_{L-2}, q_0..q_{L-2}) gives M = [[D_down, U], [L, D_up]]
(eq. M_polarized) with D_down unit block lower bidiagonal and D_up unit block
upper bidiagonal.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .discretization import LayerGrid, Problem, partition
from .bicgstab import bicgstab
from .gmres import gmres


class DirectLayerSolver:
    """(H^l)^{-1} by a sparse LU of the whole layer (the matrix-free approach
    of Sec. 4.1 with a direct local solver)."""

    def __init__(self, grid: LayerGrid, dtype=np.complex128):
        self.grid = grid
        self.dt = dtype
        self.lu = spla.splu(grid.H.astype(dtype).tocsc())

    def solve(self, g: np.ndarray) -> np.ndarray:
        """g: [HL, W] or [B, HL, W] on the layer grid."""
        shp = g.shape
        flat = np.asarray(g).astype(self.dt).reshape(-1, shp[-2] * shp[-1]).T
        return self.lu.solve(np.ascontiguousarray(flat)).T.reshape(shp).astype(complex)

    def interface_op(self, g_rows: np.ndarray, rows) -> np.ndarray:
        """(H^l)^{-1} g sampled on ``rows`` for g supported on ``rows``."""
        G = self.grid
        g = np.zeros((G.HL, G.prob.W), dtype=complex)
        g[rows, :] = g_rows
        return self.solve(g)[rows, :]


class LayeredSolver:
    """Alg. 6 (matrix-free polarized traces with the Gauss-Seidel
    preconditioner) on top of a pluggable layer solver."""

    def __init__(self, prob: Problem, layers: int, cells: int | None = None,
                 dtype=np.complex128, inner: str = "lu", inner_tol: float = 1e-6,
                 pre_plr_eps: float | None = None, pre_plr_tile: int = 64):
        """``dtype`` = complex64 gives the single-precision local solver used
        as the approximate inverse of the mixed-precision form.  ``inner``
        selects the inner solver of a nested layer: "lu" (block LU, Sec.
        4.2.2) or "pt" (nested polarized traces, Sec. 4.2.1, GMRES to
        ``inner_tol``).  ``pre_plr_eps``: the preconditioner's Green's
        integrals use the interface operators compressed in partitioned
        low-rank form at that accuracy (oracle.plr), the SIE matrix the exact
        ones (nested block-LU layers only)."""
        self.prob = prob
        self.L = layers
        self.parts = partition(prob.n, layers)
        self.grids = [LayerGrid(prob, a, b, i, layers) for i, (a, b) in enumerate(self.parts)]
        if cells is None:
            self.solvers = [DirectLayerSolver(g, dtype) for g in self.grids]
        elif inner == "pt":
            from .nested_pt import PolarizedInnerSolver
            self.solvers = [PolarizedInnerSolver(g, cells, inner_tol=inner_tol, dtype=dtype)
                            for g in self.grids]
        else:
            from .nested import NestedLayerSolver
            self.solvers = [NestedLayerSolver(g, cells, dtype=dtype) for g in self.grids]
        self.pre_solvers = None
        if pre_plr_eps is not None:
            from .plr import PLRLayerView
            assert cells is not None and inner == "lu"
            self.pre_solvers = [PLRLayerView(s, pre_plr_eps, pre_plr_tile) for s in self.solvers]
        self.W = prob.W

    # ------------------------------------------------------------------ rows
    def rows_top(self, l):
        g = self.grids[l]
        return [g.row(0), g.row(1)]

    def rows_bot(self, l):
        g = self.grids[l]
        return [g.row(g.nl), g.row(g.nl + 1)]

    def interface_rows(self, l):
        """Rows of layer l that carry equivalent sources / samples."""
        rows = []
        if l > 0:
            rows += self.rows_top(l)
        if l < self.L - 1:
            rows += self.rows_bot(l)
        return rows

    # ----------------------------------------------------- App. C sources
    def src_T(self, l: int, pair: np.ndarray) -> np.ndarray:
        """T_l(x_a, x_b) on the layer grid."""
        G = self.grids[l]
        g = np.zeros((G.HL, self.W), dtype=complex)
        g[G.row(1)] += -G.coupling(1, 0) * pair[0]
        g[G.row(0)] += G.coupling(0, 1) * pair[1]
        return g

    def src_B(self, l: int, pair: np.ndarray) -> np.ndarray:
        """B_l(y_a, y_b) on the layer grid."""
        G = self.grids[l]
        n = G.nl
        g = np.zeros((G.HL, self.W), dtype=complex)
        g[G.row(n + 1)] += G.coupling(n + 1, n) * pair[0]
        g[G.row(n)] += -G.coupling(n, n + 1) * pair[1]
        return g

    def restrict_source(self, l: int, f_ext: np.ndarray) -> np.ndarray:
        """f^l = f chi_l placed on the layer grid (Alg. 6, partition the source)."""
        G = self.grids[l]
        g = np.zeros((G.HL, self.W), dtype=complex)
        rows = np.arange(G.own_lo, G.own_hi + 1)
        g[rows] = f_ext[G.global_row(rows)]
        return g

    # --------------------------------------------------- layer operator
    def layer_op(self, l: int, top, bot, side: str, pre: bool = False) -> np.ndarray:
        """R_side (H^l)^{-1}[T_l(top) + B_l(bot)], side in {'top', 'bot'};
        ``top``/``bot`` may be None (absent).  ``pre``: inside the
        preconditioner (compressed operators when the solver has them)."""
        G = self.grids[l]
        g = np.zeros((G.HL, self.W), dtype=complex)
        if top is not None:
            g += self.src_T(l, top)
        if bot is not None:
            g += self.src_B(l, bot)
        rows = self.interface_rows(l)
        solver = self.pre_solvers[l] if (pre and self.pre_solvers) else self.solvers[l]
        w_rows = solver.interface_op(g[rows], rows)
        want = self.rows_top(l) if side == "top" else self.rows_bot(l)
        return np.stack([w_rows[rows.index(r)] for r in want])

    def newton_samples(self, l: int, f_ext: np.ndarray):
        """(R_top N^l f, R_bot N^l f) -- RHS of the polarized system (Alg. 6)."""
        w = self.solvers[l].solve(self.restrict_source(l, f_ext))
        top = w[self.rows_top(l)] if l > 0 else None
        bot = w[self.rows_bot(l)] if l < self.L - 1 else None
        return top, bot

    # ------------------------------------------------- polarized system
    def rhs(self, f_ext: np.ndarray):
        K = self.L - 1
        fd = np.zeros((K, 2, self.W), dtype=complex)
        fq = np.zeros((K, 2, self.W), dtype=complex)
        for l in range(self.L):
            top, bot = self.newton_samples(l, f_ext)
            if bot is not None:
                fd[l] = bot                 # down rows of interface l come from layer l
            if top is not None:
                fq[l - 1] = top             # up rows of interface l-1 come from layer l
        return fd, fq

    def apply_M(self, d: np.ndarray, q: np.ndarray):
        """Matrix-free application of the polarized SIE matrix (Alg. 2
        generalised, eq. integral_polarized)."""
        K = self.L - 1
        s = d + q
        od = np.zeros_like(d)
        oq = np.zeros_like(q)
        for k in range(K):
            y_bot = self.layer_op(k, s[k - 1] if k > 0 else None, q[k], "bot")
            od[k] = d[k] - y_bot
            od[k, 0] += q[k, 0]                         # E_a q_k
            y_top = self.layer_op(k + 1, d[k], s[k + 1] if k + 1 < K else None, "top")
            oq[k] = q[k] - y_top
            oq[k, 1] += d[k, 1]                         # E_b d_k
        return od, oq

    def sweep_down(self, v: np.ndarray) -> np.ndarray:
        """(D_down)^{-1} v (Alg. 3, signs of App. C)."""
        x = np.zeros_like(v)
        for k in range(self.L - 1):
            x[k] = v[k]
            if k > 0:
                x[k] = x[k] + self.layer_op(k, x[k - 1], None, "bot", pre=True)
        return x

    def sweep_up(self, v: np.ndarray) -> np.ndarray:
        """(D_up)^{-1} v (Alg. 4, signs of App. C)."""
        K = self.L - 1
        x = np.zeros_like(v)
        for k in range(K - 1, -1, -1):
            x[k] = v[k]
            if k < K - 1:
                x[k] = x[k] + self.layer_op(k + 1, None, x[k + 1], "top", pre=True)
        return x

    def apply_Lrefl(self, d: np.ndarray) -> np.ndarray:
        """The block L of M (Alg. 5, up-going reflections): d-part of the up
        rows, E_b d_k - R_top^{k+1}[G_down^{k+1}(d_k) + G_up^{k+1}(d_{k+1})]."""
        K = self.L - 1
        out = np.zeros_like(d)
        for k in range(K):
            out[k] = -self.layer_op(k + 1, d[k], d[k + 1] if k + 1 < K else None, "top", pre=True)
            out[k, 1] += d[k, 1]
        return out

    def precond_gs(self, vd: np.ndarray, vq: np.ndarray):
        """P^GS (eq. preconditioner_GS): inverse of [[D_down, 0], [L, D_up]]."""
        xd = self.sweep_down(vd)
        xq = self.sweep_up(vq - self.apply_Lrefl(xd))
        return xd, xq

    def precond_jacobi(self, vd: np.ndarray, vq: np.ndarray):
        """P^Jac (eq. preconditioner_Jac)."""
        return self.sweep_down(vd), self.sweep_up(vq)

    # -------------------------------------------------------- packing
    def pack(self, d, q):
        return np.concatenate([d.ravel(), q.ravel()])

    def unpack(self, v):
        K = self.L - 1
        half = K * 2 * self.W
        return v[:half].reshape(K, 2, self.W), v[half:].reshape(K, 2, self.W)

    # ------------------------------------------------------ full solve
    def reconstruct(self, f_ext: np.ndarray, s: np.ndarray) -> np.ndarray:
        """Alg. 6, reconstruction: u^l = (H^l)^{-1}[f^l + T_l(s_{l-1}) + B_l(s_l)]
        kept on the owned rows, concatenated."""
        u = np.zeros((self.W, self.W), dtype=complex)
        for l, G in enumerate(self.grids):
            g = self.restrict_source(l, f_ext)
            if l > 0:
                g += self.src_T(l, s[l - 1])
            if l < self.L - 1:
                g += self.src_B(l, s[l])
            w = self.solvers[l].solve(g)
            rows = np.arange(G.own_lo, G.own_hi + 1)
            u[G.global_row(rows)] = w[rows]
        return u

    def solve(self, f_ext: np.ndarray, tol: float = 1e-10, maxit: int = 200,
              precond: str = "gs", krylov: str = "gmres"):
        """Alg. 6 for one right-hand side on the extended grid; the polarized
        system is solved by left-preconditioned GMRES or right-preconditioned
        Bi-CGstab with P^GS or P^Jac (the combinations of Table 3)."""
        if self.L == 1:
            return self.solvers[0].solve(self.restrict_source(0, f_ext)), {"iters": 0}
        fd, fq = self.rhs(f_ext)
        P = self.precond_gs if precond == "gs" else self.precond_jacobi
        A = lambda v: self.pack(*self.apply_M(*self.unpack(v)))
        Pv = lambda v: self.pack(*P(*self.unpack(v)))
        if krylov == "bicgstab":
            x, info = bicgstab(A, self.pack(fd, fq), Pv, tol=tol, maxit=maxit)
        else:
            x, info = gmres(A, self.pack(fd, fq), Pv, tol=tol, maxit=maxit)
        d, q = self.unpack(x)
        s = d + q
        info["traces"] = s
        return self.reconstruct(f_ext, s), info

    # ------------------------------------------- unpolarized SIE (check)
    def apply_M_unpol(self, s: np.ndarray) -> np.ndarray:
        """SIE of Sec. 2.2 (Alg. 1): row a of interface k from layer k, row b
        from layer k+1; M = I - (Green's integrals)."""
        K = self.L - 1
        out = s.copy()
        for k in range(K):
            wa = self.layer_op(k, s[k - 1] if k > 0 else None, s[k], "bot")
            wb = self.layer_op(k + 1, s[k], s[k + 1] if k + 1 < K else None, "top")
            out[k, 0] -= wa[0]
            out[k, 1] -= wb[1]
        return out

    def rhs_unpol(self, f_ext: np.ndarray) -> np.ndarray:
        fd, fq = self.rhs(f_ext)
        out = np.zeros_like(fd)
        out[:, 0] = fd[:, 0]
        out[:, 1] = fq[:, 1]
        return out

    def dense(self, fn, K2):
        """Dense matrix of a linear map on stacked vectors (tiny grids only)."""
        n = K2
        cols = []
        for j in range(n):
            e = np.zeros(n, dtype=complex)
            e[j] = 1.0
            cols.append(fn(e))
        return np.stack(cols, axis=1)
