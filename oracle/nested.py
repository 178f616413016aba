"""Inner level of the nested solver (Sec. 4.2, Alg. 7, eq. factorization).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

A layer grid (all its rows, all W columns) is split into L_c cells along x,
with the same ownership / artificial-PML rule as the layers, transposed (the
variable swap R of Sec. 4.2).  Inner interface j (j = 0..L_c-2) lies between
cells j and j+1; its unknowns are the column pair (v_a, v_b): column a is the
last owned column of cell j, column b the first owned column of cell j+1.

Inner SIE (the transposed unpolarized SIE of Sec. 2.2, M = I - Green's
integrals):
  v_a - R_{col n}[(H^j)^{-1}(T^j(v_{j-1}) + B^j(v_j))]       = R_{col n} N^j g
  v_b - R_{col 1}[(H^{j+1})^{-1}(T^{j+1}(v_j) + B^{j+1}(v_{j+1}))] = R_{col 1} N^{j+1} g
with T^c, B^c the column versions of App. C's equivalent sources.  It is
block tridiagonal (blocks of 2 H_L) and is factorised by block LU without
pivoting with explicitly inverted diagonal blocks (Sec. 4.2.2).

Interface mode (eq. factorization): for a source g living on the layer's
interface rows, the samples of (H^l)^{-1} g on those rows equal
    D_loc g + M_u (M^l)^{-1} M_f g,
where M_f maps g to the inner right-hand side (cell Newton potentials sampled
on the cell's own interface columns), M_u maps the inner traces to samples on
the interface rows (cell Green's integrals), and D_loc -- absent from the
printed equation but present in Alg. 7's reconstruction line -- is the
cell-local Newton potential sampled on the interface rows (block diagonal
over cells).  Without D_loc the identity does not hold.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .discretization import CellGrid, LayerGrid, partition


class NestedLayerSolver:
    def __init__(self, grid: LayerGrid, cells: int, build_interface_ops: bool = True,
                 dtype=np.complex128):
        self.grid = grid
        self.dt = dtype
        prob = grid.prob
        self.Lc = cells
        self.HL = grid.HL
        self.W = prob.W
        self.cparts = partition(prob.n, cells)
        self.cells = [CellGrid(grid, a, b, i, cells) for i, (a, b) in enumerate(self.cparts)]
        self.lus = [spla.splu(c.H.astype(dtype).tocsc()) for c in self.cells]
        self.J = cells - 1                                  # inner interfaces
        self._factor_inner()
        self.rows = None
        self.ops = None
        if build_interface_ops:
            self._build_interface_ops()

    # ------------------------------------------------------------ cells
    def cell_solve(self, c: int, g: np.ndarray) -> np.ndarray:
        """(H^{l,c})^{-1} g, g of shape [HL, Wc] or [B, HL, Wc]."""
        C = self.cells[c]
        shp = g.shape
        flat = np.asarray(g).astype(self.dt).reshape(-1, shp[-2] * shp[-1]).T
        return self.lus[c].solve(np.ascontiguousarray(flat)).T.reshape(shp)

    def own_cols(self, c: int):
        C = self.cells[c]
        return np.arange(C.own_lo, C.own_hi + 1)

    def to_cell(self, c: int, g: np.ndarray) -> np.ndarray:
        """g chi_{cell c}: layer array [.., HL, W] -> cell grid [.., HL, Wc]."""
        C = self.cells[c]
        out = np.zeros(g.shape[:-1] + (C.Wc,), dtype=complex)
        own = self.own_cols(c)
        out[..., own] = g[..., C.col0 + own]
        return out

    def src_T(self, c: int, pair: np.ndarray) -> np.ndarray:
        """Column equivalent sources from the left pair (v_a, v_b): col 1 gets
        -C_{1,0} v_a, col 0 gets C_{0,1} v_b (App. C, transposed)."""
        C = self.cells[c]
        shp = pair.shape[:-2]
        g = np.zeros(shp + (C.HL, C.Wc), dtype=complex)
        g[..., :, C.col(1)] += -C.coupling(1, 0) * pair[..., 0, :]
        g[..., :, C.col(0)] += C.coupling(0, 1) * pair[..., 1, :]
        return g

    def src_B(self, c: int, pair: np.ndarray) -> np.ndarray:
        C = self.cells[c]
        n = C.nc
        shp = pair.shape[:-2]
        g = np.zeros(shp + (C.HL, C.Wc), dtype=complex)
        g[..., :, C.col(n + 1)] += C.coupling(n + 1, n) * pair[..., 0, :]
        g[..., :, C.col(n)] += -C.coupling(n, n + 1) * pair[..., 1, :]
        return g

    # -------------------------------------------------------- inner SIE
    def inner_apply(self, V: np.ndarray) -> np.ndarray:
        """M^l V for V of shape [B, J, 2, HL]."""
        J = self.J
        out = V.copy()
        for c in range(self.Lc):
            C = self.cells[c]
            g = np.zeros(V.shape[:1] + (C.HL, C.Wc), dtype=complex)
            if c > 0:
                g += self.src_T(c, V[:, c - 1])
            if c < J:
                g += self.src_B(c, V[:, c])
            w = self.cell_solve(c, g)
            if c < J:
                out[:, c, 0] -= w[..., :, C.col(C.nc)]    # row a of interface c
            if c > 0:
                out[:, c - 1, 1] -= w[..., :, C.col(1)]   # row b of interface c-1
        return out

    def inner_rhs(self, newton) -> np.ndarray:
        """Inner right-hand side from the cell Newton potentials [B, HL, Wc]."""
        B = newton[0].shape[0]
        r = np.zeros((B, self.J, 2, self.HL), dtype=complex)
        for c in range(self.Lc):
            C = self.cells[c]
            if c < self.J:
                r[:, c, 0] = newton[c][..., :, C.col(C.nc)]
            if c > 0:
                r[:, c - 1, 1] = newton[c][..., :, C.col(1)]
        return r

    def _factor_inner(self):
        """Dense inner SIE and its block LU without pivoting (Sec. 4.2.2)."""
        J, HL = self.J, self.HL
        if J == 0:
            self.M = np.zeros((0, 0), dtype=complex)
            return
        n = J * 2 * HL
        eye = np.eye(n, dtype=complex).reshape(n, J, 2, HL)
        self.M = self.inner_apply(eye).reshape(n, n).T.astype(self.dt)   # column j = M e_j
        b = 2 * HL
        blk = lambda i, j: self.M[i * b:(i + 1) * b, j * b:(j + 1) * b]
        self.Sinv = []
        self.Lfac = [None]
        self.Cup = [blk(j, j + 1) for j in range(J - 1)] + [None]
        S = blk(0, 0)
        self.Sinv.append(np.linalg.inv(S))
        for j in range(1, J):
            Lj = blk(j, j - 1) @ self.Sinv[j - 1]
            S = blk(j, j) - Lj @ blk(j - 1, j)
            self.Lfac.append(Lj)
            self.Sinv.append(np.linalg.inv(S))

    def inner_solve(self, R: np.ndarray) -> np.ndarray:
        """(M^l)^{-1} R for R of shape [B, J, 2, HL]: block forward and backward
        substitution (the inner cell-level sweeps)."""
        J, HL = self.J, self.HL
        B = R.shape[0]
        y = R.reshape(B, J, 2 * HL).astype(self.dt)
        for j in range(1, J):
            y[:, j] -= y[:, j - 1] @ self.Lfac[j].T
        x = np.zeros_like(y)
        x[:, J - 1] = y[:, J - 1] @ self.Sinv[J - 1].T
        for j in range(J - 2, -1, -1):
            x[:, j] = (y[:, j] - x[:, j + 1] @ self.Cup[j].T) @ self.Sinv[j].T
        return x.reshape(B, J, 2, HL)

    def inner_traces(self, newton) -> np.ndarray:
        """Inner traces v [B, J, 2, HL] of the layer solution from the cell
        Newton potentials: the inner SIE solved by block LU (Sec. 4.2.2)."""
        return self.inner_solve(self.inner_rhs(newton))

    # ----------------------------------------------- Alg. 7 volume mode
    def solve(self, g: np.ndarray) -> np.ndarray:
        """(H^l)^{-1} g through the cells (Alg. 7), g: [HL, W] or [B, HL, W]."""
        single = g.ndim == 2
        G = g[None] if single else g
        B = G.shape[0]
        gc = [self.to_cell(c, G) for c in range(self.Lc)]
        if self.J == 0:
            w = self.cell_solve(0, gc[0])
            out = np.zeros_like(G, dtype=complex)
            own = self.own_cols(0)
            out[..., own + self.cells[0].col0] = w[..., own]
            return out[0] if single else out
        newton = [self.cell_solve(c, gc[c]) for c in range(self.Lc)]
        v = self.inner_traces(newton)
        out = np.zeros((B, self.HL, self.W), dtype=complex)
        for c in range(self.Lc):
            C = self.cells[c]
            src = gc[c].copy()
            if c > 0:
                src += self.src_T(c, v[:, c - 1])
            if c < self.J:
                src += self.src_B(c, v[:, c])
            w = self.cell_solve(c, src)
            own = self.own_cols(c)
            out[..., C.col0 + own] = w[..., own]
        return out[0] if single else out

    # ---------------------------------------- interface mode (design B)
    def _interface_rows(self):
        G = self.grid
        rows = []
        if G.index > 0:
            rows += [G.row(0), G.row(1)]
        if G.index < G.count - 1:
            rows += [G.row(G.nl), G.row(G.nl + 1)]
        return rows

    def _build_interface_ops(self):
        """Per cell: M_f (inner RHS from interface-row sources), D_loc (cell
        Newton potential on the interface rows) and M_u (inner traces to the
        interface rows), each by solving with unit sources."""
        rows = self._interface_rows()
        self.rows = rows
        r = len(rows)
        if r == 0:
            return
        HL, J = self.HL, self.J
        self.ops = []
        for c in range(self.Lc):
            C = self.cells[c]
            own = self.own_cols(c)
            s = own.size
            # unit sources on (row, own col): [r*s, HL, Wc]
            E = np.zeros((r * s, HL, C.Wc), dtype=complex)
            for i, row in enumerate(rows):
                E[i * s + np.arange(s), row, own] = 1.0
            N = self.cell_solve(c, E)
            D_loc = np.stack([N[:, row, own] for row in rows], axis=1).reshape(r * s, r * s).T
            Mf_left = N[:, :, C.col(1)].T if c > 0 else None         # -> row b of iface c-1
            Mf_right = N[:, :, C.col(C.nc)].T if c < J else None     # -> row a of iface c
            # inner unit traces of the left / right pair: [2HL, 2, HL]
            eye = np.eye(2 * HL, dtype=complex).reshape(2 * HL, 2, HL)
            Mu_left = Mu_right = None
            if c > 0:
                w = self.cell_solve(c, self.src_T(c, eye))
                Mu_left = np.stack([w[:, row, own] for row in rows], axis=1).reshape(2 * HL, r * s).T
            if c < J:
                w = self.cell_solve(c, self.src_B(c, eye))
                Mu_right = np.stack([w[:, row, own] for row in rows], axis=1).reshape(2 * HL, r * s).T
            cast = lambda a: None if a is None else a.astype(self.dt)
            self.ops.append(dict(D_loc=cast(D_loc), Mf_left=cast(Mf_left),
                                 Mf_right=cast(Mf_right), Mu_left=cast(Mu_left),
                                 Mu_right=cast(Mu_right), own=own))

    def interface_op(self, g_rows: np.ndarray, rows) -> np.ndarray:
        """Samples of (H^l)^{-1} g on the interface rows for g supported there:
        D_loc g + M_u (M^l)^{-1} M_f g (eq. factorization, with D_loc)."""
        assert list(rows) == self.rows
        r = len(rows)
        J = self.J
        out = np.zeros((r, self.W), dtype=complex)
        xs = []
        for c in range(self.Lc):
            C = self.cells[c]
            op = self.ops[c]
            xs.append(g_rows[:, C.col0 + op["own"]].reshape(-1).astype(self.dt))
        R = np.zeros((1, J, 2, self.HL), dtype=self.dt)
        for c in range(self.Lc):
            op = self.ops[c]
            if op["Mf_right"] is not None:
                R[0, c, 0] = op["Mf_right"] @ xs[c]
            if op["Mf_left"] is not None:
                R[0, c - 1, 1] = op["Mf_left"] @ xs[c]
        v = self.inner_solve(R) if J > 0 else R
        for c in range(self.Lc):
            C = self.cells[c]
            op = self.ops[c]
            y = op["D_loc"] @ xs[c]
            if op["Mu_left"] is not None:
                y = y + op["Mu_left"] @ v[0, c - 1].reshape(-1)
            if op["Mu_right"] is not None:
                y = y + op["Mu_right"] @ v[0, c].reshape(-1)
            out[:, C.col0 + op["own"]] = y.reshape(r, -1)
        return out
