"""Nested polarized traces: the inner SIE of a layer solved by polarized
traces (Sec. 4.2.1; the inner tolerance of the experiments in Fig. 9).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The block LU of ``nested`` solves the inner SIE of layer l directly.  The
nested variant instead applies the method of polarized traces a second time,
inside the layer: the cells play the role the layers play at the outer level
(the variable swap of Sec. 4.2), and the inner system is iterated by GMRES
preconditioned with the Gauss-Seidel sweeps over the cells.  No inner block
is factorised or inverted; every block is a cell Green's integral.

Notation (transposed outer system).  Inner interface j lies between cells j
and j+1 with the column pair (a, b): a is the last owned column of cell j
(cell-local position n_c), b the first owned column of cell j+1 (position 1
there, n_c + 1 in cell j).  For cell c, with T^c and B^c the column versions
of App. C's equivalent sources of its left and right pairs,
    G_T^c = (H^c)^{-1} T^c,   G_B^c = (H^c)^{-1} B^c,
    R_right samples cell c on positions (n_c, n_c + 1),
    R_left  samples cell c on positions (0, 1).
Unknowns: the rightward pair d_j and the leftward pair q_j, with s = d + q
the inner traces (v_a, v_b).  The rows of the system are
    right rows (cell j):   d_j + E_a q_j - R_right^j[G_T^j(s_{j-1}) + G_B^j(q_j)]
                           = R_right^j N^j g
    left rows (cell j+1):  q_j + E_b d_j - R_left^{j+1}[G_B^{j+1}(s_{j+1}) + G_T^{j+1}(d_j)]
                           = R_left^{j+1} N^{j+1} g
(E_a keeps the a column of a pair, E_b the b column), i.e. the outer
polarized system (jump conditions, eq. M_polarized) with layers -> cells:
[[D_right, U], [L, D_left]] with unit block-bidiagonal D_right, D_left.
P^GS is the inverse of [[D_right, 0], [L, D_left]]: a rightward sweep, the
reflections, a leftward sweep (Algs. 3-5 transposed).

The paper fixes the inner GMRES tolerance at 1e-6 in its experiments (Fig. 9);
here it is a parameter.  Pins: the dense inner polarized system reproduces the
exact traces of the direct layer solve; its block structure; the sweeps equal
dense triangular solves; the layer solve and the outer DD solve agree with
the direct solves to the inner / outer tolerance.
"""
from __future__ import annotations

import numpy as np

from .gmres import gmres
from .nested import NestedLayerSolver


class PolarizedInnerSolver(NestedLayerSolver):
    """A layer solver whose inner SIE is solved by polarized traces and
    GMRES (no inner factorisation)."""

    def __init__(self, grid, cells: int, inner_tol: float = 1e-6, inner_maxit: int = 200,
                 dtype=np.complex128):
        self.inner_tol = inner_tol
        self.inner_maxit = inner_maxit
        self.inner_iters: list[int] = []
        super().__init__(grid, cells, build_interface_ops=False, dtype=dtype)

    def _factor_inner(self):
        """Nothing to factorise: the inner system is iterated."""

    # ------------------------------------------------- cell Green's integrals
    def cell_op(self, c: int, left, right, side: str) -> np.ndarray:
        """R_side (H^c)^{-1}[T^c(left) + B^c(right)] for pairs [B, 2, HL] (None =
        absent); side 'left' samples positions (0, 1), 'right' (n_c, n_c + 1)."""
        C = self.cells[c]
        ref = left if left is not None else right
        g = np.zeros((ref.shape[0], C.HL, C.Wc), dtype=complex)
        if left is not None:
            g += self.src_T(c, left)
        if right is not None:
            g += self.src_B(c, right)
        w = self.cell_solve(c, g)
        pos = (0, 1) if side == "left" else (C.nc, C.nc + 1)
        return np.stack([w[..., :, C.col(pos[0])], w[..., :, C.col(pos[1])]], axis=1)

    # ------------------------------------------------ inner polarized system
    def inner_rhs_pol(self, newton):
        """(R_right^j N^j g, R_left^{j+1} N^{j+1} g) from the cell Newton
        potentials, each [B, J, 2, HL]."""
        B = newton[0].shape[0]
        J, HL = self.J, self.HL
        fd = np.zeros((B, J, 2, HL), dtype=complex)
        fq = np.zeros((B, J, 2, HL), dtype=complex)
        for j in range(J):
            Cj, Cn = self.cells[j], self.cells[j + 1]
            fd[:, j, 0] = newton[j][..., :, Cj.col(Cj.nc)]
            fd[:, j, 1] = newton[j][..., :, Cj.col(Cj.nc + 1)]
            fq[:, j, 0] = newton[j + 1][..., :, Cn.col(0)]
            fq[:, j, 1] = newton[j + 1][..., :, Cn.col(1)]
        return fd, fq

    def inner_apply_pol(self, d: np.ndarray, q: np.ndarray):
        """The inner polarized matrix applied to (d, q), each [B, J, 2, HL]."""
        J = self.J
        s = d + q
        od = np.zeros_like(d)
        oq = np.zeros_like(q)
        for j in range(J):
            y = self.cell_op(j, s[:, j - 1] if j > 0 else None, q[:, j], "right")
            od[:, j] = d[:, j] - y
            od[:, j, 0] += q[:, j, 0]                        # E_a q_j
            y = self.cell_op(j + 1, d[:, j], s[:, j + 1] if j + 1 < J else None, "left")
            oq[:, j] = q[:, j] - y
            oq[:, j, 1] += d[:, j, 1]                        # E_b d_j
        return od, oq

    def sweep_right(self, v: np.ndarray) -> np.ndarray:
        """(D_right)^{-1} v: rightward sweep over the cells."""
        x = np.zeros_like(v)
        for j in range(self.J):
            x[:, j] = v[:, j]
            if j > 0:
                x[:, j] += self.cell_op(j, x[:, j - 1], None, "right")
        return x

    def sweep_left(self, v: np.ndarray) -> np.ndarray:
        """(D_left)^{-1} v: leftward sweep over the cells."""
        J = self.J
        x = np.zeros_like(v)
        for j in range(J - 1, -1, -1):
            x[:, j] = v[:, j]
            if j < J - 1:
                x[:, j] += self.cell_op(j + 1, None, x[:, j + 1], "left")
        return x

    def apply_Lrefl(self, d: np.ndarray) -> np.ndarray:
        """The block L (d-part of the left rows): reflections off each cell."""
        J = self.J
        out = np.zeros_like(d)
        for j in range(J):
            out[:, j] = -self.cell_op(j + 1, d[:, j], d[:, j + 1] if j + 1 < J else None, "left")
            out[:, j, 1] += d[:, j, 1]
        return out

    def precond_gs(self, vd: np.ndarray, vq: np.ndarray):
        """Inner P^GS: inverse of [[D_right, 0], [L, D_left]]."""
        xd = self.sweep_right(vd)
        xq = self.sweep_left(vq - self.apply_Lrefl(xd))
        return xd, xq

    def pack(self, d, q):
        return np.concatenate([d.ravel(), q.ravel()])

    def unpack(self, v):
        half = v.size // 2
        shp = (1, self.J, 2, self.HL)
        return v[:half].reshape(shp), v[half:].reshape(shp)

    def inner_traces(self, newton) -> np.ndarray:
        """Inner traces s = d + q from left-preconditioned GMRES on the inner
        polarized system, one right-hand side at a time, x0 = 0."""
        fd, fq = self.inner_rhs_pol(newton)
        B = fd.shape[0]
        v = np.zeros((B, self.J, 2, self.HL), dtype=complex)
        A = lambda x: self.pack(*self.inner_apply_pol(*self.unpack(x)))
        P = lambda x: self.pack(*self.precond_gs(*self.unpack(x)))
        for b in range(B):
            x, info = gmres(A, self.pack(fd[b:b + 1], fq[b:b + 1]), P,
                            tol=self.inner_tol, maxit=self.inner_maxit)
            if not info["converged"]:
                raise RuntimeError("inner GMRES did not reach the inner tolerance")
            self.inner_iters.append(info["iters"])
            d, q = self.unpack(x)
            v[b] = (d + q)[0]
        return v

    def interface_op(self, g_rows: np.ndarray, rows) -> np.ndarray:
        """(H^l)^{-1} g sampled on ``rows`` for g supported there (the volume
        solve of Alg. 7 with the iterated inner system)."""
        g = np.zeros((self.HL, self.W), dtype=complex)
        g[list(rows), :] = g_rows
        return self.solve(g)[list(rows), :]
