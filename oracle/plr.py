"""Partitioned low-rank compression of the interface operators (eq.
factorization and its PLR footnote; Sec. 4.3; the caption of Fig. 9:
accuracy eps = 1e-8; Table 4's "compressed direct method").

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The blocks of M_f and M_u (and the cell-local term D_loc) are samples of cell
Green's functions between well-separated point sets, hence numerically low
rank off the diagonal.  The paper compresses them in partitioned low-rank
(PLR) form: an adaptive dyadic partition whose leaves are low-rank factors
or small dense blocks, at accuracy eps.

Reading (the partition): one level of square tiles of a fixed size t.  A
tile is replaced by its truncated SVD U_r S_r V_r^H when that stores fewer
entries than the tile (r (t_r + t_c) < t_r t_c); otherwise it stays dense.
The rank r is the smallest for which the discarded singular values have
Frobenius norm at most  eps ||A||_F / sqrt(T)  (T tiles in the block), so
that the whole block satisfies  ||A - A_plr||_F <= eps ||A||_F.  The
application y = A_plr x is tile by tile: dense tiles as they are, low-rank
tiles as U_r (S_r V_r^H x).

Pins (tests/test_oracle_plr.py): an exactly rank-k tile keeps rank k; a
random full-rank block stays dense; the error bound on an operator of the
method; the nested DD solve with the compressed preconditioner equals the
global direct solve.
"""
from __future__ import annotations

import numpy as np


class PLR:
    """One-level partitioned low-rank form of a dense block A (m x k)."""

    def __init__(self, A: np.ndarray, tile: int = 64, eps: float = 1e-8):
        A = np.asarray(A)
        self.shape = A.shape
        self.dtype = A.dtype
        self.tile = tile
        m, k = A.shape
        self.row0 = list(range(0, m, tile))
        self.col0 = list(range(0, k, tile))
        T = max(1, len(self.row0) * len(self.col0))
        fro = np.linalg.norm(A)
        self.delta = eps * fro / np.sqrt(T)          # per-tile Frobenius budget
        self.tiles = {}
        self.stored = 0
        for i0 in self.row0:
            for j0 in self.col0:
                blk = A[i0:i0 + tile, j0:j0 + tile]
                tr, tc = blk.shape
                if not np.any(blk):
                    self.tiles[(i0, j0)] = ("zero", None, None)
                    continue
                U, s, Vh = np.linalg.svd(blk, full_matrices=False)
                # tail[r] = Frobenius norm of the singular values from r on
                tail = np.sqrt(np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]]))
                r = int(np.argmax(tail <= self.delta))
                if r * (tr + tc) < tr * tc:
                    self.tiles[(i0, j0)] = ("lr", U[:, :r] * s[:r], Vh[:r])
                    self.stored += r * (tr + tc)
                else:
                    self.tiles[(i0, j0)] = ("dense", blk.copy(), None)
                    self.stored += tr * tc

    @property
    def ratio(self) -> float:
        """Stored entries over the dense block's entries."""
        return self.stored / float(self.shape[0] * self.shape[1])

    def ranks(self):
        return [v[1].shape[1] for v in self.tiles.values() if v[0] == "lr"]

    def apply(self, X: np.ndarray) -> np.ndarray:
        """A_plr X for X of shape (k,) or (k, B)."""
        X = np.asarray(X)
        vec = X.ndim == 1
        X2 = X[:, None] if vec else X
        Y = np.zeros((self.shape[0], X2.shape[1]), dtype=np.result_type(self.dtype, X2.dtype))
        t = self.tile
        for (i0, j0), (kind, a, b) in self.tiles.items():
            xs = X2[j0:j0 + t]
            if kind == "dense":
                Y[i0:i0 + a.shape[0]] += a @ xs
            elif kind == "lr":
                Y[i0:i0 + a.shape[0]] += a @ (b @ xs)
        return Y[:, 0] if vec else Y

    def dense(self) -> np.ndarray:
        """The compressed block written out (for the error checks)."""
        out = np.zeros(self.shape, dtype=self.dtype)
        for (i0, j0), (kind, a, b) in self.tiles.items():
            if kind == "dense":
                out[i0:i0 + a.shape[0], j0:j0 + a.shape[1]] = a
            elif kind == "lr":
                out[i0:i0 + a.shape[0], j0:j0 + b.shape[1]] = a @ b
        return out


class PLRLayerView:
    """A nested layer solver whose interface operators D_loc, M_f and M_u
    are applied in PLR form (the compressed Green's integrals of eq.
    factorization); the inner block LU and the cell factors are shared with
    the exact solver it wraps."""

    def __init__(self, base, eps: float = 1e-8, tile: int = 64):
        self.base = base
        self.rows = base.rows
        self.ops = []
        for op in base.ops or []:
            c = {"own": op["own"]}
            for key in ("D_loc", "Mf_left", "Mf_right", "Mu_left", "Mu_right"):
                c[key] = None if op[key] is None else PLR(op[key], tile, eps)
            self.ops.append(c)

    def ratio(self) -> float:
        """Stored entries of all compressed operators over their dense size."""
        st = tot = 0.0
        for op in self.ops:
            for key in ("D_loc", "Mf_left", "Mf_right", "Mu_left", "Mu_right"):
                if op[key] is not None:
                    st += op[key].stored
                    tot += op[key].shape[0] * op[key].shape[1]
        return st / tot if tot else 1.0

    def interface_op(self, g_rows: np.ndarray, rows) -> np.ndarray:
        """D_loc g + M_u (M^l)^{-1} M_f g with the compressed operators."""
        b = self.base
        assert list(rows) == b.rows
        r = len(rows)
        J = b.J
        out = np.zeros((r, b.W), dtype=complex)
        xs = []
        for c in range(b.Lc):
            C = b.cells[c]
            xs.append(g_rows[:, C.col0 + self.ops[c]["own"]].reshape(-1))
        R = np.zeros((1, J, 2, b.HL), dtype=complex)
        for c in range(b.Lc):
            op = self.ops[c]
            if op["Mf_right"] is not None:
                R[0, c, 0] = op["Mf_right"].apply(xs[c])
            if op["Mf_left"] is not None:
                R[0, c - 1, 1] = op["Mf_left"].apply(xs[c])
        v = b.inner_solve(R) if J > 0 else R
        for c in range(b.Lc):
            C = b.cells[c]
            op = self.ops[c]
            y = op["D_loc"].apply(xs[c])
            if op["Mu_left"] is not None:
                y = y + op["Mu_left"].apply(v[0, c - 1].reshape(-1))
            if op["Mu_right"] is not None:
                y = y + op["Mu_right"].apply(v[0, c].reshape(-1))
            out[:, C.col0 + op["own"]] = y.reshape(r, -1)
        return out
