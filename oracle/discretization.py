"""Discretisation of the Helmholtz operator with PML (App. A).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions (App. A, Sec. 2.1):
* physical nodes p, q = 1..n at (p h, q h), h = 1/(n+1); the extended grid
  adds ``n_pml`` nodes per side, so local positions run from -n_pml+1 to
  n+n_pml, with homogeneous Dirichlet conditions at -n_pml and n+n_pml+1;
* sigma vanishes on the closed physical interval, so the edge nodes 0 and n+1
  are undamped and the Dirichlet node sits at depth delta = n_pml h;
* sigma(d) = (C/delta)(d/delta)^2 with C = beta omega delta, hence
  alpha = 1/(1 + i sigma/omega) = 1/(1 + i beta (d/delta)^2);
* the 5-point operator of App. A (row form) is divided row by row by
  alpha_x(p) alpha_z(q), which makes it complex symmetric and leaves every
  row inside the physical domain unchanged (alpha = 1 there).  The mass term
  is -omega^2 m u (the paper's interior stencil omits the ``u``; read as a
  typo).
* unknowns are ordered row by row in depth, x fastest (Sec. 2.1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def pml_alpha(pos, n_own: int, n_pml: int, beta: float) -> np.ndarray:
    """alpha at (possibly half-integer) positions of an axis whose own nodes
    are 1..n_own (App. A, def. of alpha and sigma)."""
    pos = np.asarray(pos, dtype=float)
    if n_pml == 0:
        return np.ones(pos.shape, dtype=complex)
    d = np.maximum(0.0, np.maximum(-pos, pos - (n_own + 1))) / n_pml
    return 1.0 / (1.0 + 1j * beta * d * d)


def axis_profile(n_own: int, n_pml: int, beta: float):
    """alpha at the nodes (length n_own+2 n_pml) and at the half positions
    between consecutive nodes, including the two half steps towards the
    Dirichlet nodes (length n_own+2 n_pml+1)."""
    nodes = np.arange(-n_pml + 1, n_own + n_pml + 1, dtype=float)
    halves = np.arange(-n_pml + 1, n_own + n_pml + 2, dtype=float) - 0.5
    return pml_alpha(nodes, n_own, n_pml, beta), pml_alpha(halves, n_own, n_pml, beta)


def assemble(m: np.ndarray, axn, axh, azn, azh, h: float, omega: float) -> sp.csr_matrix:
    """Symmetric-form 5-point operator on a grid of shape m.shape = (Wz, Wx).

    Row (j, i):
      [ax(i-1/2)(u_ij - u_i-1,j) + ax(i+1/2)(u_ij - u_i+1,j)] / (az(j) h^2)
    + [az(j-1/2)(u_ij - u_i,j-1) + az(j+1/2)(u_ij - u_i,j+1)] / (ax(i) h^2)
    - omega^2 m_ij u_ij / (ax(i) az(j)),
    with zero Dirichlet values beyond the grid.
    """
    Wz, Wx = m.shape
    N = Wz * Wx
    idx = np.arange(N).reshape(Wz, Wx)
    AX = np.asarray(axn)[None, :]
    AZ = np.asarray(azn)[:, None]
    axh = np.asarray(axh)
    azh = np.asarray(azh)
    h2 = h * h
    diag = ((axh[None, :-1] + axh[None, 1:]) / (AZ * h2)
            + (azh[:-1, None] + azh[1:, None]) / (AX * h2)
            - omega ** 2 * m / (AX * AZ))
    cx = -axh[None, 1:-1] / (AZ * h2) * np.ones((Wz, 1))
    cz = -azh[1:-1, None] / (AX * h2) * np.ones((1, Wx))
    rows = np.concatenate([idx.ravel(), idx[:, :-1].ravel(), idx[:, 1:].ravel(),
                           idx[:-1, :].ravel(), idx[1:, :].ravel()])
    cols = np.concatenate([idx.ravel(), idx[:, 1:].ravel(), idx[:, :-1].ravel(),
                           idx[1:, :].ravel(), idx[:-1, :].ravel()])
    vals = np.concatenate([diag.ravel(), cx.ravel(), cx.ravel(), cz.ravel(), cz.ravel()])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def assemble_row_form(m, axn, axh, azn, azh, h, omega) -> sp.csr_matrix:
    """The unsymmetric row form printed in App. A (before the row scaling):
    -ax(i)[ax(i+1/2)(u_i+1 - u_i) - ax(i-1/2)(u_i - u_i-1)]/h^2 - (same in z)
    - omega^2 m u.  Used only to pin the symmetric assembly."""
    D = sp.diags((np.asarray(azn)[:, None] * np.asarray(axn)[None, :]).ravel())
    return (D @ assemble(m, axn, axh, azn, azh, h, omega)).tocsr()


def partition(n: int, parts: int):
    """Split 1..n into ``parts`` contiguous blocks; the first n mod parts blocks
    get one extra node.  Returns a list of (first, last), 1-based, inclusive."""
    if parts < 1 or parts > n:
        raise ValueError("bad partition")
    base, extra = divmod(n, parts)
    out, start = [], 1
    for k in range(parts):
        size = base + (1 if k < extra else 0)
        out.append((start, start + size - 1))
        start += size
    return out


class Problem:
    """Global PML-truncated problem H u = f on the extended grid (App. A)."""

    def __init__(self, c: np.ndarray, omega: float, n_pml: int, beta: float = 2.0):
        c = np.asarray(c, dtype=float)
        assert c.ndim == 2 and c.shape[0] == c.shape[1]
        self.n = c.shape[0]
        self.p = n_pml
        self.h = 1.0 / (self.n + 1)
        self.omega = float(omega)
        self.beta = float(beta)
        self.c = c
        self.m = 1.0 / (c * c)                      # squared slowness (Sec. 2)
        self.W = self.n + 2 * n_pml
        self.ax_n, self.ax_h = axis_profile(self.n, n_pml, beta)
        self.az_n, self.az_h = self.ax_n, self.ax_h
        self.m_ext = self.m_window(-n_pml + 1, self.n + n_pml, -n_pml + 1, self.n + n_pml)
        self._H = None

    def m_window(self, z0, z1, x0, x1) -> np.ndarray:
        """m on global positions [z0..z1] x [x0..x1]; m is extended beyond the
        physical square by copying the nearest physical value."""
        zq = np.clip(np.arange(z0, z1 + 1), 1, self.n) - 1
        xq = np.clip(np.arange(x0, x1 + 1), 1, self.n) - 1
        return self.m[np.ix_(zq, xq)]

    @property
    def H(self) -> sp.csr_matrix:
        if self._H is None:
            self._H = assemble(self.m_ext, self.ax_n, self.ax_h, self.az_n, self.az_h,
                               self.h, self.omega)
        return self._H

    def extend(self, f_phys: np.ndarray) -> np.ndarray:
        """Zero-extend a physical field [.., n, n] to the extended grid (App. A)."""
        f_phys = np.asarray(f_phys)
        out = np.zeros(f_phys.shape[:-2] + (self.W, self.W), dtype=complex)
        p = self.p
        out[..., p:p + self.n, p:p + self.n] = f_phys
        return out

    def restrict(self, u_ext: np.ndarray) -> np.ndarray:
        p = self.p
        return u_ext[..., p:p + self.n, p:p + self.n]

    def apply(self, u_ext: np.ndarray) -> np.ndarray:
        """H u on the extended grid, u of shape [W, W] or [B, W, W]."""
        u = np.asarray(u_ext)
        flat = u.reshape(-1, self.W * self.W).T
        return (self.H @ flat).T.reshape(u.shape)


class LayerGrid:
    """Grid of layer l: all W columns, rows local -p+1..n_l+p (Sec. 2.1, Fig. 1).

    Owned rows are the layer's physical rows, plus the global PML rows for the
    first and last layer.  The artificial PML towards a neighbour starts at the
    first row past the owned ones (that row is undamped), so the operator of
    the layer coincides with the global one on every owned row.
    """

    def __init__(self, prob: Problem, first: int, last: int, index: int, count: int):
        self.prob = prob
        self.first, self.last = first, last        # global physical rows, 1-based
        self.index, self.count = index, count
        p = prob.p
        self.nl = last - first + 1
        self.HL = self.nl + 2 * p
        self.az_n, self.az_h = axis_profile(self.nl, p, prob.beta)
        self.ax_n, self.ax_h = prob.ax_n, prob.ax_h
        self.m = prob.m_window(first - p, last + p, -p + 1, prob.n + p)
        self.H = assemble(self.m, self.ax_n, self.ax_h, self.az_n, self.az_h, prob.h,
                          prob.omega)
        # local position -> array row: pos + p - 1
        self.own_lo = 0 if index == 0 else p            # array rows owned
        self.own_hi = self.HL - 1 if index == count - 1 else p + self.nl - 1

    def row(self, pos: int) -> int:
        """Array row of local position ``pos`` (1..n_l are the layer's own
        physical rows, 0 and n_l+1 the neighbours' interface rows)."""
        return pos + self.prob.p - 1

    def global_row(self, arr_row: int) -> int:
        """Extended-grid array row of a local array row."""
        return arr_row + self.first - 1

    def coupling(self, to_pos: int, from_pos: int) -> np.ndarray:
        """Diagonal of the block H^l[row to_pos, row from_pos] (App. C)."""
        W = self.prob.W
        r, c = self.row(to_pos), self.row(from_pos)
        blk = self.H[r * W:(r + 1) * W, c * W:(c + 1) * W]
        return np.asarray(blk.diagonal())


class CellGrid:
    """Grid of cell c of a layer: all layer rows, columns local -p+1..n_c+p
    (Sec. 4.2, Fig. 5).  Same ownership/artificial-PML rule as layers, in x."""

    def __init__(self, layer: LayerGrid, first: int, last: int, index: int, count: int):
        prob = layer.prob
        p = prob.p
        self.layer = layer
        self.first, self.last = first, last        # global physical columns, 1-based
        self.index, self.count = index, count
        self.nc = last - first + 1
        self.Wc = self.nc + 2 * p
        self.HL = layer.HL
        self.ax_n, self.ax_h = axis_profile(self.nc, p, prob.beta)
        self.az_n, self.az_h = layer.az_n, layer.az_h
        xq = np.clip(np.arange(first - p, last + p + 1), 1, prob.n) - 1
        # rows of the layer grid are already a window of m_ext; take columns
        zq_layer = np.clip(np.arange(layer.first - p, layer.last + p + 1), 1, prob.n) - 1
        self.m = prob.m[np.ix_(zq_layer, xq)]
        self.H = assemble(self.m, self.ax_n, self.ax_h, self.az_n, self.az_h, prob.h,
                          prob.omega)
        self.own_lo = 0 if index == 0 else p            # array cols owned
        self.own_hi = self.Wc - 1 if index == count - 1 else p + self.nc - 1
        # global extended-grid column of local array column 0
        self.col0 = first - 1                          # array col j -> global array col col0 + j

    def col(self, pos: int) -> int:
        return pos + self.layer.prob.p - 1

    def coupling(self, to_pos: int, from_pos: int) -> np.ndarray:
        """Diagonal (over rows) of the coupling between two columns of H^{l,c}."""
        Wc, HL = self.Wc, self.HL
        a, b = self.col(to_pos), self.col(from_pos)
        rows = np.arange(HL) * Wc + a
        cols = np.arange(HL) * Wc + b
        return np.asarray(self.H[rows, cols]).ravel()
