"""Pins of the oracle's large-grid direct solve (oracle/direct.py): the
nested-dissection order is a permutation whose separators split the grid,
and the solve equals the closed form and SuperLU's default-ordered solve."""
import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
import scipy.sparse.linalg as spla

from oracle.direct import DirectSolver, nested_dissection
from oracle.discretization import Problem
from paper_1510_01831_amd import media


def _grid_graph(nz, nx):
    idx = np.arange(nz * nx).reshape(nz, nx)
    rows = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    cols = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    A = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(nz * nx, nz * nx))
    return (A + A.T).tocsr()


def test_nested_dissection_is_a_permutation_with_separators():
    for nz, nx in [(1, 1), (5, 3), (40, 40), (37, 91), (130, 64)]:
        p = nested_dissection(nz, nx, leaf=8)
        assert np.array_equal(np.sort(p), np.arange(nz * nx))
    # the last nodes of the order are the top-level separator: removing them
    # leaves two components of the grid graph
    nz, nx = 40, 33
    p = nested_dissection(nz, nx, leaf=8)
    sep = p[-nx:]
    assert np.all(sep // nx == sep[0] // nx)          # one full grid row
    keep = np.setdiff1d(np.arange(nz * nx), sep)
    G = _grid_graph(nz, nx)[keep][:, keep]
    ncomp, _ = csg.connected_components(G, directed=False)
    assert ncomp == 2


def test_direct_solve_dst_closed_form():
    """n_pml = 0, constant m: the 2D DST-I diagonalises H (eigenvalues
    (4/h^2)(sin^2(pi i / 2(n+1)) + sin^2(pi j / 2(n+1))) - omega^2 m)."""
    n = 47
    c = np.full((n, n), 1.1)
    omega = 23.0
    prob = Problem(c, omega, 0)
    rng = np.random.default_rng(7)
    f = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    u, res = DirectSolver(prob, leaf=8).solve(prob.extend(f).ravel())
    h = prob.h
    k = np.arange(1, n + 1)
    s2 = np.sin(np.pi * k / (2 * (n + 1))) ** 2
    lam = 4.0 / h ** 2 * (s2[:, None] + s2[None, :]) - omega ** 2 / 1.1 ** 2
    fh = scipy.fft.dstn(f, type=1)
    ref = scipy.fft.idstn(fh / lam, type=1)
    assert np.linalg.norm(u.reshape(n, n) - ref) <= 1e-12 * np.linalg.norm(ref)
    assert res.max() <= 1e-13


def test_direct_solve_matches_default_superlu_with_pml():
    """A heterogeneous medium with PML (the n = 127 workload): the
    nested-dissection solve equals SuperLU with its default ordering."""
    w = media.workload("C1")
    c = media.velocity("C1")
    prob = Problem(c, w.omega, w.n_pml)
    f = media.point_sources(w.n, (20, 64, 100), w.src_z)
    F = np.stack([prob.extend(x).ravel() for x in f], axis=1)
    U, res = DirectSolver(prob).solve(F)
    ref = spla.splu(prob.H.tocsc()).solve(F)
    err = np.linalg.norm(U - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert err.max() <= 1e-12
    assert res.max() <= 1e-13
