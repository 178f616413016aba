"""Pins of the oracle's partitioned low-rank compression (oracle/plr.py):
exact recovery of a low-rank tile, a full-rank block left dense, the
Frobenius error bound on operators of the method, and the nested DD solve
with the compressed preconditioner against the global direct solve."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle.discretization import LayerGrid, Problem, partition
from oracle.nested import NestedLayerSolver
from oracle.plr import PLR, PLRLayerView
from oracle.polarized import LayeredSolver
from paper_1510_01831_amd import media


def test_low_rank_tile_is_recovered():
    rng = np.random.default_rng(0)
    for k in (1, 3, 7):
        U = rng.standard_normal((64, k)) + 1j * rng.standard_normal((64, k))
        V = rng.standard_normal((k, 64)) + 1j * rng.standard_normal((k, 64))
        A = U @ V
        c = PLR(A, tile=64, eps=1e-8)
        assert c.ranks() == [k]
        assert np.linalg.norm(c.dense() - A) <= 1e-13 * np.linalg.norm(A)
        x = rng.standard_normal(64) + 1j * rng.standard_normal(64)
        assert np.linalg.norm(c.apply(x) - A @ x) <= 1e-13 * np.linalg.norm(A @ x)


def test_full_rank_block_stays_dense():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((100, 70)) + 1j * rng.standard_normal((100, 70))
    c = PLR(A, tile=32, eps=1e-8)
    assert c.ranks() == []
    assert c.ratio == 1.0
    assert np.array_equal(c.dense(), A)


def _layer_solver():
    c, omega = media.small_problem(95, 12, 3, 3, seed=4)
    prob = Problem(c, omega, 12)
    a, b = partition(95, 3)[1]
    return NestedLayerSolver(LayerGrid(prob, a, b, 1, 3), 3)


def test_error_bound_on_interface_operators():
    """||A - A_plr||_F <= eps ||A||_F for every interface operator of an
    interior layer, with storage below the dense size overall (the
    compressibility of the cell Green's functions)."""
    ls = _layer_solver()
    for eps in (1e-6, 1e-8, 1e-10):
        view = PLRLayerView(ls, eps=eps, tile=32)
        for op, cop in zip(ls.ops, view.ops):
            for key in ("D_loc", "Mf_left", "Mf_right", "Mu_left", "Mu_right"):
                if op[key] is None:
                    continue
                A = op[key]
                err = np.linalg.norm(cop[key].dense() - A)
                assert err <= eps * np.linalg.norm(A) * (1 + 1e-12)
    # compressibility: even on cells of 31 columns, 64-tiles at 1e-8 store
    # less than the dense operators
    assert PLRLayerView(ls, eps=1e-8, tile=64).ratio() < 0.9


def test_compressed_interface_op_matches_exact():
    """The layer's Green's integral with compressed operators against the
    exact one, for random sources on the interface rows: relative error of
    the order of eps."""
    ls = _layer_solver()
    view = PLRLayerView(ls, eps=1e-8, tile=32)
    rng = np.random.default_rng(2)
    g = rng.standard_normal((len(ls.rows), ls.W)) + 1j * rng.standard_normal((len(ls.rows), ls.W))
    exact = ls.interface_op(g, ls.rows)
    approx = view.interface_op(g, ls.rows)
    rel = np.linalg.norm(approx - exact) / np.linalg.norm(exact)
    assert 0 < rel <= 1e-6


def test_dd_with_compressed_preconditioner_matches_global_direct():
    """Nested DD (block-LU layers) with the Gauss-Seidel preconditioner built
    on PLR-compressed operators (eps = 1e-8) and the exact SIE matrix:
    same solution as the global direct solve, iterations as without
    compression (within one)."""
    n, p, L, Lc = 95, 12, 4, 3
    c, omega = media.small_problem(n, p, L, Lc, seed=6)
    prob = Problem(c, omega, p)
    f = media.point_sources(n, (40,), 20)[0]
    fe = prob.extend(f)
    ref = spla.splu(prob.H.tocsc()).solve(fe.ravel()).reshape(prob.W, prob.W)
    exact = LayeredSolver(prob, L, Lc)
    u0, info0 = exact.solve(fe, tol=1e-12)
    comp = LayeredSolver(prob, L, Lc, pre_plr_eps=1e-8, pre_plr_tile=32)
    u1, info1 = comp.solve(fe, tol=1e-12)
    assert np.linalg.norm(u1 - ref) / np.linalg.norm(ref) <= 1e-9
    assert abs(info1["iters"] - info0["iters"]) <= 1
    ratios = [v.ratio() for v in comp.pre_solvers]
    assert max(ratios) < 1.0
