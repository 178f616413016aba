"""Pins of the nested polarized traces oracle (Sec. 4.2.1): the inner
polarized system of a layer against the exact traces of the direct layer
solve, its block structure, the inner sweeps against dense triangular solves,
and the layer / DD solves against the direct solves."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.discretization import Problem
from oracle.nested_pt import PolarizedInnerSolver
from oracle.polarized import DirectLayerSolver, LayeredSolver
from paper_1510_01831_amd import media


def _problem(n=31, p=8, L=3, seed=1):
    c, omega = media.small_problem(n, p, L, 2, seed=seed)
    return Problem(c, omega, p)


def _dense(S, fn):
    """Dense matrix of fn on stacked (d, q) vectors of one right-hand side."""
    n = 2 * S.J * 2 * S.HL
    cols = []
    for j in range(n):
        e = np.zeros(n, dtype=complex)
        e[j] = 1.0
        cols.append(fn(e))
    return np.stack(cols, axis=1)


@pytest.fixture(scope="module")
def layer_case():
    prob = _problem(n=23, p=6, L=3)
    lay = LayeredSolver(prob, 3)
    G = lay.grids[1]
    S = PolarizedInnerSolver(G, 3, inner_tol=1e-13)
    M = _dense(S, lambda e: S.pack(*S.inner_apply_pol(*S.unpack(e))))
    rng = np.random.default_rng(5)
    g = rng.standard_normal((G.HL, prob.W)) + 1j * rng.standard_normal((G.HL, prob.W))
    return prob, G, S, M, g


def _exact_traces(S, G, g):
    """(v_a, v_b) of every inner interface read off the direct layer solve."""
    u = DirectLayerSolver(G).solve(g)
    v = np.zeros((S.J, 2, S.HL), dtype=complex)
    for j in range(S.J):
        Cj, Cn = S.cells[j], S.cells[j + 1]
        v[j, 0] = u[:, Cj.col0 + Cj.col(Cj.nc)]
        v[j, 1] = u[:, Cn.col0 + Cn.col(1)]
    return v


def test_inner_polarized_system_gives_exact_traces(layer_case):
    prob, G, S, M, g = layer_case
    newton = [S.cell_solve(c, S.to_cell(c, g[None])) for c in range(S.Lc)]
    fd, fq = S.inner_rhs_pol(newton)
    x = np.linalg.solve(M, S.pack(fd, fq))
    d, q = S.unpack(x)
    ref = _exact_traces(S, G, g)
    assert np.abs((d + q)[0] - ref).max() < 1e-10 * np.abs(ref).max()
    # polarization: the rightward part radiates nothing back through its own
    # cell's right pair, the leftward part nothing through its left pair
    for j in range(S.J):
        a = S.cell_op(j, None, d[:, j], "right")
        assert np.abs(a[:, 0]).max() < 1e-9 * np.abs(d).max()
        assert np.abs(a[:, 1] + d[:, j, 1]).max() < 1e-9 * np.abs(d).max()
        b = S.cell_op(j + 1, q[:, j], None, "left")
        assert np.abs(b[:, 1]).max() < 1e-9 * np.abs(q).max()
        assert np.abs(b[:, 0] + q[:, j, 0]).max() < 1e-9 * np.abs(q).max()


def test_inner_polarized_block_structure(layer_case):
    prob, G, S, M, g = layer_case
    b = 2 * S.HL
    half = S.J * b
    Dd, Du = M[:half, :half], M[half:, half:]
    for i in range(S.J):
        for j in range(S.J):
            bd = Dd[i * b:(i + 1) * b, j * b:(j + 1) * b]
            bu = Du[i * b:(i + 1) * b, j * b:(j + 1) * b]
            if i == j:
                assert np.abs(bd - np.eye(b)).max() == 0 and np.abs(bu - np.eye(b)).max() == 0
            if j not in (i - 1, i):
                assert np.abs(bd).max() == 0
            if j not in (i, i + 1):
                assert np.abs(bu).max() == 0


def test_inner_sweeps_are_triangular_inverses(layer_case):
    prob, G, S, M, g = layer_case
    half = S.J * 2 * S.HL
    rng = np.random.default_rng(2)
    shp = (1, S.J, 2, S.HL)
    vd = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    vq = rng.standard_normal(shp) + 1j * rng.standard_normal(shp)
    Dd, Lb, Du = M[:half, :half], M[half:, :half], M[half:, half:]
    tol = 1e-10 * max(np.abs(vd).max(), 1)
    assert np.abs(S.sweep_right(vd).ravel() - np.linalg.solve(Dd, vd.ravel())).max() < tol * 1e2
    assert np.abs(S.sweep_left(vq).ravel() - np.linalg.solve(Du, vq.ravel())).max() < tol * 1e2
    assert np.abs(S.apply_Lrefl(vd).ravel() - Lb @ vd.ravel()).max() < tol * 1e2
    xd, xq = S.precond_gs(vd, vq)
    T = np.block([[Dd, np.zeros_like(Dd)], [Lb, Du]])
    ref = np.linalg.solve(T, np.concatenate([vd.ravel(), vq.ravel()]))
    got = np.concatenate([xd.ravel(), xq.ravel()])
    assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("cells", [2, 3, 4])
def test_pt_layer_solve_equals_direct(cells):
    prob = _problem()
    lay = LayeredSolver(prob, 3)
    rng = np.random.default_rng(11)
    for l in range(3):
        G = lay.grids[l]
        S = PolarizedInnerSolver(G, cells, inner_tol=1e-13)
        g = rng.standard_normal((2, G.HL, prob.W)) + 1j * rng.standard_normal((2, G.HL, prob.W))
        a = S.solve(g)
        b = DirectLayerSolver(G).solve(g)
        assert np.abs(a - b).max() < 1e-10 * np.abs(b).max()
        # the inner Gauss-Seidel sweeps make the inner iteration short
        assert max(S.inner_iters) <= 4 * cells


def test_pt_inner_tolerance_is_honoured():
    """A loose inner tolerance gives a correspondingly loose layer solve, and
    the inner iteration count grows as the tolerance tightens."""
    prob = _problem()
    lay = LayeredSolver(prob, 3)
    G = lay.grids[1]
    g = np.zeros((G.HL, prob.W), complex)
    g[G.HL // 2, prob.W // 2] = 1.0
    b = DirectLayerSolver(G).solve(g)
    errs, its = [], []
    for tol in (1e-4, 1e-8, 1e-12):
        S = PolarizedInnerSolver(G, 4, inner_tol=tol)
        a = S.solve(g)
        errs.append(np.abs(a - b).max() / np.abs(b).max())
        its.append(S.inner_iters[-1])
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-9
    assert its[0] < its[1] < its[2]


def test_pt_planted_sign_error_fails(layer_case):
    """Dropping the E_a term (a planted mistake) breaks the exact traces."""
    prob, G, S, M, g = layer_case

    class Broken(PolarizedInnerSolver):
        def inner_apply_pol(self, d, q):
            od, oq = super().inner_apply_pol(d, q)
            od[:, :, 0] -= q[:, :, 0]
            return od, oq

    B = Broken(G, 3, inner_tol=1e-13)
    Mb = _dense(B, lambda e: B.pack(*B.inner_apply_pol(*B.unpack(e))))
    newton = [B.cell_solve(c, B.to_cell(c, g[None])) for c in range(B.Lc)]
    x = np.linalg.solve(Mb, B.pack(*B.inner_rhs_pol(newton)))
    d, q = B.unpack(x)
    ref = _exact_traces(B, G, g)
    assert np.abs((d + q)[0] - ref).max() > 1e-3 * np.abs(ref).max()


def test_dd_with_pt_inner_matches_global_direct():
    prob = _problem(n=47, p=8, L=4)
    f = prob.extend(media.point_sources(47, (24,), 9)[0])
    u = spla.spsolve(prob.H.tocsc(), f.ravel()).reshape(prob.W, prob.W)
    S = LayeredSolver(prob, 4, 3, inner="pt", inner_tol=1e-13)
    ud, info = S.solve(f, tol=1e-11)
    assert info["converged"]
    assert np.linalg.norm(ud - u) / np.linalg.norm(u) < 1e-9
