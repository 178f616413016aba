"""Pins of the oracle's domain-decomposition method against the global direct
solve, dense assemblies and exact identities (Sec. 2-4, App. C)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.discretization import Problem
from oracle.bicgstab import bicgstab
from oracle.gmres import gmres
from oracle.nested import NestedLayerSolver
from oracle.polarized import DirectLayerSolver, LayeredSolver
from oracle import forms
from paper_1510_01831_amd import media


def _setup(n=31, p=8, L=3, seed=1, src=((16,), 6)):
    c, omega = media.small_problem(n, p, L, 2, seed=seed)
    prob = Problem(c, omega, p)
    f = prob.extend(media.point_sources(n, src[0], src[1])[0])
    u = spla.spsolve(prob.H.tocsc(), f.ravel()).reshape(prob.W, prob.W)
    return prob, f, u


def _traces(S, u):
    out = np.zeros((S.L - 1, 2, S.W), dtype=complex)
    for k in range(S.L - 1):
        G = S.grids[k]
        ra = G.global_row(G.row(G.nl))
        out[k] = u[[ra, ra + 1]]
    return out


def test_layer_rows_match_global():
    prob, f, u = _setup()
    S = LayeredSolver(prob, 3)
    H = prob.H.tocsr()
    W = prob.W
    for G in S.grids:
        for r in range(G.own_lo, G.own_hi + 1):
            gr = G.global_row(r)
            a = H[gr * W:(gr + 1) * W].toarray()
            b = G.H[r * W:(r + 1) * W].toarray()
            # columns of the layer row, placed at the global rows they refer to
            full = np.zeros_like(a)
            for rr in range(G.HL):
                g2 = G.global_row(rr)
                if 0 <= g2 < W:
                    full[:, g2 * W:(g2 + 1) * W] += b[:, rr * W:(rr + 1) * W]
            assert np.abs(full - a).max() == 0.0


def test_grf_identity_app_c():
    """(H^l)^{-1}[f^l + T_l + B_l] reproduces u on owned rows, 0 elsewhere."""
    prob, f, u = _setup()
    S = LayeredSolver(prob, 3)
    s = _traces(S, u)
    for l, G in enumerate(S.grids):
        g = S.restrict_source(l, f)
        if l > 0:
            g += S.src_T(l, s[l - 1])
        if l < S.L - 1:
            g += S.src_B(l, s[l])
        w = S.solvers[l].solve(g)
        ref = np.zeros_like(w)
        own = np.arange(G.own_lo, G.own_hi + 1)
        ref[own] = u[G.global_row(own)]
        assert np.abs(w - ref).max() < 1e-12 * np.abs(u).max()


def test_grf_identity_fails_with_flipped_sign():
    """A planted sign error in an equivalent source breaks the identity."""
    prob, f, u = _setup()
    S = LayeredSolver(prob, 3)
    s = _traces(S, u)
    l, G = 1, S.grids[1]
    g = S.restrict_source(l, f) + S.src_T(l, s[0]) - S.src_B(l, s[1])
    w = S.solvers[l].solve(g)
    own = np.arange(G.own_lo, G.own_hi + 1)
    assert np.abs(w[own] - u[G.global_row(own)]).max() > 1e-3 * np.abs(u).max()


def test_unpolarized_sie_exact():
    prob, f, u = _setup()
    S = LayeredSolver(prob, 3)
    n = (S.L - 1) * 2 * S.W
    M = S.dense(lambda e: S.apply_M_unpol(e.reshape(S.L - 1, 2, S.W)).ravel(), n)
    s = np.linalg.solve(M, S.rhs_unpol(f).ravel()).reshape(S.L - 1, 2, S.W)
    st = _traces(S, u)
    assert np.abs(s - st).max() < 1e-11 * np.abs(st).max()


@pytest.fixture(scope="module")
def dense_polarized():
    prob, f, u = _setup(n=23, p=6, L=4)
    S = LayeredSolver(prob, 4)
    K, W = S.L - 1, S.W
    n = 2 * K * 2 * W
    M = S.dense(lambda e: S.pack(*S.apply_M(*S.unpack(e))), n)
    return prob, f, u, S, M


def test_polarized_system_solution(dense_polarized):
    prob, f, u, S, M = dense_polarized
    x = np.linalg.solve(M, S.pack(*S.rhs(f)))
    d, q = S.unpack(x)
    st = _traces(S, u)
    assert np.abs(d + q - st).max() < 1e-10 * np.abs(st).max()
    # annihilation relations of the polarized pieces
    for k in range(S.L - 1):
        a = S.layer_op(k, None, d[k], "bot")
        assert np.abs(a[0]).max() < 1e-9 * np.abs(d).max()
        assert np.abs(a[1] + d[k, 1]).max() < 1e-9 * np.abs(d).max()
        b = S.layer_op(k + 1, q[k], None, "top")
        assert np.abs(b[1]).max() < 1e-9 * np.abs(q).max()
        assert np.abs(b[0] + q[k, 0]).max() < 1e-9 * np.abs(q).max()


def test_polarized_block_structure(dense_polarized):
    prob, f, u, S, M = dense_polarized
    K, W = S.L - 1, S.W
    b = 2 * W
    half = K * b
    Dd, Du = M[:half, :half], M[half:, half:]
    for i in range(K):
        for j in range(K):
            bd = Dd[i * b:(i + 1) * b, j * b:(j + 1) * b]
            bu = Du[i * b:(i + 1) * b, j * b:(j + 1) * b]
            if i == j:
                assert np.abs(bd - np.eye(b)).max() == 0 and np.abs(bu - np.eye(b)).max() == 0
            if j > i:
                assert np.abs(bd).max() == 0
            if j < i:
                assert np.abs(bu).max() == 0
            if j not in (i - 1, i):
                assert np.abs(bd).max() == 0
            if j not in (i, i + 1):
                assert np.abs(bu).max() == 0


def test_sweeps_are_triangular_inverses(dense_polarized):
    prob, f, u, S, M = dense_polarized
    K, W = S.L - 1, S.W
    half = K * 2 * W
    rng = np.random.default_rng(0)
    vd = rng.standard_normal((K, 2, W)) + 1j * rng.standard_normal((K, 2, W))
    vq = rng.standard_normal((K, 2, W)) + 1j * rng.standard_normal((K, 2, W))
    Dd, Lb, Du = M[:half, :half], M[half:, :half], M[half:, half:]
    assert np.allclose(S.sweep_down(vd).ravel(), np.linalg.solve(Dd, vd.ravel()), rtol=0, atol=1e-10)
    assert np.allclose(S.sweep_up(vq).ravel(), np.linalg.solve(Du, vq.ravel()), rtol=0, atol=1e-10)
    assert np.allclose(S.apply_Lrefl(vd).ravel(), Lb @ vd.ravel(), rtol=0, atol=1e-10)
    xd, xq = S.precond_gs(vd, vq)
    T = np.block([[Dd, np.zeros_like(Dd)], [Lb, Du]])
    ref = np.linalg.solve(T, np.concatenate([vd.ravel(), vq.ravel()]))
    assert np.abs(np.concatenate([xd.ravel(), xq.ravel()]) - ref).max() < 1e-9 * np.abs(ref).max()


def test_gmres_matches_dense_solve():
    rng = np.random.default_rng(7)
    n = 40
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    P = np.linalg.inv(A + 0.3 * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = gmres(lambda v: A @ v, b, lambda v: P @ v, tol=1e-13, maxit=n)
    assert info["converged"]
    xr = np.linalg.solve(A, b)
    assert np.abs(x - xr).max() < 1e-10 * np.abs(xr).max()
    # the recorded residual is the true preconditioned residual
    k = info["iters"]
    assert abs(np.linalg.norm(P @ (b - A @ x)) / np.linalg.norm(P @ b) - info["history"][k]) < 1e-10


def test_jacobi_is_block_diagonal_inverse(dense_polarized):
    """P^Jac = inverse of diag(D_down, D_up) (eq. preconditioner_Jac), against
    the dense blocks of the assembled polarized matrix."""
    prob, f, u, S, M = dense_polarized
    K, W = S.L - 1, S.W
    half = K * 2 * W
    rng = np.random.default_rng(3)
    vd = rng.standard_normal((K, 2, W)) + 1j * rng.standard_normal((K, 2, W))
    vq = rng.standard_normal((K, 2, W)) + 1j * rng.standard_normal((K, 2, W))
    Dd, Du = M[:half, :half], M[half:, half:]
    xd, xq = S.precond_jacobi(vd, vq)
    assert np.abs(xd.ravel() - np.linalg.solve(Dd, vd.ravel())).max() < 1e-10
    assert np.abs(xq.ravel() - np.linalg.solve(Du, vq.ravel())).max() < 1e-10


def test_bicgstab_matches_dense_solve():
    """Right-preconditioned Bi-CGstab reaches the dense solution, and the
    residual it reports is the true unpreconditioned one."""
    rng = np.random.default_rng(8)
    n = 40
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    P = np.linalg.inv(A + 0.3 * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xr = np.linalg.solve(A, b)
    for prec in (lambda v: P @ v, None):
        x, info = bicgstab(lambda v: A @ v, b, prec, tol=1e-12, maxit=200)
        assert info["converged"] and not info["breakdown"]
        assert np.abs(x - xr).max() < 1e-9 * np.abs(xr).max()
        true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        assert true <= 1e-11
        assert abs(true - info["history"][-1]) < 1e-12


def test_bicgstab_dd_matches_global_direct():
    prob, f, u = _setup(n=47, p=8, L=4, src=((24,), 9))
    S = LayeredSolver(prob, 4, 2)
    for pre in ("gs", "jacobi"):
        ud, info = S.solve(f, tol=1e-11, precond=pre, krylov="bicgstab")
        assert info["converged"]
        assert np.linalg.norm(ud - u) / np.linalg.norm(u) < 1e-9


def test_table3_iteration_pattern():
    """Soft check of Table 3's qualitative findings on a synthetic medium:
    with either Krylov method P^GS needs fewer iterations than P^Jac, and
    Bi-CGstab (two applications per iteration) needs fewer iterations than
    GMRES."""
    prob, f, u = _setup(n=63, p=10, L=6, src=((32,), 8))
    S = LayeredSolver(prob, 6)
    it = {}
    for kr in ("gmres", "bicgstab"):
        for pre in ("gs", "jacobi"):
            _, info = S.solve(f, tol=1e-7, precond=pre, krylov=kr)
            assert info["converged"]
            it[kr, pre] = info["iters"]
    assert it["gmres", "gs"] < it["gmres", "jacobi"]
    assert it["bicgstab", "gs"] < it["bicgstab", "jacobi"]
    assert it["bicgstab", "gs"] <= it["gmres", "gs"]


@pytest.mark.parametrize("cells", [1, 2, 3])
def test_nested_equals_direct_layer(cells):
    prob, f, u = _setup(n=31, p=8, L=3)
    S = LayeredSolver(prob, 3)
    rng = np.random.default_rng(11)
    for l in range(3):
        G = S.grids[l]
        nest = NestedLayerSolver(G, cells)
        direct = DirectLayerSolver(G)
        g = rng.standard_normal((G.HL, prob.W)) + 1j * rng.standard_normal((G.HL, prob.W))
        a, b = nest.solve(g), direct.solve(g)
        assert np.abs(a - b).max() < 1e-11 * np.abs(b).max()
        rows = nest.rows
        gr = rng.standard_normal((len(rows), prob.W)) + 0j
        a = nest.interface_op(gr, rows)
        b = direct.interface_op(gr, rows)
        assert np.abs(a - b).max() < 1e-11 * np.abs(b).max()


def test_nested_without_dloc_fails():
    """The interface factorisation needs the cell-local term (planted drop)."""
    prob, f, u = _setup(n=31, p=8, L=3)
    S = LayeredSolver(prob, 3)
    G = S.grids[1]
    nest = NestedLayerSolver(G, 2)
    direct = DirectLayerSolver(G)
    rows = nest.rows
    gr = np.ones((len(rows), prob.W), complex)
    ref = direct.interface_op(gr, rows)
    for op in nest.ops:
        op["D_loc"] = 0 * op["D_loc"]
    assert np.abs(nest.interface_op(gr, rows) - ref).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("cells", [None, 2])
def test_dd_matches_global_direct(cells):
    prob, f, u = _setup(n=47, p=8, L=4, src=((24,), 9))
    S = LayeredSolver(prob, 4, cells)
    ud, info = S.solve(f, tol=1e-11)
    assert info["converged"]
    assert np.linalg.norm(ud - u) / np.linalg.norm(u) < 1e-9


def test_single_layer_reduces_to_global():
    prob, f, u = _setup(n=23, p=6, L=1)
    S = LayeredSolver(prob, 1, 2)
    ud, _ = S.solve(f)
    assert np.linalg.norm(ud - u) / np.linalg.norm(u) < 1e-11


def test_gauss_seidel_beats_jacobi():
    """Soft check of Table 3's qualitative claim on a synthetic medium."""
    prob, f, u = _setup(n=63, p=10, L=6, src=((32,), 8))
    S = LayeredSolver(prob, 6)
    _, ig = S.solve(f, tol=1e-8, precond="gs")
    _, ij = S.solve(f, tol=1e-8, precond="jacobi")
    assert ig["iters"] < ij["iters"]


def test_dd_reciprocity():
    prob, _, _ = _setup(n=31, p=8, L=3)
    S = LayeredSolver(prob, 3, 2)
    f1 = prob.extend(media.point_sources(31, (7,), 5)[0])
    f2 = prob.extend(media.point_sources(31, (22,), 26)[0])
    u1, _ = S.solve(f1, tol=1e-12)
    u2, _ = S.solve(f2, tol=1e-12)
    p = prob.p
    a = u1[p + 26 - 1, p + 22 - 1]
    b = u2[p + 5 - 1, p + 7 - 1]
    assert abs(a - b) < 1e-9 * abs(a)


def test_adjoint_dot_product():
    prob, _, _ = _setup(n=23, p=6, L=1)
    lu = spla.splu(prob.H.tocsc())
    rng = np.random.default_rng(4)
    N = prob.W ** 2
    a = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    lhs = lu.solve(a) @ b                         # <H^{-1} a, b> (bilinear)
    rhs = a @ lu.solve(b, trans="T")              # <a, H^{-T} b>
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)
    assert abs(lu.solve(b, trans="T") - lu.solve(b)).max() < 1e-11 * abs(lu.solve(b)).max()


def test_gradient_finite_difference():
    n, p = 23, 6
    omega = media.omega_ppw(2.0, n, 8.0)
    true_c = media.gaussian_bump(n, 2.0, 0.4, 2 * 0.12 ** 2)
    f = media.point_sources(n, (6, 12, 18), 4)
    ref = forms.Misfit(omega, p, f, rec_row=4)
    prob, lu, U = ref.forward(1.0 / true_c ** 2)
    d_obs = ref.record(prob, U)
    mis = forms.Misfit(omega, p, f, rec_row=4, d_obs=d_obs)
    m0 = np.full((n, n), 0.25)
    J, g = mis.value_and_grad(m0)
    assert J > 0
    rng = np.random.default_rng(0)
    for _ in range(3):
        dm = rng.standard_normal((n, n))
        eps = 1e-6 * np.linalg.norm(m0) / np.linalg.norm(dm)
        fd = (mis.value(m0 + eps * dm) - mis.value(m0 - eps * dm)) / (2 * eps)
        an = float(np.sum(g * dm))
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_gradient_fd_catches_dropped_fold():
    """Without folding the PML copies onto the edge nodes the FD check fails."""
    n, p = 15, 5
    omega = media.omega_ppw(2.0, n, 8.0)
    f = media.point_sources(n, (4, 11), 3)
    ref = forms.Misfit(omega, p, f, rec_row=3)
    prob, lu, U = ref.forward(np.full((n, n), 0.2))
    mis = forms.Misfit(omega, p, f, rec_row=3, d_obs=ref.record(prob, U) * 1.1)
    m0 = np.full((n, n), 0.25)
    prob, lu, U = mis.forward(m0)
    J, g = mis.value_and_grad(m0)
    # gradient restricted to the physical copy only (planted mistake)
    r = mis.record(prob, U) - mis.d_obs
    adj = np.zeros((len(f), n, n), complex)
    adj[:, 2, :] = np.conj(r)
    MU = lu.solve(prob.extend(adj).reshape(len(f), -1).T).T.reshape(-1, prob.W, prob.W)
    g_bad = prob.restrict(omega ** 2 * np.real(forms.weight_ext(prob) * MU * U).sum(0))
    dm = np.zeros((n, n)); dm[0, :] = 1.0; dm[:, -1] = 1.0
    eps = 1e-6
    fd = (mis.value(m0 + eps * dm) - mis.value(m0 - eps * dm)) / (2 * eps)
    assert abs(fd - np.sum(g * dm)) <= 1e-6 * abs(fd)
    assert abs(fd - np.sum(g_bad * dm)) > 1e-4 * abs(fd)


def test_mixed_refinement_reaches_fp64():
    prob, f, u = _setup(n=31, p=8, L=3)
    ur, hist = forms.refine_mixed(prob, 3, 2, f, inner_tol=1e-6, target=1e-11)
    assert np.linalg.norm(ur - u) / np.linalg.norm(u) < 1e-9
    assert hist[1] < 1e-2 * hist[0]            # the correction contracts
