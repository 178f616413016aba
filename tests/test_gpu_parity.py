"""GPU parity: every building block of the HIP path, called through the C-ABI,
against the oracle on the same seeded inputs (complex128 tolerances)."""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.discretization import CellGrid, Problem  # noqa: E402
from oracle.polarized import LayeredSolver  # noqa: E402
from paper_1510_01831_amd import hz, media  # noqa: E402

N, P, L, LC = 47, 8, 4, 3


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, omega = media.small_problem(N, P, L, LC, seed=5)
    prob = Problem(c, omega, P)
    _log(f"[setup] n={N} p={P} L={L} Lc={LC} omega={omega:.3f}")
    solver = hz.Solver(torch.from_numpy(c), omega, P, L, LC, max_batch=4)
    oracle = LayeredSolver(prob, L)
    yield c, omega, prob, solver, oracle
    solver.close()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_cell_solve(setup):
    c, omega, prob, solver, oracle = setup
    rng = np.random.default_rng(0)
    for layer, cell in [(0, 0), (1, 1), (3, 2), (2, 0)]:
        _log(f"[cell_solve] layer={layer} cell={cell}")
        HL, Wc = solver.cell_shape(layer, cell)
        G = oracle.grids[layer]
        a, b = [(1, 16), (17, 32), (33, 47)][cell]
        C = CellGrid(G, a, b, cell, LC)
        assert (C.HL, C.Wc) == (HL, Wc)
        g = rng.standard_normal((HL, Wc, 3)) + 1j * rng.standard_normal((HL, Wc, 3))
        x = solver.cell_solve(layer, cell, torch.from_numpy(g).cuda()).cpu().numpy()
        lu = spla.splu(C.H.tocsc())
        for bb in range(3):
            ref = lu.solve(g[:, :, bb].ravel()).reshape(HL, Wc)
            assert _rel(x[:, :, bb], ref) < 1e-11


def test_apply_layer(setup):
    c, omega, prob, solver, oracle = setup
    W = prob.W
    rng = np.random.default_rng(1)
    B = 2
    for layer in range(L):
        for side in (0, 1):
            if (side == 0 and layer == 0) or (side == 1 and layer == L - 1):
                continue
            _log(f"[apply_layer] layer={layer} side={side}")
            top = rng.standard_normal((2, W, B)) + 1j * rng.standard_normal((2, W, B)) if layer > 0 else None
            bot = rng.standard_normal((2, W, B)) + 1j * rng.standard_normal((2, W, B)) if layer < L - 1 else None
            out = solver.apply_layer(layer, None if top is None else torch.from_numpy(top).cuda(),
                                     None if bot is None else torch.from_numpy(bot).cuda(),
                                     side, B).cpu().numpy()
            for bb in range(B):
                ref = oracle.layer_op(layer, None if top is None else top[..., bb],
                                      None if bot is None else bot[..., bb],
                                      "top" if side == 0 else "bot")
                assert _rel(out[..., bb], ref) < 1e-11


def _rand_pol(K, W, B, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((4 * K * W, B)) + 1j * rng.standard_normal((4 * K * W, B))


def test_apply_sie_and_precond(setup):
    c, omega, prob, solver, oracle = setup
    K, W = L - 1, prob.W
    x = _rand_pol(K, W, 2, 2)
    _log("[apply_sie]")
    y = solver.apply_sie(torch.from_numpy(x).cuda()).cpu().numpy()
    for bb in range(2):
        ref = oracle.pack(*oracle.apply_M(*oracle.unpack(x[:, bb])))
        assert _rel(y[:, bb], ref) < 1e-11
    _log("[apply_precond]")
    y = solver.apply_precond(torch.from_numpy(x).cuda()).cpu().numpy()
    for bb in range(2):
        ref = oracle.pack(*oracle.precond_gs(*oracle.unpack(x[:, bb])))
        assert _rel(y[:, bb], ref) < 1e-11


def test_sie_rhs(setup):
    c, omega, prob, solver, oracle = setup
    f = media.point_sources(N, (10, 30), 20)
    f[1, 40, 5] = 3.0 - 1.0j
    _log("[sie_rhs]")
    y = solver.sie_rhs(torch.from_numpy(f)).cpu().numpy()
    for bb in range(2):
        ref = oracle.pack(*oracle.rhs(prob.extend(f[bb])))
        assert _rel(y[:, bb], ref) < 1e-11


def test_full_solve_fp64(setup):
    c, omega, prob, solver, oracle = setup
    f = media.point_sources(N, (24, 7, 40), 12)
    _log("[solve fp64] B=3")
    u = solver.solve(torch.from_numpy(f), tol=1e-12).cpu().numpy()
    lu = spla.splu(prob.H.tocsc())
    for bb in range(3):
        ref = prob.restrict(lu.solve(prob.extend(f[bb]).ravel()).reshape(prob.W, prob.W))
        err = _rel(u[bb], ref)
        _log(f"  rhs {bb}: iters={solver.last_stats[bb]['iters']} err={err:.2e}")
        assert err < 1e-9


def test_uncomposed_inner_solve(monkeypatch):
    """The same operators with the inner SIE solved by block LU substitutions
    at every application (HZ_COMPOSE=0), through the composed output
    operators everywhere (2), and with the per-job-set choice (1, the
    default: sweep steps composed, parallel batches where cheaper
    substituted): all match the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, omega = media.small_problem(N, P, L, LC, seed=5)
    prob = Problem(c, omega, P)
    oracle = LayeredSolver(prob, L)
    K, W = L - 1, prob.W
    x = _rand_pol(K, W, 2, 3)
    f = media.point_sources(N, (24, 7), 12)
    lu = spla.splu(prob.H.tocsc())
    for flag in ("0", "1", "2"):
        monkeypatch.setenv("HZ_COMPOSE", flag)
        _log(f"[compose={flag}] apply_sie / apply_precond / solve")
        s = hz.Solver(torch.from_numpy(c), omega, P, L, LC, max_batch=2)
        y = s.apply_sie(torch.from_numpy(x).cuda()).cpu().numpy()
        z = s.apply_precond(torch.from_numpy(x).cuda()).cpu().numpy()
        u = s.solve(torch.from_numpy(f), tol=1e-12).cpu().numpy()
        s.close()
        for bb in range(2):
            xs = oracle.unpack(x[:, bb])
            assert _rel(y[:, bb], oracle.pack(*oracle.apply_M(*xs))) < 1e-11
            assert _rel(z[:, bb], oracle.pack(*oracle.precond_gs(*xs))) < 1e-11
            ref = prob.restrict(lu.solve(prob.extend(f[bb]).ravel()).reshape(W, W))
            assert _rel(u[bb], ref) < 1e-9


def test_volume_residual_statistic(setup):
    """The per-RHS residual reported by the solve, |f - H u| / |f| over the
    extended grid, against the same norm computed on the CPU from the GPU's
    extended solution and the oracle's matrix."""
    c, omega, prob, solver, oracle = setup
    f = media.point_sources(N, (5, 33, 41), 30)
    _log("[vol_resid] B=3")
    u = solver.solve(torch.from_numpy(f), tol=1e-11, ext=True).cpu().numpy()
    for bb in range(3):
        fe = prob.extend(f[bb]).ravel()
        ref = np.linalg.norm(fe - prob.H @ u[bb].ravel()) / np.linalg.norm(fe)
        got = solver.last_stats[bb]["vol_resid"]
        _log(f"  rhs {bb}: gpu {got:.6e} cpu {ref:.6e}")
        assert abs(got - ref) <= 1e-2 * ref + 1e-15


def test_autotuned_kernels_same_solution(monkeypatch):
    """Solves with the autotuner on (GEMM kernels and cell-solve widths timed
    and picked per launch) and off (fixed heuristic) agree to rounding, and
    both match the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, omega = media.small_problem(N, P, L, LC, seed=5)
    prob = Problem(c, omega, P)
    xs = tuple(range(2, 42, 2))                       # 20 sources: matrix-core paths
    f = media.point_sources(N, xs, 17)
    out = {}
    for flag in ("0", "1"):
        monkeypatch.setenv("HZ_TUNE", flag)
        _log(f"[tune={flag}] B={len(xs)}")
        s = hz.Solver(torch.from_numpy(c), omega, P, L, LC, max_batch=len(xs))
        out[flag] = s.solve(torch.from_numpy(f), tol=1e-12).cpu().numpy()
        out[flag + "b"] = s.solve(torch.from_numpy(f), tol=1e-12).cpu().numpy()   # tuned plans reused
        s.close()
    assert _rel(out["1"], out["0"]) < 1e-11
    assert _rel(out["1b"], out["1"]) < 1e-13
    lu = spla.splu(prob.H.tocsc())
    for bb in (0, 9, 19):
        ref = prob.restrict(lu.solve(prob.extend(f[bb]).ravel()).reshape(prob.W, prob.W))
        assert _rel(out["1"][bb], ref) < 1e-9


def test_single_layer_and_cell_counts():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, omega = media.small_problem(31, 6, 1, 1, seed=9)
    prob = Problem(c, omega, 6)
    f = media.point_sources(31, (9,), 20)
    ref = prob.restrict(spla.splu(prob.H.tocsc()).solve(prob.extend(f[0]).ravel())
                        .reshape(prob.W, prob.W))
    for Lz, Lx in [(1, 1), (1, 3), (3, 1), (2, 2)]:
        _log(f"[solve] L={Lz} Lc={Lx}")
        s = hz.Solver(torch.from_numpy(c), omega, 6, Lz, Lx)
        u = s.solve(torch.from_numpy(f), tol=1e-12).cpu().numpy()[0]
        s.close()
        assert _rel(u, ref) < 1e-9


@pytest.mark.parametrize("kind", list(range(2, 19)))
def test_every_gemm_kernel(kind, monkeypatch):
    """Every matrix-core GEMM variant the autotuner may pick, forced for all
    launches of the FP64 and the mixed form, against the sparse direct solve."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, omega = media.small_problem(N, P, L, LC, seed=5)
    prob = Problem(c, omega, P)
    xs = tuple(range(1, 41))                          # 40 sources
    f = media.point_sources(N, xs, 17)
    lu = spla.splu(prob.H.tocsc())
    monkeypatch.setenv("HZ_GEMM_KIND", str(kind))
    for prec in (hz.HZ_FP64, hz.HZ_MIXED):
        _log(f"[gemm kind={kind}] precision={prec} B={len(xs)}")
        s = hz.Solver(torch.from_numpy(c), omega, P, L, LC, precision=prec, max_batch=len(xs))
        u = s.solve(torch.from_numpy(f), tol=1e-12 if prec == hz.HZ_FP64 else 1e-11).cpu().numpy()
        s.close()
        for bb in (0, 17, 39):
            ref = prob.restrict(lu.solve(prob.extend(f[bb]).ravel()).reshape(prob.W, prob.W))
            assert _rel(u[bb], ref) < 1e-9


@pytest.mark.parametrize("n,layers", [(60, 1), (100, 1), (124, 1), (140, 1), (160, 1)])
def test_tall_cells(n, layers):
    """Cells of height 72, 112, 136, 152 and 172 (padded to 80, 112, 144, 160
    and 176): the layouts of the register-resident cell factorisation (all
    columns in registers up to order 128, part of them in LDS up to 160) and
    the general Gauss-Jordan kernel beyond; for 136 and 152 the twelve-wave
    matrix-core cell solve (nine and ten row tiles, the last one or two
    shared by two waves), in the probes and, with 16 sources, in the batched
    volume solve."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, omega = media.small_problem(n, 6, layers, 2, seed=11)
    prob = Problem(c, omega, 6)
    lu = spla.splu(prob.H.tocsc())
    f = media.point_sources(n, (n // 3,), n // 2)
    ref = prob.restrict(lu.solve(prob.extend(f[0]).ravel()).reshape(prob.W, prob.W))
    _log(f"[solve] tall cells n={n} L={layers}")
    xs = tuple(int(v) for v in np.linspace(2, n - 1, 16).round())
    fb = media.point_sources(n, xs, n // 2 + 3)
    s = hz.Solver(torch.from_numpy(c), omega, 6, layers, 2, max_batch=16)
    u = s.solve(torch.from_numpy(f), tol=1e-12).cpu().numpy()[0]
    ub = s.solve(torch.from_numpy(fb), tol=1e-12).cpu().numpy()
    s.close()
    assert _rel(u, ref) < 1e-9
    for b in (0, 7, 15):
        rb = prob.restrict(lu.solve(prob.extend(fb[b]).ravel()).reshape(prob.W, prob.W))
        assert _rel(ub[b], rb) < 1e-9


def test_residual_kernel(setup):
    c, omega, prob, solver, oracle = setup
    rng = np.random.default_rng(3)
    W = prob.W
    u = rng.standard_normal((2, W, W)) + 1j * rng.standard_normal((2, W, W))
    f = rng.standard_normal((2, W, W)) + 1j * rng.standard_normal((2, W, W))
    _log("[residual]")
    r = solver.residual(torch.from_numpy(u).cuda(), torch.from_numpy(f).cuda()).cpu().numpy()
    ref = f - prob.apply(u)
    assert _rel(r, ref) < 1e-13


@pytest.mark.parametrize("prec,tol", [("mixed", 1e-11), ("refine", 1e-10)])
def test_mixed_precision_solve(prec, tol):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, omega = media.small_problem(N, P, L, LC, seed=5)
    prob = Problem(c, omega, P)
    f = media.point_sources(N, (24, 7), 12)
    _log(f"[solve {prec}] B=2")
    code = hz.HZ_MIXED if prec == "mixed" else hz.HZ_MIXED_REFINE
    s = hz.Solver(torch.from_numpy(c), omega, P, L, LC, precision=code, max_batch=2)
    u = s.solve(torch.from_numpy(f), tol=tol).cpu().numpy()
    lu = spla.splu(prob.H.tocsc())
    for bb in range(2):
        ref = prob.restrict(lu.solve(prob.extend(f[bb]).ravel()).reshape(prob.W, prob.W))
        err = _rel(u[bb], ref)
        _log(f"  rhs {bb}: refine={s.last_stats[bb]['refine_steps']} err={err:.2e}")
        assert err < 1e-8
    s.close()


def test_adjoint_solve(setup):
    c, omega, prob, solver, oracle = setup
    rng = np.random.default_rng(8)
    f = rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))
    _log("[adjoint]")
    lam = solver.adjoint(torch.from_numpy(f), tol=1e-12).cpu().numpy()
    lu = spla.splu(prob.H.tocsc())
    for bb in range(2):
        # H^H lam = f
        ref = prob.restrict(np.conj(lu.solve(np.conj(prob.extend(f[bb]).ravel())))
                            .reshape(prob.W, prob.W))
        assert _rel(lam[bb], ref) < 1e-9


def test_misfit_gradient_vs_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import forms

    n, p = 31, 8
    omega = media.omega_ppw(2.0, n, 8.0)
    true_c = media.gaussian_bump(n, 2.0, 0.4, 2 * 0.12 ** 2)
    f = media.point_sources(n, (6, 16, 26), 4)
    ref = forms.Misfit(omega, p, f, rec_row=4)
    prob, lu, U = ref.forward(1.0 / true_c ** 2)
    d_obs = ref.record(prob, U)
    mis = forms.Misfit(omega, p, f, rec_row=4, d_obs=d_obs)
    m0 = np.full((n, n), 0.25) + 0.01 * np.random.default_rng(0).standard_normal((n, n))
    J_ref, g_ref = mis.value_and_grad(m0)
    _log("[gradient]")
    s = hz.Solver(torch.from_numpy(m0), omega, p, 3, 2, model_kind=hz.HZ_MODEL_SLOWNESS2,
                  max_batch=3)
    u = s.solve(torch.from_numpy(f), tol=1e-13, ext=True)
    J, adj = s.misfit(u, torch.from_numpy(d_obs), 4)
    lam = s.adjoint(adj, tol=1e-13, ext=True)
    g = s.misfit_gradient(u, lam).cpu().numpy()
    s.close()
    assert abs(J - J_ref) <= 1e-9 * J_ref
    assert _rel(g, g_ref) < 1e-8


def test_batched_paths_match_oracle():
    """Batches that select the matrix-core kernels (16 <= B < 64 and B >= 64)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, omega = media.small_problem(N, P, L, LC, seed=5)
    prob = Problem(c, omega, P)
    oracle = LayeredSolver(prob, L)
    s = hz.Solver(torch.from_numpy(c), omega, P, L, LC, max_batch=70)
    rng = np.random.default_rng(12)
    # cell solve with 20 and 40 right-hand sides
    for B in (20, 40):
        _log(f"[batched cell_solve] B={B}")
        HL, Wc = s.cell_shape(2, 1)
        C = CellGrid(oracle.grids[2], 17, 32, 1, LC)
        g = rng.standard_normal((HL, Wc, B)) + 1j * rng.standard_normal((HL, Wc, B))
        x = s.cell_solve(2, 1, torch.from_numpy(g).cuda()).cpu().numpy()
        lu = spla.splu(C.H.tocsc())
        ref = lu.solve(g.reshape(HL * Wc, B)).reshape(HL, Wc, B)
        assert _rel(x, ref) < 1e-11
    # M and P^GS on 20 vectors
    K, W = L - 1, prob.W
    x = _rand_pol(K, W, 20, 4)
    _log("[batched apply_sie / precond] B=20")
    y = s.apply_sie(torch.from_numpy(x).cuda()).cpu().numpy()
    z = s.apply_precond(torch.from_numpy(x).cuda()).cpu().numpy()
    for bb in (0, 7, 19):
        assert _rel(y[:, bb], oracle.pack(*oracle.apply_M(*oracle.unpack(x[:, bb])))) < 1e-11
        assert _rel(z[:, bb], oracle.pack(*oracle.precond_gs(*oracle.unpack(x[:, bb])))) < 1e-11
    # full solves with 70 sources (a row of sources and a few scattered ones)
    _log("[batched solve] B=70")
    xs = tuple(int(v) for v in np.linspace(1, N, 64).round())
    f = np.concatenate([media.point_sources(N, xs, 9),
                        media.point_sources(N, (3, 11, 19, 27, 35, 43), 40)])
    u = s.solve(torch.from_numpy(f), tol=1e-12).cpu().numpy()
    F = np.stack([prob.extend(fi).ravel() for fi in f], axis=1)
    U = spla.splu(prob.H.tocsc()).solve(F).T.reshape(-1, prob.W, prob.W)
    errs = [_rel(u[b], prob.restrict(U[b])) for b in range(len(f))]
    _log(f"  max err {max(errs):.2e}")
    assert max(errs) < 1e-9
    s.close()
