"""GPU parity of the partitioned low-rank (PLR) preconditioner operators
(eq. factorization and its PLR footnote; eps of the caption of Fig. 9):
single-right-hand-side solves whose Gauss-Seidel sweeps apply the
compressed operators, against the oracle."""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.discretization import Problem  # noqa: E402
from oracle.polarized import LayeredSolver  # noqa: E402
from paper_1510_01831_amd import hz, media  # noqa: E402

N, P, L, LC = 95, 12, 4, 3


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def small():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, omega = media.small_problem(N, P, L, LC, seed=6)
    prob = Problem(c, omega, P)
    lu = spla.splu(prob.H.tocsc())
    return c, omega, prob, lu


@pytest.mark.parametrize("tune", ["1", "0"])
@pytest.mark.parametrize("prec,bar", [(hz.HZ_FP64, 1e-9), (hz.HZ_MIXED, 1e-8)])
def test_plr_single_rhs_solve(small, prec, bar, tune, monkeypatch):
    """Solves with the compressed preconditioner (eps = 1e-8) against the
    direct solve, the same iteration count as the dense preconditioner
    (within one), and compressed storage below the dense size.  With the
    autotuner off every preconditioner launch applies the compressed form;
    with it on each launch keeps the faster of compressed and dense."""
    monkeypatch.setenv("HZ_TUNE", tune)
    c, omega, prob, lu = small
    f = media.point_sources(N, (40,), 20)
    ref = prob.restrict(lu.solve(prob.extend(f[0]).ravel()).reshape(prob.W, prob.W))
    tol = 1e-12 if prec == hz.HZ_FP64 else 1e-11
    _log(f"[plr] n={N} L={L} Lc={LC} precision={prec}")
    sd = hz.Solver(torch.from_numpy(c), omega, P, L, LC, precision=prec)
    ud = sd.solve(torch.from_numpy(f), tol=tol).cpu().numpy()[0]
    it_dense = sd.last_stats[0]["iters"]
    sd.close()
    s = hz.Solver(torch.from_numpy(c), omega, P, L, LC, precision=prec, plr=1, plr_eps=1e-8)
    u = s.solve(torch.from_numpy(f), tol=tol).cpu().numpy()[0]
    it = s.last_stats[0]["iters"]
    info = s.info
    s.close()
    ratio = info.plr_bytes / info.plr_dense_bytes
    _log(f"  err {_rel(u, ref):.2e} (dense {_rel(ud, ref):.2e}), iterations {it} (dense "
         f"{it_dense}), stored {ratio:.3f} of dense")
    assert _rel(u, ref) <= bar
    assert abs(it - it_dense) <= 1
    assert 0 < info.plr_bytes < info.plr_dense_bytes


def test_plr_preconditioner_against_oracle(small, monkeypatch):
    """P^GS applied with the compressed operators (B = 1) against the
    oracle's exact P^GS: the difference is of the order of the compression
    accuracy (each of the 3(L-1) - 2 Green's-integral applications errs by
    at most eps relative in the Frobenius norm).  The autotuner is off, so
    every launch applies the compressed form."""
    monkeypatch.setenv("HZ_TUNE", "0")
    c, omega, prob, lu = small
    s = hz.Solver(torch.from_numpy(c), omega, P, L, LC, plr=1, plr_eps=1e-8)
    oracle = LayeredSolver(prob, L, LC)
    K = L - 1
    W = prob.W
    rng = np.random.default_rng(3)
    v = rng.standard_normal((2 * K, 2, W)) + 1j * rng.standard_normal((2 * K, 2, W))
    y = s.apply_precond(torch.from_numpy(v.reshape(-1, 1)).cuda()).cpu().numpy().reshape(2 * K, 2, W)
    s.close()
    xd, xq = oracle.precond_gs(v[:K], v[K:])
    ref = np.concatenate([xd, xq])
    err = _rel(y, ref)
    _log(f"[plr] P^GS vs exact oracle: {err:.2e}")
    assert err <= 1e-6
    # the compressed form was applied: its error is far above the rounding
    # level of the dense operators (about 1e-14 here)
    assert err > 1e-11


def test_plr_rejects_iterated_inner_solver():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c, omega = media.small_problem(47, 8, 2, 2, seed=1)
    with pytest.raises(hz.HzError) as e:
        hz.Solver(torch.from_numpy(c), omega, 8, 2, 2, inner=hz.HZ_INNER_PT, plr=1)
    assert e.value.status == hz.HZ_EINVAL
