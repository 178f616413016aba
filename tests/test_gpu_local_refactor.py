"""Local re-factorisation after a local model update (the inversion-loop use
of the conclusion, Sec. 6): only the cells whose local operators change are
refactored, and the solver then gives the solution of a fresh factorisation
of the new model, which is itself checked against a sparse direct solve."""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.discretization import Problem  # noqa: E402
from paper_1510_01831_amd import hz, media  # noqa: E402

N, P, L, LC = 63, 8, 4, 3


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _models():
    c0, omega = media.small_problem(N, P, L, LC, seed=21)
    c1 = c0.copy()
    c1[8:12, 8:12] *= 1.05            # a local update near the top-left corner
    return c0, c1, omega


@pytest.mark.parametrize("prec,tol", [(hz.HZ_FP64, 1e-12), (hz.HZ_MIXED, 1e-11)])
def test_local_update_equals_fresh_factorisation(prec, tol):
    _need_gpu()
    c0, c1, omega = _models()
    f = torch.from_numpy(media.point_sources(N, (20, 40), 30))
    _log(f"[local] n={N} L={L} Lc={LC} precision={prec}")
    sa = hz.Solver(torch.from_numpy(c0), omega, P, L, LC, precision=prec, max_batch=2)
    ua0 = sa.solve(f, tol=tol).cpu().numpy()
    redone = sa.update_model_local(torch.from_numpy(c1))
    ua = sa.solve(f, tol=tol).cpu().numpy()
    sb = hz.Solver(torch.from_numpy(c1), omega, P, L, LC, precision=prec, max_batch=2)
    ub = sb.solve(f, tol=tol).cpu().numpy()
    sa.close()
    sb.close()
    # the change touches the extended grids of the two top-left cells only
    assert redone == 2
    # same operators; the autotuner may pick other kernel variants for the two
    # contexts, so agreement is to the solve tolerance rather than bitwise
    assert np.linalg.norm(ua - ub) / np.linalg.norm(ub) < 10 * tol
    assert np.linalg.norm(ua - ua0) > 1e-6 * np.linalg.norm(ua)
    prob = Problem(c1, omega, P)
    ref = prob.restrict(spla.splu(prob.H.tocsc()).solve(prob.extend(f[0].numpy()).ravel())
                        .reshape(prob.W, prob.W))
    bar = 1e-9 if prec == hz.HZ_FP64 else 1e-8
    assert np.linalg.norm(ua[0] - ref) / np.linalg.norm(ref) < bar


def test_local_update_refine_form_and_errors():
    _need_gpu()
    c0, c1, omega = _models()
    f = torch.from_numpy(media.point_sources(N, (20,), 30))
    _log("[local] refine form, error paths")
    s = hz.Solver(torch.from_numpy(c0), omega, P, L, LC, precision=hz.HZ_MIXED_REFINE,
                  max_batch=1)
    assert s.update_model_local(torch.from_numpy(c1)) == 2        # complex64 operators kept
    u = s.solve(f, tol=1e-8).cpu().numpy()
    sb = hz.Solver(torch.from_numpy(c1), omega, P, L, LC, precision=hz.HZ_MIXED_REFINE,
                   max_batch=1)
    ub = sb.solve(f, tol=1e-8).cpu().numpy()
    assert np.linalg.norm(u - ub) / np.linalg.norm(ub) < 1e-7
    sb.close()
    bad = c1.copy()
    bad[30, 30] = np.nan
    with pytest.raises(hz.HzError) as e:
        s.update_model_local(torch.from_numpy(bad))
    assert e.value.status == hz.HZ_EINVAL
    u2 = s.solve(f, tol=1e-8).cpu().numpy()              # rejected model: context unchanged
    assert np.linalg.norm(u2 - u) / np.linalg.norm(u) < 1e-7
    s.close()
    s = hz.Solver(torch.from_numpy(c0), omega, P, L, LC, max_batch=1, factor=False)
    with pytest.raises(hz.HzError) as e:                  # not factored yet
        s.update_model_local(torch.from_numpy(c1))
    assert e.value.status == hz.HZ_ESTATE
    s.close()
