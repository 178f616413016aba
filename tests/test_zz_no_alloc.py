"""The allocation-free misfit entry point (hz_misfit_noalloc) against
hz_misfit on the same inputs: two calls in a row on one context, the second
with a smaller batch, each compared with the allocating entry point."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1510_01831_amd import hz, media  # noqa: E402


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_misfit_noalloc_matches_misfit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n, p, L, Lc = 47, 8, 3, 2
    c, omega = media.small_problem(n, p, L, Lc, seed=11)
    xs = (5, 17, 29, 41)
    f = torch.from_numpy(media.point_sources(n, xs, 9))
    s = hz.Solver(torch.from_numpy(c), omega, p, L, Lc, max_batch=len(xs))
    u_ext = s.solve(f, tol=1e-12, ext=True)
    rng = np.random.default_rng(4)
    rec_row = 9
    for B in (4, 2):                           # second call: smaller input
        _log(f"[no_alloc] B={B} n={n} rec_row={rec_row}")
        d = rng.standard_normal((B, n)) + 1j * rng.standard_normal((B, n))
        d_obs = torch.from_numpy(d).cuda()
        ue = u_ext[:B].contiguous()
        J_ref, adj_ref = s.misfit(ue, d_obs, rec_row)
        adj = torch.full((B, n, n), float("nan"), dtype=torch.complex128, device="cuda")
        J = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
        s.misfit_noalloc(ue, d_obs, rec_row, adj, J)
        torch.cuda.synchronize()
        Jv = float(J.item())
        _log(f"  J = {Jv!r}, hz_misfit J = {J_ref!r}")
        assert torch.equal(adj, adj_ref)
        assert Jv == J_ref
        assert J_ref > 0.0
    # argument checks of the new entry point
    adj = torch.empty((2, n, n), dtype=torch.complex128, device="cuda")
    J = torch.empty((), dtype=torch.float64, device="cuda")
    with pytest.raises(hz.HzError) as e:
        s.misfit_noalloc(u_ext[:2].contiguous(), torch.zeros((2, n), dtype=torch.complex128,
                                                             device="cuda"), n + 1, adj, J)
    assert e.value.status == hz.HZ_EINVAL
    s.close()
