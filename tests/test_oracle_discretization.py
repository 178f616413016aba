"""Pins of the oracle's discretisation (App. A) against closed forms and
library routines that share none of its code."""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.special import hankel1

from oracle.discretization import Problem, partition
from paper_1510_01831_amd import media


def _alpha_app_a(x, omega, delta, C):
    """alpha = 1/(1 + i sigma/omega) with the quadratic sigma of App. A, written
    in physical coordinates on the unit interval (independent of the oracle)."""
    sig = np.where(x < 0, (C / delta) * (x / delta) ** 2,
                   np.where(x > 1, (C / delta) * ((x - 1) / delta) ** 2, 0.0))
    return 1.0 / (1.0 + 1j * sig / omega)


def _row_form_1d(n, p, omega, beta):
    """1D operator -alpha d/dx(alpha d/dx) of App. A on the extended axis."""
    h = 1.0 / (n + 1)
    delta = p * h
    C = beta * omega * delta
    x = np.arange(-p + 1, n + p + 1) * h
    a = _alpha_app_a(x, omega, delta, C)
    ap = _alpha_app_a(x + h / 2, omega, delta, C)
    am = _alpha_app_a(x - h / 2, omega, delta, C)
    W = x.size
    A = np.zeros((W, W), dtype=complex)
    for i in range(W):
        A[i, i] = a[i] * (ap[i] + am[i]) / h ** 2
        if i + 1 < W:
            A[i, i + 1] = -a[i] * ap[i] / h ** 2
        if i > 0:
            A[i, i - 1] = -a[i] * am[i] / h ** 2
    return A


def test_partition_rule():
    assert partition(127, 4) == [(1, 32), (33, 64), (65, 96), (97, 127)]
    assert [b - a + 1 for a, b in partition(1023, 16)] == [64] * 15 + [63]
    with pytest.raises(ValueError):
        partition(3, 4)


def test_dst_closed_form_no_pml():
    """n_pml = 0, constant m: H is diagonalised by the 2D DST-I."""
    n = 31
    c = np.full((n, n), 1.3)
    omega = 17.0
    prob = Problem(c, omega, 0)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    u = spla.spsolve(prob.H.tocsc(), prob.extend(f).ravel()).reshape(n, n)
    h = prob.h
    k = np.arange(1, n + 1)
    s2 = np.sin(np.pi * k / (2 * (n + 1))) ** 2
    lam = (4 / h ** 2) * (s2[:, None] + s2[None, :]) - omega ** 2 / 1.3 ** 2
    fr = scipy.fft.dstn(f.real, type=1) + 1j * scipy.fft.dstn(f.imag, type=1)
    v = fr / lam
    ud = scipy.fft.idstn(v.real, type=1) + 1j * scipy.fft.idstn(v.imag, type=1)
    assert np.abs(u - ud).max() / np.abs(ud).max() < 1e-12


@pytest.mark.parametrize("layered", [False, True])
def test_separable_pml_closed_form(layered):
    """Constant (or depth-only) m with PML: the row form of App. A is
    A_x (x) I + I (x) A_z - omega^2 m, solved mode by mode."""
    n, p, beta = 23, 6, 2.0
    omega = 2 * math.pi * 3.0
    zc = np.linspace(1.0, 1.6, n) if layered else np.full(n, 1.2)
    c = np.repeat(zc[:, None], n, axis=1)
    prob = Problem(c, omega, p, beta)
    rng = np.random.default_rng(5)
    f = np.zeros((n, n), dtype=complex)
    f[rng.integers(0, n, 4), rng.integers(0, n, 4)] = rng.standard_normal(4)
    u = spla.spsolve(prob.H.tocsc(), prob.extend(f).ravel()).reshape(prob.W, prob.W)
    A = _row_form_1d(n, p, omega, beta)
    lam, V = np.linalg.eig(A)
    Vi = np.linalg.inv(V)
    F = prob.extend(f)                               # alpha_x alpha_z f = f (physical support)
    Fh = F @ Vi.T                                    # transform along x
    m_ext = 1.0 / np.clip(np.concatenate([np.full(p, zc[0]), zc, np.full(p, zc[-1])]), 0, None) ** 2
    U = np.zeros_like(Fh)
    for j in range(prob.W):                          # tridiagonal solve in z per x-mode
        K = A + np.diag(lam[j] - omega ** 2 * m_ext)
        U[:, j] = np.linalg.solve(K, Fh[:, j])
    ud = U @ V.T
    assert np.abs(u - ud).max() / np.abs(ud).max() < 1e-10


def test_manufactured_solution_second_order():
    """Interior rows are the 5-point Laplacian minus omega^2 m u: O(h^2)."""
    errs = []
    for n in (31, 63, 127):
        h = 1.0 / (n + 1)
        t = np.arange(1, n + 1) * h
        z, x = np.meshgrid(t, t, indexing="ij")
        c = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.cos(np.pi * z)
        m = 1.0 / c ** 2
        omega = 9.0
        u = np.sin(np.pi * x) * np.sin(2 * np.pi * z)
        exact = (5 * np.pi ** 2 - omega ** 2 * m) * u
        prob = Problem(c, omega, 0)
        Hu = (prob.H @ u.ravel()).reshape(n, n)
        errs.append(np.sqrt(np.mean(np.abs(Hu - exact) ** 2)))
    assert errs[0] / errs[1] > 3.7 and errs[1] / errs[2] > 3.7


def test_symmetry_and_reciprocity():
    c, omega = media.small_problem(31, 8, 1, 1, seed=2)
    prob = Problem(c, omega, 8)
    H = prob.H
    assert abs(H - H.T).max() == 0.0
    lu = spla.splu(H.tocsc())
    W = prob.W
    i = (8 + 5) * W + (8 + 20)
    j = (8 + 24) * W + (8 + 3)
    ei = np.zeros(W * W, complex); ei[i] = 1
    ej = np.zeros(W * W, complex); ej[j] = 1
    ui, uj = lu.solve(ei), lu.solve(ej)
    assert abs(ui[j] - uj[i]) <= 1e-12 * abs(ui[j])


def test_row_form_relation():
    """Dividing App. A's row form by alpha_x alpha_z gives the oracle's H."""
    n, p, omega = 15, 5, 20.0
    c = np.full((n, n), 1.1)
    prob = Problem(c, omega, p)
    A = _row_form_1d(n, p, omega, 2.0)
    I = np.eye(prob.W)
    Hrow = np.kron(I, A) + np.kron(A, I) - omega ** 2 / 1.1 ** 2 * np.eye(prob.W ** 2)
    h = prob.h
    x = np.arange(-p + 1, n + p + 1) * h
    a = _alpha_app_a(x, omega, p * h, 2.0 * omega * p * h)
    D = np.outer(a, a).ravel()
    assert np.abs(Hrow / D[:, None] - prob.H.toarray()).max() < 1e-9 * np.abs(Hrow).max()


@pytest.mark.slow
def test_hankel_convergence():
    """Constant medium: the discrete point-source response approaches the
    free-space Green's function (i/4) H0^(1)(omega r) at second order."""
    omega = 2 * math.pi * 4.0
    errs = []
    for n in (63, 127, 255):
        h = 1.0 / (n + 1)
        p = int(round(0.25 / h))
        prob = Problem(np.ones((n, n)), omega, p, beta=2.0)
        f = media.point_sources(n, ((n + 1) // 2,), (n + 1) // 2)[0]
        u = spla.splu(prob.H.tocsc()).solve(prob.extend(f).ravel()).reshape(prob.W, prob.W)
        u = prob.restrict(u)
        t = np.arange(1, n + 1) * h
        z, x = np.meshgrid(t, t, indexing="ij")
        r = np.hypot(x - 0.5, z - 0.5)
        mask = r >= 0.1
        g = 0.25j * hankel1(0, omega * r[mask])
        errs.append(np.linalg.norm(u[mask] - g) / np.linalg.norm(g))
    assert errs[2] < 0.05
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_workload_sources():
    w = media.workload("C1")
    assert (w.src_x, w.src_z) == ((64,), 19)
    assert abs(w.omega - 79.796) < 1e-3
    w3 = media.workload("C3")
    assert w3.src_x == tuple(4 * k + 2 for k in range(256)) and w3.src_z == 102
    assert abs(w3.omega - 965.097) < 1e-2
    w4 = media.workload("C4")
    assert w4.src_x == tuple(32 * k + 16 for k in range(64)) and w4.src_z == 164
    w5 = media.workload("C5")
    assert w5.src_x == tuple(16 * k + 8 for k in range(32)) and w5.src_z == 26
    c = media.velocity("C2")
    assert c.shape == (1023, 1023) and abs(c.min() - 1.5) < 1e-12 and abs(c.max() - 3.0) < 1e-12
