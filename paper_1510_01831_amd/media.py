"""Seeded synthetic workloads: velocity models, point sources and receivers.

This module only *generates inputs*.  It holds none of the solver's
arithmetic, so both the CPU oracle (``oracle/``) and the GPU path may import
it.  Every random draw comes from ``numpy.random.default_rng(seed)``.

Geometry (the paper's setting, Sec. 2 and App. A): the physical domain is the
unit square, ``n`` interior nodes per side, ``h = 1/(n+1)``, node ``(p, q)`` sits
at ``x = p h`` (lateral) and ``z = q h`` (depth, pointing down).  Arrays are
stored ``c[q-1, p-1]`` -- depth rows, x fastest -- matching the ordering of the
unknowns row by row in depth (Sec. 2.1).

The five workloads stand in for the paper's BP2004 / Marmousi2 runs (Sec. 5),
which use public velocity models that are not available here: the same kind of
high-contrast media, 10 points per wavelength, sources near the top, and a
layer x cell decomposition that grows with ``n``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int                 # physical nodes per side
    n_pml: int             # PML nodes per side
    omega: float           # angular frequency
    layers: int            # L
    cells: int             # L_c
    tol: float             # GMRES tolerance (preconditioned relative residual)
    src_x: tuple           # source node indices p (1-based)
    src_z: int             # source depth node index q (1-based)
    pml_beta: float = 2.0  # sigma_max = beta * omega at the Dirichlet node
    seed: int = 0

    @property
    def h(self) -> float:
        return 1.0 / (self.n + 1)

    @property
    def n_rhs(self) -> int:
        return len(self.src_x)


def nearest_node(y: float, n: int) -> int:
    """Nearest grid node (1-based) to coordinate ``y`` in [0,1], rounding half up."""
    return int(math.floor(y * (n + 1) + 0.5))


def equally_spaced_nodes(count: int, n: int) -> tuple:
    """``count`` sources at x_k = (k + 1/2)/count, snapped to the nearest node."""
    return tuple(nearest_node((k + 0.5) / count, n) for k in range(count))


def omega_ppw(c_min: float, n: int, ppw: float = 10.0) -> float:
    """Frequency giving ``ppw`` points per wavelength at speed ``c_min``."""
    return 2.0 * math.pi * c_min * (n + 1) / ppw


# ---------------------------------------------------------------------------
# velocity models
# ---------------------------------------------------------------------------

def _coords(n: int):
    h = 1.0 / (n + 1)
    t = np.arange(1, n + 1) * h
    z, x = np.meshgrid(t, t, indexing="ij")     # c[z_index, x_index]
    return x, z


def gaussian_bump(n: int, c0: float, amp: float, width2: float,
                  centre=(0.5, 0.5)) -> np.ndarray:
    """c = c0 + amp * exp(-|x - centre|^2 / width2)."""
    x, z = _coords(n)
    r2 = (x - centre[0]) ** 2 + (z - centre[1]) ** 2
    return c0 + amp * np.exp(-r2 / width2)


def gaussian_random_field(n: int, corr_len: float, cmin: float, cmax: float,
                          seed: int = 0) -> np.ndarray:
    """White noise convolved (zero-padded FFT) with a Gaussian kernel.

    The kernel has standard deviation ``corr_len/sqrt(2)`` so that the field's
    covariance is ``exp(-r^2 / (2 corr_len^2))``; the result is min-max
    rescaled to ``[cmin, cmax]``.
    """
    from scipy.signal import fftconvolve

    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n))
    sig = (corr_len / math.sqrt(2.0)) * (n + 1)          # in grid units
    r = int(math.ceil(4.0 * sig))
    t = np.arange(-r, r + 1, dtype=float)
    k1 = np.exp(-0.5 * (t / sig) ** 2)
    field = fftconvolve(noise, np.outer(k1, k1), mode="same")
    lo, hi = field.min(), field.max()
    return cmin + (cmax - cmin) * (field - lo) / (hi - lo)


def layered_medium(n: int, seed: int = 0) -> np.ndarray:
    """Depth gradient + 12 random layers + two dipping interfaces, smoothed.

    c0 = 1.5 + 3.0 z; 11 sorted uniform depths split the column into 12
    layers with offsets U(-0.5, 0.5); two planar interfaces
    z = z_i + x tan(theta_i), theta_i ~ U(-20, 20) degrees, add a jump
    U(-0.5, 0.5) below them; a 3-node boxcar smooths every discontinuity and
    the result is clipped to [1.5, 4.5].
    """
    from scipy.ndimage import uniform_filter

    rng = np.random.default_rng(seed)
    x, z = _coords(n)
    depths = np.sort(rng.uniform(0.0, 1.0, 11))
    offsets = rng.uniform(-0.5, 0.5, 12)
    c = 1.5 + 3.0 * z + offsets[np.searchsorted(depths, z)]
    for _ in range(2):
        z0 = rng.uniform(0.2, 0.8)
        theta = math.radians(rng.uniform(-20.0, 20.0))
        jump = rng.uniform(-0.5, 0.5)
        c = c + jump * (z > z0 + x * math.tan(theta))
    c = uniform_filter(c, size=3, mode="nearest")
    return np.clip(c, 1.5, 4.5)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def workload(name: str) -> Workload:
    if name == "C1":
        n = 127
        return Workload("C1", n, 16, 2.0 * math.pi * n / 10.0, 4, 2, 1e-10,
                        (nearest_node(0.5, n),), nearest_node(0.15, n))
    if name in ("C2", "C3"):
        n = 1023
        src = (nearest_node(0.5, n),) if name == "C2" else equally_spaced_nodes(256, n)
        return Workload(name, n, 32, omega_ppw(1.5, n), 16, 4, 1e-10,
                        src, nearest_node(0.1, n))
    if name == "C4":
        n = 2047
        return Workload("C4", n, 48, omega_ppw(1.5, n), 32, 8, 1e-10,
                        equally_spaced_nodes(64, n), nearest_node(0.08, n))
    if name == "C5":
        n = 511
        return Workload("C5", n, 24, omega_ppw(2.0, n), 8, 4, 1e-13,
                        equally_spaced_nodes(32, n), nearest_node(0.05, n))
    raise KeyError(name)


def velocity(name: str, which: str = "true") -> np.ndarray:
    """Velocity model c[n, n] (float64) of a workload."""
    w = workload(name)
    if name == "C1":
        return gaussian_bump(w.n, 1.0, 0.3, 0.02)
    if name in ("C2", "C3"):
        return gaussian_random_field(w.n, 0.05, 1.5, 3.0, seed=0)
    if name == "C4":
        return layered_medium(w.n, seed=0)
    if name == "C5":
        if which == "start":
            return np.full((w.n, w.n), 2.0)
        return gaussian_bump(w.n, 2.0, 0.4, 2.0 * 0.08 ** 2)
    raise KeyError(name)


def point_sources(n: int, src_x, src_z: int, dtype=np.complex128) -> np.ndarray:
    """Right-hand sides f[B, n, n]: the discrete delta 1/h^2 at each source node
    (the paper's normalisation of a point source on the grid, Sec. 2.1)."""
    h = 1.0 / (n + 1)
    f = np.zeros((len(src_x), n, n), dtype=dtype)
    for b, px in enumerate(src_x):
        f[b, src_z - 1, px - 1] = 1.0 / (h * h)
    return f


def random_directions(n: int, count: int, seed: int = 0) -> np.ndarray:
    """i.i.d. N(0,1) perturbation directions of m on the physical grid."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((count, n, n))


def small_problem(n: int, n_pml: int, layers: int, cells: int, seed: int = 1,
                  ppw: float = 10.0, contrast: float = 0.3):
    """A tiny randomised medium used by unit tests (smooth bump + noise)."""
    rng = np.random.default_rng(seed)
    c = gaussian_bump(n, 1.0, contrast, 0.03, centre=(rng.uniform(0.3, 0.7),
                                                      rng.uniform(0.3, 0.7)))
    c = c + 0.05 * rng.uniform(-1, 1, size=(n, n))
    omega = omega_ppw(float(c.min()), n, ppw)
    return c, omega
