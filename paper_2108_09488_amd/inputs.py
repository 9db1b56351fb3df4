"""Seeded synthetic inputs for the plume problems (shared by the HIP path's tests,
the oracle's tests and the benchmark).

This module holds no arithmetic of the SPH method itself: it only draws particle
lattices, the initial Gaussian plume of the test model (Eq. 11, image-summed over
the periodic box of Section 3), sensor points and ensemble parameters.

Positions are returned as float64 arrays whose values are exact multiples of
L / 2**32, so that the library's fixed-point position format (one uint32 per
coordinate over the periodic side L) represents them without rounding.

Random numbers come from SplitMix64 (Steele, Lea & Flood 2014, the finaliser
published with it), used as a counter-based generator: the value for a counter
c under a key k is mix(k + (c + 1) * GOLDEN).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 210809488
GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
TWO32 = 4294967296.0


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    """Key of an independent stream (e.g. one plume) under a base seed."""
    with np.errstate(over="ignore"):
        k = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + GOLDEN * np.uint64(stream + 1)
    return _mix(np.array([k], dtype=np.uint64))[0]


def uniform01(key: np.uint64, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) for the given uint64 counters (53-bit mantissa)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _mix(key + (c + np.uint64(1)) * GOLDEN)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def quantize(x: np.ndarray, L: float) -> np.ndarray:
    """Round positions to the nearest multiple of L/2**32 inside [0, L)."""
    u = np.rint(np.asarray(x, dtype=np.float64) / L * TWO32)
    u = np.mod(u, TWO32)
    return u * (L / TWO32)


def lattice(n_side: int, dim: int, L: float = 1.0, jitter: float = 0.0,
            seed: int = BASE_SEED, stream: int = 0) -> np.ndarray:
    """Cell-centred lattice of n_side**dim particles, SoA float64 array (dim, N).

    Particle a = (i, j[, k]) with x fastest sits at ((i + 1/2) dp, (j + 1/2) dp, ...),
    dp = L / n_side, then moves by U[-jitter*dp, +jitter*dp) per component, and is
    wrapped into [0, L) and rounded to the L/2**32 grid.
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    dp = L / n_side
    idx = np.indices((n_side,) * dim, dtype=np.float64)  # idx[0] slowest
    comps = [idx[dim - 1 - c].reshape(-1) for c in range(dim)]  # x fastest
    n = n_side ** dim
    x = np.empty((dim, n), dtype=np.float64)
    key = stream_key(seed, stream)
    for c in range(dim):
        xc = (comps[c] + 0.5) * dp
        if jitter:
            cnt = np.arange(n, dtype=np.uint64) * np.uint64(dim) + np.uint64(c)
            xc = xc + (2.0 * uniform01(key, cnt) - 1.0) * (jitter * dp)
        x[c] = quantize(np.mod(xc, L), L)
    return x


def clustered(n_side: int, dim: int, copies: int, spread: float, L: float = 1.0,
              seed: int = BASE_SEED, stream: int = 0) -> np.ndarray:
    """Crowded particles: every site of the cell-centred n_side**dim lattice
    holds `copies` particles, each moved by U[-spread*dp, +spread*dp) per
    component (site-major order), wrapped and rounded to the L/2**32 grid."""
    sites = lattice(n_side, dim, L, 0.0, seed, stream)
    dp = L / n_side
    n = sites.shape[1] * copies
    key = stream_key(seed, stream + 1)
    x = np.empty((dim, n), dtype=np.float64)
    for c in range(dim):
        cnt = np.arange(n, dtype=np.uint64) * np.uint64(dim) + np.uint64(c)
        off = (2.0 * uniform01(key, cnt) - 1.0) * (spread * dp)
        x[c] = quantize(np.mod(np.repeat(sites[c], copies) + off, L), L)
    return x


def gaussian_plume(x: np.ndarray, centre, sigma0: float, L: float = 1.0,
                   C0: float = 1.0) -> np.ndarray:
    """Initial plume C = C0 sum_images exp(-|x - x0 - image|^2 / (2 sigma0^2))
    over the 3**dim periodic images (Eq. 11 on the periodic box)."""
    dim = x.shape[0]
    C = np.zeros(x.shape[1], dtype=np.float64)
    shifts = np.array(np.meshgrid(*([[-L, 0.0, L]] * dim), indexing="ij")).reshape(dim, -1).T
    for s in shifts:
        d2 = np.zeros(x.shape[1])
        for c in range(dim):
            d = x[c] - centre[c] - s[c]
            d2 += d * d
        C += np.exp(-d2 / (2.0 * sigma0 * sigma0))
    return C0 * C


def sensors(n_sensors: int, lo, hi, seed: int = BASE_SEED, stream: int = 7777,
            L: float = 1.0) -> np.ndarray:
    """Uniform random sensor points in the box [lo, hi] (dim, S), float64,
    rounded to the L/2**32 position grid."""
    dim = len(lo)
    key = stream_key(seed, stream)
    out = np.empty((dim, n_sensors))
    for c in range(dim):
        cnt = np.arange(n_sensors, dtype=np.uint64) * np.uint64(dim) + np.uint64(c)
        out[c] = quantize(lo[c] + (hi[c] - lo[c]) * uniform01(key, cnt), L)
    return out


def velocity_field(x: np.ndarray, L: float = 1.0, U: float = 1.0, amp: float = 0.3,
                   quantum: float = 0.0) -> np.ndarray:
    """A smooth periodic flow for the per-particle velocity path, evaluated at
    positions x (dim, n): a drift U along x with a shear and a compressive part,
        v_x = U (1 + amp sin(2 pi y / L) + amp sin(2 pi x / L)),
        v_y = U amp cos(2 pi x / L)           [, v_z = U amp sin(2 pi (x + y) / L)].
    quantum > 0 rounds every component to a multiple of it (so that dt v / L
    can be a whole number of fixed-point units per step)."""
    x = np.asarray(x, dtype=np.float64)
    dim = x.shape[0]
    k = 2.0 * math.pi / L
    v = np.zeros_like(x)
    v[0] = U * (1.0 + amp * np.sin(k * x[1]) + amp * np.sin(k * x[0]))
    v[1] = U * amp * np.cos(k * x[0])
    if dim == 3:
        v[2] = U * amp * np.sin(k * (x[0] + x[1]))
    if quantum > 0:
        v = np.rint(v / quantum) * quantum
    return v


@dataclass
class PlumeSpec:
    """One plume problem: particles on a lattice in a periodic box with uniform flow."""
    dim: int = 2
    n_side: int = 64
    L: float = 1.0
    jitter: float = 0.0
    h_over_dp: float = 1.3       # smoothing length h in units of dp; support H = 2h
    kernel: int = 4              # 2 = Wendland C2, 4 = Wendland C4 (Eq. 7)
    alpha_L: float = 1e-2
    alpha_T: float = 1e-3
    D_m: float = 1e-6
    v: tuple = (1.0, 0.0, 0.0)
    sigma0: float = 0.05
    centre: tuple = (0.25, 0.5, 0.5)
    dt: float = 1e-4
    steps: int = 200
    real_bytes: int = 4
    rho0: float = 1000.0
    seed: int = BASE_SEED
    stream: int = 0
    name: str = ""

    @property
    def n(self) -> int:
        return self.n_side ** self.dim

    @property
    def dp(self) -> float:
        return self.L / self.n_side

    @property
    def H(self) -> float:
        return 2.0 * self.h_over_dp * self.dp

    @property
    def mass(self) -> float:
        return self.rho0 * self.dp ** self.dim

    def positions(self) -> np.ndarray:
        return lattice(self.n_side, self.dim, self.L, self.jitter, self.seed, self.stream)

    def concentration(self, x: np.ndarray) -> np.ndarray:
        return gaussian_plume(x, self.centre[: self.dim], self.sigma0, self.L)

    def velocity(self) -> np.ndarray:
        return np.array(self.v[: self.dim], dtype=np.float64)


def eq10_dt(spec: PlumeSpec) -> float:
    """Time step of Eq. (10) with C = 0.1, evaluated with the config's smoothing
    length h (= H/2) and the trace of the uniform dispersion tensor."""
    v = spec.velocity()
    speed = float(np.sqrt(np.sum(v * v)))
    trD = spec.dim * (spec.alpha_T * speed + spec.D_m) + (spec.alpha_L - spec.alpha_T) * speed
    h = spec.h_over_dp * spec.dp
    return 0.1 * h * h / trD


def config(name: str, **over) -> PlumeSpec:
    """Named workloads (sizes and parameters of the plume problems).

    cfg1     2D FP64, 64^2 regular lattice, Wendland C2, h = 1.3 dp, 200 Euler steps of 1e-4.
    cfg2_*   2D FP32, 512^2 lattice jittered by +-0.1 dp, Wendland C4, h/dp in {1.3, 2, 3},
             alpha_L/alpha_T in {10, 100}, 1000 steps, dt from Eq. (10).
    cfg3     3D FP32, 128^3 jittered lattice, C4, h = 2 dp, 500 steps of 5e-5.
    cfg5     2D FP32, 256^2 regular lattice, C4, h = 1.5 dp, 500 steps of 1e-4 (adjoint problem).
    paper*   2D FP32, the paper-scale problems of Table 1 (1000^2, 1414^2, 2000^2 particles,
             31.5k-80k neighbours, jitter +-0.1 dp), dt from Eq. (10), 300 days.
    """
    if name == "cfg1":
        s = PlumeSpec(dim=2, n_side=64, jitter=0.0, h_over_dp=1.3, kernel=2, alpha_L=1e-2,
                      alpha_T=1e-3, D_m=1e-6, v=(1.0, 0.0, 0.0), sigma0=0.05,
                      centre=(0.25, 0.5, 0.5), dt=1e-4, steps=200, real_bytes=8, name=name)
    elif name.startswith("cfg2"):
        # cfg2_h{13,20,30}_r{10,100}
        parts = name.split("_")
        hod = {"h13": 1.3, "h20": 2.0, "h30": 3.0}[parts[1]]
        ratio = {"r10": 10.0, "r100": 100.0}[parts[2]]
        s = PlumeSpec(dim=2, n_side=512, jitter=0.1, h_over_dp=hod, kernel=4, alpha_L=1e-2,
                      alpha_T=1e-2 / ratio, D_m=1e-6, v=(1.0, 0.0, 0.0), sigma0=0.05,
                      centre=(0.25, 0.5, 0.5), steps=1000, real_bytes=4, name=name)
        s.dt = eq10_dt(s)
    elif name == "cfg3":
        s = PlumeSpec(dim=3, n_side=128, jitter=0.1, h_over_dp=2.0, kernel=4, alpha_L=1e-2,
                      alpha_T=1e-3, D_m=1e-6, v=(1.0, 0.0, 0.0), sigma0=0.05,
                      centre=(0.25, 0.5, 0.5), dt=5e-5, steps=500, real_bytes=4, name=name)
    elif name.startswith("paper"):
        # Table 1 resolutions: N = 1M, 2M, 4M particles with support radius
        # H/L = 0.099, 0.089, 0.079 (Table 1's h/L column, read as the support
        # radius: pi (H/L)^2 N reproduces its neighbour counts 31529, 50339,
        # 80371 to 2.5%); Section 3 model: L = 2000 m, plume centred, w = 44 m,
        # alpha_L = 10 m, alpha_T/alpha_L = 0.1 (paper1m_r100, _r1000: 0.01,
        # 0.001), D_m = 0, |v| = 1.16e-5 m/s at 45 degrees, 300 days.
        parts = name.split("_")
        side, HL = {"paper1m": (1000, 0.099), "paper2m": (1414, 0.089), "paper4m": (2000, 0.079)}[parts[0]]
        ratio = {"r10": 10.0, "r100": 100.0, "r1000": 1000.0}[parts[1] if len(parts) > 1 else "r10"]
        vv = 1.16e-5 * math.sqrt(0.5)
        s = PlumeSpec(dim=2, n_side=side, L=2000.0, jitter=0.1, h_over_dp=HL * side / 2.0, kernel=4,
                      alpha_L=10.0, alpha_T=10.0 / ratio, D_m=0.0, v=(vv, vv, 0.0), sigma0=44.0,
                      centre=(1000.0, 1000.0, 1000.0), real_bytes=4, name=name)
        # Eq. (10) with the smoothing length H/2, as for every problem here.
        # With the table's h (the support radius H) the step would be 4x
        # longer, beyond the 300-day run, and unstable: on a 150^2 lattice of
        # the same H/L the operator's most negative eigenvalue gives
        # dt lambda = -2.5, an amplification of 1.5 (Euler) and 1.6
        # (predictor-corrector) per step.
        s.dt = eq10_dt(s)
        s.steps = int(math.ceil(300 * 86400.0 / s.dt))
    elif name == "cfg5":
        s = PlumeSpec(dim=2, n_side=256, jitter=0.0, h_over_dp=1.5, kernel=4, alpha_L=2e-2,
                      alpha_T=2e-3, D_m=1e-6, v=(1.0, 0.0, 0.0), sigma0=0.05,
                      centre=(0.25, 0.5, 0.5), dt=1e-4, steps=500, real_bytes=4, name=name)
    else:
        raise KeyError(name)
    for k, val in over.items():
        setattr(s, k, val)
    return s


CFG2_CELLS = [f"cfg2_{h}_{r}" for h in ("h13", "h20", "h30") for r in ("r10", "r100")]


def ensemble(n_plumes: int = 256, seed: int = BASE_SEED, stream: int = 4242,
             sides=(32, 64, 128, 256), h_over_dp: float = 1.5):
    """The batched ensemble: per-plume lattice side drawn uniformly from `sides`,
    alpha_L log-uniform in [1e-3, 1e-1], alpha_T = alpha_L / r with r log-uniform
    in [1, 100], D_m = 1e-6, flow angle uniform in [0, 2 pi) with |v| = 1, C4,
    jitter +-0.1 dp, Gaussian sigma0 = 0.05 at (0.5, 0.5), dt from Eq. (10) per plume."""
    key = stream_key(seed, stream)
    cnt = np.arange(n_plumes, dtype=np.uint64) * np.uint64(4)
    u0 = uniform01(key, cnt)
    u1 = uniform01(key, cnt + np.uint64(1))
    u2 = uniform01(key, cnt + np.uint64(2))
    u3 = uniform01(key, cnt + np.uint64(3))
    specs = []
    for p in range(n_plumes):
        side = int(sides[min(int(u0[p] * len(sides)), len(sides) - 1)])
        aL = 10.0 ** (-3.0 + 2.0 * u1[p])
        r = 10.0 ** (2.0 * u2[p])
        ang = 2.0 * math.pi * u3[p]
        s = PlumeSpec(dim=2, n_side=side, jitter=0.1, h_over_dp=h_over_dp, kernel=4,
                      alpha_L=aL, alpha_T=aL / r, D_m=1e-6,
                      v=(math.cos(ang), math.sin(ang), 0.0), sigma0=0.05,
                      centre=(0.5, 0.5, 0.5), steps=200, real_bytes=4,
                      seed=seed, stream=1000 + p, name=f"plume{p}")
        s.dt = eq10_dt(s)
        specs.append(s)
    return specs
