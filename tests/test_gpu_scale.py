"""Large contexts: cell tables and neighbour offsets past the size where the
scans' final workgroups sum the chunk totals themselves (then the totals are
scanned in a launch of their own), and a context at the particle limit,
where the candidate lists' 32-bit byte offsets into the record array come
within 0.02% of 2^32.

Tolerances: neighbour offsets bit-exact (the oracle evaluates the same
fixed-point predicate); FP32 right-hand sides within 1e-5 relative L2 (as the
full-size sampled tests); the FP64 context at the limit within 1e-10 of the
oracle, whose positions equal the context's exactly (dyadic lattice, dyadic
time step), and solute mass conserved to 1e-11.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2108_09488_amd import inputs as I

pytestmark = pytest.mark.gpu

DIRECT_CELLS = 4096 * 1024     # cells the cell scan's final launch still sums directly
DIRECT_OFFSETS = 2048 * 4096   # neighbour-offset entries the same holds for
LIMIT = (1 << 28) - 256        # particles per context


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_scans_past_the_direct_size():
    """2900^2 jittered plume (8.4M particles; 7.5M cells, its default x cells
    coarsened to H/3 to bound the tables): both scans take the scanned-totals
    path; the neighbour offsets match the oracle's
    exactly, before and after steps, and the right-hand side matches at a
    sample of plume particles."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = I.config("cfg2_h13_r10", n_side=2900)
    spec.dt = I.eq10_dt(spec)
    assert spec.n + 1 > DIRECT_OFFSETS
    print(f"[case] scans past the direct size: n={spec.n}", flush=True)
    x = spec.positions()
    C = spec.concentration(x).astype(np.float32).astype(np.float64)
    ctx = Context([params_from_spec(spec)], [spec.n])
    ctx.init(torch.from_numpy(x), torch.from_numpy(C)).build()
    assert ctx.info()["cells"] > DIRECT_CELLS
    off = ctx.neighbour_counts().cpu().numpy()
    o_off, _ = O.neighbours_fixed(spec.dim, x, spec.L, spec.H, spec.real_bytes)
    assert np.array_equal(off, o_off)
    g = ctx.rhs().double().cpu().numpy()
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(np.flatnonzero(C > 1e-3), size=1500, replace=False))
    r = O.rhs(O.model_from_spec(spec), x, C, v_uniform=spec.velocity(), mass=spec.mass,
              rho=spec.rho0, idx=idx)
    assert _rel(g[idx], r) < 1e-5
    # every step rebuilds the cells: the lattice has moved by a whole number
    # of grid units per step, which leaves its neighbour sets as they were
    ctx.step(3)
    assert np.array_equal(ctx.neighbour_counts().cpu().numpy(), o_off)
    ctx.close()


def _limit_problem():
    """A 2D FP64 plume at the particle limit: a 16384 x 16383 lattice of
    spacing 2^-14 in the unit box (the top row left empty), so every position
    is exact in the 32-bit fixed point, with an image-summed Gaussian plume
    over the box's corner, so that the top rows and the periodic seams, whose
    candidates sit at the end of the sorted order, carry concentration."""
    nx, ny = 16384, 16383
    dp = 1.0 / nx
    xs = (np.arange(nx) + 0.5) * dp
    ys = (np.arange(ny) + 0.5) * dp
    x = np.empty((2, ny, nx))
    x[0] = xs[None, :]
    x[1] = ys[:, None]

    def g(u, c, s=0.02):
        return sum(np.exp(-(u - c + k) ** 2 / (2 * s * s)) for k in (-1.0, 0.0, 1.0))

    C = np.empty((ny, nx))
    np.multiply(g(ys, 0.985)[:, None], g(xs, 0.97)[None, :], out=C)
    x, C = x.reshape(2, nx * ny), C.reshape(nx * ny)
    spec = I.config("cfg2_h13_r10", n_side=nx, jitter=0.0, real_bytes=8, dt=2.0 ** -25)
    return spec, nx, ny, x, C


def test_particle_limit_fp64():
    """The largest lattice under the particle limit (2^28 - 16384 particles):
    the right-hand side and two Euler steps match the oracle at sampled sites
    (the top rows, the seams, the plume), and mass is conserved.  The oracle
    sees each sample's lattice patch of +-8 sites, which holds every particle
    that its value after two steps depends on (two support radii, 5.2 dp)."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec, nx, ny, x, C = _limit_problem()
    n = nx * ny
    assert LIMIT - 16384 <= n <= LIMIT
    print(f"[case] particle limit: n={n} FP64", flush=True)
    ctx = Context([params_from_spec(spec)], [n])
    ctx.init(torch.from_numpy(x), torch.from_numpy(C)).build()
    m0 = ctx.mass().cpu().numpy()[0]
    g = ctx.rhs().cpu().numpy()

    rng = np.random.default_rng(5)
    hot = np.flatnonzero(C > 1e-2)
    fixed = [(i, j) for i in (0, 1, nx // 2, nx - 2, nx - 1) for j in (0, 1, ny - 2, ny - 1)]
    picks = [(int(k % nx), int(k // nx)) for k in rng.choice(hot, size=40, replace=False)]
    sites = sorted(set(fixed + picks))
    tgt = np.array([j * nx + i for i, j in sites])
    patch = []
    for i, j in sites:
        di, dj = np.meshgrid(np.arange(-8, 9), np.arange(-8, 9))
        ii, jj = (i + di.ravel()) % nx, (j + dj.ravel()) % nx
        keep = jj < ny  # the empty top row
        patch.append(jj[keep] * nx + ii[keep])
    sub = np.unique(np.concatenate(patch))
    pos = np.searchsorted(sub, tgt)
    assert np.array_equal(sub[pos], tgt)
    m = O.model_from_spec(spec)
    r = O.rhs(m, x[:, sub], C[sub], v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0, idx=pos)
    assert _rel(g[tgt], r) < 1e-10

    ctx.step(2)
    m1 = ctx.mass().cpu().numpy()[0]
    assert abs(m1 - m0) <= 1e-11 * abs(m0)
    Cg = ctx.read_C().cpu().numpy()
    _, Co, _ = O.run(m, x[:, sub], C[sub], spec.dt, 2, v_uniform=spec.velocity(), mass=spec.mass,
                     rho=spec.rho0)
    assert _rel(Cg[tgt], Co[pos]) < 1e-10
    ctx.close()
