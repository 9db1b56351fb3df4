"""Parity cases at the edges of the problems' ranges, through the C ABI
against the FP64 oracle:

- the library's own Eq. (10) time step (a context given dt = 0);
- exact ties r = H on regular lattices (support radius a whole number of
  lattice spacings), where the inclusive predicate decides;
- velocity fields with unrounded velocities, where the library moves each
  particle on the fixed-point schedule rint((k+1) u) - rint(k u) and the
  oracle by x + dt v in FP64 (positions then differ by up to 2^-33 L);
- the paper-scale problems of Table 1 at 2 and 4 million particles;
- the 256-plume ensemble at full size over its 200 graph-replayed steps.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from oracle import spectrum as S
from paper_2108_09488_amd import _lib
from paper_2108_09488_amd import inputs as I

pytestmark = pytest.mark.gpu
TWO32 = 4294967296.0
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _sets(offsets, ids):
    offsets = np.asarray(offsets, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    seg = np.repeat(np.arange(len(offsets) - 1), np.diff(offsets))
    return offsets, ids[np.lexsort((ids, seg))]


def _context(specs, C=None, flags=0, integrator=1, cell_xsub=0, x=None, stream=None):
    from paper_2108_09488_amd.context import Context, params_from_spec
    specs = specs if isinstance(specs, list) else [specs]
    ctx = Context([params_from_spec(s, flags=flags, integrator=integrator, cell_xsub=cell_xsub) for s in specs],
                  [s.n for s in specs], stream=stream)
    if x is None:
        x = np.concatenate([s.positions() for s in specs], axis=1)
    if C is None:
        C = np.concatenate([s.concentration(s.positions()) for s in specs])
    dt = torch.float32 if specs[0].real_bytes == 4 else torch.float64
    ctx.init(torch.from_numpy(x), torch.from_numpy(C).to(dt))
    return ctx, x


# ---------------------------------------------------------------------------
# Eq. (10)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["cfg2_h20_r10", "cfg2_h13_r100", "cfg3", "cfg1"])
def test_eq10_time_step_of_the_library(name):
    """dt <= 0 makes the library take Eq. (10) with C = 0.1 and the smoothing
    length H/2; it equals the oracle's rule to round-off."""
    spec = I.config(name, n_side=16)
    spec.dt = 0.0
    print(f"[case] Eq. (10) dt of {name}", flush=True)
    ctx, _ = _context(spec)
    dt = ctx.info()["dt"]
    ref = O.dt_rule(O.model_from_spec(spec), spec.velocity(), 0.5 * spec.H)
    assert dt == pytest.approx(ref, rel=1e-14)
    assert dt == pytest.approx(I.eq10_dt(I.config(name, n_side=16)), rel=1e-14)
    ctx.close()


def test_eq10_time_step_per_plume_of_an_ensemble():
    specs = I.ensemble(6, sides=(16, 24))
    for s in specs:
        s.dt = 0.0
    print("[case] Eq. (10) dt of an ensemble", flush=True)
    ctx, _ = _context(specs)
    for p, s in enumerate(specs):
        ref = O.dt_rule(O.model_from_spec(s), s.velocity(), 0.5 * s.H)
        assert ctx.info(p)["dt"] == pytest.approx(ref, rel=1e-14)
    ctx.close()


# ---------------------------------------------------------------------------
# Exact ties at r = H
# ---------------------------------------------------------------------------
TIE_CASES = [(2, 64, 1.5, 28, 4), (2, 64, 2.5, 80, 4), (2, 64, 1.5, 28, 8), (3, 32, 1.5, 122, 4)]


@pytest.mark.parametrize("dim,n_side,hod,count,rb", TIE_CASES)
def test_exact_ties_on_regular_lattices(dim, n_side, hod, count, rb):
    """On a regular lattice with H = 2 h a whole number of spacings (3 dp or
    5 dp), lattice neighbours at exactly r = H are inside the inclusive support:
    every particle has the lattice's full count (2D: 28 at 3 dp, 80 at 5 dp;
    3D: 122 at 3 dp) and the sets equal the oracle's, also after steps."""
    base = "cfg1" if dim == 2 else "cfg3"
    spec = I.config(base, n_side=n_side, jitter=0.0, h_over_dp=hod, real_bytes=rb, kernel=4)
    print(f"[case] ties dim={dim} n_side={n_side} H={2 * hod} dp rb={rb}", flush=True)
    ctx, x = _context(spec)
    ctx.build()
    off, ids = ctx.neighbours()
    g_off, g_ids = _sets(off.cpu().numpy(), ids.cpu().numpy())
    assert np.all(np.diff(g_off) == count)
    o_off, o_ids = O.neighbours_fixed(dim, x, spec.L, spec.H, rb)
    assert np.array_equal(g_off, o_off) and np.array_equal(g_ids, o_ids)
    # the whole lattice moves by the same fixed-point shift: ties stay ties
    ctx.step(5)
    off, ids = ctx.neighbours()
    assert np.all(np.diff(off.cpu().numpy()) == count)
    ctx.close()


# ---------------------------------------------------------------------------
# Velocity fields with unrounded velocities
# ---------------------------------------------------------------------------
def _schedule_sensitivity(m, x, C0, v, dt, steps, integrator, spec):
    """How far the oracle's run moves when every position is shifted by up to
    the library's rounding, 2^-33 L per coordinate (a seeded shift held for
    the run): the scale of the difference the fixed-point schedule makes."""
    rng = np.random.default_rng(5)
    e = (rng.integers(0, 2, size=x.shape) * 2 - 1) * (spec.L * 2.0 ** -33)
    _, C1, _ = O.run(m, x, C0, dt, steps, v=v, mass=spec.mass, rho=spec.rho0, integrator=integrator)
    _, C2, _ = O.run(m, np.mod(x + e, spec.L), C0, dt, steps, v=v, mass=spec.mass, rho=spec.rho0,
                     integrator=integrator)
    return _rel(C2, C1)


@pytest.mark.parametrize("integrator", [1, 2])
@pytest.mark.parametrize("rb", [8, 4])
def test_raw_velocity_field_trajectory(integrator, rb):
    """48 steps of the velocity field of inputs.velocity_field with its
    velocities as drawn (no rounding to whole fixed-point units per step):
    positions within 2^-33 L (plus the oracle's FP64 accumulation) of the
    oracle's x + dt v, C within 1e-5 (FP32) or, in FP64, within ten times the
    oracle's own change under a shift of the positions by 2^-33 L."""
    spec = I.config("cfg1", n_side=48, real_bytes=rb, kernel=4, h_over_dp=1.5, jitter=0.1, dt=1e-4)
    x = spec.positions()
    v = I.velocity_field(x, spec.L)
    C0 = spec.concentration(x)
    if rb == 4:
        v = v.astype(np.float32).astype(np.float64)
        C0 = C0.astype(np.float32).astype(np.float64)
    steps = 48
    print(f"[case] raw velocity field rb={rb} integ={integrator}", flush=True)
    ctx, _ = _context(spec, C=C0, flags=_lib.ADE_VELOCITY_FIELD, integrator=integrator, x=x)
    ctx.set_velocities(torch.from_numpy(v)).build()
    ctx.step(steps)
    Cg = ctx.read_C().double().cpu().numpy()
    xg = ctx.read_x().cpu().numpy()
    ctx.close()
    m = O.model_from_spec(spec)
    xo, Co, _ = O.run(m, x, C0, spec.dt, steps, v=v, mass=spec.mass, rho=spec.rho0, integrator=integrator)
    d = np.abs((xg - xo + 0.5 * spec.L) % spec.L - 0.5 * spec.L)
    assert d.max() <= spec.L * (2.0 ** -33 * 1.0001 + steps * 2.0 ** -50), d.max()
    assert d.max() > 0  # the schedule did round
    err = _rel(Cg, Co)
    if rb == 4:
        tol = 1e-5
    else:
        tol = max(1e-12, 10.0 * _schedule_sensitivity(m, x, C0, v, spec.dt, steps, integrator, spec))
    print(f"[result] raw velocity field rb={rb} integ={integrator}: C rel L2 {err:.3e} (tol {tol:.2e}), "
          f"max position offset {d.max() / spec.L:.3e} L", flush=True)
    assert err <= tol


# ---------------------------------------------------------------------------
# Paper-scale problems at 2 and 4 million particles (Table 1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,table_n", [("paper2m", 50339), ("paper4m", 80371)])
def test_paper_scale_sampled_2m_4m(name, table_n):
    """Table 1's second and third resolutions at full size: the mean neighbour
    count matches the table within 3 %, and the right-hand side matches the
    oracle at a seeded sample of 400 particles inside the plume to 1e-5."""
    spec = I.config(name)
    C = spec.concentration(spec.positions()).astype(np.float32).astype(np.float64)
    print(f"[case] {name} sampled rhs", flush=True)
    ctx, x = _context(spec, C=C)
    ctx.build()
    nbar = ctx.neighbour_counts()[-1].item() / spec.n
    g = ctx.rhs().double().cpu().numpy()
    ctx.close()
    rng = np.random.default_rng(17)
    idx = np.sort(rng.choice(np.flatnonzero(C > 1e-3), size=400, replace=False))
    r = O.rhs(O.model_from_spec(spec), x, C, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0, idx=idx)
    e = _rel(g[idx], r)
    print(f"[result] {name}: mean neighbours {nbar:.1f} (Table 1: {table_n}), rhs rel L2 {e:.3e}", flush=True)
    assert abs(nbar - table_n) < 0.03 * table_n
    assert e < 1e-5


# ---------------------------------------------------------------------------
# The 256-plume ensemble at full size
# ---------------------------------------------------------------------------
def _context_xsub(specs):
    """The x cells per support radius the library picks for a context of
    these plumes (the cell-table budget may coarsen them), read off the
    workspace size of explicit choices."""
    from paper_2108_09488_amd.context import params_from_spec, workspace_bytes
    ref = workspace_bytes(specs, [s.n for s in specs])
    for xs in (8, 6, 4, 3):
        if workspace_bytes([params_from_spec(s, cell_xsub=xs) for s in specs], [s.n for s in specs]) == ref:
            return xs
    raise AssertionError("cell grid of the ensemble not found")


def test_ensemble_full_size():
    """256 plumes (5.4 M particles), 200 steps replayed from the captured
    graph.  Eight seeded plumes equal, bit for bit, the same plume run alone
    on the same cell grid and launch shape; plume 0 matches the oracle to
    1e-5 times the growth its operator allows over the run."""
    specs = I.ensemble(256)
    xsub = _context_xsub(specs)
    xs = [s.positions() for s in specs]
    Cs = [s.concentration(x).astype(np.float32).astype(np.float64) for s, x in zip(specs, xs)]
    print(f"[case] ensemble 256 plumes, {sum(s.n for s in specs)} particles, x cells H/{xsub}", flush=True)
    # graph capture needs a stream of its own
    ens, _ = _context(specs, C=np.concatenate(Cs), x=np.concatenate(xs, axis=1), stream=torch.cuda.Stream())
    ens.build()
    tuning = ens.get_tuning()
    steps = 200
    ens.step_graph(steps)
    Ce = ens.read_C().cpu().numpy()
    ens.close()
    offs = np.concatenate([[0], np.cumsum([s.n for s in specs])])
    rng = np.random.default_rng(23)
    picks = [0] + sorted(rng.choice(np.arange(1, 256), size=7, replace=False).tolist())
    for p in picks:
        s = specs[p]
        one, _ = _context(s, C=Cs[p], x=xs[p], cell_xsub=xsub)
        one.build()
        one.set_tuning(block=tuning["block"], lanes=tuning["lanes"], targets=tuning["targets"],
                       xcd_group=tuning["xcd_group"], persistent=tuning["persistent"])
        one.step(steps)
        C1 = one.read_C().cpu().numpy()
        one.close()
        assert np.array_equal(Ce[offs[p]:offs[p + 1]], C1), p
    s = specs[0]
    growth = json.load(open(os.path.join(GOLD, "spectrum.json")))["ensemble_0"]["growth_upper"]
    _, Co, _ = O.run(O.model_from_spec(s), xs[0], Cs[0], s.dt, steps, v_uniform=s.velocity(), mass=s.mass,
                     rho=s.rho0)
    e = _rel(Ce[:s.n].astype(np.float64), Co)
    print(f"[result] ensemble plume 0 ({s.n_side}^2, {steps} steps): rel L2 {e:.3e}, growth {growth:.3g}; "
          f"plumes {picks} bitwise equal to single runs", flush=True)
    assert e <= 1e-5 * max(1.0, growth)
