"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle, on the
same seeded inputs.

Tolerances: neighbour sets bit-exact (the oracle evaluates the same
fixed-point predicate in the same precision); FP64 runs within 1e-12 relative
L2; FP32 right-hand sides and FP32 trajectories on the non-growing problems
within 1e-5 relative L2.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2108_09488_amd import inputs as I

pytestmark = pytest.mark.gpu

TWO32 = 4294967296.0


def _ctx(spec, integrator=1, cell_rows=0, cell_xsub=0):
    from paper_2108_09488_amd.context import Context, params_from_spec
    print(f"[case] {spec.name} n_side={spec.n_side} dim={spec.dim} h/dp={spec.h_over_dp} "
          f"rb={spec.real_bytes} integ={integrator}", flush=True)
    ctx = Context([params_from_spec(spec, integrator=integrator, cell_rows=cell_rows,
                                    cell_xsub=cell_xsub)], [spec.n])
    x = spec.positions()
    C = spec.concentration(x)
    if spec.real_bytes == 4:
        C = C.astype(np.float32).astype(np.float64)
    ctx.init(torch.from_numpy(x), torch.from_numpy(C)).build()
    return ctx, x, C


def _sets(offsets, ids):
    offsets = np.asarray(offsets, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    seg = np.repeat(np.arange(len(offsets) - 1), np.diff(offsets))
    order = np.lexsort((ids, seg))
    return offsets, ids[order]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


NBR_CASES = [
    ("cfg1", {}),
    ("cfg2_h13_r10", {"n_side": 128}),
    ("cfg2_h20_r100", {"n_side": 128}),
    ("cfg2_h30_r10", {"n_side": 128}),
    ("cfg2_h20_r10", {"n_side": 50, "h_over_dp": 1.5}),          # ragged last tile
    ("cfg3", {"n_side": 24}),
    ("cfg1", {"real_bytes": 4, "jitter": 0.1, "n_side": 40}),
]


@pytest.mark.parametrize("name,over", NBR_CASES)
@pytest.mark.parametrize("grid", [(0, 0), (1, 1), (3, 16), (2, 3), (0, 4)])
def test_neighbour_sets_bit_exact(name, over, grid):
    spec = I.config(name, **over)
    ctx, x, _ = _ctx(spec, cell_rows=grid[0], cell_xsub=grid[1])
    off, ids = ctx.neighbours()
    g_off, g_ids = _sets(off.cpu().numpy(), ids.cpu().numpy())
    o_off, o_ids = O.neighbours_fixed(spec.dim, x, spec.L, spec.H, spec.real_bytes)
    assert np.array_equal(g_off, o_off)
    assert np.array_equal(g_ids, o_ids)
    # after some steps the lattice has moved by an exact fixed-point displacement
    k = 7
    ctx.step(k)
    off, ids = ctx.neighbours()
    g_off, g_ids = _sets(off.cpu().numpy(), ids.cpu().numpy())
    u = O.to_fixed(x, spec.L).astype(np.int64)
    v = spec.velocity()
    xk = np.empty_like(x)
    for c in range(spec.dim):
        s = int(np.rint(k * spec.dt * v[c] / spec.L * TWO32))
        xk[c] = np.mod(u[c] + s, 1 << 32).astype(np.float64) / TWO32 * spec.L
    o_off, o_ids = O.neighbours_fixed(spec.dim, xk, spec.L, spec.H, spec.real_bytes)
    assert np.array_equal(g_off, o_off) and np.array_equal(g_ids, o_ids)
    ctx.close()


@pytest.mark.parametrize("dim,real_bytes", [(2, 8), (2, 4), (3, 4)])
def test_crowded_cells(dim, real_bytes):
    """Twelve particles within +-0.02 dp of every lattice site: most sites lie
    wholly inside one cell (cells are at least 0.3 dp wide), so cells hold
    more particles than their buckets and the placement reads the overflow
    list.  Neighbour sets stay bit-exact, the right-hand side matches the
    oracle, and two contexts step to identical bits."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = I.config("cfg1" if dim == 2 else "cfg3", n_side=20 if dim == 2 else 8, real_bytes=real_bytes,
                    h_over_dp=1.3)
    x = I.clustered(spec.n_side, dim, 12, 0.02, spec.L, stream=3)
    n = x.shape[1]
    C = spec.concentration(x)
    if real_bytes == 4:
        C = C.astype(np.float32).astype(np.float64)
    outs = []
    for rep in range(2):
        print(f"[case] crowded dim={dim} rb={real_bytes} n={n} rep={rep}", flush=True)
        ctx = Context([params_from_spec(spec)], [n])
        ctx.init(torch.from_numpy(x), torch.from_numpy(C)).build()
        if rep == 0:
            off, ids = ctx.neighbours()
            g_off, g_ids = _sets(off.cpu().numpy(), ids.cpu().numpy())
            o_off, o_ids = O.neighbours_fixed(dim, x, spec.L, spec.H, real_bytes)
            assert np.array_equal(g_off, o_off) and np.array_equal(g_ids, o_ids)
            g = ctx.rhs().double().cpu().numpy()
            r = O.rhs(O.model_from_spec(spec), x, C, v_uniform=spec.velocity(), mass=spec.mass,
                      rho=spec.rho0)
            assert _rel(g, r) < (1e-12 if real_bytes == 8 else 1e-5)
        ctx.step(5)
        outs.append((ctx.read_C().cpu().numpy().copy(), ctx.read_x().cpu().numpy().copy()))
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


RHS_CASES = [(c, {"n_side": 128}) for c in I.CFG2_CELLS] + [("cfg3", {"n_side": 24}), ("cfg1", {})]


@pytest.mark.parametrize("name,over", RHS_CASES)
def test_rhs_parity(name, over):
    spec = I.config(name, **over)
    ctx, x, C = _ctx(spec)
    g = ctx.rhs().double().cpu().numpy()
    r = O.rhs(O.model_from_spec(spec), x, C, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
    tol = 1e-12 if spec.real_bytes == 8 else 1e-5
    assert _rel(g, r) < tol
    ctx.close()


@pytest.mark.parametrize("name", I.CFG2_CELLS + ["cfg3"])
def test_rhs_parity_full_size_sampled(name):
    """Full-size problems (512^2, 128^3): the oracle evaluates Eq. (4) at a
    seeded sample of particles inside the plume."""
    spec = I.config(name)
    ctx, x, C = _ctx(spec)
    g = ctx.rhs().double().cpu().numpy()
    rng = np.random.default_rng(7)
    inside = np.flatnonzero(C > 1e-3)
    idx = np.sort(rng.choice(inside, size=1500, replace=False))
    r = O.rhs(O.model_from_spec(spec), x, C, v_uniform=spec.velocity(), mass=spec.mass,
              rho=spec.rho0, idx=idx)
    assert _rel(g[idx], r) < 1e-5
    ctx.close()


@pytest.mark.parametrize("integrator", [1, 2])
def test_fp64_trajectory(integrator):
    """64^2 regular lattice, Wendland C2, 200 steps in FP64: C within 1e-12
    relative L2 of the oracle, mass conserved to 1e-12, positions to 1e-9."""
    spec = I.config("cfg1")
    ctx, x, C0 = _ctx(spec, integrator=integrator)
    m0 = ctx.mass().cpu().numpy()[0]
    ctx.step(spec.steps)
    C = ctx.read_C().cpu().numpy()
    xg = ctx.read_x().cpu().numpy()
    m1 = ctx.mass().cpu().numpy()[0]
    xo, Co, hist = O.run(O.model_from_spec(spec), x, C0, spec.dt, spec.steps, v_uniform=spec.velocity(),
                         mass=spec.mass, rho=spec.rho0, integrator=integrator)
    assert _rel(C, Co) < 1e-12
    assert abs(m1 - m0) <= 1e-12 * abs(m0)
    assert m0 == pytest.approx(hist[0], rel=1e-13)
    d = (xg - xo + 0.5) % 1.0 - 0.5
    assert np.max(np.abs(d)) < 1e-9
    ctx.close()


@pytest.mark.parametrize("name,over,steps", [("cfg2_h20_r10", {"n_side": 128}, 200),
                                             ("cfg2_h30_r10", {"n_side": 128}, 200),
                                             ("cfg2_h30_r100", {"n_side": 128}, 200),
                                             ("cfg3", {"n_side": 24}, 60)])
def test_fp32_trajectory(name, over, steps):
    spec = I.config(name, **over)
    ctx, x, C0 = _ctx(spec)
    ctx.step(steps)
    C = ctx.read_C().double().cpu().numpy()
    _, Co, _ = O.run(O.model_from_spec(spec), x, C0, spec.dt, steps, v_uniform=spec.velocity(),
                     mass=spec.mass, rho=spec.rho0)
    assert _rel(C, Co) < 1e-5
    ctx.close()


def test_determinism_and_graph_replay():
    """Two runs from the same inputs are bitwise equal; replaying a captured
    step from a HIP graph gives the same bits as eager launches."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = I.config("cfg2_h20_r10", n_side=96)
    outs = []
    for mode in ("eager", "eager", "graph"):
        stream = torch.cuda.Stream()
        ctx = Context([params_from_spec(spec)], [spec.n], stream=stream)
        x = spec.positions()
        C = spec.concentration(x)
        ctx.init(torch.from_numpy(x), torch.from_numpy(C)).build()
        if mode == "eager":
            ctx.step(30)
        else:
            for _ in range(3):  # several graph launches with host work between them
                ctx.step_graph(10)
                torch.cuda.synchronize()
        outs.append(ctx.read_C().cpu().numpy().copy())
        assert ctx.info()["step"] == 30
        stream.synchronize()
        ctx.close()
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


TUNINGS = [  # (block, lanes, persistent, xcd_group, targets per lane)
    (256, 1, 0, 0, 1), (128, 1, 0, 1, 1), (64, 1, 0, 8, 1), (256, 1, 64, 0, 1), (128, 1, 7, 3, 1),
    (256, 2, 0, 0, 1), (64, 2, 0, 128, 1), (128, 2, 40, 5, 1), (256, 2, 8, 1, 1),
    (256, 4, 0, 0, 1), (128, 4, 13, 2, 1), (64, 4, 0, 7, 1), (256, 4, 300, 4096, 1),
    (128, 1, 0, 0, 2), (64, 1, 0, 8, 2), (128, 1, 40, 3, 2), (64, 1, 7, 1, 2), (128, 1, 0, 4096, 2),
    (256, 4, 0, 0, 2), (64, 4, 0, 8, 2), (128, 4, 300, 4096, 2), (64, 4, 9, 1, 2),
]


@pytest.mark.parametrize("name,over", [("cfg2_h13_r10", {"n_side": 100}), ("cfg2_h30_r100", {"n_side": 96}),
                                       ("cfg3", {"n_side": 20}), ("cfg1", {"n_side": 45}),
                                       ("cfg3", {"n_side": 18, "real_bytes": 8})])
def test_launch_shapes_are_bitwise_equal(name, over):
    """Workgroup size, the persistent grid and the dealing of work items to
    the XCDs change which workgroup runs a target, not the order of its sums:
    for a given number of lanes per particle (or of particles per lane) every
    launch shape gives the same bits, and all match the oracle."""
    spec = I.config(name, **over)
    ctx, x, C = _ctx(spec)
    r = O.rhs(O.model_from_spec(spec), x, C, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
    by_shape = {}
    for block, lanes, pers, xg, tg in TUNINGS:
        try:
            ctx.set_tuning(block=block, lanes=lanes, persistent=pers, xcd_group=xg, targets=tg)
        except RuntimeError:
            # 3D candidate lists of 256 targets (or of 128 lanes with two
            # targets each) exceed the LDS limit; a quad serves two targets
            # only in FP32
            quad2 = tg == 2 and lanes == 4
            assert (spec.dim == 3 and not quad2 and (block // lanes == 256 or (tg == 2 and block == 128))) or \
                (quad2 and spec.real_bytes == 8)
            continue
        out = ctx.rhs().cpu().numpy().copy()
        if (lanes, tg) in by_shape:
            assert np.array_equal(out, by_shape[(lanes, tg)]), (block, lanes, pers, xg, tg)
        else:
            by_shape[(lanes, tg)] = out
        assert _rel(out.astype(np.float64), r) < (1e-12 if spec.real_bytes == 8 else 1e-5)
    ctx.set_tuning()
    ctx.close()


def test_ensemble_matches_single_plumes():
    """A context holding several plumes of different sizes, dispersivities,
    flow directions and time steps gives, for every plume, the same bits as
    that plume alone."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    specs = I.ensemble(12, sides=(16, 24, 40, 64))
    xs = [s.positions() for s in specs]
    Cs = [s.concentration(x).astype(np.float32).astype(np.float64) for s, x in zip(specs, xs)]
    ens = Context([params_from_spec(s) for s in specs], [s.n for s in specs])
    ens.init(torch.from_numpy(np.concatenate(xs, axis=1)), torch.from_numpy(np.concatenate(Cs))).build()
    ens.step(20)
    Ce = ens.read_C().cpu().numpy()
    me = ens.mass().cpu().numpy()
    off = 0
    for p, s in enumerate(specs):
        one = Context([params_from_spec(s)], [s.n])
        one.init(torch.from_numpy(xs[p]), torch.from_numpy(Cs[p])).build()
        one.step(20)
        C1 = one.read_C().cpu().numpy()
        assert np.array_equal(Ce[off:off + s.n], C1), p
        assert me[p] == one.mass().cpu().numpy()[0]
        assert one.info()["dt"] == pytest.approx(s.dt, rel=1e-15)
        off += s.n
        one.close()
    # and the first plume against the oracle
    s = specs[0]
    _, Co, _ = O.run(O.model_from_spec(s), xs[0], Cs[0], s.dt, 20, v_uniform=s.velocity(), mass=s.mass, rho=s.rho0)
    assert _rel(Ce[:s.n].astype(np.float64), Co) < 1e-5
    ens.close()


def test_autotune_keep_lanes_is_bitwise_neutral():
    """The autotuner times the update-mode kernel, whose outputs it discards:
    with the lanes and targets kept, the right-hand side and the steps after
    tuning are bitwise those of an untuned context."""
    spec = I.config("cfg2_h20_r10", n_side=80)
    ctx, x, C = _ctx(spec)
    ref, _, _ = _ctx(spec)
    before = ctx.rhs().cpu().numpy().copy()
    t = ctx.autotune(reps=2, keep_lanes=True)
    assert (t["lanes"], t["targets"]) == (ref.get_tuning()["lanes"], ref.get_tuning()["targets"])
    after = ctx.rhs().cpu().numpy()
    assert np.array_equal(before, after)
    ctx.step(5)
    ref.step(5)
    assert np.array_equal(ctx.read_C().cpu().numpy(), ref.read_C().cpu().numpy())
    assert np.array_equal(ctx.read_x().cpu().numpy(), ref.read_x().cpu().numpy())
    t2 = ctx.autotune(reps=1)
    assert t2 == ctx.get_tuning()
    ctx.step(3)
    ref.close()
    ctx.close()


# ---------------------------------------------------------------------------
# Two target particles per lane: one merged candidate list serves both
# ---------------------------------------------------------------------------
PAIRED = dict(block=128, lanes=1, targets=2)


@pytest.mark.parametrize("name,over,integrator,steps", [
    ("cfg2_h20_r10", {"n_side": 128}, 1, 100),
    ("cfg2_h13_r100", {"n_side": 101}, 2, 60),                      # odd N: a lane with one target
    ("cfg2_h30_r10", {"n_side": 96}, 1, 60),
    ("cfg1", {"n_side": 45}, 2, 100),                                # FP64, predictor-corrector
    ("cfg3", {"n_side": 20}, 1, 30),
    ("cfg3", {"n_side": 14, "real_bytes": 8}, 2, 20),
])
def test_two_targets_per_lane_trajectory(name, over, integrator, steps):
    """Steps with two targets per lane (merged lists, both integrators, 2D and
    3D, FP32 and FP64) against the oracle, and the right-hand side first."""
    spec = I.config(name, **over)
    ctx, x, C0 = _ctx(spec, integrator=integrator)
    ctx.set_tuning(**PAIRED, xcd_group=8)
    tol = 1e-12 if spec.real_bytes == 8 else 1e-5
    g = ctx.rhs().double().cpu().numpy()
    r = O.rhs(O.model_from_spec(spec), x, C0, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
    assert _rel(g, r) < tol
    ctx.step(steps)
    C = ctx.read_C().double().cpu().numpy()
    _, Co, _ = O.run(O.model_from_spec(spec), x, C0, spec.dt, steps, v_uniform=spec.velocity(),
                     mass=spec.mass, rho=spec.rho0, integrator=integrator)
    assert _rel(C, Co) < tol
    ctx.close()


def _banded(dim, rows_apart, per_row, L, H, seed):
    """Particles only in every rows_apart-th row of the default cell grid
    (rows of height L / nr, nr = floor(2 L / H') as the planner sizes them),
    per_row of them spread along x in each: consecutive particles of the cell
    order then sit in rows that far apart wherever a row's count is odd."""
    rng = np.random.default_rng(seed)
    hu = H / L * TWO32
    hc = hu * (1 + 2.0 ** -16) + 2
    nr = int(np.floor(TWO32 * 2 / hc))
    h = L / nr
    pts = []
    rows = range(0, nr, rows_apart)
    planes = range(0, nr, rows_apart) if dim == 3 else [0]
    for z in planes:
        for y in rows:
            for k in range(per_row):
                p = [rng.uniform(0, L), (y + rng.uniform(0.2, 0.8)) * h]
                if dim == 3:
                    p.append((z + rng.uniform(0.2, 0.8)) * h)
                pts.append(p)
    # on the fixed-point grid the library stores positions on, so that FP64
    # results compare at 1e-12
    return O.to_fixed(np.array(pts).T.copy(), L).astype(np.float64) / TWO32 * L


@pytest.mark.parametrize("dim,real_bytes,rows_apart,per_row,lanes", [(2, 4, 2, 7, 1), (2, 8, 3, 5, 1), (2, 4, 1, 1, 1),
                                                                     (2, 4, 2, 7, 4), (3, 4, 2, 3, 1), (3, 4, 2, 3, 4),
                                                                     (3, 4, 3, 2, 4)])
def test_two_targets_unmerged_pairs(dim, real_bytes, rows_apart, per_row, lanes):
    """Sparse rows make the two targets of many lanes (or quads of lanes)
    sit rows apart, so their candidates cannot share one list: the second
    target walks its own.  The right-hand side and a few steps match the
    oracle, and the bits match between two runs."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = I.config("cfg1" if dim == 2 else "cfg3", n_side=16 if dim == 2 else 12, real_bytes=real_bytes,
                    h_over_dp=1.5)
    x = _banded(dim, rows_apart, per_row, spec.L, spec.H, seed=rows_apart * 10 + per_row)
    n = x.shape[1]
    C = spec.concentration(x)
    if real_bytes == 4:
        C = C.astype(np.float32).astype(np.float64)
    tol = 1e-12 if real_bytes == 8 else 1e-5
    outs = []
    for rep in range(2):
        print(f"[case] banded dim={dim} rb={real_bytes} apart={rows_apart} per_row={per_row} lanes={lanes} n={n} "
              f"rep={rep}", flush=True)
        ctx = Context([params_from_spec(spec)], [n])
        ctx.init(torch.from_numpy(x), torch.from_numpy(C)).build()
        ctx.set_tuning(block=64, lanes=lanes, targets=2)
        g = ctx.rhs().double().cpu().numpy()
        r = O.rhs(O.model_from_spec(spec), x, C, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
        assert np.linalg.norm(r) > 0
        assert _rel(g, r) < tol
        ctx.step(4)
        outs.append(ctx.read_C().cpu().numpy().copy())
        if rep == 0:
            _, Co, _ = O.run(O.model_from_spec(spec), x, C, spec.dt, 4, v_uniform=spec.velocity(),
                             mass=spec.mass, rho=spec.rho0)
            assert _rel(outs[0].astype(np.float64), Co) < tol
        ctx.close()
    assert np.array_equal(outs[0], outs[1])


def test_two_targets_crowded_cells_and_ensemble():
    """Crowded cells (overflow lists) and a multi-plume context with two
    targets per lane: bitwise equal to the same plumes run one by one with
    the same launch shape, and the first plume matches the oracle."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    specs = I.ensemble(6, sides=(16, 24, 40))
    xs = [s.positions() for s in specs]
    Cs = [s.concentration(x).astype(np.float32).astype(np.float64) for s, x in zip(specs, xs)]
    ens = Context([params_from_spec(s) for s in specs], [s.n for s in specs])
    ens.init(torch.from_numpy(np.concatenate(xs, axis=1)), torch.from_numpy(np.concatenate(Cs))).build()
    ens.set_tuning(**PAIRED)
    ens.step(10)
    Ce = ens.read_C().cpu().numpy()
    off = 0
    for p, s in enumerate(specs):
        one = Context([params_from_spec(s)], [s.n])
        one.init(torch.from_numpy(xs[p]), torch.from_numpy(Cs[p])).build()
        one.set_tuning(**PAIRED)
        one.step(10)
        assert np.array_equal(Ce[off:off + s.n], one.read_C().cpu().numpy()), p
        off += s.n
        one.close()
    s = specs[0]
    _, Co, _ = O.run(O.model_from_spec(s), xs[0], Cs[0], s.dt, 10, v_uniform=s.velocity(), mass=s.mass, rho=s.rho0)
    assert _rel(Ce[:s.n].astype(np.float64), Co) < 1e-5
    ens.close()
    spec = I.config("cfg1", n_side=20, real_bytes=4, h_over_dp=1.3)
    x = I.clustered(spec.n_side, 2, 12, 0.02, spec.L, stream=3)
    C = spec.concentration(x).astype(np.float32).astype(np.float64)
    ctx = Context([params_from_spec(spec)], [x.shape[1]])
    ctx.init(torch.from_numpy(x), torch.from_numpy(C)).build()
    ctx.set_tuning(**PAIRED)
    g = ctx.rhs().double().cpu().numpy()
    r = O.rhs(O.model_from_spec(spec), x, C, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
    assert _rel(g, r) < 1e-5
    ctx.close()


def test_two_targets_graph_replay_and_validation():
    """Graph replay equals eager launches with two targets per lane, and the
    launch shapes it cannot take are refused."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = I.config("cfg2_h20_r10", n_side=96)
    outs = []
    for mode in ("eager", "graph"):
        stream = torch.cuda.Stream()
        ctx = Context([params_from_spec(spec)], [spec.n], stream=stream)
        x = spec.positions()
        ctx.init(torch.from_numpy(x), torch.from_numpy(spec.concentration(x))).build()
        ctx.set_tuning(block=64, lanes=1, targets=2, persistent=2048)
        if mode == "eager":
            ctx.step(20)
        else:
            for _ in range(2):
                ctx.step_graph(10)
                torch.cuda.synchronize()
        outs.append(ctx.read_C().cpu().numpy().copy())
        for bad in (dict(block=256, lanes=1, targets=2), dict(block=128, lanes=2, targets=2),
                    dict(block=128, lanes=1, targets=3)):
            with pytest.raises(RuntimeError):
                ctx.set_tuning(**bad)
        stream.synchronize()
        ctx.close()
    assert np.array_equal(outs[0], outs[1])
