"""Velocity-field path (per-particle velocities, the general Eqs. 4-5: the
elementwise harmonic mean of the two particles' tensors and the convective
term) against the FP64 CPU oracle, through the C ABI.

Tolerances as for the uniform flow: neighbour sets and positions bit-exact
(velocities quantised so that every step moves a particle by a whole number
of fixed-point units, as the oracle's FP64 positions then do exactly); FP64
within 1e-12 relative L2, FP32 within 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2108_09488_amd import _lib
from paper_2108_09488_amd import inputs as I

pytestmark = pytest.mark.gpu

TWO32 = 4294967296.0
DT_EXACT = 2.0 ** -12   # with v a multiple of 2^-20 and L = 1: dt v 2^32 / L is an integer
V_QUANTUM = 2.0 ** -20


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _spec(dim, real_bytes, n_side, kernel=4, hod=1.5, jitter=0.1, dt=DT_EXACT):
    base = "cfg1" if dim == 2 else "cfg3"
    return I.config(base, n_side=n_side, real_bytes=real_bytes, kernel=kernel, h_over_dp=hod,
                    jitter=jitter, dt=dt)


def _ctx(spec, v, C=None, stream=None):
    from paper_2108_09488_amd.context import Context, params_from_spec
    print(f"[case] velocity field dim={spec.dim} n={spec.n} rb={spec.real_bytes} k={spec.kernel} "
          f"h/dp={spec.h_over_dp}", flush=True)
    ctx = Context([params_from_spec(spec, flags=_lib.ADE_VELOCITY_FIELD)], [spec.n], stream=stream)
    x = spec.positions()
    if C is None:
        C = spec.concentration(x)
    if spec.real_bytes == 4:
        C = C.astype(np.float32).astype(np.float64)
    ctx.init(torch.from_numpy(x), torch.from_numpy(C)).set_velocities(torch.from_numpy(v)).build()
    return ctx, x, C


def _field(spec, quantise=True):
    x = spec.positions()
    v = I.velocity_field(x, spec.L, quantum=V_QUANTUM if quantise else 0.0)
    if spec.real_bytes == 4:  # what the context stores
        v = v.astype(np.float32).astype(np.float64)
    return v


RHS_CASES = [(2, 8, 40, 2, 1.3), (2, 8, 50, 4, 2.0), (2, 4, 96, 4, 1.5), (2, 4, 70, 4, 3.0),
             (3, 4, 16, 4, 2.0), (3, 8, 12, 2, 1.3), (3, 8, 13, 4, 1.5)]


@pytest.mark.parametrize("dim,rb,n_side,kernel,hod", RHS_CASES)
def test_velocity_field_rhs_parity(dim, rb, n_side, kernel, hod):
    spec = _spec(dim, rb, n_side, kernel, hod)
    v = _field(spec, quantise=False)
    ctx, x, C = _ctx(spec, v)
    g = ctx.rhs().double().cpu().numpy()
    r = O.rhs(O.model_from_spec(spec), x, C, v=v, mass=spec.mass, rho=spec.rho0)
    assert _rel(g, r) < (1e-12 if rb == 8 else 1e-5)
    # the convective term carries weight in this comparison
    r_disp = O.rhs(O.model_from_spec(spec), x, C, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
    assert _rel(r_disp, r) > 1e-2
    ctx.close()


def test_velocity_field_full_size_sampled():
    """The 512^2 FP32 plume of the benchmark (h = 2 dp) with the velocity field:
    the right-hand side at a seeded sample of particles against the oracle,
    then one step: every particle on its exact schedule and the sampled C."""
    spec = I.config("cfg2_h20_r10")
    x = spec.positions()
    v = I.velocity_field(x, spec.L).astype(np.float32).astype(np.float64)
    ctx, x, C = _ctx(spec, v)
    g = ctx.rhs().double().cpu().numpy()
    rng = np.random.default_rng(11)
    inside = np.flatnonzero(C > 1e-3)
    idx = np.sort(rng.choice(inside, size=1500, replace=False))
    r = O.rhs(O.model_from_spec(spec), x, C, v=v, mass=spec.mass, rho=spec.rho0, idx=idx)
    assert _rel(g[idx], r) < 1e-5
    ctx.step(1)
    C1 = ctx.read_C().double().cpu().numpy()
    assert _rel(C1[idx], C[idx] + spec.dt * r) < 1e-5
    xg = ctx.read_x().cpu().numpy()
    u0 = O.to_fixed(x, spec.L).astype(np.int64)
    u1 = np.mod(u0 + np.rint(spec.dt * v / spec.L * TWO32).astype(np.int64), 1 << 32)
    assert np.array_equal(xg, u1.astype(np.float64) / TWO32 * spec.L)
    ctx.close()


def test_uniform_field_matches_uniform_flow():
    """The same velocity for every particle gives the uniform-flow operator
    (the harmonic mean of two equal tensors is twice the tensor, and the
    convective term vanishes)."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = _spec(2, 8, 48, 4, 1.5)
    v = np.tile(spec.velocity()[:, None], (1, spec.n))
    ctx, x, C = _ctx(spec, v)
    g = ctx.rhs().cpu().numpy()
    u = Context([params_from_spec(spec)], [spec.n])
    u.init(torch.from_numpy(x), torch.from_numpy(C)).build()
    gu = u.rhs().cpu().numpy()
    assert _rel(g, gu) < 1e-12
    ctx.close()
    u.close()


@pytest.mark.parametrize("dim,rb,n_side,steps", [(2, 8, 48, 40), (2, 4, 64, 40), (3, 4, 14, 12), (3, 8, 14, 6)])
def test_velocity_field_trajectory(dim, rb, n_side, steps):
    """Explicit Euler with per-particle moves: positions bit-exact (whole
    fixed-point units per step), C within the tolerance, and the neighbour
    sets of the moved particles bit-exact."""
    spec = _spec(dim, rb, n_side, 4, 1.5 if dim == 2 else 2.0)
    v = _field(spec)
    ctx, x, C0 = _ctx(spec, v)
    ctx.step(steps)
    C = ctx.read_C().double().cpu().numpy()
    xg = ctx.read_x().cpu().numpy()
    xo, Co, _ = O.run(O.model_from_spec(spec), x, C0, spec.dt, steps, v=v, mass=spec.mass, rho=spec.rho0)
    assert np.array_equal(xg, xo)
    assert _rel(C, Co) < (1e-12 if rb == 8 else 1e-5)
    off, ids = ctx.neighbours()
    off, ids = off.cpu().numpy(), ids.cpu().numpy()
    seg = np.repeat(np.arange(len(off) - 1), np.diff(off))
    ids = ids[np.lexsort((ids, seg))]
    o_off, o_ids = O.neighbours_fixed(dim, xo, spec.L, spec.H, rb)
    assert np.array_equal(off, o_off) and np.array_equal(ids, o_ids)
    ctx.close()


@pytest.mark.parametrize("dim,rb,n_side,steps", [(2, 8, 48, 30), (2, 4, 64, 30), (3, 4, 14, 8), (3, 8, 12, 6)])
def test_velocity_field_predictor_corrector(dim, rb, n_side, steps):
    """The predictor-corrector of Eqs. (8)-(9) with per-particle velocities:
    the corrector's rhs at x^(1/2) = x + dt/2 v with C^(1/2), after a cell
    build of its own.  Velocities are multiples of 2^-19 with dt = 2^-12, so
    half steps are whole fixed-point units too: positions bit-exact, C within
    the tolerance of the oracle's PC run, neighbour sets bit-exact."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = _spec(dim, rb, n_side, 4, 1.5 if dim == 2 else 2.0)
    x = spec.positions()
    v = I.velocity_field(x, spec.L, quantum=2.0 ** -19)
    if rb == 4:
        v = v.astype(np.float32).astype(np.float64)
    C0 = spec.concentration(x)
    if rb == 4:
        C0 = C0.astype(np.float32).astype(np.float64)
    print(f"[case] velocity field PC dim={dim} rb={rb} n={spec.n}", flush=True)
    ctx = Context([params_from_spec(spec, integrator=_lib.ADE_PC, flags=_lib.ADE_VELOCITY_FIELD)], [spec.n])
    ctx.init(torch.from_numpy(x), torch.from_numpy(C0)).set_velocities(torch.from_numpy(v)).build()
    ctx.step(steps)
    assert ctx.info()["step"] == steps
    C = ctx.read_C().double().cpu().numpy()
    xg = ctx.read_x().cpu().numpy()
    xo, Co, _ = O.run(O.model_from_spec(spec), x, C0, spec.dt, steps, v=v, mass=spec.mass, rho=spec.rho0,
                      integrator=2)
    assert np.array_equal(xg, xo)
    assert _rel(C, Co) < (1e-12 if rb == 8 else 1e-5)
    # and it is not the Euler run
    _, Ce, _ = O.run(O.model_from_spec(spec), x, C0, spec.dt, steps, v=v, mass=spec.mass, rho=spec.rho0)
    assert _rel(Ce, Co) > 1e-7
    off, ids = ctx.neighbours()
    off, ids = off.cpu().numpy(), ids.cpu().numpy()
    seg = np.repeat(np.arange(len(off) - 1), np.diff(off))
    ids = ids[np.lexsort((ids, seg))]
    o_off, o_ids = O.neighbours_fixed(dim, xo, spec.L, spec.H, rb)
    assert np.array_equal(off, o_off) and np.array_equal(ids, o_ids)
    ctx.close()


def test_velocity_field_pc_graph_replay():
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = _spec(2, 4, 48, 4, 1.5)
    x = spec.positions()
    v = torch.from_numpy(I.velocity_field(x, spec.L, quantum=2.0 ** -19))
    C0 = torch.from_numpy(spec.concentration(x).astype(np.float32))
    p = params_from_spec(spec, integrator=_lib.ADE_PC, flags=_lib.ADE_VELOCITY_FIELD)
    outs = []
    for graph in (False, True):
        stream = torch.cuda.Stream()
        ctx = Context([p], [spec.n], stream=stream)
        ctx.init(torch.from_numpy(x), C0).set_velocities(v).build()
        if graph:
            for _ in range(3):
                ctx.step_graph(4)
                torch.cuda.synchronize()
        else:
            ctx.step(12)
        outs.append((ctx.read_C().cpu().numpy().copy(), ctx.read_x().cpu().numpy().copy()))
        stream.synchronize()
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_velocity_field_moves_on_the_exact_schedule():
    """Velocities that are not whole fixed-point units per step: after k steps
    a particle has moved by rint(k u) units, u = dt v / L 2^32 (FP64 state)."""
    spec = _spec(2, 8, 32, 4, 1.5, dt=1.7e-4)
    v = _field(spec, quantise=False)
    ctx, x, _ = _ctx(spec, v)
    k = 9
    ctx.step(k)
    xg = ctx.read_x().cpu().numpy()
    u0 = O.to_fixed(x, spec.L).astype(np.int64)
    us = spec.dt * v / spec.L * TWO32
    uk = np.mod(u0 + np.rint(k * us).astype(np.int64), 1 << 32)
    assert np.array_equal(xg, uk.astype(np.float64) / TWO32 * spec.L)
    ctx.close()


def test_velocity_field_graph_replay_and_determinism():
    spec = _spec(2, 4, 64, 4, 2.0)
    v = _field(spec)
    outs = []
    for graph in (False, False, True):
        stream = torch.cuda.Stream()
        ctx, _, _ = _ctx(spec, v, stream=stream)
        if graph:
            for _ in range(3):  # several graph launches with host work between them
                ctx.step_graph(3)
                torch.cuda.synchronize()
        else:
            ctx.step(9)
        outs.append((ctx.read_C().cpu().numpy().copy(), ctx.read_x().cpu().numpy().copy()))
        assert ctx.info()["step"] == 9
        stream.synchronize()
        ctx.close()
    for C, xx in outs[1:]:
        assert np.array_equal(C, outs[0][0]) and np.array_equal(xx, outs[0][1])


@pytest.mark.parametrize("shape", [None, (64, 4, 2)])
def test_velocity_field_ensemble_matches_single_plumes(shape):
    """Several plumes with velocity fields (different sizes, dispersivities and
    time steps) in one context step to the same bits as each plume alone, at
    the default launch shape and at four lanes per two targets."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    specs = [_spec(2, 4, n, 4, h) for n, h in ((24, 1.3), (40, 2.0), (33, 1.5))]
    specs[1].alpha_T = 1e-4
    specs[2].alpha_L = 3e-2
    specs[2].dt = 2.0 ** -13
    xs = [s.positions() for s in specs]
    Cs = [s.concentration(x).astype(np.float32).astype(np.float64) for s, x in zip(specs, xs)]
    vs = [_field(s) for s in specs]
    flags = _lib.ADE_VELOCITY_FIELD
    print(f"[case] velocity-field ensemble {[s.n for s in specs]}", flush=True)
    ens = Context([params_from_spec(s, flags=flags) for s in specs], [s.n for s in specs])
    ens.init(torch.from_numpy(np.concatenate(xs, axis=1)), torch.from_numpy(np.concatenate(Cs)))
    ens.set_velocities(torch.from_numpy(np.concatenate(vs, axis=1))).build()
    if shape:
        ens.set_tuning(block=shape[0], lanes=shape[1], targets=shape[2])
    ens.step(12)
    Ce, xe = ens.read_C().cpu().numpy(), ens.read_x().cpu().numpy()
    ens.close()
    off = 0
    for s, x, C, v in zip(specs, xs, Cs, vs):
        one = Context([params_from_spec(s, flags=flags)], [s.n])
        one.init(torch.from_numpy(x), torch.from_numpy(C)).set_velocities(torch.from_numpy(v)).build()
        if shape:
            one.set_tuning(block=shape[0], lanes=shape[1], targets=shape[2])
        one.step(12)
        assert np.array_equal(one.read_C().cpu().numpy(), Ce[off:off + s.n])
        assert np.array_equal(one.read_x().cpu().numpy(), xe[:, off:off + s.n])
        one.close()
        off += s.n


@pytest.mark.parametrize("rb,K,integrator,quads", [(8, 7, 1, 0), (4, 7, 1, 0), (8, 1, 1, 0), (4, 40, 1, 0),
                                                   (8, 7, 2, 0), (4, 7, 2, 0), (8, 1, 2, 0), (4, 40, 2, 0),
                                                   (4, 7, 1, 1), (4, 7, 2, 1)])
def test_velocity_field_adjoint_matches_oracle(rb, K, integrator, quads):
    """J, the gradient w.r.t. (alpha_L, alpha_T, D_m) and the final state of the
    velocity-field Euler or predictor-corrector run against the oracle's
    discrete adjoint (itself pinned by finite differences), for checkpoints
    every 1, 7 and 40 steps.  Velocities in multiples of 2^-19: half steps
    are whole fixed-point units too.  quads: the forward and its recompute
    at four lanes per two targets."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = I.config("cfg5", n_side=48, steps=30, dt=DT_EXACT, real_bytes=rb, jitter=0.1, alpha_L=1e-2,
                    alpha_T=5e-3)
    x = spec.positions()
    v = I.velocity_field(x, spec.L, quantum=2.0 ** -19)
    if rb == 4:
        v = v.astype(np.float32).astype(np.float64)
    C0 = spec.concentration(x)
    if rb == 4:
        C0 = C0.astype(np.float32).astype(np.float64)
    xs = I.sensors(64, [0.05, 0.25], [0.55, 0.75])
    truth = O.model(2, 4, spec.H, alpha_L=2e-2, alpha_T=2e-3, D_m=1e-6)
    _, _, CN = O.adjoint_field(truth, x, C0, v, spec.dt, spec.steps, xs, np.zeros(xs.shape[1]),
                               mass=spec.mass, rho=spec.rho0, integrator=integrator)
    obs, _ = O.sensor_interp(truth, (x + spec.steps * spec.dt * v) % spec.L, CN, xs)
    if rb == 4:
        obs = obs.astype(np.float32).astype(np.float64)
    print(f"[case] velocity field adjoint rb={rb} K={K} integ={integrator} quads={quads}", flush=True)
    ctx = Context([params_from_spec(spec, integrator=integrator, flags=_lib.ADE_VELOCITY_FIELD)], [spec.n])
    ctx.init(torch.from_numpy(x), torch.from_numpy(C0)).set_velocities(torch.from_numpy(v)).build()
    if quads:
        ctx.set_tuning(block=128, lanes=4, targets=2)
    J, g = ctx.adjoint(spec.steps, K, torch.from_numpy(xs), torch.from_numpy(obs))
    Jo, go, Co = O.adjoint_field(O.model_from_spec(spec), x, C0, v, spec.dt, spec.steps, xs, obs,
                                 mass=spec.mass, rho=spec.rho0, integrator=integrator)
    Cg = ctx.read_C().double().cpu().numpy()
    assert _rel(Cg, Co) < (1e-12 if rb == 8 else 1e-5)
    tol = 1e-10 if rb == 8 else 1e-4
    print(f"[vf adjoint] rb={rb} K={K} integ={integrator} J {J:.6e} vs {Jo:.6e}, grad {g} vs {list(go)}",
          flush=True)
    assert J == pytest.approx(Jo, rel=tol)
    assert np.allclose(g, go, rtol=tol, atol=tol * np.abs(go).max())
    ctx.close()


@pytest.mark.parametrize("rb", [8, 4])
def test_velocity_field_adjoint_3d(rb):
    """The velocity-field adjoint of a small 3D plume against the oracle's
    (dt = 2^-9: with velocities in multiples of 2^-20 still whole fixed-point
    units per step; truth and guess far enough apart that J is not a
    cancellation)."""
    spec = I.config("cfg3", n_side=14, steps=12, dt=2.0 ** -9, real_bytes=rb, h_over_dp=2.0, alpha_L=1e-2,
                    alpha_T=5e-3)
    x = spec.positions()
    v = _field(spec)
    C0 = spec.concentration(x)
    if rb == 4:
        C0 = C0.astype(np.float32).astype(np.float64)
    xs = I.sensors(40, [0.1, 0.3, 0.3], [0.5, 0.7, 0.7])
    truth = O.model(3, 4, spec.H, alpha_L=4e-2, alpha_T=1e-3, D_m=1e-6)
    _, _, CN = O.adjoint_field(truth, x, C0, v, spec.dt, spec.steps, xs, np.zeros(xs.shape[1]),
                               mass=spec.mass, rho=spec.rho0)
    obs, _ = O.sensor_interp(truth, (x + spec.steps * spec.dt * v) % spec.L, CN, xs)
    if rb == 4:
        obs = obs.astype(np.float32).astype(np.float64)
    ctx, _, _ = _ctx(spec, v, C=C0)
    J, g = ctx.adjoint(spec.steps, 3, torch.from_numpy(xs), torch.from_numpy(obs))
    Jo, go, _ = O.adjoint_field(O.model_from_spec(spec), x, C0, v, spec.dt, spec.steps, xs, obs,
                                mass=spec.mass, rho=spec.rho0)
    tol = 1e-10 if rb == 8 else 1e-4
    assert J == pytest.approx(Jo, rel=tol)
    assert np.allclose(g, go, rtol=tol, atol=tol * np.abs(go).max())
    ctx.close()


def test_velocity_field_validation():
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = _spec(2, 4, 32, 4, 1.5)
    x = spec.positions()
    C = spec.concentration(x).astype(np.float32).astype(np.float64)
    v = torch.from_numpy(_field(spec))
    # a uniform-flow context takes no velocities
    u = Context([params_from_spec(spec)], [spec.n])
    u.init(torch.from_numpy(x), torch.from_numpy(C))
    with pytest.raises(_lib.AdeError) as e:
        u.set_velocities(v)
    assert e.value.code == _lib.ADE_EINVAL
    u.close()
    ctx = Context([params_from_spec(spec, flags=_lib.ADE_VELOCITY_FIELD)], [spec.n])
    with pytest.raises(_lib.AdeError) as e:  # before init
        ctx.set_velocities(v)
    assert e.value.code == _lib.ADE_ESTATE
    ctx.init(torch.from_numpy(x), torch.from_numpy(C))
    with pytest.raises(_lib.AdeError) as e:  # build before the velocities
        ctx.build()
    assert e.value.code == _lib.ADE_ESTATE
    ctx.set_velocities(v).build()
    with pytest.raises(_lib.AdeError) as e:  # after build
        ctx.set_velocities(v)
    assert e.value.code == _lib.ADE_ESTATE
    # launch shapes: one target per group of lanes, or two per quad; no
    # persistent grid
    for bad in (dict(block=128, lanes=1, targets=2), dict(block=128, lanes=2, targets=2),
                dict(block=256, lanes=4, persistent=64), dict(block=96, lanes=4)):
        with pytest.raises(_lib.AdeError) as e:
            ctx.set_tuning(**bad)
        assert e.value.code == _lib.ADE_EINVAL
    ctx.set_tuning(block=128, lanes=2)
    assert (ctx.get_tuning()["block"], ctx.get_tuning()["lanes"]) == (128, 2)
    ctx.set_tuning(block=64, lanes=4, targets=2)
    assert (ctx.get_tuning()["lanes"], ctx.get_tuning()["targets"]) == (4, 2)
    t = ctx.autotune(reps=1)
    assert t["lanes"] in (1, 2, 4) and t["targets"] in (1, 2) and t["persistent"] == 0
    assert t["targets"] == 1 or t["lanes"] == 4
    # init clears the velocities: build needs them again
    ctx.init(torch.from_numpy(x), torch.from_numpy(C))
    with pytest.raises(_lib.AdeError) as e:
        ctx.build()
    assert e.value.code == _lib.ADE_ESTATE
    ctx.close()


def test_velocity_field_launch_shapes():
    """Every launch shape of the velocity-field kernel gives the oracle's
    right-hand side (FP32 1e-5, FP64 1e-12), and the same bits for the same
    lanes and targets per lane group whatever the workgroup size.  Two
    targets a quad exist in 2D FP32 only."""
    for dim, rb, n_side in [(2, 4, 80), (2, 8, 48), (3, 4, 18)]:
        spec = _spec(dim, rb, n_side, 4, 1.5)
        v = _field(spec, quantise=False)
        ctx, x, C = _ctx(spec, v)
        r = O.rhs(O.model_from_spec(spec), x, C, v=v, mass=spec.mass, rho=spec.rho0)
        by_shape = {}
        for lanes, targets in ((1, 1), (2, 1), (4, 1), (4, 2)):
            for block in (64, 128, 256):
                try:
                    ctx.set_tuning(block=block, lanes=lanes, targets=targets)
                except _lib.AdeError:
                    assert targets == 2 and (dim, rb) != (2, 4) or targets == 1
                    continue  # lists do not fit in LDS at this shape, or no such kernel
                g = ctx.rhs().cpu().numpy()
                assert _rel(g.astype(np.float64), r) < (1e-12 if rb == 8 else 1e-5), (dim, rb, block, lanes)
                if (lanes, targets) in by_shape:
                    assert np.array_equal(g, by_shape[(lanes, targets)]), (dim, rb, block, lanes, targets)
                else:
                    by_shape[(lanes, targets)] = g
        assert len(by_shape) == (4 if (dim, rb) == (2, 4) else 3)
        ctx.close()


@pytest.mark.parametrize("integrator,n_side,hod,block,steps", [("euler", 61, 1.5, 64, 30), ("euler", 80, 3.0, 256, 10),
                                                               ("pc", 53, 2.0, 128, 20)])
def test_velocity_field_two_targets_a_quad(integrator, n_side, hod, block, steps):
    """Four lanes per two targets (2D FP32): every record of the pair's
    merged list is evaluated for both targets, b's separation formed from a's.
    Positions bit-exact and C within 1e-5 of the oracle over Euler or
    predictor-corrector steps (odd plume sizes: ragged tiles and a last quad
    with one target), the neighbour sets bit-exact, and the same bits as a
    second run."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = _spec(2, 4, n_side, 4, hod)
    x = spec.positions()
    v = I.velocity_field(x, spec.L, quantum=2.0 ** -19).astype(np.float32).astype(np.float64)
    C0 = spec.concentration(x).astype(np.float32).astype(np.float64)
    integ = _lib.ADE_PC if integrator == "pc" else _lib.ADE_EULER
    outs = []
    for rep in range(2):
        print(f"[case] velocity field quads {integrator} n={spec.n} h/dp={hod} block={block} rep={rep}", flush=True)
        ctx = Context([params_from_spec(spec, integrator=integ, flags=_lib.ADE_VELOCITY_FIELD)], [spec.n])
        ctx.init(torch.from_numpy(x), torch.from_numpy(C0)).set_velocities(torch.from_numpy(v)).build()
        ctx.set_tuning(block=block, lanes=4, targets=2)
        if rep == 0:
            g = ctx.rhs().double().cpu().numpy()
            r = O.rhs(O.model_from_spec(spec), x, C0, v=v, mass=spec.mass, rho=spec.rho0)
            assert _rel(g, r) < 1e-5
        ctx.step(steps)
        outs.append((ctx.read_C().cpu().numpy().copy(), ctx.read_x().cpu().numpy().copy()))
        if rep == 0:
            xo, Co, _ = O.run(O.model_from_spec(spec), x, C0, spec.dt, steps, v=v, mass=spec.mass, rho=spec.rho0,
                              integrator=2 if integrator == "pc" else 1)
            assert np.array_equal(outs[0][1], xo)
            assert _rel(outs[0][0].astype(np.float64), Co) < 1e-5
            off, ids = ctx.neighbours()
            off, ids = off.cpu().numpy(), ids.cpu().numpy()
            seg = np.repeat(np.arange(len(off) - 1), np.diff(off))
            ids = ids[np.lexsort((ids, seg))]
            o_off, o_ids = O.neighbours_fixed(2, xo, spec.L, spec.H, 4)
            assert np.array_equal(off, o_off) and np.array_equal(ids, o_ids)
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_velocity_field_default_shape_many_neighbours():
    """A 2D FP32 velocity-field plume of more than 2000 neighbours per
    particle starts with four lanes per two targets (block 128): its
    right-hand side matches the oracle at sampled particles, and a step
    matches the same context at one target a quad (positions bit-exact)."""
    spec = _spec(2, 4, 96, 4, 14.0)
    v = _field(spec)
    ctx, x, C = _ctx(spec, v)
    t = ctx.get_tuning()
    assert (t["block"], t["lanes"], t["targets"]) == (128, 4, 2)
    g = ctx.rhs().double().cpu().numpy()
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(spec.n, size=400, replace=False))
    r = O.rhs(O.model_from_spec(spec), x, C, v=v, mass=spec.mass, rho=spec.rho0, idx=idx)
    assert _rel(g[idx], r) < 1e-5
    ctx.step(1)
    one, _, _ = _ctx(spec, v)
    one.set_tuning(block=128, lanes=4, targets=1)
    one.step(1)
    assert np.array_equal(ctx.read_x().cpu().numpy(), one.read_x().cpu().numpy())
    assert _rel(ctx.read_C().double().cpu().numpy(), one.read_C().double().cpu().numpy()) < 1e-6
    ctx.close()
    one.close()


def test_velocity_field_two_targets_unmerged_pairs():
    """Sparse rows two apart (seven particles each): the two targets of many
    quads cannot share a list, so those wavefronts walk each target's own
    list in turn.  The right-hand side and four steps match the oracle."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = _spec(2, 4, 16, 4, 1.5)
    rng = np.random.default_rng(27)
    # the rows of the default cell grid: nr = floor(2 L / H'), H' the
    # planner's widened support in grid units
    hc = spec.H / spec.L * TWO32 * (1 + 2.0 ** -16) + 2
    nr = int(np.floor(TWO32 * 2 / hc))
    h = spec.L / nr
    pts = [[rng.uniform(0, spec.L), (y + rng.uniform(0.2, 0.8)) * h] for y in range(0, nr, 2) for _ in range(7)]
    x = O.to_fixed(np.array(pts).T.copy(), spec.L).astype(np.float64) / TWO32 * spec.L
    n = x.shape[1]
    v = I.velocity_field(x, spec.L, quantum=V_QUANTUM).astype(np.float32).astype(np.float64)
    C = spec.concentration(x).astype(np.float32).astype(np.float64)
    print(f"[case] velocity field quads, banded rows n={n}", flush=True)
    ctx = Context([params_from_spec(spec, flags=_lib.ADE_VELOCITY_FIELD)], [n])
    ctx.init(torch.from_numpy(x), torch.from_numpy(C)).set_velocities(torch.from_numpy(v)).build()
    ctx.set_tuning(block=64, lanes=4, targets=2)
    g = ctx.rhs().double().cpu().numpy()
    r = O.rhs(O.model_from_spec(spec), x, C, v=v, mass=spec.mass, rho=spec.rho0)
    assert np.linalg.norm(r) > 0
    assert _rel(g, r) < 1e-5
    ctx.step(4)
    Cg = ctx.read_C().double().cpu().numpy()
    xg = ctx.read_x().cpu().numpy()
    xo, Co, _ = O.run(O.model_from_spec(spec), x, C, spec.dt, 4, v=v, mass=spec.mass, rho=spec.rho0)
    assert np.array_equal(xg, xo)
    assert _rel(Cg, Co) < 1e-5
    ctx.close()
