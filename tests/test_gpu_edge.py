"""Degenerate cases of the method through the C ABI against the FP64 CPU
oracle: no flow (D = D_m I, nothing moves), alpha_T > alpha_L (the transverse
direction dominates, the 2D pair term folds a negative a1), isotropic
dispersion (alpha_L = alpha_T), D_m = 0, particles of a velocity field with a
zero tensor (v = 0 and D_m = 0: every harmonic mean with them is 0), and
plumes of one and of seven particles beside a normal one.  Tolerances: FP64
1e-12, FP32 1e-5 relative L2 (absolute where the exact answer is 0)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2108_09488_amd import _lib
from paper_2108_09488_amd import inputs as I

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


FLOWS = [  # (dim, real_bytes, v, alpha_L, alpha_T, D_m)
    (2, 8, (0.0, 0.0, 0.0), 1e-2, 1e-3, 1e-6),
    (2, 4, (0.0, 0.0, 0.0), 1e-2, 1e-3, 1e-6),
    (2, 8, (0.6, 0.8, 0.0), 1e-3, 1e-2, 1e-6),
    (2, 4, (1.0, 0.0, 0.0), 1e-3, 2e-2, 0.0),
    (2, 8, (0.6, -0.8, 0.0), 5e-3, 5e-3, 1e-6),
    (2, 4, (-0.28, 0.96, 0.0), 2e-2, 2e-3, 0.0),
    (3, 4, (0.0, 0.0, 0.0), 1e-2, 1e-3, 1e-6),
    (3, 8, (0.48, 0.6, 0.64), 1e-3, 1e-2, 1e-6),
    (3, 4, (0.48, -0.6, 0.64), 2e-3, 3e-2, 1e-6),
]


@pytest.mark.parametrize("dim,rb,v,aL,aT,Dm", FLOWS)
def test_degenerate_flows(dim, rb, v, aL, aT, Dm):
    from paper_2108_09488_amd.context import Context, params_from_spec
    base = "cfg1" if dim == 2 else "cfg3"
    spec = I.config(base, n_side=48 if dim == 2 else 14, real_bytes=rb, kernel=4, h_over_dp=1.5,
                    jitter=0.1, v=v, alpha_L=aL, alpha_T=aT, D_m=Dm, dt=2.0 ** -14)
    print(f"[case] flow dim={dim} rb={rb} v={v} aL={aL} aT={aT} Dm={Dm}", flush=True)
    ctx = Context([params_from_spec(spec)], [spec.n])
    x = spec.positions()
    C = spec.concentration(x)
    if rb == 4:
        C = C.astype(np.float32).astype(np.float64)
    ctx.init(torch.from_numpy(x), torch.from_numpy(C)).build()
    g = ctx.rhs().double().cpu().numpy()
    m = O.model(dim, 4, spec.H, L=spec.L, alpha_L=aL, alpha_T=aT, D_m=Dm)
    r = O.rhs(m, x, C, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
    assert _rel(g, r) < (1e-12 if rb == 8 else 1e-5)
    steps = 6
    ctx.step(steps)
    Cg = ctx.read_C().double().cpu().numpy()
    xg = ctx.read_x().cpu().numpy()
    _, Co, _ = O.run(m, x, C, spec.dt, steps, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
    assert _rel(Cg, Co) < (1e-12 if rb == 8 else 1e-5)
    if not any(v[:dim]):
        assert np.array_equal(xg, x)  # no flow: nothing moves
    ctx.close()


@pytest.mark.parametrize("rb,quads", [(8, 0), (4, 0), (4, 1)])
def test_velocity_field_with_zero_tensors(rb, quads):
    """With D_m = 0, particles at rest have D = 0: their reciprocals are
    infinite and every harmonic mean with them vanishes (Eq. 5 with the zero
    product rule), while the convective term still acts.  quads: four lanes
    per two targets (b's separations formed from a's)."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = I.config("cfg1", n_side=40, real_bytes=rb, kernel=4, h_over_dp=1.5, jitter=0.1, D_m=0.0,
                    dt=2.0 ** -12)
    x = spec.positions()
    v = I.velocity_field(x, spec.L, quantum=2.0 ** -20)
    rest = (np.arange(spec.n) % 3) == 0  # every third particle at rest
    v[:, rest] = 0.0
    v[1, ~rest & ((np.arange(spec.n) % 3) == 1)] = 0.0  # others along x only: D_xy = 0
    C = spec.concentration(x)
    if rb == 4:
        C = C.astype(np.float32).astype(np.float64)
    print(f"[case] velocity field with zero tensors rb={rb} quads={quads}", flush=True)
    ctx = Context([params_from_spec(spec, flags=_lib.ADE_VELOCITY_FIELD)], [spec.n])
    ctx.init(torch.from_numpy(x), torch.from_numpy(C)).set_velocities(torch.from_numpy(v)).build()
    if quads:
        ctx.set_tuning(block=64, lanes=4, targets=2)
    g = ctx.rhs().double().cpu().numpy()
    assert np.all(np.isfinite(g))
    m = O.model_from_spec(spec)
    r = O.rhs(m, x, C, v=v, mass=spec.mass, rho=spec.rho0)
    assert _rel(g, r) < (1e-12 if rb == 8 else 1e-5)
    ctx.step(5)
    Cg = ctx.read_C().double().cpu().numpy()
    xo, Co, _ = O.run(m, x, C, spec.dt, 5, v=v, mass=spec.mass, rho=spec.rho0)
    assert np.array_equal(ctx.read_x().cpu().numpy(), xo)
    assert _rel(Cg, Co) < (1e-12 if rb == 8 else 1e-5)
    ctx.close()


def test_tiny_plumes_in_an_ensemble():
    """Plumes of one particle (no neighbours: rhs 0, C unchanged) and of seven
    (one ragged tile, a few neighbours) beside a normal plume: each matches the
    oracle and the normal plume matches itself alone."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    big = I.config("cfg1", n_side=32, real_bytes=8, kernel=4, h_over_dp=1.5)
    one = I.config("cfg1", n_side=1, real_bytes=8, kernel=4, h_over_dp=0.15)
    seven = I.config("cfg1", n_side=1, real_bytes=8, kernel=4, h_over_dp=0.15)
    x_one = np.array([[0.3], [0.7]])
    # seven particles within H = 0.3 of each other around (0.5, 0.5)
    ang = np.arange(7) * 2 * np.pi / 7
    x_seven = I.quantize(np.stack([0.5 + 0.08 * np.cos(ang), 0.5 + 0.08 * np.sin(ang)]), 1.0)
    x_big = big.positions()
    C_big = big.concentration(x_big)
    C_one = np.array([0.8])
    C_seven = np.linspace(0.1, 0.9, 7)
    specs = [big, one, seven]
    xs, Cs, ns = [x_big, x_one, x_seven], [C_big, C_one, C_seven], [big.n, 1, 7]
    print("[case] tiny plumes", flush=True)
    ens = Context([params_from_spec(s) for s in specs], ns)
    ens.init(torch.from_numpy(np.concatenate(xs, axis=1)), torch.from_numpy(np.concatenate(Cs))).build()
    g = ens.rhs().cpu().numpy()
    off = 0
    for s, x, C, n in zip(specs, xs, Cs, ns):
        r = O.rhs(O.model_from_spec(s), x, C, v_uniform=s.velocity(), mass=s.mass, rho=s.rho0)
        if n == 1:
            assert g[off] == 0.0 and r[0] == 0.0
        else:
            assert np.max(np.abs(r)) > 0
            assert _rel(g[off:off + n], r) < 1e-12
        off += n
    ens.step(4)
    Ce = ens.read_C().cpu().numpy()
    assert Ce[big.n] == C_one[0]
    alone = Context([params_from_spec(big)], [big.n])
    alone.init(torch.from_numpy(x_big), torch.from_numpy(C_big)).build()
    alone.step(4)
    assert np.array_equal(alone.read_C().cpu().numpy(), Ce[:big.n])
    alone.close()
    ens.close()


@pytest.mark.parametrize("flags", [0, _lib.ADE_CHECK_FINITE])
def test_finite_check(flags):
    """A NaN forced into C from the host: with ADE_CHECK_FINITE the step
    reports ADE_ENONFINITE (eager and graph replay); without it the steps run
    and the NaN spreads to the neighbours."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = I.config("cfg1", n_side=32, real_bytes=4, kernel=4, h_over_dp=1.5)
    x = spec.positions()
    C = spec.concentration(x).astype(np.float32)
    clean = C.copy()
    C[spec.n // 2] = np.nan
    print(f"[case] finite check flags={flags}", flush=True)
    for graph in (False, True):
        stream = torch.cuda.Stream()
        ctx = Context([params_from_spec(spec, flags=flags)], [spec.n], stream=stream)
        ctx.init(torch.from_numpy(x), torch.from_numpy(clean)).build()
        (ctx.step_graph if graph else ctx.step)(2)  # finite: no error either way
        ctx.init(torch.from_numpy(x), torch.from_numpy(C)).build()
        if flags:
            with pytest.raises(_lib.AdeError) as e:
                (ctx.step_graph if graph else ctx.step)(2)
            assert e.value.code == _lib.ADE_ENONFINITE
        else:
            (ctx.step_graph if graph else ctx.step)(2)
            assert np.isnan(ctx.read_C().cpu().numpy()).sum() > 1
        stream.synchronize()
        ctx.close()


@pytest.mark.parametrize("velocity_field,integrator", [(False, 1), (False, 2), (True, 1), (True, 2)])
def test_save_and_resume_is_bit_identical(velocity_field, integrator):
    """ade_save_state after some steps, ade_load_state into a fresh context of
    the same parameters: the resumed run matches the uninterrupted one bit for
    bit (C, positions, step counter).  A state of other parameters, or a
    short buffer, is rejected."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = I.config("cfg2_h20_r10", n_side=96)
    x = spec.positions()
    C = spec.concentration(x).astype(np.float32)
    flags = _lib.ADE_VELOCITY_FIELD if velocity_field else 0
    p = params_from_spec(spec, integrator=integrator, flags=flags)
    v = torch.from_numpy(I.velocity_field(x, spec.L, quantum=2.0 ** -20))
    print(f"[case] save/resume vf={velocity_field} integ={integrator}", flush=True)

    def fresh():
        c = Context([p], [spec.n])
        c.init(torch.from_numpy(x), torch.from_numpy(C))
        if velocity_field:
            c.set_velocities(v)
        return c.build()

    a = fresh()
    a.step(7)
    state = a.save_state()
    a.step(9)
    Ca, xa, sa = a.read_C().cpu().numpy(), a.read_x().cpu().numpy(), a.info()["step"]
    b = Context([p], [spec.n])
    b.load_state(state)
    assert b.info()["step"] == 7
    b.step(9)
    assert np.array_equal(b.read_C().cpu().numpy(), Ca)
    assert np.array_equal(b.read_x().cpu().numpy(), xa)
    assert b.info()["step"] == sa == 16
    with pytest.raises(_lib.AdeError) as e:
        b.load_state(state[: len(state) - 1])
    assert e.value.code == _lib.ADE_EINVAL
    other = Context([params_from_spec(I.config("cfg2_h20_r10", n_side=64), integrator=integrator, flags=flags)],
                    [64 * 64])
    with pytest.raises(_lib.AdeError) as e:
        other.load_state(state)
    assert e.value.code == _lib.ADE_EINVAL
    for c in (a, b, other):
        c.close()


def test_state_of_another_plume_split_is_rejected():
    """Two contexts of the same particle and cell totals whose plumes are
    split differently (the same support radius on two lattices, in either
    order) do not share a saved state; a context of the saving one's split
    takes it."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    a = I.config("cfg2_h20_r10", n_side=64, h_over_dp=4.0)
    b = I.config("cfg2_h20_r10", n_side=32, h_over_dp=2.0)
    assert a.H == b.H
    print("[case] state of another plume split", flush=True)

    def ctx(specs):
        return Context([params_from_spec(s) for s in specs], [s.n for s in specs])

    xs = [s.positions() for s in (a, b)]
    Cs = [s.concentration(x).astype(np.float32) for s, x in zip((a, b), xs)]
    src = ctx((a, b))
    src.init(torch.from_numpy(np.concatenate(xs, axis=1)), torch.from_numpy(np.concatenate(Cs))).build()
    src.step(3)
    state = src.save_state()
    swapped, same = ctx((b, a)), ctx((a, b))
    assert swapped.info()["cells"] == same.info()["cells"]
    with pytest.raises(_lib.AdeError) as e:
        swapped.load_state(state)
    assert e.value.code == _lib.ADE_EINVAL
    same.load_state(state)
    src.step(2)
    same.step(2)
    assert np.array_equal(same.read_C().cpu().numpy(), src.read_C().cpu().numpy())
    for c in (src, swapped, same):
        c.close()


def test_concentration_range_per_plume():
    """ade_conc_range gives each plume's smallest and largest C exactly
    (min and max do not depend on the order), also after steps that push
    concentrations below zero."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    specs = I.ensemble(5, sides=(16, 24, 40))
    xs = [s.positions() for s in specs]
    Cs = [s.concentration(x).astype(np.float32) for s, x in zip(specs, xs)]
    print("[case] concentration range", flush=True)
    ens = Context([params_from_spec(s) for s in specs], [s.n for s in specs])
    ens.init(torch.from_numpy(np.concatenate(xs, axis=1)), torch.from_numpy(np.concatenate(Cs))).build()
    for steps in (0, 25):
        ens.step(steps)
        C = ens.read_C().double().cpu().numpy()
        got = ens.conc_range().cpu().numpy()
        off = 0
        for p, s in enumerate(specs):
            assert got[p, 0] == C[off:off + s.n].min() and got[p, 1] == C[off:off + s.n].max()
            off += s.n
    ens.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_coincident_particles(dim):
    """Distinct particles at one position: the sum of Eq. (4) leaves such
    pairs out (r = 0).  The cell build finds them, so the context keeps the
    pair kernels that test every candidate for r > 0, and the rhs and a few
    FP32 steps match the oracle; the same plume without them is reported
    free of coincidences (and its kernels skip the test)."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    base = "cfg1" if dim == 2 else "cfg3"
    spec = I.config(base, n_side=48 if dim == 2 else 14, real_bytes=4, kernel=4, h_over_dp=1.5,
                    jitter=0.1, dt=2.0 ** -14)
    x = spec.positions()
    C = spec.concentration(x).astype(np.float32).astype(np.float64)
    xc = x.copy()
    xc[:, 500:510] = x[:, 10:20]  # ten particles moved onto ten others (their C differ)
    assert np.any(C[500:510] != C[10:20])
    m = O.model_from_spec(spec)
    # in 3D also with two targets a quad (which a context with coincident
    # particles runs as one target a quad)
    shapes = [None] + ([dict(block=64, lanes=4, targets=2)] if dim == 3 else [])
    for (pos, coincident), shape in [(pc, sh) for pc in ((x, False), (xc, True)) for sh in shapes]:
        print(f"[case] coincident particles dim={dim} planted={coincident} shape={shape}", flush=True)
        ctx = Context([params_from_spec(spec)], [spec.n])
        ctx.init(torch.from_numpy(pos), torch.from_numpy(C))
        assert ctx.coincident()  # unchecked before the cell build
        ctx.build()
        assert ctx.coincident() == coincident
        if shape:
            ctx.set_tuning(**shape)
        g = ctx.rhs().double().cpu().numpy()
        r = O.rhs(m, pos, C, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
        assert _rel(g, r) < 1e-5
        steps = 6
        ctx.step(steps)
        Cg = ctx.read_C().double().cpu().numpy()
        _, Co, _ = O.run(m, pos, C, spec.dt, steps, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
        assert _rel(Cg, Co) < 1e-5
        ctx.close()
