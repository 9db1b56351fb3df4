"""Full-length FP32 trajectories of the HIP path against the FP64 oracle, at
the problems' own sizes: the six cells of the 2D consistency sweep (512^2
particles, 1000 steps) and the 3D plume (128^3 particles, 500 steps).

The oracle's concentrations after the run, at a seeded sample of 24 000
particles (20 000 inside the plume), come from tests/golden/traj_<case>.npz,
written by tests/golden/make_trajectory_golden.py from the oracle alone.  The
context runs the same steps in the launch shape the benchmark uses (autotuned,
steps replayed from the captured graph) from the same initial state (the
Gaussian rounded to FP32).

Tolerance.  FP32 C carries a rounding of each step into the next; a step
multiplies every eigencomponent of the error by 1 + dt lambda, so a run whose
operator has growing modes amplifies that round-off by up to the growth
max |1 + dt lambda|^steps.  The growth of each case comes from the oracle's
Lanczos report (tests/golden/spectrum.json, with the residual bound added):
the gate is 1e-5 relative L2 times max(1, growth), and a case whose growth
passes 100 (the sweep's h/dp = 1.3 cells, where the operator amplifies some
modes by 1e5 and 1e31 over the run) is compared and reported, not gated.
The FP64 mass of the FP32 state is reported beside it and bounded by 1e-5.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_2108_09488_amd import inputs as I

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CASES = list(I.CFG2_CELLS) + ["cfg3"]
GATE_GROWTH_MAX = 100.0


def _spectrum():
    with open(os.path.join(GOLD, "spectrum.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("case", CASES)
def test_fp32_trajectory_full_length(case):
    from paper_2108_09488_amd.context import Context, params_from_spec
    path = os.path.join(GOLD, f"traj_{case}.npz")
    gold = np.load(path)
    spec = I.config(case)
    steps = int(gold["steps"])
    assert steps == spec.steps and float(gold["dt"]) == spec.dt
    growth = float(_spectrum()[case]["growth_upper"])
    print(f"[case] trajectory {case}: {spec.n} particles, {steps} steps, growth {growth:.3g}", flush=True)
    x = spec.positions()
    C0 = spec.concentration(x).astype(np.float32)
    ctx = Context([params_from_spec(spec)], [spec.n], stream=torch.cuda.Stream())  # graph capture: own stream
    ctx.init(torch.from_numpy(x), torch.from_numpy(C0)).build()
    tuning = ctx.autotune(reps=1)
    m0 = ctx.mass().cpu().numpy()[0]
    ctx.step_graph(steps)
    C = ctx.read_C().double().cpu().numpy()
    m1 = ctx.mass().cpu().numpy()[0]
    ctx.close()
    ids = gold["ids"]
    ref = gold["C"]
    err = float(np.linalg.norm(C[ids] - ref) / np.linalg.norm(ref))
    drift = abs(m1 - m0) / abs(m0)
    gated = growth <= GATE_GROWTH_MAX
    tol = 1e-5 * max(1.0, growth)
    print(f"[result] {case}: rel L2 {err:.3e} (gate {tol:.2e}{'' if gated else ', not gated'}), "
          f"FP64 mass drift of the FP32 state {drift:.2e}, max |C| {np.max(np.abs(C)):.4g}, tuning {tuning}",
          flush=True)
    if gated:
        assert err <= tol, (case, err, tol)
        assert drift <= 1e-5, (case, drift)


def test_fp32_sweep_context_full_length():
    """The six sweep cells in one context, the way the benchmark runs them
    (autotuned launch shape, one graph-replayed step for all six), 1000 steps:
    each plume against its own golden, with its own gate."""
    from paper_2108_09488_amd.context import Context, params_from_spec
    specs = [I.config(c) for c in I.CFG2_CELLS]
    steps = specs[0].steps
    assert all(s.steps == steps for s in specs)
    xs = [s.positions() for s in specs]
    Cs = [s.concentration(x).astype(np.float32) for s, x in zip(specs, xs)]
    print(f"[case] trajectory of the six-plume sweep context, {steps} steps", flush=True)
    ctx = Context([params_from_spec(s) for s in specs], [s.n for s in specs], stream=torch.cuda.Stream())
    ctx.init(torch.from_numpy(np.concatenate(xs, axis=1)), torch.from_numpy(np.concatenate(Cs))).build()
    tuning = ctx.autotune(reps=1)
    ctx.step_graph(steps)
    C = ctx.read_C().double().cpu().numpy()
    ctx.close()
    spec_all = _spectrum()
    off = 0
    for name, s in zip(I.CFG2_CELLS, specs):
        gold = np.load(os.path.join(GOLD, f"traj_{name}.npz"))
        Cp = C[off:off + s.n]
        off += s.n
        err = float(np.linalg.norm(Cp[gold["ids"]] - gold["C"]) / np.linalg.norm(gold["C"]))
        growth = float(spec_all[name]["growth_upper"])
        gated = growth <= GATE_GROWTH_MAX
        print(f"[result] sweep context {name}: rel L2 {err:.3e} ({'gate %.2e' % (1e-5 * max(1.0, growth)) if gated else 'not gated'}), "
              f"tuning {tuning}", flush=True)
        if gated:
            assert err <= 1e-5 * max(1.0, growth), (name, err)
