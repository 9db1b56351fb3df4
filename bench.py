"""Benchmark: particle-neighbour interactions per second of the SPH
advection-dispersion step on one MI355X.

Workload (default): the 2D consistency sweep -- six 512^2-particle plumes on
jittered lattices (+-0.1 dp), Wendland C4, h/dp in {1.3, 2, 3} x
alpha_L/alpha_T in {10, 100}, FP32, dt from Eq. (10), held in one context.
One bench step advances each of the six plumes by one explicit step (pair sum
of Eqs. 4-5, update of C and x, cell-list rebuild), one launch per kernel for
all six.  value = sum over plumes of the
directed interactions per step (pairs b != a with 0 < r <= H) times the
steps, divided by the wall time of the timed region.

Also reported: the HIP-event time of the pair kernel and its roofline, the
same sweep replayed from HIP graphs, the batched ensemble (256 plumes of
32^2..256^2 particles in one context), and the FP64 CPU oracle on a bounded
sample of the same workload (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic floating-point work of one directed interaction (FMA = 2 flops):
# separation (d), r^2 (2d - 1), rsqrt (1), q (2), Wendland C4 polynomial (7),
# quadratic form x^T (Gamma D) x (7 in 2D, 14 in 3D), A = Q / r^2 - tr D (3),
# C_a - C_b (1), accumulation (3).
FLOPS_PER_INTERACTION = {2: 29, 3: 39}
# the velocity-field pair term in 2D: the uniform term's separation, kernel and
# sum, plus three harmonic means (a division each), the tensor quadratic form
# and the convective dot product
FLOPS_PER_INTERACTION_FIELD = {2: 57}
PEAK_FP32_VECTOR_TFLOPS = 157.3      # MI355X published vector FP32 (packed FMA)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pair_kernel_traffic.md")
PAIR_SOURCES = ["kernels_pair.hip", "ade_walk.h", "ade_geom.h", "ade_device.h", "ade_internal.h"]
PEAK_FP32_NONPACKED_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA)
# single-issue VALU roof: 256 CU x 64 lanes x 2.4 GHz lane-slots per second, and
# the issue slots one directed interaction needs (the pair term's operations,
# the reciprocal square root at 4 slots): the VALU fraction of a pair kernel
VALU_SLOTS_PER_S = 256 * 64 * 2.4e9
ISSUE_SLOTS_PER_INTERACTION = {2: 27, 3: 36}


def valu_issue_frac(dim, interactions, seconds):
    return ISSUE_SLOTS_PER_INTERACTION[dim] * interactions / seconds / VALU_SLOTS_PER_S


def step_kernel_name(tuning):
    """The update-mode pair kernel a launch shape runs (2D, FP32, Wendland C4)."""
    if tuning.get("targets", 1) == 2:
        return "k_pair2<2, float, 4, 0>"
    return f"k_pair<2, float, 4, 0, {tuning['lanes']}>"


def pair_profile(kernel, key="traffic_bytes_per_launch"):
    """A figure of the pair kernel from the committed counter profile (HBM
    bytes per launch from FETCH_SIZE/WRITE_SIZE, or the L2 and L1 hit rates),
    or None when the kernel sources changed since it was taken or the profile
    covers another launch shape's kernel."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    vals = dict(l.split(":", 1) for l in text.splitlines()
                if l.startswith((key + ":", "source_sha256:", "kernel:")))
    if vals.get("kernel", "").strip() != kernel or key not in vals:
        return None
    h = hashlib.sha256()
    for f in PAIR_SOURCES:
        with open(os.path.join(ROOT, "paper_2108_09488_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if vals.get("source_sha256", "").strip() != h.hexdigest():
        return None
    return float(vals[key])


def pair_traffic(kernel):
    return pair_profile(kernel, "traffic_bytes_per_launch")


def _sync():
    import torch
    torch.cuda.synchronize()


def build_sweep(cells, device):
    """The sweep plumes in one context: every kernel of a step is one launch
    over all plumes (each plume keeps its own cell grid, dt and parameters)."""
    import numpy as np
    import torch
    from paper_2108_09488_amd import inputs as I
    from paper_2108_09488_amd.context import Context, params_from_spec

    specs = [I.config(name) for name in cells]
    stream = torch.cuda.Stream(device=device)
    ctx = Context([params_from_spec(s) for s in specs], [s.n for s in specs], device=device,
                  stream=stream)
    xs = [s.positions() for s in specs]
    Cs = [s.concentration(x).astype(np.float32) for s, x in zip(specs, xs)]
    ctx.init(torch.from_numpy(np.concatenate(xs, axis=1)),
             torch.from_numpy(np.concatenate(Cs))).build()
    off, _ = ctx.neighbours()
    bounds = np.concatenate([[0], np.cumsum([s.n for s in specs])])
    per = [int(off[bounds[p + 1]].item() - off[bounds[p]].item()) for p in range(len(specs))]
    return {"ctx": ctx, "specs": specs, "names": list(cells), "interactions": per}


def time_sweep(sweep, steps, warmup, graph):
    ctx = sweep["ctx"]
    (ctx.step_graph if graph else ctx.step)(warmup)
    _sync()
    if not graph:
        ctx.timing_start()
    t0 = time.perf_counter()
    (ctx.step_graph if graph else ctx.step)(steps)
    _sync()
    wall = time.perf_counter() - t0
    pair = None
    if not graph:
        ms, c = ctx.timing_stop()
        flops = sum(i * FLOPS_PER_INTERACTION[s.dim] for i, s in zip(sweep["interactions"], sweep["specs"]))
        pair = {"ms_total": ms, "launches": c, "flops": flops * c}
    return wall, pair


def batched(device, steps, warmup, n_plumes=256):
    """The ensemble: 256 plumes of 32^2..256^2 particles with their own
    dispersivities, flow directions and time steps, in one context: one
    launch per kernel per step, the pair kernel on a persistent grid, steps
    replayed from a HIP graph, launch shape picked by the autotuner."""
    import numpy as np
    import torch
    from paper_2108_09488_amd import inputs as I
    from paper_2108_09488_amd.context import Context, params_from_spec

    specs = I.ensemble(n_plumes)
    stream = torch.cuda.Stream(device=device)
    ctx = Context([params_from_spec(s) for s in specs], [s.n for s in specs], device=device, stream=stream)
    xs = np.concatenate([s.positions() for s in specs], axis=1)
    Cs = np.concatenate([s.concentration(s.positions()) for s in specs])
    ctx.init(torch.from_numpy(xs), torch.from_numpy(Cs.astype(np.float32))).build()
    off, _ = ctx.neighbours()
    inter = int(off[-1].item())
    tuned = ctx.autotune(reps=3)
    ctx.step_graph(warmup)
    _sync()
    t0 = time.perf_counter()
    ctx.step_graph(steps)
    _sync()
    wall = time.perf_counter() - t0
    n = ctx.N
    ctx.close()
    # plain reference at the ensemble's neighbour count: one 512^2 plume with
    # h = 1.5 dp (the ensemble's smoothing length), the same kernel and jitter
    ref = I.config("cfg2_h20_r10", h_over_dp=1.5)
    rc = Context([params_from_spec(ref)], [ref.n], device=device, stream=stream)
    xr = ref.positions()
    rc.init(torch.from_numpy(xr), torch.from_numpy(ref.concentration(xr).astype(np.float32))).build()
    rinter = int(rc.neighbour_counts()[-1].item())
    rc.autotune(reps=3)
    rc.step_graph(warmup)
    _sync()
    t0 = time.perf_counter()
    rc.step_graph(steps)
    _sync()
    rwall = time.perf_counter() - t0
    rc.close()
    plain = rinter * steps / rwall
    rate = inter * steps / wall
    return {"plumes": n_plumes, "particles": n, "interactions_per_step": inter,
            "steps": steps, "ms_per_step": 1e3 * wall / steps, "tuning": tuned,
            "interactions_per_s": rate,
            "plain_same_nbar": {"workload": "one 512^2 plume, h/dp 1.5, C4, FP32, graph replay",
                                "neighbours_mean": rinter / ref.n, "interactions_per_s": plain},
            "vs_plain_same_nbar": rate / plain}


def fwd_adjoint(device):
    """The inverse problem: 256^2 particles, 500 Euler steps of 1e-4, 1024
    sensors; J and dJ/d(alpha_L, alpha_T, D_m) by the adjoint with a
    checkpoint every 50 steps (forward + recompute + reverse sweep), against
    the plain forward of the same plume.  Observations come from a GPU forward
    run at alpha_L = 2e-2, alpha_T = 2e-3 (timing only, no parity claim)."""
    import numpy as np
    import torch
    from paper_2108_09488_amd import inputs as I
    from paper_2108_09488_amd.context import Context, params_from_spec

    xs = torch.from_numpy(I.sensors(1024, [0.05, 0.25], [0.55, 0.75]))
    truth = I.config("cfg5")
    guess = I.config("cfg5", alpha_L=1e-2, alpha_T=5e-3)
    x = truth.positions()
    C0 = torch.from_numpy(truth.concentration(x).astype(np.float32))
    c = Context([params_from_spec(truth)], [truth.n], device=device)
    c.init(torch.from_numpy(x), C0).build()
    c.step(truth.steps)
    obs = c.sensor_interp(xs)
    c.close()
    c = Context([params_from_spec(guess)], [guess.n], device=device)
    c.init(torch.from_numpy(x), C0).build()
    tuning = c.autotune(reps=3)
    off, _ = c.neighbours()
    inter = int(off[-1].item())
    c.adjoint(guess.steps, 50, xs, obs)  # warm-up
    c.init(torch.from_numpy(x), C0).build()
    _sync()
    t0 = time.perf_counter()
    J, g = c.adjoint(guess.steps, 50, xs, obs)
    _sync()
    wall_adj = time.perf_counter() - t0
    c.init(torch.from_numpy(x), C0).build()
    _sync()
    t0 = time.perf_counter()
    c.step(guess.steps)
    _sync()
    wall_fwd = time.perf_counter() - t0
    c.close()
    return {"particles": guess.n, "steps": guess.steps, "interactions_per_step": inter, "tuning": tuning,
            "ms_fwd_adjoint": 1e3 * wall_adj, "ms_fwd": 1e3 * wall_fwd,
            "interactions_per_s": inter * guess.steps / wall_adj,
            "fwd_interactions_per_s": inter * guess.steps / wall_fwd,
            "vs_plain": wall_fwd / wall_adj, "J": J, "grad": g}


def single_3d(device, steps=10):
    """One 3D plume, 128^3 particles, h = 2 dp (about 270 neighbours)."""
    import numpy as np
    import torch
    from paper_2108_09488_amd import inputs as I
    from paper_2108_09488_amd.context import Context, params_from_spec

    s = I.config("cfg3")
    c = Context([params_from_spec(s)], [s.n], device=device)
    x = s.positions()
    c.init(torch.from_numpy(x), torch.from_numpy(s.concentration(x).astype(np.float32))).build()
    off, _ = c.neighbours()
    inter = int(off[-1].item())
    tuned = c.autotune(reps=2)
    c.step(2)
    _sync()
    t0 = time.perf_counter()
    c.step(steps)
    _sync()
    wall = time.perf_counter() - t0
    c.close()
    return {"particles": s.n, "interactions_per_step": inter, "steps": steps, "tuning": tuned,
            "ms_per_step": 1e3 * wall / steps, "interactions_per_s": inter * steps / wall,
            "valu_issue_frac_of_step": valu_issue_frac(3, inter * steps, wall)}


def velocity_field(device, steps=50, warmup=3):
    """One 512^2 sweep plume (h = 2 dp, FP32) with a velocity per particle (the
    smooth periodic field of inputs.velocity_field: harmonic means of the
    per-particle tensors and the convective term active), beside the same plume
    in the uniform flow; eager steps with the pair kernel timed by HIP events."""
    import numpy as np
    import torch
    from paper_2108_09488_amd import _lib
    from paper_2108_09488_amd import inputs as I
    from paper_2108_09488_amd.context import Context, params_from_spec

    s = I.config("cfg2_h20_r10")
    x = s.positions()
    C = s.concentration(x).astype(np.float32)
    v = I.velocity_field(x, s.L)
    out = {}
    for kind in ("uniform", "field"):
        stream = torch.cuda.Stream(device=device)
        flags = _lib.ADE_VELOCITY_FIELD if kind == "field" else 0
        c = Context([params_from_spec(s, flags=flags)], [s.n], device=device, stream=stream)
        c.init(torch.from_numpy(x), torch.from_numpy(C))
        if kind == "field":
            c.set_velocities(torch.from_numpy(v))
        c.build()
        off, _ = c.neighbours()
        inter = int(off[-1].item())
        if kind == "uniform":
            c.autotune(reps=2)
        c.step(warmup)
        _sync()
        c.timing_start()
        t0 = time.perf_counter()
        c.step(steps)
        _sync()
        wall = time.perf_counter() - t0
        ms, n = c.timing_stop()
        c.close()
        out[kind] = {"ms_per_step": 1e3 * wall / steps, "pair_kernel_ms": ms / n,
                     "interactions_per_step": inter, "interactions_per_s": inter * steps / wall}
    f = out["field"]
    f["vs_uniform"] = f["interactions_per_s"] / out["uniform"]["interactions_per_s"]
    out["fwd_adjoint"] = velocity_field_adjoint(device)
    achieved = FLOPS_PER_INTERACTION_FIELD[2] * f["interactions_per_step"] / (f["pair_kernel_ms"] * 1e-3) / 1e12
    f["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "flops_per_interaction": FLOPS_PER_INTERACTION_FIELD[2],
                     "kernel": "k_pair_gen<2, float, 4, 0, 4> (update mode)"}
    out["workload"] = ("cfg2 plume h/dp 2, alpha_L/alpha_T 10, 512^2 FP32, explicit Euler; "
                       "interactions counted at the initial positions")
    return out


def paper_scale(device, steps=3):
    """The paper-scale problems of Table 1: 10^6 particles with ~31k neighbours
    each (autotuned) and 4x10^6 with ~78k (the default launch shape of such
    plumes), FP32, eager steps with the pair kernel timed by HIP events."""
    import numpy as np
    import torch
    from paper_2108_09488_amd import inputs as I
    from paper_2108_09488_amd.context import Context, params_from_spec

    out = {}
    for name, tune in (("paper1m", True), ("paper4m", False)):
        s = I.config(name)
        stream = torch.cuda.Stream(device=device)
        c = Context([params_from_spec(s)], [s.n], device=device, stream=stream)
        x = s.positions()
        c.init(torch.from_numpy(x), torch.from_numpy(s.concentration(x).astype(np.float32))).build()
        inter = int(c.neighbour_counts()[-1].item())
        tuning = c.autotune(reps=1) if tune else c.get_tuning()
        c.step(1)
        _sync()
        c.timing_start()
        t0 = time.perf_counter()
        c.step(steps)
        _sync()
        wall = time.perf_counter() - t0
        ms, n = c.timing_stop()
        cells = c.info()["cells"]
        c.close()
        achieved = FLOPS_PER_INTERACTION[2] * inter / (ms / n * 1e-3) / 1e12
        out[name] = {"particles": s.n, "neighbours_mean": inter / s.n, "interactions_per_step": inter,
                     "cells": cells, "steps": steps, "tuning": tuning, "ms_per_step": 1e3 * wall / steps,
                     "pair_kernel_ms": ms / n, "interactions_per_s": inter * steps / wall,
                     "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
                                  "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                                  "valu_issue_frac": valu_issue_frac(2, inter, ms / n * 1e-3)}}
        _sync()
        print(f"[bench] {name}: {out[name]['ms_per_step']:.1f} ms/step, "
              f"{out[name]['interactions_per_s']:.3e} interactions/s", file=sys.stderr, flush=True)
    return out


def velocity_field_adjoint(device, steps=200, ckpt=20):
    """The inverse problem of fwd_adjoint (256^2 particles, 1024 sensors, guess
    alpha_L = 1e-2, alpha_T = 5e-3) with the velocity field of
    inputs.velocity_field: forward + recompute + reverse sweep with a
    checkpoint every 20 steps against the plain forward, 200 steps.
    Observations from a GPU forward run at the true parameters (timing only)."""
    import numpy as np
    import torch
    from paper_2108_09488_amd import _lib
    from paper_2108_09488_amd import inputs as I
    from paper_2108_09488_amd.context import Context, params_from_spec

    xs = torch.from_numpy(I.sensors(1024, [0.05, 0.25], [0.55, 0.75]))
    truth = I.config("cfg5", steps=steps)
    guess = I.config("cfg5", steps=steps, alpha_L=1e-2, alpha_T=5e-3)
    x = truth.positions()
    v = torch.from_numpy(I.velocity_field(x, truth.L))
    C0 = torch.from_numpy(truth.concentration(x).astype(np.float32))
    flags = _lib.ADE_VELOCITY_FIELD

    def fresh(spec):
        c = Context([params_from_spec(spec, flags=flags)], [spec.n], device=device)
        c.init(torch.from_numpy(x), C0).set_velocities(v).build()
        return c

    c = fresh(truth)
    c.step(steps)
    obs = c.sensor_interp(xs)
    c.close()
    c = fresh(guess)
    inter = int(c.neighbour_counts()[-1].item())
    c.adjoint(steps, ckpt, xs, obs)  # warm-up
    c.close()
    c = fresh(guess)
    _sync()
    t0 = time.perf_counter()
    J, g = c.adjoint(steps, ckpt, xs, obs)
    _sync()
    wall_adj = time.perf_counter() - t0
    c.close()
    c = fresh(guess)
    _sync()
    t0 = time.perf_counter()
    c.step(steps)
    _sync()
    wall_fwd = time.perf_counter() - t0
    c.close()
    return {"particles": guess.n, "steps": steps, "ckpt_every": ckpt, "interactions_per_step": inter,
            "ms_fwd_adjoint": 1e3 * wall_adj, "ms_fwd": 1e3 * wall_fwd,
            "interactions_per_s": inter * steps / wall_adj, "vs_plain": wall_fwd / wall_adj,
            "J": J, "grad": g}


def cpu_baseline(cells, budget_s=20.0):
    """The FP64 oracle on the host cores: one explicit step of each plume of
    the sweep (full 512^2 size), repeated while within the time budget."""
    import numpy as np
    import oracle as O
    from paper_2108_09488_amd import inputs as I

    total_inter = 0
    total_wall = 0.0
    reps = 0
    specs = [I.config(c) for c in cells]
    prepared = []
    for s in specs:
        x = s.positions()
        C = s.concentration(x).astype(np.float32).astype(np.float64)
        m = O.model_from_spec(s)
        off, _ = O.neighbours_cells(m, x)
        prepared.append((s, m, x, C, int(off[-1])))
    while total_wall < budget_s and reps < 3:
        for s, m, x, C, inter in prepared:
            t0 = time.perf_counter()
            O.run(m, x, C, s.dt, 1, v_uniform=s.velocity(), mass=s.mass, rho=s.rho0)
            total_wall += time.perf_counter() - t0
            total_inter += inter
        reps += 1
    return {"value": total_inter / total_wall, "unit": "interactions/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{reps} explicit step(s) of each of the {len(cells)} 512^2 sweep plumes, FP64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip graph replay and batched runs")
    ap.add_argument("--extras", default="batched,fwd_adjoint,single_3d,velocity_field,paper_scale",
                    help="comma-separated extras to run (unless --no-extras)")
    ap.add_argument("--cells", default="", help="comma-separated subset of the sweep plumes")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of this many MiB (a known-size "
                         "reference for the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sweep and the "
              "ensemble are single-GPU workloads here.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2108_09488_amd import inputs as I

    device = "cuda:0"
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration * (1 << 20) // 4, dtype=torch.float32, device=device)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cells = args.cells.split(",") if args.cells else list(I.CFG2_CELLS)
    sweep = build_sweep(cells, device)
    sweep["tuning"] = sweep["ctx"].autotune(reps=3)
    inter_step = sum(sweep["interactions"])
    print(f"[bench] sweep built: {len(cells)} plumes, {inter_step} interactions per step, "
          f"tuning {sweep['tuning']}", file=sys.stderr, flush=True)

    # timed region: every plume's captured step replayed from its HIP graph
    wall, _ = time_sweep(sweep, args.steps, args.warmup, graph=True)
    value = inter_step * args.steps / wall
    print(f"[bench] graph: {1e3 * wall / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    # the same steps launched eagerly, with HIP events around every pair kernel
    ewall, pair = time_sweep(sweep, args.steps, args.warmup, graph=False)
    print(f"[bench] eager: {1e3 * ewall / args.steps:.3f} ms/step", file=sys.stderr, flush=True)
    avg_ms = pair["ms_total"] / pair["launches"]
    achieved = pair["flops"] / (pair["ms_total"] * 1e-3) / 1e12
    extras = {"eager": {"ms_per_step": 1e3 * ewall / args.steps,
                        "interactions_per_s": inter_step * args.steps / ewall,
                        "pair_kernel_ms_per_step": pair["ms_total"] / args.steps}}
    want = set() if args.no_extras else set(args.extras.split(","))
    if "batched" in want:
        b = batched(device, steps=min(args.steps, 200), warmup=args.warmup)
        b["vs_plain"] = b["interactions_per_s"] / value
        extras["batched"] = b
        print(f"[bench] batched: {b['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if "fwd_adjoint" in want:
        extras["fwd_adjoint"] = fwd_adjoint(device)
        print(f"[bench] fwd+adjoint: {extras['fwd_adjoint']['ms_fwd_adjoint']:.1f} ms", file=sys.stderr, flush=True)
    if "single_3d" in want:
        extras["single_3d"] = single_3d(device)
        print(f"[bench] 3D: {extras['single_3d']['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if "paper_scale" in want:
        extras["paper_scale"] = paper_scale(device)
    if "velocity_field" in want:
        vf = velocity_field(device, steps=min(args.steps, 100))
        extras["velocity_field"] = vf
        print(f"[bench] velocity field: {vf['field']['ms_per_step']:.3f} ms/step "
              f"(pair kernel {1e3 * vf['field']['pair_kernel_ms']:.1f} us), uniform "
              f"{vf['uniform']['ms_per_step']:.3f} ms/step; fwd+adjoint "
              f"{vf['fwd_adjoint']['ms_fwd_adjoint']:.1f} ms vs fwd {vf['fwd_adjoint']['ms_fwd']:.1f} ms",
              file=sys.stderr, flush=True)
    per_cell = {n: {"interactions_per_step": i, "neighbours_mean": i / s.n}
                for n, i, s in zip(sweep["names"], sweep["interactions"], sweep["specs"])}
    sweep["ctx"].close()

    line = {
        "metric": "particle-neighbour interactions/s per ADE step (fwd, fwd+adjoint, batched) vs plain",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D consistency sweep: 6 plumes x 512^2 particles, jitter 0.1 dp, "
                               "Wendland C4, h/dp {1.3,2,3} x alpha_L/alpha_T {10,100}, FP32, "
                               "explicit Euler, dt Eq. (10)",
                   "plumes": cells, "interactions_per_step": inter_step, "per_plume": per_cell,
                   "tuning": sweep["tuning"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": pair_traffic(step_kernel_name(sweep["tuning"])),
                     "kernel": step_kernel_name(sweep["tuning"]) + " (update mode)", "avg_launch_ms": avg_ms,
                     "launches": pair["launches"],
                     "flops_per_interaction": FLOPS_PER_INTERACTION[2],
                     "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED_TFLOPS,
                     "valu_issue_frac": valu_issue_frac(2, inter_step * pair["launches"], pair["ms_total"] * 1e-3),
                     "l2_hit_rate": pair_profile(step_kernel_name(sweep["tuning"]), "l2_hit_rate"),
                     "l1_hit_rate": pair_profile(step_kernel_name(sweep["tuning"]), "l1_hit_rate")},
        "extras": extras,
    }
    if not args.no_cpu:
        print("[bench] cpu baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(cells)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
