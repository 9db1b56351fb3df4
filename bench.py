"""Benchmark: particle-neighbour interactions per second of the SPH
advection-dispersion step on one MI355X.

Workload (default, the headline): the 3D plume -- 128^3 = 2,097,152 particles
on a lattice jittered by +-0.1 dp, Wendland C4, h = 2 dp (support H = 4 dp,
~256 neighbours), alpha_L = 1e-2, alpha_T = 1e-3, D_m = 1e-6, v = (1, 0, 0),
FP32 state, explicit Euler steps of 5e-5.  One bench step is one step of the
plume (pair sum of Eqs. 4-5 fused with the update of C and x and the hashing
of the moved particles, then the cell-list rebuild), replayed from the HIP
graph of one captured step, inputs resident in HBM.  value = the directed
interactions of a step (pairs b != a with 0 < r <= H) times the steps,
divided by the wall time of the timed region.

Also reported: the roofline of the pair kernel (HIP events on its eager
launches), the 2D consistency sweep (six 512^2 plumes in one context), the
batched ensemble (256 plumes of 32^2..256^2 particles, 200 graph-replayed
steps), the inverse problem (forward + adjoint), the velocity-field plume and
the paper-scale problems, each with the pair kernel's roofline, and the FP64
CPU oracle on a bounded sample of the headline workload (cpu_baseline).
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
TRAFFIC_PROFILE_3D = os.path.join(ROOT, "profiles", "pair_kernel_traffic_3d.md")
PAIR_SOURCES = ["kernels_pair.hip", "ade_walk.h", "ade_geom.h", "ade_device.h", "ade_internal.h"]
PEAK_FP32_NONPACKED_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA)
# single-issue VALU roof: 256 CU x 64 lanes x 2.4 GHz lane-slots per second, and
# the issue slots one directed interaction needs (the pair term's operations,
# the reciprocal square root at 4 slots): the VALU fraction of a pair kernel
VALU_SLOTS_PER_S = 256 * 64 * 2.4e9
ISSUE_SLOTS_PER_INTERACTION = {2: 27, 3: 36}


def valu_issue_frac(dim, interactions, seconds):
    return ISSUE_SLOTS_PER_INTERACTION[dim] * interactions / seconds / VALU_SLOTS_PER_S


def step_kernel_name(tuning, dim=2, coincident=False):
    """The update-mode pair kernel a launch shape runs (FP32, Wendland C4;
    the last template argument: whether it tests every candidate for r > 0,
    which it does only in a context where two particles share a position)."""
    zc = "true" if coincident else "false"
    if tuning.get("targets", 1) == 2 and tuning["lanes"] == 4:
        # two targets a quad (3D, no coincident particles; else one a quad)
        if dim == 3 and not coincident:
            return "k_pair42<3, float, 4, 0, false>"
        return f"k_pair<{dim}, float, 4, 0, 4, {zc}>"
    if tuning.get("targets", 1) == 2:
        return f"k_pair2<{dim}, float, 4, 0, {zc}>"
    return f"k_pair<{dim}, float, 4, 0, {tuning['lanes']}, {zc}>"


def pair_profile(kernel, key="traffic_bytes_per_launch", profile=None):
    """A figure of the pair kernel from a committed counter profile (HBM bytes
    per launch from FETCH_SIZE/WRITE_SIZE, or the L2 and L1 hit rates), or
    None when the kernel sources changed since it was taken or the profile
    covers another launch shape's kernel."""
    import hashlib
    try:
        text = open(profile or TRAFFIC_PROFILE).read()
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
    launch per kernel per step for all plumes, steps replayed from a HIP
    graph, launch shape (work-item size, lanes and targets per lane,
    persistent grid or not, XCD dealing) picked by the autotuner."""
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
    tuned = ctx.autotune(reps=8)
    ctx.step_graph(warmup)
    _sync()
    t0 = time.perf_counter()
    ctx.step_graph(steps)
    _sync()
    wall = time.perf_counter() - t0
    # the pair kernel's roofline from eager steps with HIP events on its launches
    ectx_steps = min(steps, 20)
    ctx.timing_start()
    ctx.step(ectx_steps)
    _sync()
    pms, pn = ctx.timing_stop()
    n = ctx.N
    coincident = ctx.coincident()
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
            "vs_plain_same_nbar": rate / plain,
            "roofline": roofline_alu(2, inter, pms / pn, step_kernel_name(tuned, coincident=coincident), pn)}


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


def roofline_alu(dim, interactions, ms_per_launch, kernel, launches, profile=None, field=False):
    """Roofline entry of a pair kernel bound by its plain FP32 arithmetic:
    algorithmic flops of one launch (the interactions it evaluates times the
    flops of one) over its mean HIP-event duration, against the published
    FP32 vector peak; with the single-issue VALU fraction and, while the
    kernel sources match a committed counter profile, its HBM bytes, cache
    hit rates and the share of the VALU issue slots it kept busy."""
    fpi = FLOPS_PER_INTERACTION_FIELD[dim] if field else FLOPS_PER_INTERACTION[dim]
    achieved = fpi * interactions / (ms_per_launch * 1e-3) / 1e12
    out = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
           "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
           "traffic": pair_profile(kernel, "traffic_bytes_per_launch", profile) if profile else None,
           "kernel": kernel + " (update mode)", "avg_launch_ms": ms_per_launch, "launches": launches,
           "flops_per_interaction": fpi, "frac_of_nonpacked_peak": achieved / PEAK_FP32_NONPACKED_TFLOPS}
    if not field:
        out["valu_issue_frac"] = valu_issue_frac(dim, interactions, ms_per_launch * 1e-3)
    if profile:
        out["l2_hit_rate"] = pair_profile(kernel, "l2_hit_rate", profile)
        out["l1_hit_rate"] = pair_profile(kernel, "l1_hit_rate", profile)
        # measured share of the VALU issue slots the kernel used (counter run)
        out["valu_slot_util"] = pair_profile(kernel, "valu_slot_util", profile)
    return out


def parse_shape(text):
    """A launch shape given as block,lanes,targets,xcd_group (None if empty)."""
    if not text:
        return None
    b, l, t, x = (int(v) for v in text.split(","))
    return {"block": b, "lanes": l, "targets": t, "xcd_group": x}


def headline_3d(device, steps, warmup, shape=None):
    """The 3D plume (128^3 particles, h = 2 dp, FP32): autotuned launch shape
    (or the given one), `steps` steps replayed from the captured graph after
    `warmup` (the timed region), then the same number of eager steps with HIP
    events around every pair-kernel launch (the roofline)."""
    import numpy as np
    import torch
    from paper_2108_09488_amd import inputs as I
    from paper_2108_09488_amd.context import Context, params_from_spec

    s = I.config("cfg3")
    stream = torch.cuda.Stream(device=device)
    c = Context([params_from_spec(s)], [s.n], device=device, stream=stream)
    x = s.positions()
    c.init(torch.from_numpy(x), torch.from_numpy(s.concentration(x).astype(np.float32))).build()
    inter = int(c.neighbour_counts()[-1].item())
    if shape:
        c.set_tuning(**shape)
        tuned = c.get_tuning()
    else:
        tuned = c.autotune(reps=5)
    print(f"[bench] 3D plume built: {inter} interactions per step, tuning {tuned}", file=sys.stderr, flush=True)
    c.step_graph(warmup)
    _sync()
    t0 = time.perf_counter()
    c.step_graph(steps)
    _sync()
    wall = time.perf_counter() - t0
    c.timing_start()
    t1 = time.perf_counter()
    c.step(steps)
    _sync()
    ewall = time.perf_counter() - t1
    ms, n = c.timing_stop()
    cells = c.info()["cells"]
    coincident = c.coincident()
    c.close()
    kernel = step_kernel_name(tuned, dim=3, coincident=coincident)
    return {"spec": s, "interactions_per_step": inter, "tuning": tuned, "wall": wall, "cells": cells,
            "eager": {"ms_per_step": 1e3 * ewall / steps, "interactions_per_s": inter * steps / ewall,
                      "pair_kernel_ms_per_step": ms / n},
            "roofline": roofline_alu(3, inter, ms / n, kernel, n, profile=TRAFFIC_PROFILE_3D)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_single_thread_sample(n_targets=30000):
    """Child-process body: the oracle's right-hand side of the 3D plume at a
    seeded sample of target particles on one thread; prints JSON."""
    import numpy as np
    import oracle as O
    from paper_2108_09488_amd import inputs as I

    s = I.config("cfg3")
    x = s.positions()
    C = s.concentration(x).astype(np.float32).astype(np.float64)
    m = O.model_from_spec(s)
    idx = np.sort(np.random.default_rng(3).choice(s.n, n_targets, replace=False))
    t0 = time.perf_counter()
    O.rhs(m, x, C, v_uniform=s.velocity(), mass=s.mass, rho=s.rho0, idx=idx)
    wall = time.perf_counter() - t0
    print(json.dumps({"targets": n_targets, "seconds": wall, "threads": O.num_threads()}))


def cpu_baseline_3d(inter_per_step, budget_steps=2):
    """The FP64 oracle on the host cores: whole explicit steps of the 3D plume
    (cell list, pair sum, update) on every core, and the pair sum of a seeded
    sample of targets on one thread (a child process with OMP_NUM_THREADS=1),
    scaled by the sample's share of the step's interactions."""
    import subprocess
    import numpy as np
    import oracle as O
    from paper_2108_09488_amd import inputs as I

    s = I.config("cfg3")
    x = s.positions()
    C = s.concentration(x).astype(np.float32).astype(np.float64)
    m = O.model_from_spec(s)
    t0 = time.perf_counter()
    O.run(m, x, C, s.dt, budget_steps, v_uniform=s.velocity(), mass=s.mass, rho=s.rho0)
    wall = time.perf_counter() - t0
    out = {"value": inter_per_step * budget_steps / wall, "unit": "interactions/s", "cores": O.num_threads(),
           "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "sample": f"{budget_steps} explicit FP64 steps of the 128^3 plume on all host cores "
                     f"({1e3 * wall / budget_steps:.0f} ms per step)"}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-single-thread"], env=env,
                           capture_output=True, text=True, timeout=300)
        st = json.loads(r.stdout.strip().splitlines()[-1])
        # the sample's targets hold the step's mean neighbour count (seeded
        # uniform draw over a near-uniform lattice)
        rate = st["targets"] / s.n * inter_per_step / st["seconds"]
        out["single_thread"] = {"value": rate, "unit": "interactions/s", "threads": st["threads"],
                                "sample": f"the rhs of {st['targets']} seeded targets of the 128^3 plume, "
                                          f"one thread ({st['seconds']:.2f} s, cell list included)"}
    except Exception as e:  # the single-thread figure is context only
        out["single_thread"] = {"error": str(e)[:200]}
    return out


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
    f["roofline"] = roofline_alu(2, f["interactions_per_step"], f["pair_kernel_ms"], "k_pair_gen<2, float, 4, 0, 4>",
                                 steps, field=True)
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


def velocity_paper_scale(device, rounds=3, steps=2):
    """Table 1's first problem (10^6 particles, ~31k neighbours, FP32) with a
    velocity per particle (inputs.velocity_field at the paper's flow speed,
    1.16e-5 m/s): the default launch shape of such plumes (four lanes per two
    targets) against one target a quad, both contexts stepped in lockstep,
    the pair kernel timed by HIP events round by round (the particles move
    under the field, so the rounds differ; the two shapes see the same
    states)."""
    import numpy as np
    import torch
    from paper_2108_09488_amd import _lib
    from paper_2108_09488_amd import inputs as I
    from paper_2108_09488_amd.context import Context, params_from_spec

    s = I.config("paper1m")
    x = s.positions()
    C = torch.from_numpy(s.concentration(x).astype(np.float32))
    v = torch.from_numpy(I.velocity_field(x, s.L, U=1.16e-5))
    shapes = {"two_targets_a_quad": None, "one_target_a_quad": {"block": 128, "lanes": 4, "targets": 1}}
    ctxs = {}
    for k, t in shapes.items():
        c = Context([params_from_spec(s, flags=_lib.ADE_VELOCITY_FIELD)], [s.n], device=device,
                    stream=torch.cuda.Stream(device=device))
        c.init(torch.from_numpy(x), C).set_velocities(v).build()
        if t:
            c.set_tuning(**t)
        ctxs[k] = c
    inter = int(ctxs["two_targets_a_quad"].neighbour_counts()[-1].item())
    res = {k: [] for k in shapes}
    for _ in range(rounds):
        for k, c in ctxs.items():
            c.timing_start()
            c.step(steps)
            _sync()
            ms, n = c.timing_stop()
            res[k].append(ms / n)
    out = {"particles": s.n, "interactions_per_step_initial": inter, "steps_per_round": steps}
    for k, c in ctxs.items():
        out[k] = {"tuning": c.get_tuning(), "pair_kernel_ms_min": min(res[k]), "pair_kernel_ms_rounds": res[k]}
        c.close()
    out["speedup"] = out["one_target_a_quad"]["pair_kernel_ms_min"] / out["two_targets_a_quad"]["pair_kernel_ms_min"]
    print(f"[bench] velocity field, 10^6 particles: pair kernel {out['two_targets_a_quad']['pair_kernel_ms_min']:.1f} "
          f"ms (two targets a quad) vs {out['one_target_a_quad']['pair_kernel_ms_min']:.1f} ms (one)",
          file=sys.stderr, flush=True)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip every workload but the headline")
    ap.add_argument("--extras", default="sweep,batched,fwd_adjoint,velocity_field,paper_scale,velocity_paper",
                    help="comma-separated extras to run (unless --no-extras)")
    ap.add_argument("--cells", default="", help="comma-separated subset of the sweep plumes")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of this many MiB (a known-size "
                         "reference for the HBM byte counters of a profiler run)")
    ap.add_argument("--shape-3d", default="", metavar="B,L,T,X",
                    help="launch shape of the 3D plume (block,lanes,targets,xcd_group) instead of "
                         "the autotuner's, so that profiler runs see one kernel configuration")
    ap.add_argument("--shape-sweep", default="", metavar="B,L,T,X",
                    help="the same for the sweep context")
    ap.add_argument("--cpu-single-thread", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_single_thread:  # child process of cpu_baseline_3d (no GPU use)
        cpu_single_thread_sample()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): every workload here is "
              "a single-GPU workload, and no multi-GPU path is built.", file=sys.stderr)
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

    # the headline: the 3D plume, graph-replayed steps
    h = headline_3d(device, args.steps, args.warmup, parse_shape(args.shape_3d))
    inter3 = h["interactions_per_step"]
    value = inter3 * args.steps / h["wall"]
    print(f"[bench] 3D plume: {1e3 * h['wall'] / args.steps:.3f} ms/step (graph), pair kernel "
          f"{1e3 * h['roofline']['avg_launch_ms']:.1f} us", file=sys.stderr, flush=True)
    extras = {"eager": h["eager"]}
    want = set() if args.no_extras else set(args.extras.split(","))
    if "sweep" in want:
        cells = args.cells.split(",") if args.cells else list(I.CFG2_CELLS)
        sweep = build_sweep(cells, device)
        if args.shape_sweep:
            sweep["ctx"].set_tuning(**parse_shape(args.shape_sweep))
            sweep["tuning"] = sweep["ctx"].get_tuning()
        else:
            sweep["tuning"] = sweep["ctx"].autotune(reps=8)
        inter_step = sum(sweep["interactions"])
        wall, _ = time_sweep(sweep, args.steps, args.warmup, graph=True)
        ewall, pair = time_sweep(sweep, args.steps, args.warmup, graph=False)
        coincident = sweep["ctx"].coincident()
        sweep["ctx"].close()
        kname = step_kernel_name(sweep["tuning"], coincident=coincident)
        extras["sweep"] = {
            "workload": "2D consistency sweep: 6 plumes x 512^2 particles, jitter 0.1 dp, Wendland C4, "
                        "h/dp {1.3,2,3} x alpha_L/alpha_T {10,100}, FP32, explicit Euler, dt Eq. (10), "
                        "one context",
            "interactions_per_step": inter_step, "tuning": sweep["tuning"],
            "per_plume": {n: {"interactions_per_step": i, "neighbours_mean": i / s.n}
                          for n, i, s in zip(sweep["names"], sweep["interactions"], sweep["specs"])},
            "ms_per_step": 1e3 * wall / args.steps, "interactions_per_s": inter_step * args.steps / wall,
            "eager_ms_per_step": 1e3 * ewall / args.steps,
            "roofline": roofline_alu(2, inter_step, pair["ms_total"] / pair["launches"], kname,
                                     pair["launches"], profile=TRAFFIC_PROFILE)}
        print(f"[bench] sweep: {1e3 * wall / args.steps:.3f} ms/step (graph)", file=sys.stderr, flush=True)
    if "batched" in want:
        b = batched(device, steps=200, warmup=args.warmup)
        b["vs_plain"] = b["interactions_per_s"] / extras["sweep"]["interactions_per_s"] if "sweep" in extras else None
        b["vs_plain_workload"] = "the six-plume 2D sweep context (graph replay)"
        extras["batched"] = b
        print(f"[bench] batched: {b['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    if "fwd_adjoint" in want:
        extras["fwd_adjoint"] = fwd_adjoint(device)
        print(f"[bench] fwd+adjoint: {extras['fwd_adjoint']['ms_fwd_adjoint']:.1f} ms", file=sys.stderr, flush=True)
    if "paper_scale" in want:
        extras["paper_scale"] = paper_scale(device)
    if "velocity_paper" in want:
        extras["velocity_paper"] = velocity_paper_scale(device)
    if "velocity_field" in want:
        vf = velocity_field(device, steps=min(args.steps, 100))
        extras["velocity_field"] = vf
        print(f"[bench] velocity field: {vf['field']['ms_per_step']:.3f} ms/step "
              f"(pair kernel {1e3 * vf['field']['pair_kernel_ms']:.1f} us), uniform "
              f"{vf['uniform']['ms_per_step']:.3f} ms/step; fwd+adjoint "
              f"{vf['fwd_adjoint']['ms_fwd_adjoint']:.1f} ms vs fwd {vf['fwd_adjoint']['ms_fwd']:.1f} ms",
              file=sys.stderr, flush=True)

    s3 = h["spec"]
    line = {
        "metric": "particle-neighbour interactions/s per ADE step (fwd, fwd+adjoint, batched) vs plain",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * h["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D plume: 128^3 particles, jitter 0.1 dp, Wendland C4, h = 2 dp (support 4 dp), "
                               "alpha_L 1e-2, alpha_T 1e-3, D_m 1e-6, v = (1, 0, 0), FP32 state, explicit Euler, "
                               "dt 5e-5, graph-replayed steps",
                   "particles": s3.n, "interactions_per_step": inter3,
                   "neighbours_mean": inter3 / s3.n, "cells": h["cells"], "tuning": h["tuning"]},
        "roofline": h["roofline"],
        "extras": extras,
    }
    if not args.no_cpu:
        print("[bench] cpu baseline ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline_3d(inter3)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
