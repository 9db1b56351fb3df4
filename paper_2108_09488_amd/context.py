"""Thin Python front end of the C ABI: torch tensors provide the device memory
and the HIP stream, libadesph.so does all of the work."""
from __future__ import annotations

import ctypes as ct
from typing import Sequence

import numpy as np
import torch

from . import _lib
from ._lib import AdeParams, AdeTuning, check, lib


def params_from_spec(spec, integrator: int = _lib.ADE_EULER, flags: int = 0,
                     cell_rows: int = 0, cell_xsub: int = 0) -> AdeParams:
    """ade_params of a PlumeSpec (support radius H = 2 h)."""
    v = list(spec.v) + [0.0] * (3 - len(spec.v))
    return AdeParams(spec.dim, spec.real_bytes, spec.kernel, integrator, spec.H, spec.L,
                     spec.alpha_L, spec.alpha_T, spec.D_m, (ct.c_double * 3)(*v[:3]), spec.dt,
                     spec.rho0, spec.mass, flags, cell_rows, cell_xsub, 0)


def _ptr(t: torch.Tensor) -> ct.c_void_p:
    return ct.c_void_p(t.data_ptr())


def _tuning_dict(t: AdeTuning) -> dict:
    return {"block": t.block, "lanes": t.lanes, "xcd_group": t.xcd_group, "persistent": t.persistent,
            "targets": t.targets if t.targets else 1}


class Context:
    """One context of nplumes plumes (an ensemble when nplumes > 1).

    params  : sequence of AdeParams (or PlumeSpec), one per plume
    counts  : particles per plume
    stream  : torch.cuda.Stream to enqueue on (default: the current stream)
    """

    def __init__(self, params: Sequence, counts: Sequence[int], device="cuda:0", stream=None):
        L = lib()
        ps = [p if isinstance(p, AdeParams) else params_from_spec(p) for p in params]
        self.nplumes = len(ps)
        self._params = (AdeParams * self.nplumes)(*ps)
        self._counts = (ct.c_int64 * self.nplumes)(*[int(c) for c in counts])
        self.dim = ps[0].dim
        self.real_bytes = ps[0].real_bytes
        self.dtype = torch.float32 if self.real_bytes == 4 else torch.float64
        self.device = torch.device(device)
        self.N = int(sum(int(c) for c in counts))
        nb = ct.c_size_t(0)
        check(L.ade_workspace_bytes(self._params, self._counts, self.nplumes, ct.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ct.c_void_p()
        check(L.ade_create(self._params, self._counts, self.nplumes, _ptr(self.ws),
                           self.ws_bytes, ct.c_void_p(self.stream.cuda_stream), ct.byref(h)))
        self._h = h

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().ade_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- stream hand-over ---------------------------------------------------
    def _inputs_ready(self, *ts):
        """Inputs produced on torch's current stream are consumed on the context's."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
            for t in ts:
                t.record_stream(self.stream)

    def _out(self, t: torch.Tensor) -> torch.Tensor:
        """Outputs written on the context's stream become visible to torch's current stream."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            t.record_stream(self.stream)
            cur.wait_stream(self.stream)
        return t

    def _empty(self, *shape, dtype):
        t = torch.empty(*shape, dtype=dtype, device=self.device)
        self._inputs_ready(t)
        return t

    # -- state ---------------------------------------------------------------
    def init(self, x: torch.Tensor, C: torch.Tensor):
        """x: float64 (dim, N) positions; C: (N,) concentrations of the working dtype."""
        x = x.to(self.device, torch.float64).contiguous()
        C = C.to(self.device, self.dtype).contiguous()
        assert x.shape == (self.dim, self.N) and C.shape == (self.N,)
        self._inputs_ready(x, C)
        self._x_in, self._C_in = x, C  # keep alive until the kernels ran
        check(lib().ade_init_particles(self._h, _ptr(x), _ptr(C)))
        return self

    def set_velocities(self, v: torch.Tensor):
        """v: float64 (dim, N) per-particle velocities in id order (contexts made
        with ADE_VELOCITY_FIELD; after init, before build)."""
        v = v.to(self.device, torch.float64).contiguous()
        assert v.shape == (self.dim, self.N)
        self._inputs_ready(v)
        self._v_in = v  # keep alive until the kernel ran
        check(lib().ade_set_velocities(self._h, _ptr(v)))
        return self

    def build(self):
        check(lib().ade_build_cells(self._h))
        return self

    def step(self, n: int = 1):
        check(lib().ade_step(self._h, int(n)))
        return self

    def step_graph(self, n: int = 1):
        check(lib().ade_step_graph(self._h, int(n)))
        return self

    def rhs(self) -> torch.Tensor:
        out = self._empty(self.N, dtype=self.dtype)
        check(lib().ade_rhs(self._h, _ptr(out)))
        return self._out(out)

    def read_C(self) -> torch.Tensor:
        out = self._empty(self.N, dtype=self.dtype)
        check(lib().ade_read_C(self._h, _ptr(out)))
        return self._out(out)

    def read_x(self) -> torch.Tensor:
        out = self._empty((self.dim, self.N), dtype=torch.float64)
        check(lib().ade_read_x(self._h, _ptr(out)))
        return self._out(out)

    def mass(self) -> torch.Tensor:
        out = self._empty(self.nplumes, dtype=torch.float64)
        check(lib().ade_mass(self._h, _ptr(out)))
        return self._out(out)

    def neighbours(self):
        """(offsets (N+1,), ids) as int64 / int32 device tensors (id order)."""
        offsets = self._empty(self.N + 1, dtype=torch.int64)
        need = ct.c_int64(0)
        check(lib().ade_neighbours(self._h, _ptr(offsets), None, 0, ct.byref(need)))
        ids = self._empty(max(need.value, 1), dtype=torch.int32)
        check(lib().ade_neighbours(self._h, _ptr(offsets), _ptr(ids), need.value, ct.byref(need)))
        return self._out(offsets), self._out(ids)[: need.value]

    def save_state(self) -> np.ndarray:
        """The context's state (ade_save_state) as a host byte array."""
        nb = ct.c_size_t(0)
        check(lib().ade_state_bytes(self._h, ct.byref(nb)))
        buf = np.zeros(nb.value, dtype=np.uint8)
        check(lib().ade_save_state(self._h, buf.ctypes.data_as(ct.c_void_p), nb.value))
        return buf

    def load_state(self, buf: np.ndarray):
        """Resume from a state saved by a context of the same parameters."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        check(lib().ade_load_state(self._h, buf.ctypes.data_as(ct.c_void_p), buf.nbytes))
        return self

    def conc_range(self) -> torch.Tensor:
        """(nplumes, 2) float64: the smallest and largest C of each plume."""
        out = self._empty(2 * self.nplumes, dtype=torch.float64)
        check(lib().ade_conc_range(self._h, _ptr(out)))
        return self._out(out).view(self.nplumes, 2)

    def neighbour_counts(self) -> torch.Tensor:
        """offsets (N+1,) int64 of the neighbour lists (id order), without the ids."""
        offsets = self._empty(self.N + 1, dtype=torch.int64)
        need = ct.c_int64(0)
        check(lib().ade_neighbours(self._h, _ptr(offsets), None, 0, ct.byref(need)))
        return self._out(offsets)

    def sensor_interp(self, xs: torch.Tensor) -> torch.Tensor:
        xs = xs.to(self.device, torch.float64).contiguous()
        self._inputs_ready(xs)
        out = self._empty(xs.shape[1], dtype=self.dtype)
        check(lib().ade_sensor_interp(self._h, _ptr(xs), xs.shape[1], _ptr(out)))
        return self._out(out)

    def info(self, plume: int = 0) -> dict:
        n, c, t, st = ct.c_int64(), ct.c_int64(), ct.c_int64(), ct.c_int64()
        dt = ct.c_double()
        check(lib().ade_info(self._h, plume, ct.byref(n), ct.byref(c), ct.byref(t), ct.byref(dt),
                             ct.byref(st)))
        return {"n": n.value, "cells": c.value, "tiles": t.value, "dt": dt.value, "step": st.value}

    def coincident(self) -> bool:
        """Whether two particles of a plume share a position (or the context
        has not been checked): the pair kernels then test every candidate
        for r > 0."""
        v = ct.c_int32()
        check(lib().ade_coincident(self._h, ct.byref(v)))
        return bool(v.value)

    def timing_start(self):
        """Start HIP-event timing of the pair kernel launches."""
        check(lib().ade_kernel_timing(self._h, 1, None, None))

    def timing_stop(self):
        """Stop timing; returns (summed pair-kernel ms, number of launches)."""
        ms, n = ct.c_double(), ct.c_int64()
        check(lib().ade_kernel_timing(self._h, 0, ct.byref(ms), ct.byref(n)))
        return ms.value, n.value

    def autotune(self, reps: int = 5, keep_lanes: bool = False) -> dict:
        """Time the pair kernel over the launch shapes and keep the fastest."""
        t = AdeTuning()
        check(lib().ade_autotune(self._h, int(reps), _lib.ADE_TUNE_KEEP_LANES if keep_lanes else 0,
                                 ct.byref(t)))
        return _tuning_dict(t)

    def set_tuning(self, block=256, lanes=2, persistent=0, xcd_group=0, targets=1):
        t = AdeTuning(block, lanes, xcd_group, persistent, targets)
        check(lib().ade_set_tuning(self._h, ct.byref(t)))

    def get_tuning(self) -> dict:
        t = AdeTuning()
        check(lib().ade_get_tuning(self._h, ct.byref(t)))
        return _tuning_dict(t)

    def adjoint(self, nsteps: int, ckpt_every: int, xs: torch.Tensor, obs: torch.Tensor):
        """J and dJ/d(alpha_L, alpha_T, D_m) of plume 0 after nsteps Euler steps."""
        xs = xs.to(self.device, torch.float64).contiguous()
        obs = obs.to(self.device, self.dtype).contiguous()
        nb = ct.c_size_t(0)
        check(lib().ade_adjoint_workspace_bytes(self._h, int(nsteps), int(ckpt_every), xs.shape[1],
                                                ct.byref(nb)))
        ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device)
        J = ct.c_double()
        g = (ct.c_double * 3)()
        check(lib().ade_adjoint(self._h, int(nsteps), int(ckpt_every), _ptr(xs), xs.shape[1],
                                _ptr(obs), _ptr(ws), nb.value, ct.byref(J), g))
        return J.value, [g[0], g[1], g[2]]

    def adjoint_noalloc(self, nsteps: int, ckpt_every: int, xs: torch.Tensor, obs: torch.Tensor):
        """adjoint() through ade_adjoint_noalloc: the library's static scratch
        array serves as the adjoint workspace (no device allocation in the call;
        xs and obs must already be device tensors of the right type)."""
        assert xs.device == self.device and xs.dtype == torch.float64 and xs.is_contiguous()
        assert obs.device == self.device and obs.dtype == self.dtype and obs.is_contiguous()
        self._inputs_ready(xs, obs)
        J = ct.c_double()
        g = (ct.c_double * 3)()
        check(lib().ade_adjoint_noalloc(self._h, int(nsteps), int(ckpt_every), _ptr(xs), xs.shape[1],
                                        _ptr(obs), ct.byref(J), g))
        return J.value, [g[0], g[1], g[2]]


def workspace_bytes(params, counts) -> int:
    ps = [p if isinstance(p, AdeParams) else params_from_spec(p) for p in params]
    arr = (AdeParams * len(ps))(*ps)
    cn = (ct.c_int64 * len(ps))(*[int(c) for c in counts])
    nb = ct.c_size_t(0)
    check(lib().ade_workspace_bytes(arr, cn, len(ps), ct.byref(nb)))
    return nb.value


class ADEMisfit(torch.autograd.Function):
    """J(theta) = sum_s (C_s(T) - d_s)^2 for theta = (alpha_L, alpha_T, D_m),
    with its gradient from the library's discrete adjoint (ade_adjoint).

    problem: dict with keys spec (PlumeSpec of the plume), x0 (float64 (dim, N)
    positions), C0 (initial concentrations), xs (float64 (dim, S) sensor
    points), obs (S observations), nsteps, ckpt_every, and optionally device.
    When theta requires a gradient the forward pass runs the adjoint (forward,
    recompute and reverse sweep) and keeps the gradient for backward;
    otherwise it only steps the plume and interpolates at the sensors.  The
    gradient comes back on theta's device and in its dtype.
    """

    @staticmethod
    def forward(ctx, theta, problem):
        import copy
        spec = copy.copy(problem["spec"])
        th = theta.detach().to("cpu", torch.float64)
        spec.alpha_L, spec.alpha_T, spec.D_m = float(th[0]), float(th[1]), float(th[2])
        dev = problem.get("device", "cuda:0")
        x0 = torch.as_tensor(problem["x0"], dtype=torch.float64)
        xs = torch.as_tensor(problem["xs"], dtype=torch.float64)
        obs = torch.as_tensor(problem["obs"])
        c = Context([params_from_spec(spec)], [x0.shape[1]], device=dev)
        try:
            c.init(x0, torch.as_tensor(problem["C0"])).build()
            if ctx.needs_input_grad[0]:
                J, g = c.adjoint(problem["nsteps"], problem["ckpt_every"], xs, obs)
            else:
                c.step(problem["nsteps"])
                Cs = c.sensor_interp(xs).double()
                J = float(((Cs - obs.to(Cs.device, torch.float64)) ** 2).sum().item())
                g = [0.0, 0.0, 0.0]
        finally:
            c.close()
        ctx.save_for_backward(torch.tensor(g, dtype=torch.float64))
        ctx.theta_meta = (theta.device, theta.dtype)
        return torch.tensor(J, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, gJ):
        (g,) = ctx.saved_tensors
        dev, dt = ctx.theta_meta
        return (gJ.to(dev, torch.float64) * g.to(dev)).to(dt), None
