"""Python access to the FP64 CPU oracle (oracle.c), via ctypes.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the HIP implementation; inputs come from the seeded generators in
``paper_2108_09488_amd.inputs`` (which hold none of the method's arithmetic).

Each function names the equation of Klapp et al. (arXiv:2108.09488) it follows;
the C source carries the equations and the readings of ambiguous points.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Compile oracle.c with gcc (FP64, OpenMP, no contraction of a*b+c)."""
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wno-unused-function",
           _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Model(ct.Structure):
    """or_model: dim, kernel (2 = Wendland C2, 4 = Wendland C4), support radius H,
    box side L, alpha_L, alpha_T, D_m (Eq. 3), Gamma (Eq. 5)."""
    _fields_ = [("dim", ct.c_int32), ("kernel", ct.c_int32), ("H", ct.c_double),
                ("L", ct.c_double), ("alpha_L", ct.c_double), ("alpha_T", ct.c_double),
                ("D_m", ct.c_double), ("gamma", ct.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ct.CDLL(_LIB)
        d, i32, i64, p = ct.c_double, ct.c_int, ct.c_int64, ct.c_void_p
        mp = ct.POINTER(Model)
        L.or_kernel_B.restype = d
        L.or_kernel_B.argtypes = [i32, i32, d]
        L.or_kernel_W.restype = d
        L.or_kernel_W.argtypes = [i32, i32, d, d]
        L.or_kernel_dWdr.restype = d
        L.or_kernel_dWdr.argtypes = [i32, i32, d, d]
        L.or_dispersion.argtypes = [i32, d, d, d, p, p]
        L.or_harmonic.argtypes = [i32, p, p, p]
        L.or_neighbours_brute.argtypes = [mp, i64, p, p, p, p]
        L.or_neighbours_cells.argtypes = [mp, i64, p, p, p, p]
        L.or_neighbours_fixed.argtypes = [i32, i64, p, d, d, i32, i32, p, p, p]
        L.or_rhs.argtypes = [mp, i64, p, p, p, p, p, p, p, i64, p, p]
        L.or_rhs_brute.argtypes = [mp, i64, p, p, p, p, p, p, p]
        L.or_mass.restype = d
        L.or_mass.argtypes = [i64, p, p]
        L.or_run.argtypes = [mp, i64, p, p, p, p, p, p, d, i64, i32, p]
        L.or_dt_rule.restype = d
        L.or_dt_rule.argtypes = [mp, p, d]
        L.or_analytic.argtypes = [mp, p, p, d, d, d, i64, p, p]
        L.or_sensor_interp.argtypes = [mp, i64, p, p, i64, p, p, p]
        L.or_apply_LT.argtypes = [mp, i64, p, p, p, p, p, p]
        L.or_adjoint.argtypes = [mp, i64, p, p, p, p, p, d, i64, i64, p, p, i32, p, p, p]
        L.or_misfit.restype = d
        L.or_misfit.argtypes = [mp, i64, p, p, p, p, p, d, i64, i64, p, p, i32, p]
        L.or_rhs_deriv.argtypes = [mp, i64, p, p, p, p, p, i32, p]
        L.or_apply_LT_field.argtypes = [mp, i64, p, p, p, p, p, p]
        L.or_adjoint_field.argtypes = [mp, i64, p, p, p, p, p, d, i64, i64, p, p, i32, p, p, p]
        L.or_misfit_field.restype = d
        L.or_misfit_field.argtypes = [mp, i64, p, p, p, p, p, d, i64, i64, p, p, i32]
        L.or_num_threads.restype = ct.c_int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def model(dim, kernel, H, L=1.0, alpha_L=1e-2, alpha_T=1e-3, D_m=1e-6, gamma=None) -> Model:
    """Gamma defaults to d + 2 (= 4 in 2D as printed in Eq. 5)."""
    return Model(dim, kernel, H, L, alpha_L, alpha_T, D_m, float(dim + 2) if gamma is None else gamma)


def model_from_spec(spec) -> Model:
    return model(spec.dim, spec.kernel, spec.H, spec.L, spec.alpha_L, spec.alpha_T, spec.D_m)


def kernel_B(kernel, dim, H):
    return lib().or_kernel_B(kernel, dim, H)


def kernel_W(kernel, dim, H, r):
    return lib().or_kernel_W(kernel, dim, H, float(r))


def kernel_dWdr(kernel, dim, H, r):
    return lib().or_kernel_dWdr(kernel, dim, H, float(r))


def dispersion(dim, aL, aT, Dm, v):
    """Eq. (3) tensor, shape (dim, dim)."""
    v = _f64(v)
    D = np.zeros(dim * dim)
    lib().or_dispersion(dim, aL, aT, Dm, _ptr(v), _ptr(D))
    return D.reshape(dim, dim)


def harmonic(Da, Db):
    """Eq. (5) elementwise 4 D_a D_b / (D_a + D_b), 0 where D_a D_b <= 0."""
    Da, Db = _f64(Da), _f64(Db)
    dim = Da.shape[0]
    h = np.zeros(dim * dim)
    lib().or_harmonic(dim, _ptr(Da), _ptr(Db), _ptr(h))
    return h.reshape(dim, dim)


def _csr(fn, n, *args):
    counts = np.zeros(n, dtype=np.int64)
    fn(*args, _ptr(counts), None, None)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    ids = np.zeros(max(int(offsets[-1]), 1), dtype=np.int32)
    fn(*args, _ptr(counts), _ptr(offsets), _ptr(ids))
    return offsets, ids[: offsets[-1]]


def neighbours_brute(m: Model, x):
    """Neighbour sets (CSR: offsets, ascending ids) with the FP64 predicate, O(N^2)."""
    x = _f64(x)
    n = x.shape[1]
    return _csr(lambda *a: lib().or_neighbours_brute(ct.byref(m), n, _ptr(x), *a), n)


def neighbours_cells(m: Model, x):
    """Same sets via the cell-linked list."""
    x = _f64(x)
    n = x.shape[1]
    return _csr(lambda *a: lib().or_neighbours_cells(ct.byref(m), n, _ptr(x), *a), n)


def to_fixed(x, L=1.0):
    """Positions as uint32 fractions of the box: round(x / L * 2^32) mod 2^32."""
    u = np.mod(np.rint(_f64(x) / L * 4294967296.0), 4294967296.0)
    return np.ascontiguousarray(u.astype(np.uint64).astype(np.uint32))


def neighbours_fixed(dim, x, L, H, real_bytes, force_brute=False):
    """Neighbour sets under the fixed-point predicate in the working precision
    (cell list, or all pairs when force_brute)."""
    u = to_fixed(x, L)
    n = u.shape[1]
    return _csr(lambda *a: lib().or_neighbours_fixed(dim, n, _ptr(u), L, H, real_bytes,
                                                     int(force_brute), *a), n)


def _particle_arrays(n, mass, rho):
    m_arr = _f64(np.broadcast_to(mass, (n,)))
    r_arr = _f64(np.broadcast_to(rho, (n,)))
    return m_arr, r_arr


def rhs(m: Model, x, C, v_uniform=None, v=None, mass=1.0, rho=1.0, idx=None, Dfix=None):
    """Eq. (4)-(5) right-hand side (dispersion + convective part) for all
    particles or for the particle indices idx."""
    x, C = _f64(x), _f64(C)
    n = x.shape[1]
    vu = _f64(np.zeros(3) if v_uniform is None else np.pad(np.asarray(v_uniform, float), (0, 3 - len(v_uniform))))
    vv = None if v is None else _f64(v)
    m_arr, r_arr = _particle_arrays(n, mass, rho)
    if idx is None:
        out = np.zeros(n)
        nidx, ip = n, None
    else:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        out = np.zeros(len(idx))
        nidx, ip = len(idx), _ptr(idx)
    Df = None if Dfix is None else _f64(Dfix)
    lib().or_rhs(ct.byref(m), n, _ptr(x), _ptr(C), _ptr(vv), _ptr(vu), _ptr(m_arr), _ptr(r_arr),
                 _ptr(Df), nidx, ip, _ptr(out))
    return out


def rhs_brute(m: Model, x, C, v_uniform=None, v=None, mass=1.0, rho=1.0):
    x, C = _f64(x), _f64(C)
    n = x.shape[1]
    vu = _f64(np.zeros(3) if v_uniform is None else np.pad(np.asarray(v_uniform, float), (0, 3 - len(v_uniform))))
    vv = None if v is None else _f64(v)
    m_arr, r_arr = _particle_arrays(n, mass, rho)
    out = np.zeros(n)
    lib().or_rhs_brute(ct.byref(m), n, _ptr(x), _ptr(C), _ptr(vv), _ptr(vu), _ptr(m_arr),
                       _ptr(r_arr), _ptr(out))
    return out


def run(m: Model, x, C, dt, nsteps, v_uniform=None, v=None, mass=1.0, rho=1.0, integrator=1):
    """Explicit Euler (1) or predictor-corrector (2, Eqs. 8-9) run; returns
    (x, C, mass history)."""
    x, C = _f64(x).copy(), _f64(C).copy()
    n = x.shape[1]
    vu = _f64(np.zeros(3) if v_uniform is None else np.pad(np.asarray(v_uniform, float), (0, 3 - len(v_uniform))))
    vv = None if v is None else _f64(v)
    m_arr, r_arr = _particle_arrays(n, mass, rho)
    hist = np.zeros(nsteps + 1)
    lib().or_run(ct.byref(m), n, _ptr(x), _ptr(C), _ptr(vv), _ptr(vu), _ptr(m_arr), _ptr(r_arr),
                 dt, nsteps, integrator, _ptr(hist))
    return x, C, hist


def mass_sum(mass, C):
    C = _f64(C)
    m_arr = _f64(np.broadcast_to(mass, C.shape))
    return lib().or_mass(C.shape[0], _ptr(m_arr), _ptr(C))


def dt_rule(m: Model, v_uniform, hs):
    vu = _f64(np.pad(np.asarray(v_uniform, float), (0, 3 - len(v_uniform))))
    return lib().or_dt_rule(ct.byref(m), _ptr(vu), hs)


def analytic(m: Model, v_uniform, x0, w, C0, t, x):
    """Closed-form plume (Eqs. 12-13, corrected denominator, advected centre)."""
    x = _f64(x)
    vu = _f64(np.pad(np.asarray(v_uniform, float), (0, 3 - len(v_uniform))))
    c0 = _f64(np.pad(np.asarray(x0, float), (0, 3 - len(x0))))
    out = np.zeros(x.shape[1])
    lib().or_analytic(ct.byref(m), _ptr(vu), _ptr(c0), w, C0, t, x.shape[1], _ptr(x), _ptr(out))
    return out


def sensor_interp(m: Model, x, C, xs):
    """Shepard interpolation at sensor points; returns (C_s, sum_b W_sb)."""
    x, C, xs = _f64(x), _f64(C), _f64(xs)
    ns = xs.shape[1]
    out = np.zeros(ns)
    den = np.zeros(ns)
    lib().or_sensor_interp(ct.byref(m), x.shape[1], _ptr(x), _ptr(C), ns, _ptr(xs), _ptr(out), _ptr(den))
    return out, den


def apply_LT(m: Model, x, lam, v_uniform, mass=1.0, rho=1.0):
    """y = L^T lam for the uniform-velocity operator (rhs = L C)."""
    x, lam = _f64(x), _f64(lam)
    n = x.shape[1]
    vu = _f64(np.pad(np.asarray(v_uniform, float), (0, 3 - len(v_uniform))))
    m_arr, r_arr = _particle_arrays(n, mass, rho)
    y = np.zeros(n)
    lib().or_apply_LT(ct.byref(m), n, _ptr(x), _ptr(vu), _ptr(m_arr), _ptr(r_arr), _ptr(lam), _ptr(y))
    return y


def adjoint(m: Model, x0, C0, v_uniform, dt, nsteps, xs, obs, mass=1.0, rho=1.0, integrator=1):
    """Discrete adjoint of the Euler (1) or predictor-corrector (2, Eqs. 8-9)
    run: returns (J, grad[alpha_L, alpha_T, D_m], C^N)."""
    x0, C0, xs, obs = _f64(x0), _f64(C0), _f64(xs), _f64(obs)
    n = x0.shape[1]
    vu = _f64(np.pad(np.asarray(v_uniform, float), (0, 3 - len(v_uniform))))
    m_arr, r_arr = _particle_arrays(n, mass, rho)
    J = np.zeros(1)
    g = np.zeros(3)
    CN = np.zeros(n)
    lib().or_adjoint(ct.byref(m), n, _ptr(x0), _ptr(C0), _ptr(vu), _ptr(m_arr), _ptr(r_arr), dt,
                     nsteps, xs.shape[1], _ptr(xs), _ptr(obs), int(integrator), _ptr(J), _ptr(g), _ptr(CN))
    return float(J[0]), g, CN


def misfit(m: Model, x0, C0, v_uniform, dt, nsteps, xs, obs=None, mass=1.0, rho=1.0, integrator=1):
    """Forward run (Euler 1, predictor-corrector 2) and J = sum_s (C_s - d_s)^2;
    returns (J, C_s)."""
    x0, C0, xs = _f64(x0), _f64(C0), _f64(xs)
    ob = None if obs is None else _f64(obs)
    n = x0.shape[1]
    vu = _f64(np.pad(np.asarray(v_uniform, float), (0, 3 - len(v_uniform))))
    m_arr, r_arr = _particle_arrays(n, mass, rho)
    pred = np.zeros(xs.shape[1])
    J = lib().or_misfit(ct.byref(m), n, _ptr(x0), _ptr(C0), _ptr(vu), _ptr(m_arr), _ptr(r_arr), dt,
                        nsteps, xs.shape[1], _ptr(xs), _ptr(ob), int(integrator), _ptr(pred))
    return J, pred


def rhs_deriv(m: Model, x, C, v, k, mass=1.0, rho=1.0):
    """L_k C: the derivative of the right-hand side with respect to theta_k
    (0: alpha_L, 1: alpha_T, 2: D_m) for per-particle velocities v (dim, n)."""
    x, C, v = _f64(x), _f64(C), _f64(v)
    n = x.shape[1]
    m_arr, r_arr = _particle_arrays(n, mass, rho)
    out = np.zeros(n)
    lib().or_rhs_deriv(ct.byref(m), n, _ptr(x), _ptr(C), _ptr(v), _ptr(m_arr), _ptr(r_arr), int(k), _ptr(out))
    return out


def apply_LT_field(m: Model, x, lam, v, mass=1.0, rho=1.0):
    """y = L^T lam for per-particle velocities v (dim, n)."""
    x, lam, v = _f64(x), _f64(lam), _f64(v)
    n = x.shape[1]
    m_arr, r_arr = _particle_arrays(n, mass, rho)
    y = np.zeros(n)
    lib().or_apply_LT_field(ct.byref(m), n, _ptr(x), _ptr(v), _ptr(m_arr), _ptr(r_arr), _ptr(lam), _ptr(y))
    return y


def adjoint_field(m: Model, x0, C0, v, dt, nsteps, xs, obs, mass=1.0, rho=1.0, integrator=1):
    """Discrete adjoint of the Euler (1) or predictor-corrector (2) run with
    per-particle velocities v (dim, n): returns (J, grad[alpha_L, alpha_T, D_m], C^N)."""
    x0, C0, v, xs, obs = _f64(x0), _f64(C0), _f64(v), _f64(xs), _f64(obs)
    n = x0.shape[1]
    m_arr, r_arr = _particle_arrays(n, mass, rho)
    J = np.zeros(1)
    g = np.zeros(3)
    CN = np.zeros(n)
    lib().or_adjoint_field(ct.byref(m), n, _ptr(x0), _ptr(C0), _ptr(v), _ptr(m_arr), _ptr(r_arr), dt, nsteps,
                           xs.shape[1], _ptr(xs), _ptr(obs), int(integrator), _ptr(J), _ptr(g), _ptr(CN))
    return float(J[0]), g, CN


def misfit_field(m: Model, x0, C0, v, dt, nsteps, xs, obs, mass=1.0, rho=1.0, integrator=1):
    """Euler (1) or predictor-corrector (2) run with per-particle velocities and
    J = sum_s (C_s - d_s)^2."""
    x0, C0, v, xs, obs = _f64(x0), _f64(C0), _f64(v), _f64(xs), _f64(obs)
    n = x0.shape[1]
    m_arr, r_arr = _particle_arrays(n, mass, rho)
    return lib().or_misfit_field(ct.byref(m), n, _ptr(x0), _ptr(C0), _ptr(v), _ptr(m_arr), _ptr(r_arr), dt,
                                 nsteps, xs.shape[1], _ptr(xs), _ptr(obs), int(integrator))


def num_threads():
    return lib().or_num_threads()
