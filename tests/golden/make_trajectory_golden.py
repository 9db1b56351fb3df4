"""Writes traj_<case>.npz: the FP64 CPU oracle's concentrations after the full
run of a plume problem, at a seeded sample of particles, for the GPU
trajectory-parity tests (the FP32 state stepped the same number of steps is
compared with them element by element).

Cases: the six cells of the 2D consistency sweep (512^2 particles jittered by
+-0.1 dp, Wendland C4, h/dp in {1.3, 2, 3}, alpha_L/alpha_T in {10, 100},
dt from Eq. (10), 1000 explicit steps) and the 3D plume (128^3 particles,
h = 2 dp, 500 steps of 5e-5).  The oracle starts from the seeded lattice and
the initial Gaussian rounded to FP32 (the values the FP32 state starts from),
promoted to FP64; positions are exact on both sides.

Sample: 20 000 particles drawn (seeded) from those where the oracle's final
|C| exceeds 1e-4 of its maximum, and 4 000 from the rest.  Each file also
holds the oracle's FP64 mass at the start and the end of the run.

Only oracle/ and the seeded input generators are called.

Run: python tests/golden/make_trajectory_golden.py [case ...]
     (about 15 minutes for the sweep and 70 minutes for the 3D plume on 8 cores)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2108_09488_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = list(I.CFG2_CELLS) + ["cfg3"]
N_PLUME, N_REST = 20000, 4000
SEED = 1802


def path_of(case):
    return os.path.join(HERE, f"traj_{case}.npz")


def make(case):
    t0 = time.time()
    spec = I.config(case)
    x = spec.positions()
    C0 = spec.concentration(x).astype(np.float32).astype(np.float64)
    m = O.model_from_spec(spec)
    _, C, hist = O.run(m, x, C0, spec.dt, spec.steps, v_uniform=spec.velocity(), mass=spec.mass,
                       rho=spec.rho0)
    rng = np.random.default_rng(SEED)
    cmax = np.max(np.abs(C)) if np.all(np.isfinite(C)) else np.inf
    inside = np.flatnonzero(np.abs(C) > 1e-4 * cmax) if np.isfinite(cmax) else np.arange(spec.n)
    rest = np.setdiff1d(np.arange(spec.n), inside)
    ids = np.concatenate([rng.choice(inside, min(N_PLUME, len(inside)), replace=False),
                          rng.choice(rest, min(N_REST, len(rest)), replace=False)])
    ids = np.sort(ids).astype(np.int64)
    np.savez(path_of(case), ids=ids, C=C[ids], steps=spec.steps, dt=spec.dt,
             mass0=hist[0], massN=hist[-1], seconds=time.time() - t0)
    print(f"{case}: {spec.steps} steps in {time.time() - t0:.0f} s, max C {cmax:.4g}, "
          f"mass drift {abs(hist[-1] - hist[0]) / abs(hist[0]):.2e}", flush=True)


def main():
    cases = sys.argv[1:] or CASES
    for c in cases:
        if c not in CASES:
            raise SystemExit(f"unknown case {c}; one of {CASES}")
        make(c)


if __name__ == "__main__":
    main()
