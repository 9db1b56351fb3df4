"""Writes spectrum.json: the extreme eigenvalues of the SPH operator L
(rhs = L C, uniform flow) of each plume problem, from the oracle's Lanczos
iteration (oracle/spectrum.py), and the largest amplification of any mode
over the problem's run, max |1 + dt lam|^steps (explicit Euler).

The GPU trajectory tests take their gate from this report: a problem whose
run amplifies some mode (growth > 1) carries the FP32 round-off of every step
along with it, so its tolerance is 1e-5 times the growth, and a problem whose
growth passes 100 is compared and reported but not gated.

Cases: the FP64 problem (64^2, C2), the six cells of the 2D sweep, the 3D
plume, the adjoint problem at its true and guessed parameters, and every plume
of the 256-plume ensemble (200 steps each).

Only oracle/ and the seeded input generators are called.

Run: python tests/golden/make_spectrum.py [case ...]   (cases: cfg1 cfg2 cfg3 cfg5 ensemble;
     the 3D plume takes about half an hour on 8 cores, the rest a few minutes)
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import spectrum as S  # noqa: E402
from paper_2108_09488_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "spectrum.json")


def entry(spec, iters):
    t0 = time.time()
    lo, hi, rlo, rhi = S.operator_extremes(spec, iters=iters)
    return {"n": spec.n, "dt": spec.dt, "steps": spec.steps, "lam_min": lo, "lam_max": hi,
            "res_min": rlo, "res_max": rhi, "iters": iters,
            "growth": S.run_growth(lo, hi, spec.dt, spec.steps),
            "growth_upper": S.run_growth(lo - rlo, hi + rhi, spec.dt, spec.steps),
            "seconds": time.time() - t0}


def main():
    groups = sys.argv[1:] or ["cfg1", "cfg2", "cfg5", "ensemble", "cfg3"]
    out = json.load(open(PATH)) if os.path.exists(PATH) else {}
    out["what"] = ("extreme eigenvalues of the uniform-flow SPH operator (oracle Lanczos, full "
                   "reorthogonalisation) at the initial positions, and max |1 + dt lam|^steps")
    for g in groups:
        if g == "cfg1":
            todo = [("cfg1", I.config("cfg1"), 300)]
        elif g == "cfg2":
            todo = [(c, I.config(c), 300) for c in I.CFG2_CELLS]
        elif g == "cfg3":
            todo = [("cfg3", I.config("cfg3"), 120)]
        elif g == "cfg5":
            todo = [("cfg5_truth", I.config("cfg5"), 300),
                    ("cfg5_guess", I.config("cfg5", alpha_L=1e-2, alpha_T=5e-3), 300)]
        elif g == "ensemble":
            todo = [(f"ensemble_{p}", s, 150) for p, s in enumerate(I.ensemble(256))]
        else:
            raise SystemExit(f"unknown group {g}")
        for name, spec, iters in todo:
            out[name] = entry(spec, iters)
            e = out[name]
            print(f"{name}: lam [{e['lam_min']:.6g}, {e['lam_max']:.6g}] (res {e['res_min']:.1e}, "
                  f"{e['res_max']:.1e}), growth {e['growth']:.4g} in {e['seconds']:.0f} s", flush=True)
            with open(PATH, "w") as f:
                json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
