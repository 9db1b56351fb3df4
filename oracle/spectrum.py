"""Extreme eigenvalues of the oracle's SPH operator, and the growth they give a run.

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: used by the tests and by
the script that writes the committed spectrum report, never by the product
library.

For a uniform flow and equal particle volumes the right-hand side of
Eqs. (4)-(5) is linear in C, rhs = L C, and L is symmetric: the pair weight
of a and b is the same function of |x_ab| and (e . x_ab)^2 seen from either
side.  Section 2.3 (the consistency requirement around Eq. (6)) is about the
discrete operator reproducing the second derivative; where the particle
distribution and the anisotropy are such that it does not, L can have
positive eigenvalues, so that an explicit run amplifies the matching modes
instead of damping them -- the negative-concentration behaviour that
Section 4 discusses.  An explicit Euler step multiplies the component of C
along an eigenvector of eigenvalue lam by 1 + dt lam; the predictor-corrector
of Eqs. (8)-(9) by 1 + dt lam + (dt lam)^2 / 2.  Over n steps the largest
amplification of any mode is max over the spectrum of |g(dt lam)|^n, reached
at the smallest or the largest eigenvalue.

The extreme eigenvalues come from the Lanczos iteration (Lanczos 1950; as in
Golub & Van Loan, Matrix Computations, Section 10.1) with full
reorthogonalisation, using the oracle's rhs as the matrix-vector product.
The Ritz values of the tridiagonal matrix lie inside the spectrum, and
|beta_k s_k| bounds the distance of each from an eigenvalue.
"""
from __future__ import annotations

import numpy as np

from . import model_from_spec, rhs


def lanczos_extremes(matvec, n: int, iters: int = 200, seed: int = 1802):
    """Smallest and largest eigenvalue estimates of the symmetric operator
    matvec (n x n) after `iters` Lanczos steps from a seeded random start.

    Returns (lam_min, lam_max, res_min, res_max): the extreme Ritz values and
    their residual bounds |beta_k s_k|.
    """
    k = min(iters, n)
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(n)
    q /= np.linalg.norm(q)
    Q = np.empty((k, n))
    alpha, beta = [], []
    q_prev = np.zeros(n)
    b = 0.0
    for j in range(k):
        Q[j] = q
        w = matvec(q)
        a = float(q @ w)
        w = w - a * q - b * q_prev
        # full reorthogonalisation against every Lanczos vector so far (twice)
        for _ in range(2):
            w -= Q[: j + 1].T @ (Q[: j + 1] @ w)
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        if b <= 1e-13 * max(1.0, abs(a)):
            break
        q_prev, q = q, w / b
    m = len(alpha)
    T = np.diag(alpha) + np.diag(beta[: m - 1], 1) + np.diag(beta[: m - 1], -1)
    theta, S = np.linalg.eigh(T)
    res = np.abs(beta[m - 1] * S[-1, :])
    return float(theta[0]), float(theta[-1]), float(res[0]), float(res[-1])


def operator_extremes(spec, x=None, iters: int = 200, seed: int = 1802):
    """Extreme eigenvalues of the uniform-flow operator L (rhs = L C) of a plume
    problem at its initial positions (the geometry is the same at every step
    of a uniform flow)."""
    x = spec.positions() if x is None else x
    m = model_from_spec(spec)
    v = spec.velocity()

    def matvec(c):
        return rhs(m, x, c, v_uniform=v, mass=spec.mass, rho=spec.rho0)

    return lanczos_extremes(matvec, x.shape[1], iters, seed)


def amplification(lam, dt, integrator: int = 1):
    """Amplification factor of one step for an eigenvalue lam: explicit Euler
    (1) or the predictor-corrector of Eqs. (8)-(9) (2)."""
    z = dt * np.asarray(lam, dtype=np.float64)
    return 1.0 + z if integrator == 1 else 1.0 + z + 0.5 * z * z


def run_growth(lam_min, lam_max, dt, steps, integrator: int = 1) -> float:
    """Largest amplification of any mode over `steps` steps,
    max(|g(dt lam_min)|, |g(dt lam_max)|)^steps."""
    g = max(abs(float(amplification(lam_min, dt, integrator))), abs(float(amplification(lam_max, dt, integrator))))
    return float(g ** steps)
