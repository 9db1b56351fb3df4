"""Pins of the oracle's spectrum report (oracle/spectrum.py): the Lanczos
extremes of the SPH operator L (rhs = L C) against a dense eigensolver and
against the exact Fourier symbol on a regular lattice, and the per-step
amplification against the oracle's own Euler run.  CPU only."""
import numpy as np
import pytest

import oracle as O
from oracle import spectrum as S
from paper_2108_09488_amd import inputs as I


def _dense_operator(spec):
    x = spec.positions()
    m = O.model_from_spec(spec)
    n = x.shape[1]
    Lm = np.empty((n, n))
    e = np.zeros(n)
    for b in range(n):
        e[b] = 1.0
        Lm[:, b] = O.rhs(m, x, e, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
        e[b] = 0.0
    return Lm


@pytest.mark.parametrize("hod,ratio", [(1.3, 100.0), (2.0, 10.0)])
def test_lanczos_matches_dense_eigensolver(hod, ratio):
    """Jittered 20^2 lattice: L is symmetric; the Lanczos extremes equal those
    of numpy's dense symmetric eigensolver, and with fewer steps stay inside
    the spectrum within their residual bounds."""
    spec = I.config("cfg2_h13_r10", n_side=20, h_over_dp=hod, alpha_T=1e-2 / ratio)
    Lm = _dense_operator(spec)
    rho = np.max(np.abs(Lm)) * Lm.shape[0]
    assert np.max(np.abs(Lm - Lm.T)) <= 1e-13 * np.max(np.abs(Lm))
    ev = np.linalg.eigvalsh(0.5 * (Lm + Lm.T))
    lo, hi, rlo, rhi = S.operator_extremes(spec, iters=400)
    assert abs(lo - ev[0]) <= 1e-10 * rho
    assert abs(hi - ev[-1]) <= 1e-10 * rho
    lo, hi, rlo, rhi = S.operator_extremes(spec, iters=40)
    assert ev[0] - 1e-12 * rho <= lo and hi <= ev[-1] + 1e-12 * rho
    # the residual bound covers the distance to the nearest eigenvalue
    assert np.min(np.abs(ev - lo)) <= rlo + 1e-12 * rho
    assert np.min(np.abs(ev - hi)) <= rhi + 1e-12 * rho


def test_lanczos_matches_lattice_symbol():
    """Regular 64^2 lattice (h = 2 dp, alpha_L/alpha_T = 100, where the
    operator has growing modes): L is a circulant convolution, its eigenvalues
    are the Fourier transform of one column; the Lanczos extremes match them."""
    spec = I.config("cfg2_h20_r100", n_side=64, jitter=0.0)
    x = spec.positions()
    m = O.model_from_spec(spec)
    col = np.zeros(spec.n)
    col[0] = 1.0
    col = O.rhs(m, x, col, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
    lam = np.fft.fft2(col.reshape(64, 64)).real
    lo, hi, rlo, rhi = S.operator_extremes(spec, iters=300)
    scale = np.max(np.abs(lam))
    assert lam.max() > 0  # the growing modes exist
    assert abs(hi - lam.max()) <= max(rhi, 1e-9 * scale) and abs(hi - lam.max()) <= 1e-6 * scale
    assert abs(lo - lam.min()) <= max(rlo, 1e-9 * scale) and abs(lo - lam.min()) <= 1e-6 * scale


def test_amplification_of_the_growing_mode():
    """The fastest-growing Fourier mode of the regular lattice, run through 20
    of the oracle's Euler steps and 20 of its predictor-corrector steps, grows
    by exactly the factor run_growth gives from its eigenvalue."""
    spec = I.config("cfg2_h20_r100", n_side=64, jitter=0.0)
    x = spec.positions()
    m = O.model_from_spec(spec)
    col = np.zeros(spec.n)
    col[0] = 1.0
    col = O.rhs(m, x, col, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0)
    lam = np.fft.fft2(col.reshape(64, 64)).real
    ky, kx = np.unravel_index(np.argmax(lam), lam.shape)
    j = np.arange(64)
    mode = np.cos(2 * np.pi * (ky * j[:, None] + kx * j[None, :]) / 64).reshape(-1)
    dt = 50.0 * spec.dt  # long steps, so that the growth is large
    for integ in (1, 2):
        _, C, _ = O.run(m, x, mode, dt, 20, v_uniform=spec.velocity(), mass=spec.mass, rho=spec.rho0,
                        integrator=integ)
        g = S.run_growth(lam.max(), lam.max(), dt, 20, integ)
        assert g > 1.01
        assert np.linalg.norm(C) / np.linalg.norm(mode) == pytest.approx(g, rel=1e-10)


def test_run_growth_takes_the_larger_end():
    assert S.run_growth(-3.0, -1.0, 0.5, 10) == pytest.approx(0.5 ** 10)
    assert S.run_growth(-3.0, 0.0, 0.5, 10) == pytest.approx(1.0)
    assert S.run_growth(-5.0, 0.0, 0.5, 3) == pytest.approx(1.5 ** 3)
    assert S.run_growth(-1.0, 2.0, 0.5, 4) == pytest.approx(2.0 ** 4)
    # predictor-corrector: 1 + z + z^2/2 at z = -2 is 1
    assert S.run_growth(-4.0, 0.0, 0.5, 7, integrator=2) == pytest.approx(1.0)
