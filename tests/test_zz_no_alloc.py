"""The allocation-free adjoint entry point (ade_adjoint_noalloc) against
ade_adjoint with a caller's workspace: the same kernels in the same order on
the same inputs, so J and the gradient must agree bit for bit.  Two calls in
a row on the library's static scratch array, the second on a smaller problem
(the array keeps the first call's contents), and a run too large for the
array is refused without touching the state."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2108_09488_amd import _lib
from paper_2108_09488_amd import inputs as I

pytestmark = pytest.mark.gpu


def _problem(n_side, steps, ns, integrator=1, rb=4):
    from paper_2108_09488_amd.context import Context, params_from_spec
    spec = I.config("cfg5", n_side=n_side, steps=steps, dt=2.0 ** -12, real_bytes=rb, v=(0.75, 0.5, 0.0),
                    alpha_L=1e-2, alpha_T=5e-3)
    print(f"[case] no-alloc adjoint n_side={n_side} steps={steps} sensors={ns} integ={integrator} rb={rb}",
          flush=True)
    x = spec.positions()
    C0 = spec.concentration(x)
    if rb == 4:
        C0 = C0.astype(np.float32).astype(np.float64)
    xs = I.sensors(ns, [0.05, 0.25], [0.55, 0.75])
    truth = O.model(2, 4, spec.H, alpha_L=2e-2, alpha_T=2e-3, D_m=1e-6)
    _, obs = O.misfit(truth, x, C0, spec.velocity(), spec.dt, steps, xs, None, mass=spec.mass, rho=spec.rho0,
                      integrator=integrator)

    def fresh():
        c = Context([params_from_spec(spec, integrator=integrator)], [spec.n])
        c.init(torch.from_numpy(x), torch.from_numpy(C0)).build()
        return c

    dt = torch.float32 if rb == 4 else torch.float64
    return fresh, torch.from_numpy(xs).cuda(), torch.from_numpy(obs).to("cuda", dt), spec


@pytest.mark.parametrize("integrator", [1, 2])
def test_noalloc_adjoint_equals_adjoint(integrator):
    # the larger problem first, then a smaller one on the same scratch array
    for n_side, steps, ns, K in [(64, 40, 64, 7), (40, 25, 32, 4)]:
        fresh, xs, obs, spec = _problem(n_side, steps, ns, integrator)
        c = fresh()
        J, g = c.adjoint(steps, K, xs, obs)
        C_ref = c.read_C().cpu().numpy()
        c.close()
        c = fresh()
        Jn, gn = c.adjoint_noalloc(steps, K, xs, obs)
        C_n = c.read_C().cpu().numpy()
        c.close()
        torch.cuda.synchronize()
        assert Jn == J and gn == g, (J, Jn, g, gn)
        assert np.array_equal(C_n, C_ref)
        assert np.isfinite(J) and J > 0 and all(np.isfinite(g))


def test_noalloc_refuses_runs_beyond_the_array():
    fresh, xs, obs, spec = _problem(64, 40, 64)
    c = fresh()
    import ctypes as ct
    cap = ct.c_size_t(0)
    _lib.check(_lib.lib().ade_adjoint_noalloc_max_bytes(ct.byref(cap)))
    nb = ct.c_size_t(0)
    _lib.check(_lib.lib().ade_adjoint_workspace_bytes(c._h, 4000, 4000, 64, ct.byref(nb)))
    assert nb.value > cap.value  # 4001 steps kept in one segment
    C0 = c.read_C().cpu().numpy()
    with pytest.raises(_lib.AdeError) as e:
        c.adjoint_noalloc(4000, 4000, xs, obs)
    assert e.value.code == _lib.ADE_EWORKSPACE
    assert np.array_equal(c.read_C().cpu().numpy(), C0)
    c.close()
