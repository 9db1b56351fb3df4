"""CPU-side checks of the C ABI: the library loads, exports every entry point
that include/adesph.h declares, and validates its arguments on the host
(no device work is started by these calls)."""
import ctypes as ct
import os
import re

import pytest

from paper_2108_09488_amd import _lib, inputs as I
from paper_2108_09488_amd.context import params_from_spec

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "adesph.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ade_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    declared = _declared()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(_lib.EXPORTS) == declared
    assert b"gfx950" in L.ade_version()


def _wsbytes(params, counts):
    arr = (_lib.AdeParams * len(params))(*params)
    cn = (ct.c_int64 * len(counts))(*counts)
    nb = ct.c_size_t(0)
    rc = _lib.lib().ade_workspace_bytes(arr, cn, len(params), ct.byref(nb))
    return rc, nb.value


def test_workspace_bytes_scales_with_particles():
    s = I.config("cfg2_h20_r10")
    rc, nb = _wsbytes([params_from_spec(s)], [s.n])
    assert rc == 0 and nb > s.n * 40
    s2 = I.config("cfg2_h20_r10", n_side=256)
    rc2, nb2 = _wsbytes([params_from_spec(s2)], [s2.n])
    assert rc2 == 0 and nb2 < nb


@pytest.mark.parametrize("field,value", [("dim", 4), ("real_bytes", 2), ("kernel", 3),
                                         ("integrator", 7), ("H", -1.0), ("H", 0.5),
                                         ("alpha_L", -1e-3), ("rho0", 0.0), ("mass", float("nan")),
                                         ("reserved", 1), ("cell_rows", 9)])
def test_invalid_parameters_are_rejected(field, value):
    p = params_from_spec(I.config("cfg1"))
    setattr(p, field, value)
    rc, _ = _wsbytes([p], [4096])
    assert rc == _lib.ADE_EINVAL
    assert len(_lib.lib().ade_last_error()) > 0


def test_mixed_plumes_and_counts_rejected():
    a = params_from_spec(I.config("cfg1"))
    b = params_from_spec(I.config("cfg2_h20_r10"))
    assert _wsbytes([a, b], [4096, 4096])[0] == _lib.ADE_EINVAL
    assert _wsbytes([a], [0])[0] == _lib.ADE_EINVAL


def test_strict_dt_flags_unstable_step():
    s = I.config("cfg2_h20_r10")
    p = params_from_spec(s, flags=_lib.ADE_STRICT_DT)
    assert _wsbytes([p], [s.n])[0] == 0
    p.dt = s.dt * 40 * 4  # Eq. (10) with h = H/2 is the reference: 4x the config's h-based dt
    assert _wsbytes([p], [s.n])[0] == _lib.ADE_EUNSTABLE


def test_velocity_field_flag_validation():
    """ADE_VELOCITY_FIELD: a given dt, the same on every plume; its workspace
    holds the per-particle velocities and tensors (and, for the
    predictor-corrector, C^n carried through the predictor's build)."""
    s = I.config("cfg1")
    base = params_from_spec(s)
    p = params_from_spec(s, flags=_lib.ADE_VELOCITY_FIELD)
    rc0, nb0 = _wsbytes([base], [s.n])
    rc, nb = _wsbytes([p], [s.n])
    assert rc0 == 0 and rc == 0
    # two buffers (sorted and hashed) of 2 velocity and 3 tensor components, FP64
    assert nb - nb0 >= 2 * 5 * 8 * s.n
    pc = params_from_spec(s, integrator=_lib.ADE_PC, flags=_lib.ADE_VELOCITY_FIELD)
    rc_pc, nb_pc = _wsbytes([pc], [s.n])
    assert rc_pc == 0 and nb_pc >= nb + 2 * 8 * s.n  # C^n carried through the predictor's build
    p0 = params_from_spec(s, flags=_lib.ADE_VELOCITY_FIELD)
    p0.dt = 0.0
    assert _wsbytes([p0], [s.n])[0] == _lib.ADE_EINVAL
    assert _wsbytes([p, base], [s.n, s.n])[0] == _lib.ADE_EINVAL
    bad = params_from_spec(s, flags=64)
    assert _wsbytes([bad], [s.n])[0] == _lib.ADE_EINVAL


def test_create_rejects_null_and_small_workspace():
    p = params_from_spec(I.config("cfg1"))
    arr = (_lib.AdeParams * 1)(p)
    cn = (ct.c_int64 * 1)(4096)
    out = ct.c_void_p()
    assert _lib.lib().ade_create(arr, cn, 1, None, 0, None, ct.byref(out)) == _lib.ADE_EINVAL
    # misaligned pointer is rejected before any device call
    assert _lib.lib().ade_create(arr, cn, 1, ct.c_void_p(0x1001), 1 << 30, None, ct.byref(out)) == _lib.ADE_EINVAL


def test_particle_limit_per_context():
    """A context holds at most 2^28 - 256 particles (32-bit byte offsets of the
    16-byte candidate records); the plan rejects one more, before any device
    work."""
    p = params_from_spec(I.config("cfg2_h20_r10"))
    lim = (1 << 28) - 256
    rc, nb = _wsbytes([p, p], [lim // 2, lim - lim // 2])
    assert rc == 0 and nb > lim * 40
    assert _wsbytes([p, p], [lim // 2, lim - lim // 2 + 1])[0] == _lib.ADE_EINVAL


def test_default_x_cells_coarsen_for_large_cell_tables():
    """A context whose default cell tables (40 bytes per cell) would pass
    160 MiB gets coarser x cells: the 256-plume ensemble (9.6M cells at H/8)
    is sized as with H/3 cells, the six-plume sweep (2M cells) as with H/8
    (H/12 for its plumes of 111 neighbours), the 128^3 plume (256 neighbours) as with H/28 and a 3D plume of
    137 neighbours as with H/16 (the 3D defaults), and an explicit cell_xsub is kept."""
    from paper_2108_09488_amd.context import workspace_bytes

    def ws(specs, xsub=0):
        return workspace_bytes([params_from_spec(s, cell_xsub=xsub) for s in specs], [s.n for s in specs])

    ens = I.ensemble(256)
    assert ws(ens) == ws(ens, 3) < ws(ens, 4) < ws(ens, 8)
    sweep = [I.config(n) for n in I.CFG2_CELLS]
    # H/12 for the plumes of 80 or more expected neighbours (h/dp = 3), H/8 for the rest
    mixed = workspace_bytes([params_from_spec(s, cell_xsub=12 if s.h_over_dp == 3.0 else 8) for s in sweep],
                            [s.n for s in sweep])
    assert ws(sweep) == mixed > ws(sweep, 8)
    cube = [I.config("cfg3")]  # 3D, 256 neighbours: H/28 by default
    assert ws(cube) == ws(cube, 28) > ws(cube, 16) > ws(cube, 8)
    thin = [I.config("cfg3", h_over_dp=1.6)]  # 3D, 137 neighbours: H/16
    assert ws(thin) == ws(thin, 16) < ws(thin, 28)
