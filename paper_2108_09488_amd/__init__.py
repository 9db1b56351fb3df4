"""MI355X (gfx950) SPH advection-dispersion library: the hot path of the
consistent-SPH solver of Klapp et al., "Consistent SPH simulations of the
anisotropic dispersion of a contaminant plume" (arXiv:2108.09488).

The compute runs in hand-written HIP kernels behind the C ABI of
include/adesph.h (libadesph.so); this package only marshals torch tensors
(device memory and streams) into that ABI.
"""
from __future__ import annotations

from . import inputs  # noqa: F401  (seeded synthetic inputs; no method arithmetic)

__all__ = ["inputs", "Context", "params_from_spec"]


def __getattr__(name):
    # the HIP binding is loaded lazily so that `inputs` can be used without a GPU
    if name in ("Context", "params_from_spec", "ADEMisfit"):
        from . import context
        return getattr(context, name)
    raise AttributeError(name)
