// adjoint.hip -- sensors and the discrete adjoint (filled in below).
#include <hip/hip_runtime.h>

#include "../../include/adesph.h"

extern "C" {
int ade_sensor_interp(ade_ctx*, const double*, int32_t, void*) { return ADE_EINVAL; }
int ade_adjoint_workspace_bytes(const ade_ctx*, int64_t, int32_t, int32_t, size_t*) { return ADE_EINVAL; }
int ade_adjoint(ade_ctx*, int64_t, int32_t, const double*, int32_t, const void*, void*, size_t, double*,
                double*) {
    return ADE_EINVAL;
}
}
