// 3D time step (not built yet in this file's first version).
#include "esi_internal.h"

namespace esi {

esi_status_t launch_step3d(Plan* P, unsigned flags, const StepArgs& a) {
    (void)P; (void)flags; (void)a;
    return fail(ESI_ERR_ARG, "3D kernels are not available in this build");
}

void step3d_tile_shape(int* tx, int* ty, int* tz) { *tx = 64; *ty = 4; *tz = 1; }

}  // namespace esi
