// Forward modelling that allocates no device memory: the wavefield ring of
// the shots lives in a fixed device array of the library instead of plan
// scratch grown with hipMalloc.  For callers that cannot allocate (work under
// HIP graph capture, tight serving loops).
//
// The array is a file-scope device variable.  Its host-side name is only a
// stand-in for the device address, so host code never passes `scratch` to a
// kernel: each device's address is looked up once with hipGetSymbolAddress
// (when the first plan is created on that device) and kept per device.
#include <mutex>

#include "esi_internal.h"

namespace esi {
// the largest wavefield ring one call may use (bytes)
constexpr int64_t NOALLOC_SCRATCH_BYTES = 64ll << 20;
}  // namespace esi

static __device__ __align__(256) float scratch[esi::NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace esi {

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
bool g_looked_up[MAX_DEVICES] = {};
float* g_ptr[MAX_DEVICES] = {};
hipError_t g_err[MAX_DEVICES] = {};

}  // namespace

// Look up this device's copy of `scratch` (the device must be current).  The
// result, or the failure, is kept for the no-allocation call to report.
void noalloc_init_device(int device) {
    if (device < 0 || device >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_looked_up[device]) return;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_err[device] = e;
    g_ptr[device] = e == hipSuccess ? static_cast<float*>(p) : nullptr;
    g_looked_up[device] = true;
}

namespace {

esi_status_t scratch_for(int device, float** out) {
    if (device < 0 || device >= MAX_DEVICES) return fail(ESI_ERR_ARG, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_looked_up[device]) return fail(ESI_ERR_HIP, "no-allocation scratch not set up on this device");
    if (!g_ptr[device])
        return fail(ESI_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(g_err[device]));
    *out = g_ptr[device];
    return ESI_OK;
}

// The plan's tiling for `tx x tz (x ty)` tiles if it has been built (plan
// creation builds the default tilings; the autotuner builds those of the
// shapes it picks), else an error: this path must not build lists, which
// would allocate.
esi_status_t existing_lists(Plan* P, int tx, int tz, int ty, TileLists** out) {
    for (TileLists* L : P->lists)
        if (L->tx == tx && L->tz == tz && L->ty == ty) { *out = L; return ESI_OK; }
    return fail(ESI_ERR_ARG, "tile lists of this tiling were not built at plan creation");
}

}  // namespace

}  // namespace esi

using namespace esi;

extern "C" esi_status_t esi_forward_noalloc(esi_plan_t plan, int32_t shot0, int32_t nshots, int32_t src_kind,
                                            const float* src, float* data) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, nshots));
    if (src_kind != ESI_SRC_POINT && src_kind != ESI_SRC_DENSE) return fail(ESI_ERR_ARG, "bad src_kind");
    if (!src) return fail(ESI_ERR_ARG, "null src");
    if (!data && data_len(P, shot0, nshots) > 0) return fail(ESI_ERR_ARG, "null data");
    const int64_t ring_floats = (int64_t)nshots * RING * P->fsize;
    if (ring_floats * (int64_t)sizeof(float) > NOALLOC_SCRATCH_BYTES)
        return fail(ESI_ERR_SHAPE, "the wavefield ring of " + std::to_string(nshots) + " shots needs " +
                                       std::to_string(ring_floats * (int64_t)sizeof(float)) +
                                       " bytes; the no-allocation scratch holds " +
                                       std::to_string(NOALLOC_SCRATCH_BYTES) + " (call with fewer shots)");
    float* ring = nullptr;
    ESI_TRY(scratch_for(P->device, &ring));
    // every tiling the loop uses must exist already
    int tx, ty, tz;
    shape_tile(P, LS_ONE, &tx, &ty, &tz);
    TileLists* L;
    ESI_TRY(existing_lists(P, tx, tz, ty, &L));
    const unsigned fl = F_GATHER | (src_kind == ESI_SRC_POINT ? F_SRC_POINT : F_SRC_DENSE);
    const int shape = loop_shape(P, fl, false);
    if (shape != LS_ONE) {
        TileLists* L2;
        shape_tile(P, shape, &tx, &ty, &tz);
        ESI_TRY(existing_lists(P, tx, tz, ty, &L2));
    }
    // the scratch keeps the last call's contents: the state starts at zero
    ESI_TRY(launch_fill(P, ring, ring_floats, 0.f));
    StepArgs a = base_args(P, L, shot0, nshots);
    if (src_kind == ESI_SRC_POINT) a.wavelet = src;
    else a.dsrc = src;
    a.gat_data = data;
    int cs = 0;
    ESI_TRY(forward_loop(P, a, fl, ring, &cs, 0, P->nt));
    return launch_final_gather(P, ring + (int64_t)cs * P->fsize, RING * P->fsize, data, shot0, nshots);
}
