// Internal declarations of the ESI library: plan layout, device helpers and
// the launchers each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "esi.h"

namespace esi {

constexpr int HALO = 4;          // 8th-order stencil half width
constexpr int GH = 8;            // zero ghost cells around the padded grid in storage
                                 // (two stencil radii: enough for two-step blocking)
constexpr int XCDS = 8;          // MI355X: 8 accelerator complex dies, 32 CUs each

// Launch shapes of 2D time loops (the autotuner's candidates): one step per
// launch on 64 x 32 tiles, or two steps per launch on 56-column tiles of 32,
// 24 or 40 rows.  3D loops use LS_ONE.
enum : int { LS_ONE = 1, LS_T2_32 = 2, LS_T2_24 = 3, LS_T2_40 = 4 };
constexpr int LS_COUNT = 4;


// Thread-local error text.
void set_error(const std::string& s);

// Throw-free status helper: record text, return code.
esi_status_t fail(esi_status_t code, const std::string& s);

#define ESI_HIP_TRY(expr)                                                            \
    do {                                                                             \
        hipError_t _e = (expr);                                                      \
        if (_e != hipSuccess)                                                        \
            return ::esi::fail(_e == hipErrorOutOfMemory ? ESI_ERR_OOM : ESI_ERR_HIP, \
                               std::string(#expr) + ": " + hipGetErrorString(_e));   \
    } while (0)

#define ESI_TRY(expr)                        \
    do {                                     \
        esi_status_t _s = (expr);            \
        if (_s != ESI_OK) return _s;         \
    } while (0)

// Per-tile sparse lists for one tile shape, all shots of the plan.
//  inj: unique injection cells (receivers sharing a cell are summed in a fixed
//       order); each cell has a CSR range into inj_rid (receiver ids).
//  gat: one entry per receiver (tile-local cell, receiver id).
//  src: one entry per shot (tile id, tile-local cell) for the point source.
struct TileLists {
    int tx = 0, tz = 0, ty = 0;          // tile shape the lists were built for
    int tiles_x = 0, tiles_y = 0, tiles_z = 0, tiles = 0;
    int32_t* inj_ptr = nullptr;          // [nshots][tiles+1] into inj_cell
    int32_t* inj_cell = nullptr;         // tile-local cell index
    int32_t* inj_rptr = nullptr;         // [ncell+1] into inj_rid
    int32_t* inj_rid = nullptr;          // receiver index within its shot
    int32_t* gat_ptr = nullptr;          // [nshots][tiles+1]
    int32_t* gat_cell = nullptr;         // tile-local cell index
    int32_t* gat_rid = nullptr;          // receiver index within its shot
    int32_t* src_tile = nullptr;         // [nshots]
    int32_t* src_cell = nullptr;         // [nshots]
    // injection cells of the tile grown by one stencil radius (two-step
    // launches inject on that region in their first step); cells are indexed
    // on the grown tile, (tz + 8) x (tx + 8) in 2D
    int32_t* inj2_ptr = nullptr;
    int32_t* inj2_cell = nullptr;
    int32_t* inj2_rptr = nullptr;
    int32_t* inj2_rid = nullptr;
    // with apertures: the (shot, tile) items whose tile meets the shot's
    // window plus its absorbing layer, shot-major; work_ptr[gs] indexes it
    int32_t* work = nullptr;
    std::vector<int64_t> work_ptr;
};

struct Plan {
    // grid
    int ndim = 2, nz = 0, nx = 0, ny = 1, nb = 0, nt = 0;
    double dx = 0, dt = 0, eta_max = 0, beta = 0, b_eps = 1;
    int w_identity = 0;                  // penalty weight B = I (WRI) instead of the annihilator
    // DTFT frequencies (Hz), twiddle table [nt][nf] (cos, sin) and F G as a
    // real 2nf x 2nf matrix (row (k, re/im), column (m, re/im))
    std::vector<double> dft_freqs;
    float2* dft_tw = nullptr;
    double* dft_C = nullptr;
    // DTFT passes in blocks of dft_block steps (0: per step inside the step
    // kernel): the block's dense sources or adjoint fields, [nshots][block][phys]
    int dft_block = 64;
    float* dft_blk = nullptr; int64_t dft_blk_cap = 0;
    // data-space solver scratch: adjoint field [nshots][nt][phys], W^{-1}
    // [nshots][phys], data segment offsets [nshots + 1]
    float* ds_mu = nullptr; int64_t ds_mu_cap = 0;
    // ds_ckpt > 0: the adjoint field is not kept whole; the adjoint state is
    // checkpointed every ds_ckpt steps into ds_ck [nshots][segments][2][fsize]
    // and each segment's field recomputed into ds_mu [nshots][ds_ckpt][phys]
    int ds_ckpt = 0;
    float* ds_ck = nullptr; int64_t ds_ck_cap = 0;
    float* ds_winv = nullptr; int64_t ds_winv_cap = 0;
    int64_t* ds_seg = nullptr; int64_t ds_seg_cap = 0;
    int nzp = 0, nyp = 1, nxp = 0;       // padded grid
    int ZS = 0, YS = 1, XS = 0;          // storage grid (padded + zero ghost halo)
    int64_t fsize = 0;                   // floats per stored field (one shot)
    int64_t nphys = 0;                   // physical cells
    hipStream_t stream = nullptr;
    int device = 0;

    // geometry (host copies + device copies)
    int nshots = 0;
    std::vector<int32_t> h_src;          // [nshots][ndim]
    std::vector<int64_t> h_rec_ptr;      // [nshots+1]
    std::vector<int32_t> h_rec;          // [nrec][ndim]
    int32_t* d_src = nullptr;            // [nshots][3] (ix, iz, iy), iy = 0 in 2D
    int64_t* d_rec_ptr = nullptr;        // [nshots+1]
    int32_t* d_rec = nullptr;            // [nrec][3] (ix, iz, iy)
    int max_nrec = 0;

    // model-derived coefficients
    float* c2 = nullptr;                 // storage layout: v^2 dt^2 / dx^2
    float* kx = nullptr;                 // [nxp] damping contribution per column
    float* kz = nullptr;                 // [nzp]
    float* ky = nullptr;                 // [nyp]
    float vmax = 0.f;
    float lap_w[5] = {0, 0, 0, 0, 0};    // a_0..a_4 rounded once to float32

    // scratch, grown on demand
    float* ring = nullptr;               // [cap][4][fsize]: u slots 0/1, increment d slots 0/1
    int ring_cap = 0;
    float* ring2 = nullptr;              // second ring (gradient recompute)
    int ring2_cap = 0;
    float* dscr = nullptr;               // data scratch (CSR layout)
    int64_t dscr_cap = 0;
    float* dscr2 = nullptr;
    int64_t dscr2_cap = 0;
    double* part = nullptr;              // reduction partials
    int64_t part_cap = 0;
    int part_stride = 0;                 // partials per shot of the last N p
    double* scal = nullptr;              // CG scalars [8][nshots]
    float* gshot = nullptr;              // per-shot gradient accumulators
    int64_t gshot_cap = 0;
    float* store = nullptr;              // (dA/dm)u storage or segment buffer
    int64_t store_cap = 0;
    float* ckpt = nullptr;               // checkpoints
    int64_t ckpt_cap = 0;
    int* flags = nullptr;                // per-shot active / finish flags [2][nshots]
    int* cgi = nullptr;                  // CG bookkeeping: iters [nshots], status [nshots], ctl [2]
    double* cg_hist = nullptr;           // residual history [nshots][max_iter + 1]
    int64_t cg_hist_cap = 0;
    int* h_ctl = nullptr;                // pinned host copy of ctl
    // CG iterations captured as graphs (one per parity of the iteration index:
    // the direction and N p buffers trade places every iteration)
    bool cg_graph = false;
    bool cg_rfuse = true;                // 2D CG: residual update fused into the adjoint pass
    hipStream_t cap_stream = nullptr;    // capture and replay stream
    hipEvent_t cap_ev[2] = {nullptr, nullptr};
    hipGraph_t cg_g[2] = {nullptr, nullptr};
    hipGraphExec_t cg_exec[2] = {nullptr, nullptr};
    std::vector<uintptr_t> cg_key;       // what the captured graphs were built for
    float* vphys = nullptr;              // physical velocity [nphys] (network features)
    std::vector<int32_t> h_win;          // per-shot apertures [nshots][2] (empty: whole grid)
    int32_t* d_win = nullptr;
    // flexible CG scratch: cell scale, sum_t r^2 and sum_t r Np [nshots][nphys],
    // network input [nshots][3][Hp][Wp] and output [nshots][Hp][Wp], scalars
    float* fcg_s = nullptr; int64_t fcg_s_cap = 0;
    float* fcg_a = nullptr; int64_t fcg_a_cap = 0;
    double* fcg_g = nullptr; int64_t fcg_g_cap = 0;
    float* fcg_in = nullptr; int64_t fcg_in_cap = 0;
    float* fcg_o = nullptr; int64_t fcg_o_cap = 0;
    double* fcg_d = nullptr; int64_t fcg_d_cap = 0;   // pr, zAp, zr[3], mean, best [7][nshots]
    int* fcg_i = nullptr; int64_t fcg_i_cap = 0;      // mode, restart, fallback, kbest, cg_at [5][nshots]

    std::vector<TileLists*> lists;       // one per tile shape used
    int tb_fwd = LS_T2_32, tb_adj = LS_T2_32;   // launch shape of forward / adjoint loops (2D)
    // the autotuner's last candidate table: shape, forward ms, adjoint ms
    struct TuneRow { int shape; double fwd_ms, adj_ms; };
    std::vector<TuneRow> tune_rows;
    // checkpoints retained by esi_forward_ckpt for a SEED_REUSE gradient
    bool ck_valid = false;
    int ck_shot0 = 0, ck_nshots = 0, ck_kind = 0, ck_K = 0;
    const float* ck_src = nullptr;
    int64_t model_version = 0;

    // profiling: event pairs around time loops, folded into totals on read
    struct ProfRec { unsigned flags; int64_t launches, shot_launches; hipEvent_t e0, e1; };
    struct ProfTot { unsigned flags; int64_t launches, shot_launches; double ms; };
    bool prof_on = false;
    std::vector<ProfRec> prof_pending;
    std::vector<ProfTot> prof_tot;
};

// ---- allocation helpers -------------------------------------------------
esi_status_t grow(void** p, int64_t* cap, int64_t need_bytes, hipStream_t stream);
template <class T>
esi_status_t grow_t(T** p, int64_t* cap_elems, int64_t need_elems, hipStream_t stream) {
    int64_t capb = *cap_elems * (int64_t)sizeof(T);
    esi_status_t s = grow((void**)p, &capb, need_elems * (int64_t)sizeof(T), stream);
    *cap_elems = capb / (int64_t)sizeof(T);
    return s;
}

// Lists for a tile shape (built on first use).
esi_status_t get_lists(Plan* P, int tx, int tz, int ty, TileLists** out);

// Look up the no-allocation scratch array of `device` (current) once per
// process; called when a plan is created (noalloc.hip).
void noalloc_init_device(int device);

// ---- launch-side descriptions -----------------------------------------------
// Everything a time step needs; passed by value to the kernels.
struct StepArgs {
    // fields
    const float* cur;        // u^n (shot 0); shots are fstride apart
    float* nxt;              // u^{n+1} (or u^{n+2} for a two-step launch) out
    const float* din;        // d^n = u^n - u^{n-1} in
    float* dnx;              // d^{n+1} (or d^{n+2}) out
    int dir;                 // +1 forward in time, -1 adjoint (two-step launches)
    int64_t fstride;
    const float* c2;
    const float* kx;
    const float* kz;
    const float* ky;
    int nzp, nyp, nxp, XS, YS;
    int nb, nz, ny, nx;
    int64_t nphys;
    float w0, w1, w2, w3, w4;
    float dx2;               // dx^2 (source scale inside c2 (lap + dx^2 q))
    float inv_dt2;           // 1 / dt^2
    float beta;
    float b_eps;
    int w_identity;          // 1: beta B^2 = beta (WRI); 0: B = distance to the source + b_eps
    int step;                // n (forward) or j (adjoint)
    int nt;
    int tiles_x, tiles_y, tiles_z, tiles;   // per shot
    int nshots;
    int shot0;               // global index of the first shot
    const int32_t* src_pos;  // [global shots][3]
    const int64_t* rec_ptr;  // [global shots + 1]
    const int* active;       // [nshots] or null (all active)
    // tile lists
    const int32_t* inj_ptr; const int32_t* inj_cell; const int32_t* inj_rptr; const int32_t* inj_rid;
    const int32_t* gat_ptr; const int32_t* gat_cell; const int32_t* gat_rid;
    const int32_t* src_tile; const int32_t* src_cell;
    const int32_t* inj2_ptr; const int32_t* inj2_cell; const int32_t* inj2_rptr; const int32_t* inj2_rid;
    // sparse values
    const float* wavelet;    // point source [nshots][nt]
    const float* inj_data;   // data injected (adjoint), CSR layout
    float* gat_data;         // data recorded (forward), CSR layout
    // dense vectors, [nshots][nt][phys]
    const float* dsrc;       // dense source q^n (forward)
    float* dout;             // dense output (adjoint mu^j, or N p)
    const float* dp;         // p for N p = mu + beta B^2 p
    double* part;            // per-(shot, tile) float64 partial sums, accumulated
    int part_stride;         // partials per shot (the largest tile count in use)
    // CG fused direction update (forward): p = r + b p_old; x += a p_old
    const float* cg_r;
    const float* cg_p;       // p_old (read)
    float* cg_pn;            // p_new (written; a different buffer from cg_p)
    float* cg_x;
    const float* cg_s;           // F_SCALE: per-shot cell scale [nshots][nphys], z = s r
    float* cg_rw;                // F_RUPD with F_NORMAL: r, updated in place (adjoint)
    // per-shot apertures (2D): physical columns [win[2 gs], win[2 gs + 1]) of
    // global shot gs, or nullptr for the whole grid; damping table of shot gs
    // at kx + kx_stride * gs; work list of (shot, tile) items gs * tiles + t
    // of this batch (nwork of them), or nullptr for every tile of every shot
    const int32_t* win;
    int kx_stride;
    const int32_t* work;
    int nwork;
    const double* cg_alpha;  // [nshots]
    const double* cg_beta;   // [nshots]
    // gradient
    float* gacc;             // [nshots][phys] per-shot accumulators
    float* store;            // (dA/dm)u store [nshots][slots][phys]
    int64_t store_stride;    // floats per shot in store
    int store_slot;          // slot of this step
    int store_slot2;         // slot of the second step of a two-step launch; with
                             // corr_pair, slot of the previous step
    int corr_pair;           // one-step CORR launch (3D): also add the previous
                             // step's product, its input field times slot
                             // store_slot2, before this step's
    float* src_rec;          // [nshots][nt] adjoint field at the source cell
    // DTFT at dft_nf frequencies; frequency vectors [nshots][dft_nf][phys] of
    // (re, im) pairs; dft_tw[n][m] = (cos w_m t_n, sin w_m t_n)
    const float2* dft_src;   // F_DTFT_SRC: q^n = inv_nt sum_m Re(src_m exp(-j w_m t_n))
    float2* dft_acc;         // F_DTFT_ACC: acc_m += mu^j exp(+j w_m t_j)
    const float2* dft_tw;
    int dft_nf;
    float inv_nt;
    // blk_T > 0: dsrc and dout hold blk_T steps, step n in slot n % blk_T
    // ([nshots][blk_T][phys]); 0: the whole time axis
    int blk_T;
};

// kernel flag bits
enum : unsigned {
    F_SRC_POINT = 1u << 0,   // inject wavelet at the shot's source cell
    F_SRC_DENSE = 1u << 1,   // inject dense q^n
    F_CG_FUSE = 1u << 2,     // q^n = p_new = r + beta p_old, x += alpha p_old
    F_INJ = 1u << 3,         // inject R^T data^j (adjoint)
    F_GATHER = 1u << 4,      // record data^{n-1} = R u^n (forward)
    F_OUT = 1u << 5,         // write mu^j to dout (adjoint)
    F_NORMAL = 1u << 6,      // write mu^j + beta B^2 p^j to dout, accumulate p.Np
    F_PENALTY = 1u << 7,     // gacc += beta B^2 q^n (dA/dm) u^n (forward)
    F_STORE = 1u << 8,       // store (dA/dm) u^n into store slot (forward)
    F_CORR = 1u << 9,        // gacc += mu^j * store slot (adjoint)
    F_SRC_REC = 1u << 10,    // src_rec[s][j] = mu^j at the shot's source cell (adjoint)
    F_SCALE = 1u << 11,      // with F_CG_FUSE: the new direction is s r + beta p (flexible CG);
                             // p_new . r accumulates into the (shot, tile) partials;
                             // with F_SRC_DENSE: the dense source times the cell scale cg_s
    F_DTFT_SRC = 1u << 12,   // dense source from frequency slices (inverse DTFT on the fly)
    F_DTFT_ACC = 1u << 13,   // accumulate the DTFT of the output mu^j (adjoint)
    F_RUPD = 1u << 14,       // CG residual update fused into the normal operator:
                             // with F_CG_FUSE (or F_SRC_DENSE: p is the dense source)
                             // the partials of beta B^2 p . p;
                             // with F_NORMAL r -= alpha (mu^j + beta B^2 p^j) in place
                             // (cg_rw) and the partials of r . r, no dout
};

// Gather of the last trace d^{nt-1} = R u^{nt} (after the time loop).
esi_status_t launch_final_gather(Plan* P, const float* field, int64_t fstride, float* data,
                                 int shot0, int nshots);

// ---- vector kernels (vec.hip) ---------------------------------------------
esi_status_t launch_fill(Plan* P, float* p, int64_t n, float v);
esi_status_t launch_copy(Plan* P, float* dst, const float* src, int64_t n);
// per shot s < nshots: dst[s * dst_stride + i] = src[s * src_stride + i], i < n
esi_status_t launch_copy_shots(Plan* P, float* dst, int64_t dst_stride, const float* src,
                               int64_t src_stride, int64_t n, int nshots);
// One stored field per shot s < nshots (global shot shot0 + s), dst[s * dst_stride
// + i] = src[s * src_stride + i]: with 2D apertures only the window's cells
// (with its absorbing layer), the only ones a step ever makes non-zero.
esi_status_t launch_copy_fields(Plan* P, float* dst, int64_t dst_stride, const float* src, int64_t src_stride,
                                int shot0, int nshots);
// r -= alpha_s Np (float32), partial r.r (float64) per block into part;
// then reduce into out[s].  Vectors are [nshots][len].
esi_status_t launch_r_update(Plan* P, float* r, const float* Ap, const double* alpha,
                             const int* active, int nshots, int64_t len, double* rr_out);
// x += alpha_s p for the shots whose flag equals `which`.
esi_status_t launch_axpy_flag(Plan* P, float* x, const float* p, const double* alpha,
                              const int* flag, int which, int nshots, int64_t len);
// out[s] = sum of part[s][0..n)
// Fused-residual CG: pAp[s] holds sum beta B^2 p.p of shot s on entry and
// leaves as that plus ||S p||^2 over the shot's data (data of shots shot0..
// back to back, CSR layout); alpha[s] = rr[s] / pAp[s].  Needs P->part to
// hold DATA_BLOCKS partials per shot; tmp takes nshots doubles.
constexpr int DATA_BLOCKS = 64;
esi_status_t launch_cg_alpha_data(Plan* P, int shot0, int nshots, const float* data, const int* active,
                                  const double* rr, double* pAp, double* tmp, double* alpha);
esi_status_t launch_reduce_parts(Plan* P, const double* part, int64_t n, int nshots,
                                 double* out);
// per-shot scalar updates of CG
esi_status_t launch_cg_alpha(Plan* P, const double* rr, const double* pAp, double* alpha,
                             int nshots);
esi_status_t launch_cg_beta(Plan* P, const double* rr_new, double* rr, double* beta, int nshots);
esi_status_t launch_cg_init(Plan* P, const double* rr0, int* active, int* finish, int* iters,
                            int* status, double* hist, int hstride, int* ctl, int nshots);
esi_status_t launch_cg_control(Plan* P, const double* rr0, const double* rr_new, const double* pAp,
                               int* active, int* finish, int* iters, int* status, double* hist,
                               int hstride, int* ctl, double rtol, int max_iter, int nshots);
// grad[phys] += sum_s gacc[s][phys] (fixed order over s)
esi_status_t launch_sum_shots(Plan* P, const float* gacc, int nshots, int64_t len, float sign,
                              float* grad);
// out = a - b elementwise
esi_status_t launch_sub(Plan* P, float* out, const float* a, const float* b, int64_t n);
// grad_src point: out[s][n] = mu at the source cell, from a dense [nshots][nt][phys] field
esi_status_t launch_trace_at_src(Plan* P, const float* dense, int shot0, int nshots, float* out);
// grad_v = -2 grad_m / v^3
esi_status_t launch_grad_velocity(Plan* P, const float* vel, const float* gm, float* gv, int64_t n);

// per-shot ring: u slot 0, u slot 1, d slot 0, d slot 1.  The current state is
// (u[cs], d[cs]); every launch writes (u[1-cs], d[1-cs]) and flips cs.
constexpr int RING = 4;

// time-loop plumbing of the entry points (api.hip)
esi_status_t check_shots(Plan* P, int shot0, int nshots);
esi_status_t lists_for(Plan* P, TileLists** L);
// launch shape a loop of `flags` runs with (the plan's choice, or 32-row
// two-step tiles for variants without other heights), and its tiling
int loop_shape(Plan* P, unsigned flags, bool adjoint);
esi_status_t shape_lists(Plan* P, int shape, TileLists** L);
void shape_tile(Plan* P, int shape, int* tx, int* ty, int* tz);
// the largest tile count of the plan's tilings (stride of per-tile partials)
int max_tiles(Plan* P);
StepArgs base_args(Plan* P, const TileLists* L, int shot0, int nshots);
esi_status_t ring_for(Plan* P, float** ring, int* cap, int nshots);
int64_t data_len(Plan* P, int shot0, int nshots);
// forward steps [n0, n1) (checkpoints of (u, d) every K steps into ckpt when given)
esi_status_t forward_loop(Plan* P, StepArgs a, unsigned flags, float* ring, int* cs, int n0, int n1,
                          float* ckpt = nullptr, int K = 0, int nseg = 0);
// adjoint steps j = j1 - 1 down to j0 (segment length K for the store slots)
esi_status_t adjoint_loop(Plan* P, StepArgs a, unsigned flags, float* ring, int* cs, int j0, int j1,
                          int K = 0);

// forward pass of q (+ point wavelets bg) with the PENALTY correlation into
// gshot, the data S(q [+ f]) into dsyn and the per-shot penalty beta W q^2 sums
// into pen (api.hip; used by the outer loop)
esi_status_t penalty_eval(Plan* P, int shot0, int ns, const float* q, const float* bg, float* gshot,
                          float* dsyn, double* pen);

// flexible CG (fcg.hip) and the network (unet.hip)
esi_status_t launch_energy(Plan* P, const float* r, const int* active, float* a, int ns);
esi_status_t launch_stats(Plan* P, const float* r, const float* x, const float* p, const double* alpha,
                          const float* xref, const int* iters, int k, float* out, int ns);
esi_status_t launch_features(Plan* P, int shot0, int ns, const float* a, const float* c, double* mean, int Hp,
                             int Wp, const float* base, float* xin, float* apad, float* cpad);
esi_status_t launch_fcg_zr_check_scale(Plan* P, const float* o, const float* fixed, const float* a,
                                       const int* active, int* mode, int* restart, int* fallback, int* cg_at,
                                       double* best, int* kbest, const double* hist, int hstride, int k,
                                       int Hp, int Wp, double* zr, float* S, int ns);
esi_status_t launch_scale_vec(Plan* P, float* p, const float* r, const float* S, int ns);
// r -= alpha Np for active shots; per cell en = sum_t r^2 and rnp = sum_t r Np of
// the new r; rr_out[s] = sum of r^2 (all FP64 sums)
esi_status_t launch_r_update_cells(Plan* P, float* r, const float* Np, const double* alpha, const int* active,
                                   int ns, float* en, double* rnp, double* rr_out);
// out[s] = sum_x S[s][x] g[s][x]
esi_status_t launch_dot_cells(Plan* P, const float* S, const double* g, int ns, double* out);
esi_status_t launch_fcg_beta(Plan* P, const double* zAp, const double* pAp, const int* restart, double* beta,
                             int ns);
esi_status_t launch_fcg_init(Plan* P, int* mode, int* restart, int* fallback, int* cg_at, double* best, int* kbest,
                             int ns);
esi_status_t launch_fcg_control(Plan* P, const double* rr0, const double* rr_new, const double* pAp, int* active,
                                int* finish, int* iters, int* status, double* hist, int hstride, int* ctl,
                                double rtol, int max_iter, int* mode, int* restart, int* fallback, int* cg_at,
                                double stall, int window, double* best, int* kbest, bool has_net, int ns);
esi_status_t unet_dims(esi_unet_t u, int* H, int* W, int* maxb);
esi_status_t unet_forward_on(esi_unet_t u, hipStream_t stream, const float* x, float* o, int batch);

}  // namespace esi
