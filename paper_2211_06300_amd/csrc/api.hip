// C-ABI entry points: modelling, adjoint modelling, normal operator, CG and
// gradient (the calls of the ESI hot path, Sec. 2-3 and Algorithms 1-2).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "esi_internal.h"

namespace esi {

esi_status_t launch_step2d(Plan* P, unsigned flags, const StepArgs& a, int shape);
int step2d_loop_shape(unsigned flags, int shape);
void step2d_tile_shape(int* tx, int* tz);
void step2d_shape_tile(int shape, int* tx, int* tz);
esi_status_t launch_step3d(Plan* P, unsigned flags, const StepArgs& a);
esi_status_t launch_step3d_t2(Plan* P, unsigned flags, const StepArgs& a);
bool step3d_t2_has(unsigned flags);
void step3d_tile_shape(int* tx, int* ty, int* tz);
void step3d_t2_tile_shape(int* tx, int* ty, int* tz);
esi_status_t launch_dot(Plan* P, const float* x, const float* y, int nshots, int64_t len,
                        double* out);
esi_status_t launch_fill_d(Plan* P, double* p, int64_t n);

esi_status_t check_shots(Plan* P, int shot0, int nshots) {
    if (nshots < 1 || shot0 < 0 || shot0 + nshots > P->nshots)
        return fail(ESI_ERR_ARG, "shot range [" + std::to_string(shot0) + ", " +
                                     std::to_string(shot0 + nshots) + ") outside [0, " +
                                     std::to_string(P->nshots) + ")");
    return ESI_OK;
}

esi_status_t lists_for(Plan* P, TileLists** L) {
    int tx, ty = 1, tz;
    if (P->ndim == 2) step2d_tile_shape(&tx, &tz);
    else step3d_tile_shape(&tx, &ty, &tz);
    return get_lists(P, tx, tz, ty, L);
}

esi_status_t launch_step(Plan* P, unsigned flags, const StepArgs& a, int shape) {
    if (P->ndim == 2) return launch_step2d(P, flags, a, shape);
    return shape == LS_ONE ? launch_step3d(P, flags, a) : launch_step3d_t2(P, flags, a);
}

// 2D: the plan's shape (32-row tiles for variants without other heights);
// 3D: two steps per launch (LS_T2_32) for the variants the two-step kernel has
int loop_shape(Plan* P, unsigned flags, bool adjoint) {
    const int want = adjoint ? P->tb_adj : P->tb_fwd;
    if (P->ndim == 2) return step2d_loop_shape(flags, want);
    return want != LS_ONE && step3d_t2_has(flags) ? LS_T2_32 : LS_ONE;
}

void shape_tile(Plan* P, int shape, int* tx, int* ty, int* tz) {
    *ty = 1;
    if (P->ndim == 2) step2d_shape_tile(shape, tx, tz);
    else if (shape == LS_ONE) step3d_tile_shape(tx, ty, tz);
    else step3d_t2_tile_shape(tx, ty, tz);
}

esi_status_t shape_lists(Plan* P, int shape, TileLists** L) {
    int tx, ty, tz;
    shape_tile(P, shape, &tx, &ty, &tz);
    return get_lists(P, tx, tz, ty, L);
}

int max_tiles(Plan* P) {
    int m = 0;
    for (const TileLists* L : P->lists) m = std::max(m, L->tiles);
    return m;
}

namespace {
// Build the tilings of the time loops of `fflags` (forward) and `aflags`
// (adjoint) before per-tile partials are sized by max_tiles.
esi_status_t loop_lists(Plan* P, unsigned fflags, unsigned aflags) {
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    ESI_TRY(shape_lists(P, loop_shape(P, fflags, false), &L));
    return shape_lists(P, loop_shape(P, aflags, true), &L);
}
}  // namespace

// Point the tile fields and sparse lists of `a` at the tiling `L`.
void apply_lists(StepArgs& a, const TileLists* L) {
    a.tiles_x = L->tiles_x; a.tiles_y = L->tiles_y; a.tiles_z = L->tiles_z; a.tiles = L->tiles;
    a.inj_ptr = L->inj_ptr; a.inj_cell = L->inj_cell; a.inj_rptr = L->inj_rptr; a.inj_rid = L->inj_rid;
    a.gat_ptr = L->gat_ptr; a.gat_cell = L->gat_cell; a.gat_rid = L->gat_rid;
    a.src_tile = L->src_tile; a.src_cell = L->src_cell;
    a.inj2_ptr = L->inj2_ptr; a.inj2_cell = L->inj2_cell; a.inj2_rptr = L->inj2_rptr; a.inj2_rid = L->inj2_rid;
    if (L->work) {
        a.work = L->work + L->work_ptr[a.shot0];
        a.nwork = (int)(L->work_ptr[a.shot0 + a.nshots] - L->work_ptr[a.shot0]);
    } else {
        a.work = nullptr;
        a.nwork = 0;
    }
}

// Fill the fields every step of a call shares.
StepArgs base_args(Plan* P, const TileLists* L, int shot0, int nshots) {
    StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.fstride = RING * P->fsize;
    a.c2 = P->c2; a.kx = P->kx; a.kz = P->kz; a.ky = P->ky;
    a.nzp = P->nzp; a.nyp = P->nyp; a.nxp = P->nxp; a.XS = P->XS; a.YS = P->YS;
    a.nb = P->nb; a.nz = P->nz; a.ny = P->ny; a.nx = P->nx; a.nphys = P->nphys;
    a.w0 = P->lap_w[0]; a.w1 = P->lap_w[1]; a.w2 = P->lap_w[2]; a.w3 = P->lap_w[3]; a.w4 = P->lap_w[4];
    a.dx2 = (float)(P->dx * P->dx);
    a.inv_dt2 = (float)(1.0 / (P->dt * P->dt));
    a.beta = (float)P->beta;
    a.b_eps = (float)P->b_eps;
    a.w_identity = P->w_identity;
    a.nt = P->nt;
    a.dir = 1;
    a.nshots = nshots; a.shot0 = shot0;
    a.src_pos = P->d_src; a.rec_ptr = P->d_rec_ptr;
    a.win = P->d_win;
    a.kx_stride = P->d_win ? P->nxp : 0;
    apply_lists(a, L);
    return a;
}

// A zeroed ring for `nshots` shots; the state starts in slot 0.
esi_status_t ring_for(Plan* P, float** ring, int* cap, int nshots) {
    if (nshots > *cap || !*ring) {
        int64_t capb = (int64_t)(*ring ? *cap : 0) * RING * P->fsize * (int64_t)sizeof(float);
        ESI_TRY(grow((void**)ring, &capb, (int64_t)nshots * RING * P->fsize * (int64_t)sizeof(float), P->stream));
        *cap = nshots;
    }
    return launch_fill(P, *ring, (int64_t)nshots * RING * P->fsize, 0.f);
}

void set_fields(Plan* P, StepArgs& a, float* ring, int cs) {
    a.cur = ring + (int64_t)cs * P->fsize;
    a.nxt = ring + (int64_t)(1 - cs) * P->fsize;
    a.din = ring + (int64_t)(2 + cs) * P->fsize;
    a.dnx = ring + (int64_t)(3 - cs) * P->fsize;
}

int64_t data_len(Plan* P, int shot0, int nshots) {
    return (int64_t)P->nt * (P->h_rec_ptr[shot0 + nshots] - P->h_rec_ptr[shot0]);
}

// Profiling brackets around a time loop.
struct ProfScope {
    Plan* P; unsigned flags; int64_t launches, shots; hipEvent_t e0 = nullptr, e1 = nullptr;
    ProfScope(Plan* p, unsigned f, int64_t ns) : P(p), flags(f), launches(0), shots(ns) {
        if (!P->prof_on) return;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { e0 = e1 = nullptr; return; }
        hipEventRecord(e0, P->stream);
    }
    ~ProfScope() {
        if (!e0) return;
        hipEventRecord(e1, P->stream);
        if (launches > 0) P->prof_pending.push_back({flags, launches, launches * shots, e0, e1});
        else { hipEventDestroy(e0); hipEventDestroy(e1); }
    }
};

// Forward time loop over [n0, n1) on `ring` whose state is in slot *cs.
// Two-step launches are used where allowed; a checkpoint of (u^n, d^n) is
// saved at every n = k*K into ckpt[s][k][2][fsize] (two-step launches never
// straddle a checkpoint).  Profiling records two-step launches with bit 1<<15
// and their launch shape in bits 16-18.
esi_status_t forward_loop(Plan* P, StepArgs a, unsigned flags, float* ring, int* cs, int n0,
                          int n1, float* ckpt, int K, int nseg) {
    const int shape = loop_shape(P, flags, false);
    ProfScope p1(P, flags, a.nshots), p2(P, flags | (1u << 15) | ((unsigned)shape << 16), a.nshots);
    TileLists* L2 = nullptr;
    if (shape != LS_ONE) ESI_TRY(shape_lists(P, shape, &L2));
    const bool t2 = L2 != nullptr;
    StepArgs b = a;
    if (t2) apply_lists(b, L2);
    a.dir = b.dir = 1;
    for (int n = n0; n < n1;) {
        if (ckpt && n % K == 0) {
            const int k = n / K;
            const int64_t cstr = (int64_t)nseg * 2 * P->fsize;   // per-shot checkpoint stride
            ESI_TRY(launch_copy_fields(P, ckpt + (int64_t)k * 2 * P->fsize, cstr,
                                       ring + (int64_t)(*cs) * P->fsize, RING * P->fsize, a.shot0,
                                       a.nshots));
            ESI_TRY(launch_copy_fields(P, ckpt + (int64_t)k * 2 * P->fsize + P->fsize, cstr,
                                       ring + (int64_t)(2 + *cs) * P->fsize, RING * P->fsize, a.shot0,
                                       a.nshots));
        }
        const bool two = t2 && n + 1 < n1 && !(ckpt && (n + 1) % K == 0);
        StepArgs& c = two ? b : a;
        c.step = n;
        set_fields(P, c, ring, *cs);
        if (flags & F_STORE) {
            c.store_slot = K > 0 ? n % K : n;
            c.store_slot2 = K > 0 ? (n + 1) % K : n + 1;
        }
        ESI_TRY(launch_step(P, flags, c, two ? shape : LS_ONE));
        (two ? p2 : p1).launches++;
        *cs ^= 1;
        n += two ? 2 : 1;
    }
    return ESI_OK;
}

// Adjoint time loop over j = j1-1 .. j0 on `ring` whose state is in slot *cs.
esi_status_t adjoint_loop(Plan* P, StepArgs a, unsigned flags, float* ring, int* cs, int j0,
                          int j1, int K) {
    const int shape = loop_shape(P, flags, true);
    ProfScope p1(P, flags, a.nshots), p2(P, flags | (1u << 15) | ((unsigned)shape << 16), a.nshots);
    TileLists* L2 = nullptr;
    if (shape != LS_ONE) ESI_TRY(shape_lists(P, shape, &L2));
    const bool t2 = L2 != nullptr;
    StepArgs b = a;
    if (t2) apply_lists(b, L2);
    a.dir = b.dir = -1;
    // One-step correlating launches in 3D go in pairs: the first without the
    // correlation, the second adding both steps' products in the order a
    // two-step launch chains them, so the accumulator crosses HBM once per
    // pair and the bits are those of unpaired launches.
    const bool pair = !t2 && (flags & F_CORR) && P->ndim == 3;
    for (int j = j1 - 1; j >= j0;) {
        if (pair && j - 1 >= j0) {
            a.step = j;
            set_fields(P, a, ring, *cs);
            ESI_TRY(launch_step(P, flags & ~F_CORR, a, LS_ONE));
            *cs ^= 1;
            a.step = j - 1;
            set_fields(P, a, ring, *cs);
            a.store_slot = K > 0 ? (j - 1) % K : j - 1;
            a.store_slot2 = K > 0 ? j % K : j;
            a.corr_pair = 1;
            const esi_status_t st = launch_step(P, flags, a, LS_ONE);
            a.corr_pair = 0;
            ESI_TRY(st);
            p1.launches += 2;
            *cs ^= 1;
            j -= 2;
            continue;
        }
        const bool two = t2 && j - 1 >= j0;
        StepArgs& c = two ? b : a;
        c.step = j;
        set_fields(P, c, ring, *cs);
        if (flags & F_CORR) {
            c.store_slot = K > 0 ? j % K : j;
            c.store_slot2 = K > 0 ? (j - 1) % K : j - 1;
        }
        ESI_TRY(launch_step(P, flags, c, two ? shape : LS_ONE));
        (two ? p2 : p1).launches++;
        *cs ^= 1;
        j -= two ? 2 : 1;
    }
    return ESI_OK;
}

esi_status_t do_forward(Plan* P, int shot0, int ns, int kind, const float* src, float* data,
                        const TileLists* L) {
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs a = base_args(P, L, shot0, ns);
    unsigned fl = F_GATHER;
    if (kind == ESI_SRC_POINT) { fl |= F_SRC_POINT; a.wavelet = src; }
    else { fl |= F_SRC_DENSE; a.dsrc = src; }
    a.gat_data = data;
    int cs = 0;
    ESI_TRY(forward_loop(P, a, fl, P->ring, &cs, 0, P->nt));
    return launch_final_gather(P, P->ring + (int64_t)cs * P->fsize, RING * P->fsize, data, shot0, ns);
}

namespace {

// N p into Ap (+ p.Np partials in P->part [ns][tiles]) for the active shots.
// With cg_fuse the forward pass first forms p_new = r + beta p (p = p_old is
// read, p_new written to `pnew`) and x += alpha p_old; N is applied to p_new.
// Ap may be the p_old buffer (it is dead once the forward pass has run).
//
// With cg_s (flexible CG) the forward pass forms p = s r + beta p_old and
// writes the per-shot p . r (FP64) to pr.
esi_status_t do_normal(Plan* P, int shot0, int ns, const float* p, float* Ap, const TileLists* L,
                       const int* active, bool cg_fuse, float* pnew, const float* r, float* x,
                       const double* alpha, const double* beta, const float* cg_s = nullptr,
                       double* pr = nullptr) {
    if (cg_s && (!cg_fuse || !pr)) return fail(ESI_ERR_ARG, "internal: scaled direction needs p.r output");
    const int64_t dl = data_len(P, shot0, ns);
    ESI_TRY(grow_t(&P->dscr, &P->dscr_cap, std::max<int64_t>(dl, 1), P->stream));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    ESI_TRY(loop_lists(P, cg_fuse ? F_CG_FUSE | F_GATHER | (cg_s ? F_SCALE : 0u) : F_SRC_DENSE | F_GATHER,
                       F_INJ | F_NORMAL));
    P->part_stride = max_tiles(P);
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)ns * P->part_stride, P->stream));
    StepArgs a = base_args(P, L, shot0, ns);
    a.active = active;
    a.gat_data = P->dscr;
    int cs = 0;
    if (cg_fuse) {
        a.cg_r = r; a.cg_p = p; a.cg_pn = pnew; a.cg_x = x; a.cg_alpha = alpha; a.cg_beta = beta;
        a.cg_s = cg_s;
        if (cg_s) {
            ESI_TRY(launch_fill_d(P, P->part, (int64_t)ns * P->part_stride));
            a.part = P->part;
            a.part_stride = P->part_stride;
        }
        ESI_TRY(forward_loop(P, a, F_CG_FUSE | F_GATHER | (cg_s ? F_SCALE : 0u), P->ring, &cs, 0, P->nt));
        if (cg_s) ESI_TRY(launch_reduce_parts(P, P->part, P->part_stride, ns, pr));
    } else {
        a.dsrc = p;
        ESI_TRY(forward_loop(P, a, F_SRC_DENSE | F_GATHER, P->ring, &cs, 0, P->nt));
    }
    ESI_TRY(launch_final_gather(P, P->ring + (int64_t)cs * P->fsize, RING * P->fsize, P->dscr,
                                shot0, ns));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    ESI_TRY(launch_fill_d(P, P->part, (int64_t)ns * P->part_stride));
    StepArgs b = base_args(P, L, shot0, ns);
    b.active = active;
    b.inj_data = P->dscr;
    b.dp = cg_fuse ? pnew : p;
    b.dout = Ap;
    b.part = P->part;
    b.part_stride = P->part_stride;
    cs = 0;
    return adjoint_loop(P, b, F_INJ | F_NORMAL, P->ring, &cs, 0, P->nt);
}

// Iteration k of Algorithm 1 with the residual update fused into the normal
// operator.  For k >= 1 the forward pass forms p_k = r_k + beta p_{k-1} into
// pnew and x_k = x_{k-1} + alpha p_{k-1}; for k = 0 (first) it takes p = p_0
// as its dense source and pnew is unused.  It records S p_k and the partials
// of beta B^2 p_k . p_k; with p_k . N p_k = ||S p_k||^2 + beta ||B p_k||^2 the
// step length is known before the adjoint pass, which then takes
// r_{k+1} = r_k - alpha_k N p_k cell by cell in place, with the partials of
// ||r_{k+1}||^2.  N p_k is never stored: per step, the adjoint reads r and
// writes it back instead of writing N p for a separate pass to read.
esi_status_t do_normal_rupd(Plan* P, int shot0, int ns, const float* p, float* pnew, const TileLists* L,
                            const int* active, float* r, float* x, double* alpha, const double* beta,
                            const double* rr, double* pAp, double* rr_new, bool first) {
    const int64_t dl = data_len(P, shot0, ns);
    ESI_TRY(grow_t(&P->dscr, &P->dscr_cap, std::max<int64_t>(dl, 1), P->stream));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    ESI_TRY(loop_lists(P, (first ? F_SRC_DENSE : F_CG_FUSE) | F_GATHER | F_RUPD, F_INJ | F_NORMAL | F_RUPD));
    P->part_stride = max_tiles(P);
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)ns * std::max(P->part_stride, DATA_BLOCKS), P->stream));
    ESI_TRY(launch_fill_d(P, P->part, (int64_t)ns * P->part_stride));
    StepArgs a = base_args(P, L, shot0, ns);
    a.active = active;
    a.gat_data = P->dscr;
    if (first) {
        a.dsrc = p;
    } else {
        a.cg_r = r; a.cg_p = p; a.cg_pn = pnew; a.cg_x = x; a.cg_alpha = alpha; a.cg_beta = beta;
    }
    a.part = P->part;
    a.part_stride = P->part_stride;
    int cs = 0;
    ESI_TRY(forward_loop(P, a, (first ? F_SRC_DENSE : F_CG_FUSE) | F_GATHER | F_RUPD, P->ring, &cs, 0, P->nt));
    ESI_TRY(launch_final_gather(P, P->ring + (int64_t)cs * P->fsize, RING * P->fsize, P->dscr,
                                shot0, ns));
    ESI_TRY(launch_reduce_parts(P, P->part, P->part_stride, ns, pAp));
    ESI_TRY(launch_cg_alpha_data(P, shot0, ns, P->dscr, active, rr, pAp, rr_new, alpha));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    ESI_TRY(launch_fill_d(P, P->part, (int64_t)ns * P->part_stride));
    StepArgs b = base_args(P, L, shot0, ns);
    b.active = active;
    b.inj_data = P->dscr;
    b.dp = first ? p : pnew;
    b.cg_rw = r;
    b.cg_alpha = alpha;
    b.part = P->part;
    b.part_stride = P->part_stride;
    cs = 0;
    ESI_TRY(adjoint_loop(P, b, F_INJ | F_NORMAL | F_RUPD, P->ring, &cs, 0, P->nt));
    return launch_reduce_parts(P, P->part, P->part_stride, ns, rr_new);
}

}  // namespace
}  // namespace esi

using namespace esi;

extern "C" esi_status_t esi_forward(esi_plan_t plan, int32_t shot0, int32_t nshots,
                                    int32_t src_kind, const float* src, float* data) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, nshots));
    if (src_kind != ESI_SRC_POINT && src_kind != ESI_SRC_DENSE) return fail(ESI_ERR_ARG, "bad src_kind");
    if (!src) return fail(ESI_ERR_ARG, "null src");
    if (!data && data_len(P, shot0, nshots) > 0) return fail(ESI_ERR_ARG, "null data");
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    return do_forward(P, shot0, nshots, src_kind, src, data, L);
}

extern "C" esi_status_t esi_adjoint(esi_plan_t plan, int32_t shot0, int32_t nshots,
                                    const float* data, float* out) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, nshots));
    if (!out || (!data && data_len(P, shot0, nshots) > 0)) return fail(ESI_ERR_ARG, "null pointer");
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, nshots));
    StepArgs a = base_args(P, L, shot0, nshots);
    a.inj_data = data;
    a.dout = out;
    int cs = 0;
    return adjoint_loop(P, a, F_INJ | F_OUT, P->ring, &cs, 0, P->nt);
}

extern "C" esi_status_t esi_normal_apply(esi_plan_t plan, int32_t shot0, int32_t nshots,
                                         const float* p, float* Ap, double* pAp) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, nshots));
    if (!p || !Ap) return fail(ESI_ERR_ARG, "null pointer");
    const int64_t n = (int64_t)nshots * P->nt * P->nphys;
    if ((Ap < p + n) && (p < Ap + n)) return fail(ESI_ERR_ARG, "p and Ap overlap");
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    ESI_TRY(do_normal(P, shot0, nshots, p, Ap, L, nullptr, false, nullptr, nullptr, nullptr, nullptr,
                      nullptr));
    if (pAp) ESI_TRY(launch_reduce_parts(P, P->part, P->part_stride, nshots, pAp));
    return ESI_OK;
}

namespace esi {
namespace {

// Buffers and scalars of one CG solve (Algorithm 1, one system per shot).
struct CgState {
    int shot0, ns, max_iter;
    double rtol;
    int64_t len;
    const TileLists* L;
    float *x, *r, *p, *Ap;
    double *rr, *pAp, *alpha, *beta, *rr_new, *rr0;
    int *active, *finish, *iters, *status, *ctl;
    double* hist;
};

// Enqueue iteration k (kernels only: no host decision, no allocation, so it
// can be captured).  k = 0 applies N to p_0 = r_0; later iterations form
// p_k = r_k + beta p_{k-1} and x_k = x_{k-1} + alpha p_{k-1} inside the forward
// pass, writing p_k into the buffer that held N p_{k-1}, and N p_k over p_{k-1}.
// The caller swaps p and Ap after every iteration k >= 1.
esi_status_t cg_iteration(Plan* P, const CgState& c, int k, const float* p, float* Ap) {
    const float* dir = p;
    if (P->cg_rfuse) {
        ESI_TRY(do_normal_rupd(P, c.shot0, c.ns, p, Ap, c.L, c.active, c.r, c.x, c.alpha, c.beta, c.rr,
                               c.pAp, c.rr_new, k == 0));
        ESI_TRY(launch_cg_control(P, c.rr0, c.rr_new, c.pAp, c.active, c.finish, c.iters, c.status,
                                  c.hist, c.max_iter + 1, c.ctl, c.rtol, c.max_iter, c.ns));
        ESI_TRY(launch_cg_beta(P, c.rr_new, c.rr, c.beta, c.ns));
        // shots leaving now take x += alpha p_k; p_k is p_0 itself at k = 0 and lives in Ap later
        return launch_axpy_flag(P, c.x, k == 0 ? p : Ap, c.alpha, c.finish, 1, c.ns, c.len);
    }
    if (k == 0) {
        ESI_TRY(do_normal(P, c.shot0, c.ns, p, Ap, c.L, c.active, false, nullptr, c.r, c.x,
                          c.alpha, c.beta));
    } else {
        ESI_TRY(do_normal(P, c.shot0, c.ns, p, const_cast<float*>(p), c.L, c.active, true, Ap,
                          c.r, c.x, c.alpha, c.beta));
        dir = Ap;                        // p_k lives in the old N p buffer
        Ap = const_cast<float*>(p);      // N p_k over p_{k-1}
    }
    ESI_TRY(launch_reduce_parts(P, P->part, P->part_stride, c.ns, c.pAp));
    ESI_TRY(launch_cg_alpha(P, c.rr, c.pAp, c.alpha, c.ns));
    ESI_TRY(launch_r_update(P, c.r, Ap, c.alpha, c.active, c.ns, c.len, c.rr_new));
    ESI_TRY(launch_cg_control(P, c.rr0, c.rr_new, c.pAp, c.active, c.finish, c.iters, c.status,
                              c.hist, c.max_iter + 1, c.ctl, c.rtol, c.max_iter, c.ns));
    ESI_TRY(launch_cg_beta(P, c.rr_new, c.rr, c.beta, c.ns));
    // shots leaving now take their last update x_{k+1} = x_k + alpha_k p_k
    return launch_axpy_flag(P, c.x, dir, c.alpha, c.finish, 1, c.ns, c.len);
}

uintptr_t beta_bits(double b) {
    uint64_t u;
    std::memcpy(&u, &b, sizeof u);
    return (uintptr_t)u;
}

// Everything a captured iteration depends on besides its parity.
std::vector<uintptr_t> cg_graph_key(Plan* P, const CgState& c) {
    return {(uintptr_t)c.shot0, (uintptr_t)c.ns, (uintptr_t)c.max_iter,
            (uintptr_t)std::llround(c.rtol * 1e18), (uintptr_t)c.L, (uintptr_t)c.x,
            (uintptr_t)c.r, (uintptr_t)c.hist, (uintptr_t)P->ring, (uintptr_t)P->dscr,
            (uintptr_t)P->part, (uintptr_t)(P->tb_fwd * 8 + P->tb_adj), (uintptr_t)P->part_stride,
            (uintptr_t)P->w_identity, beta_bits(P->beta), (uintptr_t)P->cg_rfuse};
}

void cg_graph_drop(Plan* P) {
    for (int i = 0; i < 2; ++i) {
        if (P->cg_exec[i]) hipGraphExecDestroy(P->cg_exec[i]);
        if (P->cg_g[i]) hipGraphDestroy(P->cg_g[i]);
        P->cg_exec[i] = nullptr;
        P->cg_g[i] = nullptr;
    }
    P->cg_key.clear();
}

// Capture iteration k (parity k & 1, k >= 1) on the plan's capture stream.
esi_status_t cg_graph_capture(Plan* P, const CgState& c, int k, const float* p, float* Ap) {
    const int i = k & 1;
    hipStream_t user = P->stream;
    const bool prof = P->prof_on;
    P->stream = P->cap_stream;
    P->prof_on = false;
    ESI_HIP_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    esi_status_t st = cg_iteration(P, c, k, p, Ap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
    P->stream = user;
    P->prof_on = prof;
    if (st != ESI_OK) {
        if (g) hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(ESI_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    P->cg_g[i] = g;
    e = hipGraphInstantiate(&P->cg_exec[i], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        P->cg_exec[i] = nullptr;
        return fail(ESI_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return ESI_OK;
}

// Replay a captured iteration after the work already queued on the plan's
// stream, and make later work on that stream wait for it.
esi_status_t cg_graph_launch(Plan* P, int i) {
    ESI_HIP_TRY(hipEventRecord(P->cap_ev[0], P->stream));
    ESI_HIP_TRY(hipStreamWaitEvent(P->cap_stream, P->cap_ev[0], 0));
    ESI_HIP_TRY(hipGraphLaunch(P->cg_exec[i], P->cap_stream));
    ESI_HIP_TRY(hipEventRecord(P->cap_ev[1], P->cap_stream));
    ESI_HIP_TRY(hipStreamWaitEvent(P->stream, P->cap_ev[1], 0));
    return ESI_OK;
}

}  // namespace
}  // namespace esi

extern "C" esi_status_t esi_plan_set_cg_graph(esi_plan_t plan, int32_t enable) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    if (enable && !P->cap_stream) {
        ESI_HIP_TRY(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
        ESI_HIP_TRY(hipEventCreateWithFlags(&P->cap_ev[0], hipEventDisableTiming));
        ESI_HIP_TRY(hipEventCreateWithFlags(&P->cap_ev[1], hipEventDisableTiming));
    }
    if (!enable) {
        if (P->cap_stream) ESI_HIP_TRY(hipStreamSynchronize(P->cap_stream));
        cg_graph_drop(P);
    }
    P->cg_graph = enable != 0;
    return ESI_OK;
}

extern "C" esi_status_t esi_plan_set_cg_rfuse(esi_plan_t plan, int32_t enable) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    ((Plan*)plan)->cg_rfuse = enable != 0;
    return ESI_OK;
}

namespace esi {
namespace {

// Algorithm 1 from x_0 = 0 (resume = NULL) or from a saved state, optionally
// leaving the state of the last iteration in `save`.
esi_status_t cg_solve_impl(Plan* P, int32_t shot0, int32_t ns, const float* d_obs, float* x, float* work,
                           int32_t max_iter, double rtol, const esi_cg_state_t* resume, esi_cg_state_t* save,
                           esi_cg_report_t* rep) {
    ESI_TRY(check_shots(P, shot0, ns));
    if (!x || !work || (!resume && !d_obs && data_len(P, shot0, ns) > 0)) return fail(ESI_ERR_ARG, "null pointer");
    if (max_iter < 1) return fail(ESI_ERR_ARG, "max_iter must be >= 1");
    if (!(rtol >= 0)) return fail(ESI_ERR_ARG, "rtol must be >= 0");
    if (P->nshots < ns) return fail(ESI_ERR_ARG, "internal: scalar space");
    auto state_ok = [](const esi_cg_state_t* st) {
        return st->rr0 && st->rr && st->beta && st->iterating && st->iters && st->status && st->res_hist;
    };
    if (resume && (!state_ok(resume) || resume->k < 1 || resume->k > max_iter || resume->hist_cap < resume->k + 1))
        return fail(ESI_ERR_ARG, "resume state: null arrays, or k outside [1, max_iter], or hist_cap < k + 1");
    if (save && (!state_ok(save) || save->hist_cap < max_iter + 1))
        return fail(ESI_ERR_ARG, "save state: null arrays or hist_cap < max_iter + 1");
    CgState c;
    ESI_TRY(lists_for(P, const_cast<TileLists**>(&c.L)));
    c.shot0 = shot0; c.ns = ns; c.max_iter = max_iter; c.rtol = rtol;
    c.len = (int64_t)P->nt * P->nphys;
    c.x = x;
    c.r = work;
    c.p = work + (int64_t)ns * c.len;
    c.Ap = work + 2 * (int64_t)ns * c.len;
    c.rr = P->scal; c.pAp = P->scal + P->nshots; c.alpha = P->scal + 2 * P->nshots;
    c.beta = P->scal + 3 * P->nshots; c.rr_new = P->scal + 4 * P->nshots;
    c.rr0 = P->scal + 5 * P->nshots;
    c.active = P->flags; c.finish = P->flags + P->nshots;
    c.iters = P->cgi; c.status = P->cgi + P->nshots; c.ctl = P->cgi + 2 * P->nshots;
    const int hs = max_iter + 1;
    ESI_TRY(grow_t(&P->cg_hist, &P->cg_hist_cap, (int64_t)ns * hs, P->stream));
    c.hist = P->cg_hist;
    // the fused-residual iterations' data partials (sized here, outside any capture)
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)ns * DATA_BLOCKS, P->stream));

    std::vector<int> h_status(ns, 0);
    auto read_status = [&]() -> esi_status_t {
        ESI_HIP_TRY(hipMemcpyAsync(h_status.data(), c.status, ns * sizeof(int), hipMemcpyDeviceToHost,
                                   P->stream));
        ESI_HIP_TRY(hipStreamSynchronize(P->stream));
        for (int s = 0; s < ns; ++s)
            if (h_status[s] == ESI_ERR_NONFINITE) return fail(ESI_ERR_NONFINITE, "CG: non-finite scalar");
        for (int s = 0; s < ns; ++s)
            if (h_status[s] == ESI_ERR_BREAKDOWN) return fail(ESI_ERR_BREAKDOWN, "CG breakdown: p.Np <= 0");
        return ESI_OK;
    };
    int k0 = 0;
    if (!resume) {
        // b = S^T d (adjoint modelling, Sec. 3); r_0 = b, p_0 = r_0, x_0 = 0
        ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
        {
            StepArgs a = base_args(P, c.L, shot0, ns);
            a.inj_data = d_obs;
            a.dout = c.r;
            int cs = 0;
            ESI_TRY(adjoint_loop(P, a, F_INJ | F_OUT, P->ring, &cs, 0, P->nt));
        }
        ESI_TRY(launch_copy(P, c.p, c.r, ns * c.len));
        ESI_TRY(launch_fill(P, x, ns * c.len, 0.f));
        ESI_TRY(launch_dot(P, c.r, c.r, ns, c.len, c.rr));
        ESI_HIP_TRY(hipMemcpyAsync(c.rr0, c.rr, ns * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
        ESI_TRY(launch_cg_init(P, c.rr0, c.active, c.finish, c.iters, c.status, c.hist, hs, c.ctl, ns));
        ESI_HIP_TRY(hipMemcpyAsync(P->h_ctl, c.ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipStreamSynchronize(P->stream));
        if (read_status() == ESI_ERR_NONFINITE) return fail(ESI_ERR_NONFINITE, "non-finite right-hand side");
    } else {
        // x = x_k, work[0] = r_k, work[1] = p_{k-1} come from the caller; the
        // next iteration forms p_k = r_k + beta p_{k-1} and, with alpha = 0,
        // leaves x as it is (x_k already holds the last step)
        k0 = resume->k;
        std::vector<int> act(ns), fin(ns, 0);
        std::vector<double> hist((size_t)ns * hs, -1.0), zero(ns, 0.0);
        int cnt = 0;
        for (int s = 0; s < ns; ++s) {
            act[s] = resume->iterating[s] ? 1 : 0;
            cnt += act[s];
            for (int j = 0; j <= k0; ++j) hist[(size_t)s * hs + j] = resume->res_hist[(size_t)s * resume->hist_cap + j];
        }
        const int ctl[2] = {k0, cnt};
        ESI_HIP_TRY(hipMemcpy(c.rr0, resume->rr0, ns * sizeof(double), hipMemcpyHostToDevice));
        ESI_HIP_TRY(hipMemcpy(c.rr, resume->rr, ns * sizeof(double), hipMemcpyHostToDevice));
        ESI_HIP_TRY(hipMemcpy(c.beta, resume->beta, ns * sizeof(double), hipMemcpyHostToDevice));
        ESI_HIP_TRY(hipMemcpy(c.alpha, zero.data(), ns * sizeof(double), hipMemcpyHostToDevice));
        ESI_HIP_TRY(hipMemcpy(c.active, act.data(), ns * sizeof(int), hipMemcpyHostToDevice));
        ESI_HIP_TRY(hipMemcpy(c.finish, fin.data(), ns * sizeof(int), hipMemcpyHostToDevice));
        ESI_HIP_TRY(hipMemcpy(c.iters, resume->iters, ns * sizeof(int), hipMemcpyHostToDevice));
        ESI_HIP_TRY(hipMemcpy(c.status, resume->status, ns * sizeof(int), hipMemcpyHostToDevice));
        ESI_HIP_TRY(hipMemcpy(c.hist, hist.data(), hist.size() * sizeof(double), hipMemcpyHostToDevice));
        ESI_HIP_TRY(hipMemcpy(c.ctl, ctl, 2 * sizeof(int), hipMemcpyHostToDevice));
        P->h_ctl[0] = ctl[0];
        P->h_ctl[1] = ctl[1];
    }

    // graph replay assumes the direction buffers of a fresh solve
    const bool graph = P->cg_graph && P->cap_stream && !resume;
    if (graph && P->cg_key != cg_graph_key(P, c)) cg_graph_drop(P);
    float* p = c.p;
    float* Ap = c.Ap;
    int done_iters = k0;
    for (int k = k0; k < max_iter && P->h_ctl[1] > 0; ++k) {
        if (graph && k >= 1) {
            const int i = k & 1;
            if (!P->cg_exec[i]) {
                ESI_TRY(cg_graph_capture(P, c, k, p, Ap));
                P->cg_key = cg_graph_key(P, c);
            }
            ESI_TRY(cg_graph_launch(P, i));
        } else {
            ESI_TRY(cg_iteration(P, c, k, p, Ap));
        }
        if (k >= 1) std::swap(p, Ap);
        ESI_HIP_TRY(hipMemcpyAsync(P->h_ctl, c.ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipStreamSynchronize(P->stream));
        done_iters = k + 1;
    }
    esi_status_t status = read_status();
    if (save) {
        // p_{k-1} into work[1] (the direction buffers alternate)
        if (p != c.p) ESI_TRY(launch_copy(P, c.p, p, ns * c.len));
        std::vector<double> hist((size_t)ns * hs);
        ESI_HIP_TRY(hipMemcpyAsync(save->rr0, c.rr0, ns * sizeof(double), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipMemcpyAsync(save->rr, c.rr, ns * sizeof(double), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipMemcpyAsync(save->beta, c.beta, ns * sizeof(double), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipMemcpyAsync(save->iters, c.iters, ns * sizeof(int), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipMemcpyAsync(save->status, c.status, ns * sizeof(int), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipMemcpyAsync(hist.data(), c.hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost,
                                   P->stream));
        ESI_HIP_TRY(hipStreamSynchronize(P->stream));
        save->k = done_iters;
        for (int s = 0; s < ns; ++s) {
            for (int j = 0; j < hs; ++j) save->res_hist[(size_t)s * save->hist_cap + j] = hist[(size_t)s * hs + j];
            // still iterating: stopped by the iteration limit alone
            const double rel = hist[(size_t)s * hs + done_iters];
            save->iterating[s] = save->status[s] == ESI_OK && save->rr0[s] > 0.0 && save->iters[s] == done_iters &&
                                 !(rel < rtol);
        }
    }
    if (rep) {
        rep->iters = done_iters;
        if (rep->shot_iters)
            ESI_HIP_TRY(hipMemcpyAsync(rep->shot_iters, c.iters, ns * sizeof(int),
                                       hipMemcpyDeviceToHost, P->stream));
        if (rep->res_hist)
            ESI_HIP_TRY(hipMemcpyAsync(rep->res_hist, c.hist, (size_t)ns * hs * sizeof(double),
                                       hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipStreamSynchronize(P->stream));
    }
    return status;
}

}  // namespace
}  // namespace esi

extern "C" esi_status_t esi_cg_solve(esi_plan_t plan, int32_t shot0, int32_t ns,
                                     const float* d_obs, float* x, float* work, int32_t max_iter,
                                     double rtol, esi_cg_report_t* rep) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    return cg_solve_impl((Plan*)plan, shot0, ns, d_obs, x, work, max_iter, rtol, nullptr, nullptr, rep);
}

extern "C" esi_status_t esi_cg_solve_state(esi_plan_t plan, int32_t shot0, int32_t ns, const float* d_obs,
                                           float* x, float* work, int32_t max_iter, double rtol,
                                           const esi_cg_state_t* resume, esi_cg_state_t* save,
                                           esi_cg_report_t* rep) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    return cg_solve_impl((Plan*)plan, shot0, ns, d_obs, x, work, max_iter, rtol, resume, save, rep);
}

extern "C" esi_status_t esi_fpcg_solve(esi_plan_t plan, int32_t shot0, int32_t ns,
                                       const float* d_obs, float* x, float* work, int32_t max_iter,
                                       double rtol, esi_unet_t net, int32_t net_every, const float* scale,
                                       esi_cg_report_t* rep) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    if (P->ndim != 2) return fail(ESI_ERR_ARG, "flexible CG runs on 2D plans");
    if (P->w_identity) return fail(ESI_ERR_ARG, "flexible CG scales model the annihilator weight, not B = I");
    if (!x || !work || (!d_obs && data_len(P, shot0, ns) > 0)) return fail(ESI_ERR_ARG, "null pointer");
    if (max_iter < 1) return fail(ESI_ERR_ARG, "max_iter must be >= 1");
    if (!(rtol >= 0)) return fail(ESI_ERR_ARG, "rtol must be >= 0");
    if (net_every < 0) return fail(ESI_ERR_ARG, "net_every must be >= 0");
    const int Hp = (P->nz + 7) / 8 * 8, Wp = (P->nx + 7) / 8 * 8;
    if (net) {
        int H, W, mb;
        ESI_TRY(unet_dims(net, &H, &W, &mb));
        if (H != Hp || W != Wp || mb < ns)
            return fail(ESI_ERR_SHAPE, "network must take " + std::to_string(Hp) + " x " + std::to_string(Wp) +
                                           " images and batches of " + std::to_string(ns) + " shots");
    }
    const bool stats = rep && rep->stat_out;
    if (stats && !rep->stat_xref) return fail(ESI_ERR_ARG, "stat_out needs stat_xref");
    CgState c;
    ESI_TRY(lists_for(P, const_cast<TileLists**>(&c.L)));
    c.shot0 = shot0; c.ns = ns; c.max_iter = max_iter; c.rtol = rtol;
    c.len = (int64_t)P->nt * P->nphys;
    c.x = x;
    c.r = work;
    c.p = work + (int64_t)ns * c.len;
    c.Ap = work + 2 * (int64_t)ns * c.len;
    c.rr = P->scal; c.pAp = P->scal + P->nshots; c.alpha = P->scal + 2 * P->nshots;
    c.beta = P->scal + 3 * P->nshots; c.rr_new = P->scal + 4 * P->nshots;
    c.rr0 = P->scal + 5 * P->nshots;
    c.active = P->flags; c.finish = P->flags + P->nshots;
    c.iters = P->cgi; c.status = P->cgi + P->nshots; c.ctl = P->cgi + 2 * P->nshots;
    ESI_TRY(grow_t(&P->cg_hist, &P->cg_hist_cap, (int64_t)ns * (max_iter + 1), P->stream));
    c.hist = P->cg_hist;
    const int64_t cells = (int64_t)ns * P->nphys;
    ESI_TRY(grow_t(&P->fcg_s, &P->fcg_s_cap, cells, P->stream));
    ESI_TRY(grow_t(&P->fcg_a, &P->fcg_a_cap, cells, P->stream));
    ESI_TRY(grow_t(&P->fcg_g, &P->fcg_g_cap, cells, P->stream));
    ESI_TRY(grow_t(&P->fcg_d, &P->fcg_d_cap, (int64_t)7 * ns, P->stream));
    ESI_TRY(grow_t(&P->fcg_i, &P->fcg_i_cap, (int64_t)5 * ns, P->stream));
    if (net) {
        ESI_TRY(grow_t(&P->fcg_in, &P->fcg_in_cap, (int64_t)ns * 3 * Hp * Wp, P->stream));
        ESI_TRY(grow_t(&P->fcg_o, &P->fcg_o_cap, (int64_t)ns * Hp * Wp, P->stream));
    }
    float* S = P->fcg_s;
    float* en = P->fcg_a;
    double* pr = P->fcg_d;
    double* zAp = P->fcg_d + ns;
    double* zr = P->fcg_d + 2 * ns;          // [ns][3]
    double* fmean = P->fcg_d + 5 * ns;
    double* best = P->fcg_d + 6 * ns;
    int* mode = P->fcg_i;
    int* restart = P->fcg_i + ns;
    int* fallback = P->fcg_i + 2 * ns;
    int* kbest = P->fcg_i + 3 * ns;
    int* cg_at = P->fcg_i + 4 * ns;
    const float* o = net ? P->fcg_o : nullptr;
    const double stall = 0.99;
    const int window = 20;

    double* rnp = P->fcg_g;                  // sum_t r Np per cell (FP64)

    // z = M(r) for the shots still iterating, k = the iteration count so far;
    // `en` holds sum_t r^2 per cell of the current r
    auto precondition = [&](int k) -> esi_status_t {
        if (net && (k == 0 || (net_every > 0 && k % net_every == 0))) {
            ESI_TRY(launch_features(P, shot0, ns, en, nullptr, fmean, Hp, Wp, nullptr, P->fcg_in, nullptr,
                                    nullptr));
            ESI_TRY(unet_forward_on(net, P->stream, P->fcg_in, P->fcg_o, ns));
        }
        return launch_fcg_zr_check_scale(P, o, scale, en, c.active, mode, restart, fallback, cg_at, best, kbest,
                                         c.hist, max_iter + 1, k, Hp, Wp, zr, S, ns);
    };

    // b = S^T d; r_0 = b, x_0 = 0
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    {
        StepArgs a = base_args(P, c.L, shot0, ns);
        a.inj_data = d_obs;
        a.dout = c.r;
        int cs = 0;
        ESI_TRY(adjoint_loop(P, a, F_INJ | F_OUT, P->ring, &cs, 0, P->nt));
    }
    ESI_TRY(launch_fill(P, x, ns * c.len, 0.f));
    ESI_TRY(launch_dot(P, c.r, c.r, ns, c.len, c.rr));
    ESI_HIP_TRY(hipMemcpyAsync(c.rr0, c.rr, ns * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
    ESI_TRY(launch_cg_init(P, c.rr0, c.active, c.finish, c.iters, c.status, c.hist, max_iter + 1, c.ctl, ns));
    ESI_TRY(launch_fcg_init(P, mode, restart, fallback, cg_at, best, kbest, ns));
    if (stats) ESI_TRY(launch_stats(P, c.r, x, nullptr, nullptr, rep->stat_xref, c.iters, 0, rep->stat_out, ns));
    ESI_HIP_TRY(hipMemcpyAsync(P->h_ctl, c.ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
    ESI_HIP_TRY(hipStreamSynchronize(P->stream));
    std::vector<int> h_status(ns, 0);
    ESI_HIP_TRY(hipMemcpy(h_status.data(), c.status, ns * sizeof(int), hipMemcpyDeviceToHost));
    for (int s = 0; s < ns; ++s)
        if (h_status[s] == ESI_ERR_NONFINITE) return fail(ESI_ERR_NONFINITE, "non-finite right-hand side");

    // p_0 = z_0 = M(r_0)
    ESI_TRY(launch_energy(P, c.r, c.active, en, ns));
    ESI_TRY(precondition(0));
    ESI_TRY(launch_scale_vec(P, c.p, c.r, S, ns));
    float* p = c.p;
    float* Ap = c.Ap;
    int done_iters = 0;
    const int64_t stat_stride = (int64_t)ns * 2 * P->nphys;
    for (int k = 0; k < max_iter && P->h_ctl[1] > 0; ++k) {
        // N p_k; from k = 1 on the forward pass forms p_k = S r_k + beta p_{k-1}
        // and x_k = x_{k-1} + alpha p_{k-1} (into the old N p buffer)
        float* dir = p;
        float* Apk = Ap;
        if (k == 0) {
            ESI_TRY(do_normal(P, shot0, ns, p, Ap, c.L, c.active, false, nullptr, c.r, x, c.alpha, c.beta));
        } else {
            ESI_TRY(do_normal(P, shot0, ns, p, p, c.L, c.active, true, Ap, c.r, x, c.alpha, c.beta, S, pr));
            dir = Ap;
            Apk = p;
        }
        ESI_TRY(launch_reduce_parts(P, P->part, P->part_stride, ns, c.pAp));
        if (k == 0) ESI_TRY(launch_dot(P, dir, c.r, ns, c.len, pr));
        ESI_TRY(launch_cg_alpha(P, pr, c.pAp, c.alpha, ns));          // alpha = p.r / p.Np
        // r -= alpha Np, with sum_t r^2 (network input, z.r) and sum_t r Np (z.Np) per cell
        ESI_TRY(launch_r_update_cells(P, c.r, Apk, c.alpha, c.active, ns, en, rnp, c.rr_new));
        ESI_TRY(launch_fcg_control(P, c.rr0, c.rr_new, c.pAp, c.active, c.finish, c.iters, c.status, c.hist,
                                   max_iter + 1, c.ctl, rtol, max_iter, mode, restart, fallback, cg_at, stall,
                                   window, best, kbest, net != nullptr, ns));
        if (stats)
            ESI_TRY(launch_stats(P, c.r, x, dir, c.alpha, rep->stat_xref, c.iters, k + 1,
                                 rep->stat_out + (k + 1) * stat_stride, ns));
        ESI_TRY(launch_axpy_flag(P, x, dir, c.alpha, c.finish, 1, ns, c.len));
        ESI_HIP_TRY(hipMemcpyAsync(P->h_ctl, c.ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipStreamSynchronize(P->stream));
        done_iters = k + 1;
        if (k >= 1) std::swap(p, Ap);
        if (P->h_ctl[1] == 0 || k == max_iter - 1) break;
        // z_{k+1} = M(r_{k+1}); beta = -z.Np / p.Np (0 when the direction restarts)
        ESI_TRY(precondition(k + 1));
        ESI_TRY(launch_dot_cells(P, S, rnp, ns, zAp));                // z.Np = sum_x s(x) sum_t r Np
        ESI_TRY(launch_fcg_beta(P, zAp, c.pAp, restart, c.beta, ns));
    }
    std::vector<int> h_fb(ns, -1), h_cg(ns, -1);
    ESI_HIP_TRY(hipMemcpyAsync(h_status.data(), c.status, ns * sizeof(int), hipMemcpyDeviceToHost, P->stream));
    ESI_HIP_TRY(hipMemcpyAsync(h_fb.data(), fallback, ns * sizeof(int), hipMemcpyDeviceToHost, P->stream));
    ESI_HIP_TRY(hipMemcpyAsync(h_cg.data(), cg_at, ns * sizeof(int), hipMemcpyDeviceToHost, P->stream));
    if (rep) {
        rep->iters = done_iters;
        if (rep->shot_iters)
            ESI_HIP_TRY(hipMemcpyAsync(rep->shot_iters, c.iters, ns * sizeof(int), hipMemcpyDeviceToHost, P->stream));
        if (rep->res_hist)
            ESI_HIP_TRY(hipMemcpyAsync(rep->res_hist, c.hist, (size_t)ns * (max_iter + 1) * sizeof(double),
                                       hipMemcpyDeviceToHost, P->stream));
    }
    ESI_HIP_TRY(hipStreamSynchronize(P->stream));
    if (rep && rep->shot_fallback)
        for (int s = 0; s < ns; ++s) rep->shot_fallback[s] = h_fb[s];
    if (rep && rep->shot_cg)
        for (int s = 0; s < ns; ++s) rep->shot_cg[s] = h_cg[s];
    for (int s = 0; s < ns; ++s)
        if (h_status[s] == ESI_ERR_NONFINITE) return fail(ESI_ERR_NONFINITE, "flexible CG: non-finite scalar");
    for (int s = 0; s < ns; ++s)
        if (h_status[s] == ESI_ERR_BREAKDOWN) return fail(ESI_ERR_BREAKDOWN, "flexible CG breakdown: p.Np <= 0");
    return ESI_OK;
}

extern "C" esi_status_t esi_precond_features(esi_plan_t plan, int32_t shot0, int32_t ns, const float* a,
                                             const float* cmap, const float* base, int32_t Hp, int32_t Wp,
                                             float* xin, float* apad, float* cpad) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    if (P->ndim != 2) return fail(ESI_ERR_ARG, "network features are 2D");
    if (!a || !xin) return fail(ESI_ERR_ARG, "null pointer");
    if (Hp < P->nz || Wp < P->nx || Hp % 8 || Wp % 8) return fail(ESI_ERR_SHAPE, "Hp, Wp: multiples of 8 covering the grid");
    ESI_TRY(grow_t(&P->fcg_d, &P->fcg_d_cap, (int64_t)7 * std::max(ns, P->nshots), P->stream));
    return launch_features(P, shot0, ns, a, cmap, P->fcg_d + 5 * ns, Hp, Wp, base, xin, apad, cpad);
}

namespace esi {
namespace {

// The gradients of esi_gradient; bg (nullable, [nshots][nt]) adds the physical
// point source f to the forward pass of the PENALTY and ADJOINT modes, so that
// u = A^{-1}(f + q) (WRI).
esi_status_t gradient_impl(Plan* P, int32_t shot0, int32_t ns, int32_t mode, int32_t src_kind,
                           const float* src, const float* bg, const float* data, float* grad_m,
                           float* grad_src, int32_t K) {
    if (mode != ESI_GRAD_PENALTY && mode != ESI_GRAD_ADJOINT && mode != ESI_GRAD_SEED &&
        mode != ESI_GRAD_SEED_REUSE)
        return fail(ESI_ERR_ARG, "bad gradient mode");
    const bool reuse = mode == ESI_GRAD_SEED_REUSE;
    if (reuse && !(P->ck_valid && P->ck_shot0 == shot0 && P->ck_nshots == ns &&
                   P->ck_kind == src_kind && P->ck_src == src && P->ck_K == K))
        return fail(ESI_ERR_ARG, "no checkpoints from esi_forward_ckpt for these shots, source and K");
    if (reuse) mode = ESI_GRAD_SEED;
    if (src_kind != ESI_SRC_POINT && src_kind != ESI_SRC_DENSE) return fail(ESI_ERR_ARG, "bad src_kind");
    if (mode != ESI_GRAD_SEED && src_kind != ESI_SRC_DENSE)
        return fail(ESI_ERR_ARG, "PENALTY and ADJOINT modes take a dense extended source");
    if (!src || !grad_m) return fail(ESI_ERR_ARG, "null pointer");
    if (mode != ESI_GRAD_PENALTY && !data && data_len(P, shot0, ns) > 0) return fail(ESI_ERR_ARG, "null data");
    if (K < 0) return fail(ESI_ERR_ARG, "ckpt_every must be >= 0");
    if (bg && mode != ESI_GRAD_PENALTY && mode != ESI_GRAD_ADJOINT)
        return fail(ESI_ERR_ARG, "internal: a physical source applies to PENALTY and ADJOINT");
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    const int64_t nph = P->nphys;
    ESI_TRY(grow_t(&P->gshot, &P->gshot_cap, (int64_t)ns * nph, P->stream));
    ESI_TRY(launch_fill(P, P->gshot, (int64_t)ns * nph, 0.f));
    const unsigned srcfl = (src_kind == ESI_SRC_POINT ? F_SRC_POINT : F_SRC_DENSE) | (bg ? F_SRC_POINT : 0u);

    if (mode == ESI_GRAD_PENALTY) {
        // one forward pass of q (plus f) correlating beta B^2 q with (dA/dm) u (Algorithm 2)
        ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
        StepArgs a = base_args(P, L, shot0, ns);
        a.dsrc = src;
        a.wavelet = bg;
        a.gacc = P->gshot;
        int cs = 0;
        ESI_TRY(forward_loop(P, a, srcfl | F_PENALTY, P->ring, &cs, 0, P->nt));
        return launch_sum_shots(P, P->gshot, ns, nph, 1.f, grad_m);
    }

    // ADJOINT and SEED: adjoint field of G (G = S q - d_obs for ADJOINT, G = data for SEED),
    // correlated with the stored or recomputed (dA/dm) u.
    const int nt = P->nt;
    const int64_t dl = data_len(P, shot0, ns);
    const bool ckpt = reuse || (K > 0 && K < nt);
    P->ck_valid = false;
    const int Kc = ckpt ? K : 0;
    const int nseg = ckpt ? (nt + K - 1) / K : 1;
    const int slots = ckpt ? K : nt;
    ESI_TRY(grow_t(&P->store, &P->store_cap, (int64_t)ns * slots * nph, P->stream));
    if (ckpt) ESI_TRY(grow_t(&P->ckpt, &P->ckpt_cap, (int64_t)ns * nseg * 2 * P->fsize, P->stream));
    ESI_TRY(grow_t(&P->dscr, &P->dscr_cap, std::max<int64_t>(dl, 1), P->stream));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs a = base_args(P, L, shot0, ns);
    if (src_kind == ESI_SRC_POINT) a.wavelet = src; else a.dsrc = src;
    if (bg) a.wavelet = bg;
    a.store = P->store;
    a.store_stride = (int64_t)slots * nph;
    const float* G = data;
    int fcs = 0;
    if (mode == ESI_GRAD_ADJOINT) {
        a.gat_data = P->dscr;
        ESI_TRY(forward_loop(P, a, srcfl | F_GATHER | (ckpt ? 0u : F_STORE), P->ring, &fcs, 0, nt,
                             ckpt ? P->ckpt : nullptr, Kc, nseg));
        ESI_TRY(launch_final_gather(P, P->ring + (int64_t)fcs * P->fsize, RING * P->fsize, P->dscr,
                                    shot0, ns));
        ESI_TRY(launch_sub(P, P->dscr, P->dscr, data, dl));   // G = S q - d_obs
        G = P->dscr;
    } else if (!reuse) {
        ESI_TRY(forward_loop(P, a, srcfl | (ckpt ? 0u : F_STORE), P->ring, &fcs, 0, nt,
                             ckpt ? P->ckpt : nullptr, Kc, nseg));
    }
    // backward sweep
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    if (ckpt) ESI_TRY(ring_for(P, &P->ring2, &P->ring2_cap, ns));
    float* adj_ring = P->ring;
    StepArgs b = base_args(P, L, shot0, ns);
    b.inj_data = G;
    b.gacc = P->gshot;
    b.store = P->store;
    b.store_stride = (int64_t)slots * nph;
    unsigned bfl = F_INJ | F_CORR;
    if (mode == ESI_GRAD_SEED && grad_src) {
        if (src_kind == ESI_SRC_DENSE) { bfl |= F_OUT; b.dout = grad_src; }
        else { bfl |= F_SRC_REC; b.src_rec = grad_src; }
    }
    int acs = 0;
    if (!ckpt) {
        ESI_TRY(adjoint_loop(P, b, bfl, adj_ring, &acs, 0, nt));
    } else {
        for (int k = nseg - 1; k >= 0; --k) {
            const int n0 = k * K, n1 = std::min(nt, n0 + K);
            // restore (u^{n0}, d^{n0}) into slot 0 of the recompute ring
            const int64_t cstr = (int64_t)nseg * 2 * P->fsize;
            ESI_TRY(launch_copy_fields(P, P->ring2, RING * P->fsize,
                                       P->ckpt + (int64_t)k * 2 * P->fsize, cstr, shot0, ns));
            ESI_TRY(launch_copy_fields(P, P->ring2 + 2 * P->fsize, RING * P->fsize,
                                       P->ckpt + (int64_t)k * 2 * P->fsize + P->fsize, cstr, shot0, ns));
            int rcs = 0;
            ESI_TRY(forward_loop(P, a, srcfl | F_STORE, P->ring2, &rcs, n0, n1, nullptr, K, nseg));
            ESI_TRY(adjoint_loop(P, b, bfl, adj_ring, &acs, n0, n1, K));
        }
    }
    // ADJOINT: lambda = S^T (d_obs - S q) = -S^T G; SEED: grad_m = -sum S^T G (dA/dm) u
    return launch_sum_shots(P, P->gshot, ns, nph, -1.f, grad_m);
}

}  // namespace

// One forward pass of q (plus the point wavelets bg, when given) that adds each
// shot's PENALTY gradient (lambda = beta W q) to gshot [ns][phys], records
// S q (or S(f + q)) into dsyn and writes the per-shot penalty sum of
// beta W q^2 to pen (device, FP64 [ns]).
esi_status_t penalty_eval(Plan* P, int shot0, int ns, const float* q, const float* bg, float* gshot,
                          float* dsyn, double* pen) {
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    const unsigned pfl = F_SRC_DENSE | F_PENALTY | F_GATHER | (bg ? F_SRC_POINT : 0u);
    ESI_TRY(loop_lists(P, pfl, F_INJ));
    P->part_stride = max_tiles(P);
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)ns * P->part_stride, P->stream));
    ESI_TRY(launch_fill_d(P, P->part, (int64_t)ns * P->part_stride));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs a = base_args(P, L, shot0, ns);
    a.dsrc = q;
    a.wavelet = bg;
    a.gacc = gshot;
    a.gat_data = dsyn;
    a.part = P->part;
    a.part_stride = P->part_stride;
    int cs = 0;
    ESI_TRY(forward_loop(P, a, pfl, P->ring, &cs, 0, P->nt));
    ESI_TRY(launch_final_gather(P, P->ring + (int64_t)cs * P->fsize, RING * P->fsize, dsyn, shot0, ns));
    return launch_reduce_parts(P, P->part, P->part_stride, ns, pen);
}

}  // namespace esi

extern "C" esi_status_t esi_gradient(esi_plan_t plan, int32_t shot0, int32_t ns, int32_t mode,
                                     int32_t src_kind, const float* src, const float* data,
                                     float* grad_m, float* grad_src, int32_t K) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    return gradient_impl(P, shot0, ns, mode, src_kind, src, nullptr, data, grad_m, grad_src, K);
}

extern "C" esi_status_t esi_plan_set_beta(esi_plan_t plan, double beta) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    if (!std::isfinite(beta)) return fail(ESI_ERR_ARG, "beta must be finite");
    ((Plan*)plan)->beta = beta;
    return ESI_OK;
}

extern "C" esi_status_t esi_wri_gradient(esi_plan_t plan, int32_t shot0, int32_t ns, int32_t mode,
                                         const float* wavelet, const float* q, const float* d_obs,
                                         float* grad_m, int32_t ckpt_every) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    if (mode != ESI_GRAD_PENALTY && mode != ESI_GRAD_ADJOINT)
        return fail(ESI_ERR_ARG, "WRI gradient modes are PENALTY and ADJOINT");
    if (!wavelet) return fail(ESI_ERR_ARG, "null wavelet");
    return gradient_impl(P, shot0, ns, mode, ESI_SRC_DENSE, q, wavelet, d_obs, grad_m, nullptr, ckpt_every);
}

extern "C" esi_status_t esi_data_residual(esi_plan_t plan, int32_t shot0, int32_t ns, const float* wavelet,
                                          const float* d_obs, float* d_res) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    const int64_t dl = data_len(P, shot0, ns);
    if (!wavelet || (dl > 0 && (!d_obs || !d_res))) return fail(ESI_ERR_ARG, "null pointer");
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    if (dl == 0) return ESI_OK;
    // S f into plan scratch, so that d_res may alias d_obs
    ESI_TRY(grow_t(&P->dscr2, &P->dscr2_cap, dl, P->stream));
    ESI_TRY(do_forward(P, shot0, ns, ESI_SRC_POINT, wavelet, P->dscr2, L));
    return launch_sub(P, d_res, d_obs, P->dscr2, dl);                         // d - S f
}

extern "C" esi_status_t esi_plan_set_weight(esi_plan_t plan, int32_t kind) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    if (kind != ESI_WEIGHT_ANNIHILATOR && kind != ESI_WEIGHT_IDENTITY) return fail(ESI_ERR_ARG, "bad weight kind");
    Plan* P = (Plan*)plan;
    P->w_identity = kind == ESI_WEIGHT_IDENTITY;
    return ESI_OK;
}

extern "C" esi_status_t esi_plan_profile(esi_plan_t plan, int32_t enable) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_HIP_TRY(hipStreamSynchronize(P->stream));
    for (auto& r : P->prof_pending) { hipEventDestroy(r.e0); hipEventDestroy(r.e1); }
    P->prof_pending.clear();
    if (enable) P->prof_tot.clear();
    P->prof_on = enable != 0;
    return ESI_OK;
}

namespace {
esi_status_t fold_profile(Plan* P);
}

extern "C" esi_status_t esi_plan_profile_read(esi_plan_t plan, int32_t cap, int32_t* count,
                                              uint32_t* flags, int64_t* launches,
                                              int64_t* shot_launches, double* ms) {
    set_error("");
    if (!plan || !count) return fail(ESI_ERR_ARG, "null argument");
    if (cap > 0 && (!flags || !launches || !shot_launches || !ms)) return fail(ESI_ERR_ARG, "null output array");
    Plan* P = (Plan*)plan;
    ESI_TRY(fold_profile(P));
    *count = (int32_t)P->prof_tot.size();
    for (int i = 0; i < cap && i < (int)P->prof_tot.size(); ++i) {
        flags[i] = P->prof_tot[i].flags;
        launches[i] = P->prof_tot[i].launches;
        shot_launches[i] = P->prof_tot[i].shot_launches;
        ms[i] = P->prof_tot[i].ms;
    }
    return ESI_OK;
}

extern "C" esi_status_t esi_plan_set_time_block(esi_plan_t plan, int32_t steps) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    if (steps != 1 && steps != 2) return fail(ESI_ERR_ARG, "time block must be 1 or 2");
    ((Plan*)plan)->tb_fwd = ((Plan*)plan)->tb_adj = steps == 1 ? LS_ONE : LS_T2_32;
    return ESI_OK;
}

namespace {

// Fold the pending event pairs of the plan's profile into its totals.
esi_status_t fold_profile(Plan* P) {
    for (auto& r : P->prof_pending) {
        ESI_HIP_TRY(hipEventSynchronize(r.e1));
        float t = 0.f;
        ESI_HIP_TRY(hipEventElapsedTime(&t, r.e0, r.e1));
        bool found = false;
        for (auto& q : P->prof_tot)
            if (q.flags == r.flags) { q.launches += r.launches; q.shot_launches += r.shot_launches; q.ms += t; found = true; }
        if (!found) P->prof_tot.push_back({r.flags, r.launches, r.shot_launches, (double)t});
        hipEventDestroy(r.e0);
        hipEventDestroy(r.e1);
    }
    P->prof_pending.clear();
    return ESI_OK;
}

// Process-wide cache of tuned choices, keyed by the grid, the shots (count,
// apertures), nt and the kind of timing run.
struct TuneEntry { std::vector<int64_t> key; int fwd, adj; std::vector<Plan::TuneRow> rows; };
std::vector<TuneEntry> g_tune_cache;

// FNV-1a over the apertures of shots [shot0, shot0 + ns) (0 without apertures)
int64_t window_hash(Plan* P, int shot0, int ns) {
    if (P->h_win.empty()) return 0;
    uint64_t h = 1469598103934665603ull;
    for (int i = 2 * shot0; i < 2 * (shot0 + ns); ++i) {
        h ^= (uint64_t)(uint32_t)P->h_win[i];
        h *= 1099511628211ull;
    }
    return (int64_t)(h >> 1);
}

// One timing run of the forward-type and adjoint-type loops of candidate
// `shape`: the normal operator on p (probe = false), or a point-source forward
// pass of nprobe steps and a gradient's adjoint pass, injecting its data and
// correlating with a two-slot store (probe = true).
esi_status_t tune_run(Plan* P, int shot0, int ns, const float* p, float* Ap, bool probe, int nprobe,
                      const TileLists* L) {
    if (!probe) return do_normal(P, shot0, ns, p, Ap, L, nullptr, false, nullptr, nullptr, nullptr, nullptr, nullptr);
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs a = base_args(P, L, shot0, ns);
    a.wavelet = P->dscr2;                  // zeros
    a.gat_data = P->dscr;
    int cs = 0;
    ESI_TRY(forward_loop(P, a, F_SRC_POINT | F_GATHER, P->ring, &cs, 0, nprobe));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs b = base_args(P, L, shot0, ns);
    b.inj_data = P->dscr;
    b.store = P->store;
    b.store_stride = 2 * P->nphys;
    b.gacc = P->gshot;
    cs = 0;
    return adjoint_loop(P, b, F_INJ | F_CORR, P->ring, &cs, P->nt - nprobe, P->nt, 2);
}

}  // namespace

extern "C" esi_status_t esi_plan_autotune(esi_plan_t plan, int32_t shot0, int32_t ns, const float* p,
                                          float* Ap, int32_t force, int32_t* choice) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    if (!p != !Ap) return fail(ESI_ERR_ARG, "p and Ap: both device vectors, or both NULL");
    const bool probe = !p;
    if (!probe) {
        const int64_t n = (int64_t)ns * P->nt * P->nphys;
        if ((Ap < p + n) && (p < Ap + n)) return fail(ESI_ERR_ARG, "p and Ap overlap");
    }
    P->tune_rows.clear();
    const int nprobe = std::min(P->nt, 64);
    const std::vector<int64_t> key = {P->ndim, P->nzp, P->nyp, P->nxp, ns, P->nt, probe ? 1 : 0,
                                      window_hash(P, shot0, ns)};
    if (!force)
        for (const TuneEntry& e : g_tune_cache)
            if (e.key == key) {
                P->tb_fwd = e.fwd;
                P->tb_adj = e.adj;
                P->tune_rows = e.rows;
                if (choice) { choice[0] = e.fwd; choice[1] = e.adj; }
                return ESI_OK;
            }
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    if (probe) {
        ESI_TRY(grow_t(&P->dscr, &P->dscr_cap, std::max<int64_t>(data_len(P, shot0, ns), 1), P->stream));
        ESI_TRY(grow_t(&P->dscr2, &P->dscr2_cap, (int64_t)ns * P->nt, P->stream));
        ESI_TRY(launch_fill(P, P->dscr2, (int64_t)ns * P->nt, 0.f));
        ESI_TRY(launch_fill(P, P->dscr, std::max<int64_t>(data_len(P, shot0, ns), 1), 0.f));
        // the correlation's two-slot store and per-shot images (gradient scratch)
        ESI_TRY(grow_t(&P->store, &P->store_cap, (int64_t)ns * 2 * P->nphys, P->stream));
        ESI_TRY(grow_t(&P->gshot, &P->gshot_cap, (int64_t)ns * P->nphys, P->stream));
        ESI_TRY(launch_fill(P, P->store, (int64_t)ns * 2 * P->nphys, 0.f));
        ESI_TRY(launch_fill(P, P->gshot, (int64_t)ns * P->nphys, 0.f));
    }
    // keep the caller's profile aside and time each candidate on its own
    const bool prof = P->prof_on;
    std::vector<Plan::ProfRec> pend;
    std::vector<Plan::ProfTot> tot;
    pend.swap(P->prof_pending);
    tot.swap(P->prof_tot);
    const int tf0 = P->tb_fwd, ta0 = P->tb_adj;
    double best_f = 1e300, best_a = 1e300;
    int sf = LS_T2_32, sa = LS_T2_32;
    esi_status_t st = ESI_OK;
    std::vector<Plan::TuneRow> rows;
    const std::vector<int> cands = P->ndim == 2 ? std::vector<int>{LS_ONE, LS_T2_24, LS_T2_32, LS_T2_40}
                                                : std::vector<int>{LS_ONE, LS_T2_32};
    for (int shape : cands) {
        P->tb_fwd = P->tb_adj = shape;
        P->prof_on = false;   // first run builds the tile lists of this shape and warms up
        st = tune_run(P, shot0, ns, p, Ap, probe, nprobe, L);
        if (st != ESI_OK) break;
        P->prof_on = true;
        st = tune_run(P, shot0, ns, p, Ap, probe, nprobe, L);
        if (st != ESI_OK) break;
        P->prof_on = false;
        st = fold_profile(P);
        if (st != ESI_OK) break;
        double f = 0.0, a = 0.0;
        for (const auto& q : P->prof_tot) (q.flags & F_INJ ? a : f) += q.ms;
        P->prof_tot.clear();
        rows.push_back({shape, f, a});
        if (f < best_f) { best_f = f; sf = shape; }
        if (a < best_a) { best_a = a; sa = shape; }
    }
    P->prof_on = prof;
    P->prof_pending.swap(pend);
    P->prof_tot.swap(tot);
    if (st != ESI_OK) {
        P->tb_fwd = tf0;
        P->tb_adj = ta0;
        return st;
    }
    P->tb_fwd = sf;
    P->tb_adj = sa;
    P->tune_rows = rows;
    g_tune_cache.push_back({key, sf, sa, rows});
    if (choice) { choice[0] = sf; choice[1] = sa; }
    return ESI_OK;
}

extern "C" esi_status_t esi_plan_tune_table(esi_plan_t plan, int32_t cap, int32_t* count, int32_t* shape,
                                            double* fwd_ms, double* adj_ms) {
    set_error("");
    if (!plan || !count) return fail(ESI_ERR_ARG, "null argument");
    if (cap > 0 && (!shape || !fwd_ms || !adj_ms)) return fail(ESI_ERR_ARG, "null output array");
    Plan* P = (Plan*)plan;
    *count = (int32_t)P->tune_rows.size();
    for (int i = 0; i < cap && i < (int)P->tune_rows.size(); ++i) {
        shape[i] = P->tune_rows[i].shape;
        fwd_ms[i] = P->tune_rows[i].fwd_ms;
        adj_ms[i] = P->tune_rows[i].adj_ms;
    }
    return ESI_OK;
}

extern "C" esi_status_t esi_plan_set_launch_shape(esi_plan_t plan, int32_t forward, int32_t adjoint) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    if (forward < LS_ONE || forward > LS_COUNT || adjoint < LS_ONE || adjoint > LS_COUNT)
        return fail(ESI_ERR_ARG, "launch shapes are 1 .. 4");
    if (P->ndim != 2 && (forward > LS_T2_32 || adjoint > LS_T2_32))
        return fail(ESI_ERR_ARG, "3D plans run shape 1 (one step per launch) or 2 (two steps)");
    P->tb_fwd = forward;
    P->tb_adj = adjoint;
    return ESI_OK;
}

extern "C" esi_status_t esi_forward_ckpt(esi_plan_t plan, int32_t shot0, int32_t nshots,
                                         int32_t src_kind, const float* src, float* data,
                                         int32_t K) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, nshots));
    if (src_kind != ESI_SRC_POINT && src_kind != ESI_SRC_DENSE) return fail(ESI_ERR_ARG, "bad src_kind");
    if (!src) return fail(ESI_ERR_ARG, "null src");
    if (!data && data_len(P, shot0, nshots) > 0) return fail(ESI_ERR_ARG, "null data");
    if (K < 1) return fail(ESI_ERR_ARG, "ckpt_every must be >= 1");
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    P->ck_valid = false;
    const int nseg = (P->nt + K - 1) / K;
    ESI_TRY(grow_t(&P->ckpt, &P->ckpt_cap, (int64_t)nshots * nseg * 2 * P->fsize, P->stream));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, nshots));
    StepArgs a = base_args(P, L, shot0, nshots);
    unsigned fl = F_GATHER;
    if (src_kind == ESI_SRC_POINT) { fl |= F_SRC_POINT; a.wavelet = src; }
    else { fl |= F_SRC_DENSE; a.dsrc = src; }
    a.gat_data = data;
    int cs = 0;
    ESI_TRY(forward_loop(P, a, fl, P->ring, &cs, 0, P->nt, P->ckpt, K, nseg));
    ESI_TRY(launch_final_gather(P, P->ring + (int64_t)cs * P->fsize, RING * P->fsize, data, shot0,
                                nshots));
    P->ck_valid = true;
    P->ck_shot0 = shot0; P->ck_nshots = nshots; P->ck_kind = src_kind; P->ck_src = src; P->ck_K = K;
    return ESI_OK;
}

extern "C" esi_status_t esi_grad_velocity(esi_plan_t plan, const float* vel, const float* grad_m,
                                          float* grad_v) {
    set_error("");
    if (!plan || !vel || !grad_m || !grad_v) return fail(ESI_ERR_ARG, "null argument");
    Plan* P = (Plan*)plan;
    return launch_grad_velocity(P, vel, grad_m, grad_v, P->nphys);
}
