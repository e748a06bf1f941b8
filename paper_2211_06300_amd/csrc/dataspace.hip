// Data-space solution of the normal equation (Sec. 5.1, the Sherman-Morrison-
// Woodbury route): CG on (beta I + S W^{-1} S^T) w = v, v = S W^{-1} S^T d,
// over the data vector of each shot, then q = (beta W)^{-1} S^T (d - w).
// An application of S W^{-1} S^T is an adjoint pass writing the adjoint
// field, then a forward pass whose dense source is that field times W^{-1}
// (scaled inside the stencil kernel) and which records the data.  The CG
// vectors hold nt x nrec values per shot; the one field-sized buffer is the
// adjoint field between the two passes.
#include <algorithm>
#include <cmath>
#include <vector>

#include "esi_internal.h"

namespace esi {
namespace {

constexpr int NT = 256;
constexpr int DB = 64;    // blocks per shot of the data-vector kernels

__device__ __forceinline__ double block_sum(double v, double* sm) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < NT / 64; ++k) t += sm[k];
    return t;
}

// W^{-1} per cell of each shot: 1 / B^2, or 1 for B = I (cells [nz][ny][nx],
// ny = 1 in 2D, where the source's third coordinate is 0)
__global__ void k_winv(const int32_t* __restrict__ src, int shot0, int ns, int nz, int ny, int nx, double b_eps,
                       int identity, float* __restrict__ out) {
    const int64_t n = (int64_t)nz * ny * nx;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < ns * n; i += (int64_t)gridDim.x * NT) {
        const int k = (int)(i / n);
        const int64_t c = i - k * n;
        if (identity) {
            out[i] = 1.f;
            continue;
        }
        const int64_t zy = c / nx;
        const int ix = (int)(c - zy * nx), iz = (int)(zy / ny), iy = (int)(zy - (int64_t)iz * ny);
        const double dx = ix - src[(shot0 + k) * 3 + 0], dz = iz - src[(shot0 + k) * 3 + 1],
                     dy = iy - src[(shot0 + k) * 3 + 2];
        const double b = sqrt(dx * dx + dz * dz + dy * dy) + b_eps;
        out[i] = (float)(1.0 / (b * b));
    }
}

// part[s][b] = block sums of a . b over shot s's data segment
__global__ __launch_bounds__(NT) void k_ds_dot(const float* __restrict__ a, const float* __restrict__ b,
                                               const int64_t* __restrict__ seg, double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.y;
    double acc = 0.0;
    for (int64_t i = seg[s] + blockIdx.x * (int64_t)NT + threadIdx.x; i < seg[s + 1]; i += (int64_t)gridDim.x * NT)
        acc += (double)a[i] * (double)b[i];
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

// Ap = beta p + Kp; part = block sums of p . Ap
__global__ __launch_bounds__(NT) void k_ds_ap(const float* __restrict__ p, const float* __restrict__ Kp, float beta,
                                              float* __restrict__ Ap, const int64_t* __restrict__ seg,
                                              double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.y;
    double acc = 0.0;
    for (int64_t i = seg[s] + blockIdx.x * (int64_t)NT + threadIdx.x; i < seg[s + 1]; i += (int64_t)gridDim.x * NT) {
        const float v = fmaf(beta, p[i], Kp[i]);
        Ap[i] = v;
        acc += (double)p[i] * (double)v;
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

// r -= alpha Ap for active shots; part = block sums of r . r
__global__ __launch_bounds__(NT) void k_ds_r(float* __restrict__ r, const float* __restrict__ Ap,
                                             const double* __restrict__ alpha, const int* __restrict__ active,
                                             const int64_t* __restrict__ seg, double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.y;
    double acc = 0.0;
    if (active[s]) {   // uniform over the block
        const float al = (float)alpha[s];
        for (int64_t i = seg[s] + blockIdx.x * (int64_t)NT + threadIdx.x; i < seg[s + 1];
             i += (int64_t)gridDim.x * NT) {
            const float v = fmaf(-al, Ap[i], r[i]);
            r[i] = v;
            acc += (double)v * (double)v;
        }
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

// w += alpha p (active or leaving normally); p = r + beta p (active)
__global__ void k_ds_wp(float* __restrict__ w, float* __restrict__ p, const float* __restrict__ r,
                        const double* __restrict__ alpha, const double* __restrict__ beta,
                        const int* __restrict__ active, const int* __restrict__ finish,
                        const int64_t* __restrict__ seg) {
    const int s = blockIdx.y;
    const bool act = active[s] != 0;
    if (!act && finish[s] != 1) return;
    const float al = (float)alpha[s], be = (float)beta[s];
    for (int64_t i = seg[s] + blockIdx.x * (int64_t)NT + threadIdx.x; i < seg[s + 1]; i += (int64_t)gridDim.x * NT) {
        const float pv = p[i];
        w[i] = fmaf(al, pv, w[i]);
        if (act) p[i] = fmaf(be, pv, r[i]);
    }
}

// q[s][t][c] *= winv[s][c] * scale
__global__ void k_ds_scale_q(float* __restrict__ q, const float* __restrict__ winv, float scale, int ns, int nt,
                             int64_t n) {
    const int64_t total = (int64_t)ns * nt * n;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
        const int64_t c = i % n;
        const int s = (int)(i / ((int64_t)nt * n));
        q[i] = q[i] * (winv[(int64_t)s * n + c] * scale);
    }
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 8192)); }

// y = S W^{-1} S^T x with the adjoint field checkpointed: one adjoint pass
// saves the adjoint state (mu, its increment) after every step j = kK, k >= 1;
// then, segment by segment in forward time, the segment's field is recomputed
// from the checkpoint above it into a K-step buffer and the forward pass runs
// the segment with it as its source.  The same kernels run on the same
// states, so y equals the resident-field result bit for bit.
esi_status_t K_apply_ckpt(Plan* P, const TileLists* L, int shot0, int ns, const float* x, float* y,
                          const int* active) {
    const int nt = P->nt, K = std::min(P->ds_ckpt, nt), nseg = (nt + K - 1) / K;
    const int64_t cstr = (int64_t)nseg * 2 * P->fsize;       // floats per shot of ds_ck
    ESI_TRY(grow_t(&P->ds_ck, &P->ds_ck_cap, (int64_t)ns * cstr, P->stream));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs a = base_args(P, L, shot0, ns);
    a.active = active;
    a.inj_data = x;
    int cs = 0;
    for (int k = nseg - 1; k >= 1; --k) {
        ESI_TRY(adjoint_loop(P, a, F_INJ, P->ring, &cs, k * K, std::min(nt, (k + 1) * K)));
        ESI_TRY(launch_copy_shots(P, P->ds_ck + (int64_t)k * 2 * P->fsize, cstr, P->ring + (int64_t)cs * P->fsize,
                                  RING * P->fsize, P->fsize, ns));
        ESI_TRY(launch_copy_shots(P, P->ds_ck + (int64_t)k * 2 * P->fsize + P->fsize, cstr,
                                  P->ring + (int64_t)(2 + cs) * P->fsize, RING * P->fsize, P->fsize, ns));
    }
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs b = base_args(P, L, shot0, ns);
    b.active = active;
    b.inj_data = x;
    b.dout = P->ds_mu;
    b.blk_T = K;
    StepArgs f = base_args(P, L, shot0, ns);
    f.active = active;
    f.dsrc = P->ds_mu;
    f.blk_T = K;
    f.cg_s = P->ds_winv;
    f.gat_data = y;
    int fcs = 0;
    for (int k = 0; k < nseg; ++k) {
        const int j0 = k * K, j1 = std::min(nt, j0 + K);
        // the adjoint state after step j1 into slot 0 of the recompute ring
        // (zero above the last step)
        ESI_TRY(ring_for(P, &P->ring2, &P->ring2_cap, ns));
        if (k + 1 < nseg) {
            ESI_TRY(launch_copy_shots(P, P->ring2, RING * P->fsize, P->ds_ck + (int64_t)(k + 1) * 2 * P->fsize, cstr,
                                      P->fsize, ns));
            ESI_TRY(launch_copy_shots(P, P->ring2 + 2 * P->fsize, RING * P->fsize,
                                      P->ds_ck + (int64_t)(k + 1) * 2 * P->fsize + P->fsize, cstr, P->fsize, ns));
        }
        int rcs = 0;
        ESI_TRY(adjoint_loop(P, b, F_INJ | F_OUT, P->ring2, &rcs, j0, j1));
        ESI_TRY(forward_loop(P, f, F_SRC_DENSE | F_SCALE | F_GATHER, P->ring, &fcs, j0, j1));
    }
    return launch_final_gather(P, P->ring + (int64_t)fcs * P->fsize, RING * P->fsize, y, shot0, ns);
}

// y = S W^{-1} S^T x (data vectors of the call's shots)
esi_status_t K_apply(Plan* P, const TileLists* L, int shot0, int ns, const float* x, float* y, const int* active) {
    if (P->ds_ckpt > 0) return K_apply_ckpt(P, L, shot0, ns, x, y, active);
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs a = base_args(P, L, shot0, ns);
    a.active = active;
    a.inj_data = x;
    a.dout = P->ds_mu;
    int cs = 0;
    ESI_TRY(adjoint_loop(P, a, F_INJ | F_OUT, P->ring, &cs, 0, P->nt));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs b = base_args(P, L, shot0, ns);
    b.active = active;
    b.dsrc = P->ds_mu;
    b.cg_s = P->ds_winv;
    b.gat_data = y;
    cs = 0;
    ESI_TRY(forward_loop(P, b, F_SRC_DENSE | F_SCALE | F_GATHER, P->ring, &cs, 0, P->nt));
    return launch_final_gather(P, P->ring + (int64_t)cs * P->fsize, RING * P->fsize, y, shot0, ns);
}

}  // namespace
}  // namespace esi

using namespace esi;

extern "C" esi_status_t esi_plan_set_ds_ckpt(esi_plan_t plan, int32_t every) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    if (every < 0) return fail(ESI_ERR_ARG, "checkpoint interval must be >= 0");
    ((Plan*)plan)->ds_ckpt = every;
    return ESI_OK;
}

extern "C" esi_status_t esi_ds_cg_solve(esi_plan_t plan, int32_t shot0, int32_t ns, const float* d, float* w,
                                        float* q, float* work, int32_t max_iter, double rtol,
                                        esi_cg_report_t* rep) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    const int64_t dl = data_len(P, shot0, ns);
    if (dl == 0) return fail(ESI_ERR_ARG, "the shots record no data");
    if (!d || !w || !work) return fail(ESI_ERR_ARG, "null pointer");
    if (max_iter < 1) return fail(ESI_ERR_ARG, "max_iter must be >= 1");
    if (!(rtol >= 0)) return fail(ESI_ERR_ARG, "rtol must be >= 0");
    if (!(P->beta > 0)) return fail(ESI_ERR_ARG, "the data-space route needs beta > 0");
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    const int64_t fl = (int64_t)ns * P->nt * P->nphys;
    const int64_t mu_len = (int64_t)ns * (P->ds_ckpt > 0 ? std::min(P->ds_ckpt, P->nt) : P->nt) * P->nphys;
    ESI_TRY(grow_t(&P->ds_mu, &P->ds_mu_cap, mu_len, P->stream));
    ESI_TRY(grow_t(&P->ds_winv, &P->ds_winv_cap, (int64_t)ns * P->nphys, P->stream));
    ESI_TRY(grow_t(&P->ds_seg, &P->ds_seg_cap, (int64_t)ns + 1, P->stream));
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)DB * ns, P->stream));
    ESI_TRY(grow_t(&P->cg_hist, &P->cg_hist_cap, (int64_t)ns * (max_iter + 1), P->stream));
    std::vector<int64_t> seg(ns + 1);
    for (int s = 0; s <= ns; ++s) seg[s] = (int64_t)P->nt * (P->h_rec_ptr[shot0 + s] - P->h_rec_ptr[shot0]);
    ESI_HIP_TRY(hipMemcpyAsync(P->ds_seg, seg.data(), seg.size() * sizeof(int64_t), hipMemcpyHostToDevice, P->stream));
    hipLaunchKernelGGL(k_winv, dim3(grid_for((int64_t)ns * P->nphys)), dim3(NT), 0, P->stream, P->d_src, shot0, ns,
                       P->nz, P->ny, P->nx, P->b_eps, P->w_identity, P->ds_winv);
    ESI_HIP_TRY(hipGetLastError());
    float* r = work;
    float* p = work + dl;
    float* Ap = work + 2 * dl;
    double* rr = P->scal;
    double* pAp = P->scal + P->nshots;
    double* alpha = P->scal + 2 * P->nshots;
    double* beta = P->scal + 3 * P->nshots;
    double* rr_new = P->scal + 4 * P->nshots;
    double* rr0 = P->scal + 5 * P->nshots;
    int* active = P->flags;
    int* finish = P->flags + P->nshots;
    int* iters = P->cgi;
    int* status = P->cgi + P->nshots;
    int* ctl = P->cgi + 2 * P->nshots;
    const dim3 g2(DB, ns);
    // v = S W^{-1} S^T d; w_0 = 0, r_0 = v, p_0 = r_0
    ESI_TRY(K_apply(P, L, shot0, ns, d, r, nullptr));
    ESI_TRY(launch_copy(P, p, r, dl));
    ESI_TRY(launch_fill(P, w, dl, 0.f));
    hipLaunchKernelGGL(k_ds_dot, g2, dim3(NT), 0, P->stream, r, r, P->ds_seg, P->part);
    ESI_HIP_TRY(hipGetLastError());
    ESI_TRY(launch_reduce_parts(P, P->part, DB, ns, rr));
    ESI_HIP_TRY(hipMemcpyAsync(rr0, rr, ns * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
    ESI_TRY(launch_cg_init(P, rr0, active, finish, iters, status, P->cg_hist, max_iter + 1, ctl, ns));
    ESI_HIP_TRY(hipMemcpyAsync(P->h_ctl, ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
    ESI_HIP_TRY(hipStreamSynchronize(P->stream));
    int done = 0;
    for (int k = 0; k < max_iter && P->h_ctl[1] > 0; ++k) {
        ESI_TRY(K_apply(P, L, shot0, ns, p, Ap, active));
        hipLaunchKernelGGL(k_ds_ap, g2, dim3(NT), 0, P->stream, p, Ap, (float)P->beta, Ap, P->ds_seg, P->part);
        ESI_HIP_TRY(hipGetLastError());
        ESI_TRY(launch_reduce_parts(P, P->part, DB, ns, pAp));
        ESI_TRY(launch_cg_alpha(P, rr, pAp, alpha, ns));
        hipLaunchKernelGGL(k_ds_r, g2, dim3(NT), 0, P->stream, r, Ap, alpha, active, P->ds_seg, P->part);
        ESI_HIP_TRY(hipGetLastError());
        ESI_TRY(launch_reduce_parts(P, P->part, DB, ns, rr_new));
        ESI_TRY(launch_cg_control(P, rr0, rr_new, pAp, active, finish, iters, status, P->cg_hist, max_iter + 1, ctl,
                                  rtol, max_iter, ns));
        ESI_TRY(launch_cg_beta(P, rr_new, rr, beta, ns));
        hipLaunchKernelGGL(k_ds_wp, g2, dim3(NT), 0, P->stream, w, p, r, alpha, beta, active, finish, P->ds_seg);
        ESI_HIP_TRY(hipGetLastError());
        ESI_HIP_TRY(hipMemcpyAsync(P->h_ctl, ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipStreamSynchronize(P->stream));
        done = k + 1;
    }
    if (q) {
        // q = (beta W)^{-1} S^T (d - w)
        ESI_TRY(launch_sub(P, r, d, w, dl));
        ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
        StepArgs a = base_args(P, L, shot0, ns);
        a.inj_data = r;
        a.dout = q;
        int cs = 0;
        ESI_TRY(adjoint_loop(P, a, F_INJ | F_OUT, P->ring, &cs, 0, P->nt));
        hipLaunchKernelGGL(k_ds_scale_q, dim3(grid_for(fl)), dim3(NT), 0, P->stream, q, P->ds_winv,
                           (float)(1.0 / P->beta), ns, P->nt, P->nphys);
        ESI_HIP_TRY(hipGetLastError());
    }
    std::vector<int> hs(ns);
    ESI_HIP_TRY(hipMemcpy(hs.data(), status, ns * sizeof(int), hipMemcpyDeviceToHost));
    if (rep) {
        rep->iters = done;
        if (rep->shot_iters) ESI_HIP_TRY(hipMemcpy(rep->shot_iters, iters, ns * sizeof(int), hipMemcpyDeviceToHost));
        if (rep->res_hist)
            ESI_HIP_TRY(hipMemcpy(rep->res_hist, P->cg_hist, (size_t)ns * (max_iter + 1) * sizeof(double),
                                  hipMemcpyDeviceToHost));
    }
    for (int s = 0; s < ns; ++s)
        if (hs[s] == ESI_ERR_NONFINITE) return fail(ESI_ERR_NONFINITE, "data-space CG: non-finite scalar");
    for (int s = 0; s < ns; ++s)
        if (hs[s] == ESI_ERR_BREAKDOWN) return fail(ESI_ERR_BREAKDOWN, "data-space CG breakdown: p.Ap <= 0");
    return ESI_OK;
}
