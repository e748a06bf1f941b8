// Frequency-domain ESI solved with time-domain modelling (Sec. 5.2):
// CG on M q_bar = F S^T G F d (eq. (normaldtft)) with q_bar the DTFT of the
// extended source at N_f frequencies, M = F (S^T S + beta W) G.  The inverse
// DTFT G (real part, scaled by 1/nt) feeds the forward pass as its dense
// source inside the stencil kernel, and the DTFT F of the adjoint field is
// accumulated in the adjoint pass into complex float32 slices, so no vector
// with a time axis is ever stored: the CG vectors hold N_f slices per cell.
// The penalty term uses F (beta W) G = beta W (F G), with F G a 2 N_f x 2 N_f
// real matrix per plan.  Inner products are the real ones, Re sum conj(a) b.
//
// In blocks of K steps (the default), the slices meet the time loops once per
// block instead of at every step: before the forward pass runs steps
// [n0, n1), one kernel forms their sources G x_bar into a K-step buffer that
// the pass reads as a dense source; after the adjoint pass has run steps
// [j0, j1) writing its field into that buffer, one kernel folds the K fields
// into the slices.  Each cell's operations run in the same order as inside
// the step kernel, so both ways give the same bits.
#include <algorithm>
#include <cmath>
#include <vector>

#include "esi_internal.h"

namespace esi {

esi_status_t launch_dot(Plan* P, const float* x, const float* y, int nshots, int64_t len, double* out);

namespace {

constexpr int NT = 256;
constexpr int MAX_NF = 32;

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 8192)); }

__device__ __forceinline__ double block_sum(double v, double* sm) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < NT / 64; ++k) t += sm[k];
    return t;
}

// out = acc + beta W (F G) p per cell, and part[s][b] = block sums of p . out.
__global__ __launch_bounds__(NT) void k_dtft_finish(const float2* __restrict__ acc, const float2* __restrict__ p,
                                                    const double* __restrict__ C, int nf, int nz, int ny, int nx,
                                                    const int32_t* __restrict__ src, int shot0, double beta,
                                                    double b_eps, int w_identity, float2* __restrict__ out,
                                                    double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.y, b = blockIdx.x, bps = gridDim.x;
    const int64_t n = (int64_t)nz * ny * nx;
    const int64_t base = (int64_t)s * nf * n;
    double dot = 0.0;
    for (int64_t c = (int64_t)b * NT + threadIdx.x; c < n; c += (int64_t)bps * NT) {
        double w = beta;
        if (!w_identity) {
            const int64_t zy = c / nx;   // cells [nz][ny][nx]; ny = 1 and source y = 0 in 2D
            const int ix = (int)(c - zy * nx), iz = (int)(zy / ny), iy = (int)(zy - (int64_t)iz * ny);
            const double dx = ix - src[(shot0 + s) * 3 + 0], dz = iz - src[(shot0 + s) * 3 + 1],
                         dy = iy - src[(shot0 + s) * 3 + 2];
            const double bb = sqrt(dx * dx + dz * dz + dy * dy) + b_eps;
            w = beta * bb * bb;
        }
        double pv[2 * MAX_NF];
        for (int m = 0; m < nf; ++m) {
            const float2 v = p[base + m * n + c];
            pv[2 * m] = v.x;
            pv[2 * m + 1] = v.y;
        }
        for (int k = 0; k < nf; ++k) {
            double cr = 0.0, ci = 0.0;
            for (int j = 0; j < 2 * nf; ++j) {
                cr += C[(2 * k) * (2 * nf) + j] * pv[j];
                ci += C[(2 * k + 1) * (2 * nf) + j] * pv[j];
            }
            const float2 a = acc[base + k * n + c];
            float2 o;
            o.x = (float)((double)a.x + w * cr);
            o.y = (float)((double)a.y + w * ci);
            out[base + k * n + c] = o;
            dot += pv[2 * k] * (double)o.x + pv[2 * k + 1] * (double)o.y;
        }
    }
    const double t = block_sum(dot, sm);
    if (threadIdx.x == 0) part[(int64_t)s * bps + b] = t;
}

// d_out = G F d_in per receiver trace (the data represented through the
// inverse DTFT of their DTFT); one thread per receiver of the call's shots.
__global__ void k_data_band(const float* __restrict__ din, float* __restrict__ dout,
                            const int64_t* __restrict__ rec_ptr, int shot0, int nshots, int nt,
                            const float2* __restrict__ tw, int nf, double inv_nt) {
    const int64_t base = rec_ptr[shot0];
    const int64_t nr = rec_ptr[shot0 + nshots] - base;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nr; r += (int64_t)gridDim.x * blockDim.x) {
        int s = 0;
        while (rec_ptr[shot0 + s + 1] <= base + r) ++s;
        const int64_t nrs = rec_ptr[shot0 + s + 1] - rec_ptr[shot0 + s];
        const int64_t col = base + r - rec_ptr[shot0 + s];
        const int64_t off = (int64_t)nt * (rec_ptr[shot0 + s] - base) + col;
        double fr[MAX_NF], fi[MAX_NF];
        for (int m = 0; m < nf; ++m) fr[m] = fi[m] = 0.0;
        for (int t = 0; t < nt; ++t) {
            const double v = din[off + (int64_t)t * nrs];
            for (int m = 0; m < nf; ++m) {
                const float2 w = tw[(int64_t)t * nf + m];
                fr[m] += v * (double)w.x;
                fi[m] += v * (double)w.y;
            }
        }
        for (int t = 0; t < nt; ++t) {
            double q = 0.0;
            for (int m = 0; m < nf; ++m) {
                const float2 w = tw[(int64_t)t * nf + m];
                q += fr[m] * (double)w.x + fi[m] * (double)w.y;
            }
            dout[off + (int64_t)t * nrs] = (float)(q * inv_nt);
        }
    }
}

// q[s][t][c] = inv_nt sum_m (re_m cos + im_m sin)(w_m t)
__global__ void k_to_time(const float2* __restrict__ xb, const float2* __restrict__ tw, int nf, int nt,
                          int64_t n, int nshots, float inv_nt, float* __restrict__ q) {
    const int64_t total = (int64_t)nshots * nt * n;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
        const int64_t c = i % n;
        const int64_t st = i / n;
        const int t = (int)(st % nt), s = (int)(st / nt);
        float acc = 0.f;
        for (int m = 0; m < nf; ++m) {
            const float2 v = xb[((int64_t)s * nf + m) * n + c];
            const float2 w = tw[(int64_t)t * nf + m];
            acc = fmaf(v.y, w.y, fmaf(v.x, w.x, acc));
        }
        q[i] = acc * inv_nt;
    }
}

// The block kernels give a thread CPT cells 64 apart (a wave then moves runs
// of 64 * CPT consecutive floats of a time step) and take a cell's frequency
// slices in registers; CPT shrinks as the frequency count grows.

// q[s][n % K][c] = inv_nt sum_m (re_m cos + im_m sin)(w_m t_n), n in [n0, n1):
// the step kernel's per-step source, the frequencies in the same order.
template <int NFC, int CPT>
__global__ __launch_bounds__(NT) void k_dtft_qgen(const float2* __restrict__ xb, const float2* __restrict__ tw,
                                                  int nf, int n0, int n1, int K, int64_t n,
                                                  const int* __restrict__ active, float inv_nt,
                                                  float* __restrict__ q) {
    const int s = blockIdx.y;
    if (active && !active[s]) return;   // uniform over the block
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t c0 = ((int64_t)blockIdx.x * (NT / 64) + wv) * 64 * CPT + lane; c0 < n;
         c0 += (int64_t)gridDim.x * NT * CPT) {
        float2 v[CPT][NFC];
        bool on[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            on[j] = c0 + 64 * j < n;
#pragma unroll
            for (int m = 0; m < NFC; ++m)
                v[j][m] = (on[j] && m < nf) ? xb[((int64_t)s * nf + m) * n + c0 + 64 * j] : make_float2(0.f, 0.f);
        }
        for (int t = n0; t < n1; ++t) {
            const float2* __restrict__ w = tw + (int64_t)t * nf;
            float* __restrict__ qt = q + ((int64_t)s * K + t % K) * n + c0;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                float acc = 0.f;
#pragma unroll
                for (int m = 0; m < NFC; ++m)
                    if (m < nf) acc = fmaf(v[j][m].y, w[m].y, fmaf(v[j][m].x, w[m].x, acc));
                if (on[j]) qt[64 * j] = acc * inv_nt;
            }
        }
    }
}

// acc_m[s][c] += mu^j (cos, sin)(w_m t_j) for j = j1-1 down to j0, mu^j in
// slot j % K: the step kernel's per-step accumulation, in the same order.  U
// steps of mu are loaded before they are folded in.
template <int NFC, int CPT>
__global__ __launch_bounds__(NT) void k_dtft_bacc(float2* __restrict__ acc, const float* __restrict__ mu,
                                                  const float2* __restrict__ tw, int nf, int j0, int j1, int K,
                                                  int64_t n, const int* __restrict__ active) {
    constexpr int U = 4;
    const int s = blockIdx.y;
    if (active && !active[s]) return;   // uniform over the block
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t c0 = ((int64_t)blockIdx.x * (NT / 64) + wv) * 64 * CPT + lane; c0 < n;
         c0 += (int64_t)gridDim.x * NT * CPT) {
        float2 v[CPT][NFC];
        bool on[CPT];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            on[j] = c0 + 64 * j < n;
#pragma unroll
            for (int m = 0; m < NFC; ++m)
                v[j][m] = (on[j] && m < nf) ? acc[((int64_t)s * nf + m) * n + c0 + 64 * j] : make_float2(0.f, 0.f);
        }
        for (int jt = j1 - 1; jt >= j0; jt -= U) {
            float u[U][CPT];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int jj = jt - k;
                const float* __restrict__ mt = mu + ((int64_t)s * K + (jj >= j0 ? jj % K : 0)) * n + c0;
#pragma unroll
                for (int j = 0; j < CPT; ++j) u[k][j] = (on[j] && jj >= j0) ? mt[64 * j] : 0.f;
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                if (jt - k < j0) break;   // uniform over the block
                const float2* __restrict__ w = tw + (int64_t)(jt - k) * nf;
#pragma unroll
                for (int j = 0; j < CPT; ++j) {
#pragma unroll
                    for (int m = 0; m < NFC; ++m) {
                        if (m < nf) {
                            v[j][m].x = fmaf(u[k][j], w[m].x, v[j][m].x);
                            v[j][m].y = fmaf(u[k][j], w[m].y, v[j][m].y);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if (!on[j]) continue;
#pragma unroll
            for (int m = 0; m < NFC; ++m)
                if (m < nf) acc[((int64_t)s * nf + m) * n + c0 + 64 * j] = v[j][m];
        }
    }
}

// CG update after the stopping test: x += alpha p for shots still active or
// leaving normally; p = r + beta p for shots still active.
__global__ void k_xp(float* __restrict__ x, float* __restrict__ p, const float* __restrict__ r,
                     const double* __restrict__ alpha, const double* __restrict__ beta,
                     const int* __restrict__ active, const int* __restrict__ finish, int64_t len) {
    const int s = blockIdx.y;
    const bool act = active[s] != 0, upd = act || finish[s] == 1;
    if (!upd) return;
    const float al = (float)alpha[s], be = (float)beta[s];
    float* xs = x + (int64_t)s * len;
    float* ps = p + (int64_t)s * len;
    const float* rs = r + (int64_t)s * len;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < len; i += (int64_t)gridDim.x * NT) {
        const float pv = ps[i];
        xs[i] = fmaf(al, pv, xs[i]);
        if (act) ps[i] = fmaf(be, pv, rs[i]);
    }
}

esi_status_t need_freqs(Plan* P) {
    if (P->dft_freqs.empty() || !P->dft_tw) return fail(ESI_ERR_ARG, "no DTFT frequencies: call esi_dtft_set_freqs");
    if (P->ndim != 2 && P->dft_block <= 0)
        return fail(ESI_ERR_ARG, "the per-step DTFT runs on 2D plans; 3D plans take blocks of steps");
    return ESI_OK;
}

int dft_block(Plan* P) { return P->dft_block > 0 ? std::min(P->dft_block, P->nt) : 0; }

template <int CPT>
dim3 cell_grid(Plan* P, int ns) {
    const int64_t per = (int64_t)NT * CPT;
    return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((P->nphys + per - 1) / per, 1024)), (unsigned)ns);
}

esi_status_t launch_qgen(Plan* P, const float2* xb, int n0, int n1, int K, int ns, const int* active, float* q) {
    const int nf = (int)P->dft_freqs.size();
    const float inv_nt = (float)(1.0 / P->nt);
    if (nf <= 8)
        hipLaunchKernelGGL((k_dtft_qgen<8, 4>), cell_grid<4>(P, ns), dim3(NT), 0, P->stream, xb, P->dft_tw, nf, n0,
                           n1, K, P->nphys, active, inv_nt, q);
    else if (nf <= 16)
        hipLaunchKernelGGL((k_dtft_qgen<16, 2>), cell_grid<2>(P, ns), dim3(NT), 0, P->stream, xb, P->dft_tw, nf, n0,
                           n1, K, P->nphys, active, inv_nt, q);
    else
        hipLaunchKernelGGL((k_dtft_qgen<MAX_NF, 1>), cell_grid<1>(P, ns), dim3(NT), 0, P->stream, xb, P->dft_tw, nf,
                           n0, n1, K, P->nphys, active, inv_nt, q);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_bacc(Plan* P, float2* acc, const float* mu, int j0, int j1, int K, int ns, const int* active) {
    const int nf = (int)P->dft_freqs.size();
    if (nf <= 8)
        hipLaunchKernelGGL((k_dtft_bacc<8, 4>), cell_grid<4>(P, ns), dim3(NT), 0, P->stream, acc, mu, P->dft_tw, nf,
                           j0, j1, K, P->nphys, active);
    else if (nf <= 16)
        hipLaunchKernelGGL((k_dtft_bacc<16, 2>), cell_grid<2>(P, ns), dim3(NT), 0, P->stream, acc, mu, P->dft_tw, nf,
                           j0, j1, K, P->nphys, active);
    else
        hipLaunchKernelGGL((k_dtft_bacc<MAX_NF, 1>), cell_grid<1>(P, ns), dim3(NT), 0, P->stream, acc, mu, P->dft_tw,
                           nf, j0, j1, K, P->nphys, active);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

StepArgs dft_args(Plan* P, const TileLists* L, int shot0, int ns) {
    StepArgs a = base_args(P, L, shot0, ns);
    a.dft_tw = P->dft_tw;
    a.dft_nf = (int)P->dft_freqs.size();
    a.inv_nt = (float)(1.0 / P->nt);
    return a;
}

// The forward pass over all steps with the dense source G x_bar and the
// extra flags (F_GATHER, F_PENALTY); the ring state ends in slot *cs.
esi_status_t dtft_forward(Plan* P, StepArgs a, unsigned extra, const float2* xb, int ns, int* cs) {
    *cs = 0;
    const int K = dft_block(P);
    if (K == 0) {
        a.dft_src = xb;
        return forward_loop(P, a, F_DTFT_SRC | extra, P->ring, cs, 0, P->nt);
    }
    ESI_TRY(grow_t(&P->dft_blk, &P->dft_blk_cap, (int64_t)ns * K * P->nphys, P->stream));
    a.dsrc = P->dft_blk;
    a.blk_T = K;
    for (int n0 = 0; n0 < P->nt; n0 += K) {
        const int n1 = std::min(P->nt, n0 + K);
        ESI_TRY(launch_qgen(P, xb, n0, n1, K, ns, a.active, P->dft_blk));
        ESI_TRY(forward_loop(P, a, F_SRC_DENSE | extra, P->ring, cs, n0, n1));
    }
    return ESI_OK;
}

// The adjoint pass over all steps (injection set in b) with the DTFT of its
// field accumulated into acc.
esi_status_t dtft_adjoint(Plan* P, StepArgs b, float2* acc, int ns) {
    int cs = 0;
    const int K = dft_block(P);
    if (K == 0) {
        b.dft_acc = acc;
        return adjoint_loop(P, b, F_INJ | F_DTFT_ACC, P->ring, &cs, 0, P->nt);
    }
    ESI_TRY(grow_t(&P->dft_blk, &P->dft_blk_cap, (int64_t)ns * K * P->nphys, P->stream));
    b.dout = P->dft_blk;
    b.blk_T = K;
    for (int j1 = P->nt, j0 = ((P->nt - 1) / K) * K; j1 > 0; j1 = j0, j0 -= K) {
        ESI_TRY(adjoint_loop(P, b, F_INJ | F_OUT, P->ring, &cs, j0, j1));
        ESI_TRY(launch_bacc(P, acc, P->dft_blk, j0, j1, K, ns, b.active));
    }
    return ESI_OK;
}

// M p_bar into Mp (device [ns][nf][phys] (re, im)); p.Mp per shot into pMp
// (device, nullable); inactive shots (active != nullptr) are skipped by the
// time loops.
esi_status_t dtft_normal(Plan* P, int shot0, int ns, const float2* p, float2* Mp, double* pMp, const int* active) {
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    const int nf = (int)P->dft_freqs.size();
    const int64_t dl = data_len(P, shot0, ns);
    ESI_TRY(grow_t(&P->dscr, &P->dscr_cap, std::max<int64_t>(dl, 1), P->stream));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs a = dft_args(P, L, shot0, ns);
    a.active = active;
    a.gat_data = P->dscr;
    int cs = 0;
    ESI_TRY(dtft_forward(P, a, F_GATHER, p, ns, &cs));
    ESI_TRY(launch_final_gather(P, P->ring + (int64_t)cs * P->fsize, RING * P->fsize, P->dscr, shot0, ns));
    ESI_TRY(launch_fill(P, (float*)Mp, (int64_t)ns * nf * P->nphys * 2, 0.f));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs b = dft_args(P, L, shot0, ns);
    b.active = active;
    b.inj_data = P->dscr;
    ESI_TRY(dtft_adjoint(P, b, Mp, ns));
    const int bps = (int)std::max<int64_t>(1, std::min<int64_t>(64, (P->nphys + 4095) / 4096));
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)bps * ns, P->stream));
    hipLaunchKernelGGL(k_dtft_finish, dim3(bps, ns), dim3(NT), 0, P->stream, Mp, p, P->dft_C, nf, P->nz, P->ny, P->nx,
                       P->d_src, shot0, P->beta, P->b_eps, P->w_identity, Mp, P->part);
    ESI_HIP_TRY(hipGetLastError());
    return pMp ? launch_reduce_parts(P, P->part, bps, ns, pMp) : ESI_OK;
}

// b = F S^T G F d_obs
esi_status_t dtft_rhs(Plan* P, int shot0, int ns, const float* d_obs, float2* b) {
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    const int nf = (int)P->dft_freqs.size();
    const int64_t dl = data_len(P, shot0, ns);
    ESI_TRY(grow_t(&P->dscr, &P->dscr_cap, std::max<int64_t>(dl, 1), P->stream));
    if (dl > 0) {
        const int64_t nr = P->h_rec_ptr[shot0 + ns] - P->h_rec_ptr[shot0];
        hipLaunchKernelGGL(k_data_band, dim3((int)std::min<int64_t>((nr + 63) / 64, 4096)), dim3(64), 0, P->stream,
                           d_obs, P->dscr, P->d_rec_ptr, shot0, ns, P->nt, P->dft_tw, nf, 1.0 / P->nt);
        ESI_HIP_TRY(hipGetLastError());
    }
    ESI_TRY(launch_fill(P, (float*)b, (int64_t)ns * nf * P->nphys * 2, 0.f));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs a = dft_args(P, L, shot0, ns);
    a.inj_data = P->dscr;
    return dtft_adjoint(P, a, b, ns);
}

}  // namespace
}  // namespace esi

using namespace esi;

extern "C" esi_status_t esi_dtft_set_freqs(esi_plan_t plan, int32_t nf, const double* freqs) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    if (nf < 1 || nf > MAX_NF || !freqs) return fail(ESI_ERR_ARG, "need 1 to 32 frequencies");
    for (int m = 0; m < nf; ++m)
        if (!std::isfinite(freqs[m]) || freqs[m] < 0) return fail(ESI_ERR_ARG, "frequencies must be finite and >= 0");
    const int nt = P->nt;
    std::vector<float2> tw((size_t)nt * nf);
    std::vector<double> cs((size_t)nt * nf), sn((size_t)nt * nf);
    for (int t = 0; t < nt; ++t)
        for (int m = 0; m < nf; ++m) {
            const double ph = 2.0 * M_PI * freqs[m] * t * P->dt;
            cs[(size_t)t * nf + m] = std::cos(ph);
            sn[(size_t)t * nf + m] = std::sin(ph);
            tw[(size_t)t * nf + m] = make_float2((float)std::cos(ph), (float)std::sin(ph));
        }
    // F G on (re, im) pairs: column (m, re) is F of cos(w_m t)/nt, column
    // (m, im) is F of sin(w_m t)/nt
    const int n2 = 2 * nf;
    std::vector<double> C((size_t)n2 * n2, 0.0);
    for (int m = 0; m < nf; ++m)
        for (int part = 0; part < 2; ++part)
            for (int k = 0; k < nf; ++k) {
                double re = 0.0, im = 0.0;
                for (int t = 0; t < nt; ++t) {
                    const double g = (part == 0 ? cs[(size_t)t * nf + m] : sn[(size_t)t * nf + m]) / nt;
                    re += g * cs[(size_t)t * nf + k];
                    im += g * sn[(size_t)t * nf + k];
                }
                C[(size_t)(2 * k) * n2 + 2 * m + part] = re;
                C[(size_t)(2 * k + 1) * n2 + 2 * m + part] = im;
            }
    if (P->dft_tw) ESI_HIP_TRY(hipFree(P->dft_tw));
    if (P->dft_C) ESI_HIP_TRY(hipFree(P->dft_C));
    P->dft_tw = nullptr;
    P->dft_C = nullptr;
    P->dft_freqs.clear();
    ESI_HIP_TRY(hipMalloc((void**)&P->dft_tw, tw.size() * sizeof(float2)));
    ESI_HIP_TRY(hipMalloc((void**)&P->dft_C, C.size() * sizeof(double)));
    ESI_HIP_TRY(hipMemcpy(P->dft_tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice));
    ESI_HIP_TRY(hipMemcpy(P->dft_C, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice));
    P->dft_freqs.assign(freqs, freqs + nf);
    return ESI_OK;
}

extern "C" esi_status_t esi_plan_set_dtft_block(esi_plan_t plan, int32_t block) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    if (block < 0 || block > 1024) return fail(ESI_ERR_ARG, "DTFT block must be 0..1024 steps");
    ((Plan*)plan)->dft_block = block;
    return ESI_OK;
}

extern "C" esi_status_t esi_dtft_normal_apply(esi_plan_t plan, int32_t shot0, int32_t ns, const float* p,
                                              float* Mp, double* pMp) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    ESI_TRY(need_freqs(P));
    if (!p || !Mp) return fail(ESI_ERR_ARG, "null pointer");
    if (p == Mp) return fail(ESI_ERR_ARG, "p and Mp must not alias");
    return dtft_normal(P, shot0, ns, (const float2*)p, (float2*)Mp, pMp, nullptr);
}

extern "C" esi_status_t esi_dtft_rhs(esi_plan_t plan, int32_t shot0, int32_t ns, const float* d_obs, float* b) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    ESI_TRY(need_freqs(P));
    if (!b || (!d_obs && data_len(P, shot0, ns) > 0)) return fail(ESI_ERR_ARG, "null pointer");
    return dtft_rhs(P, shot0, ns, d_obs, (float2*)b);
}

extern "C" esi_status_t esi_dtft_to_time(esi_plan_t plan, int32_t shot0, int32_t ns, const float* xbar, float* q) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    ESI_TRY(need_freqs(P));
    if (!xbar || !q) return fail(ESI_ERR_ARG, "null pointer");
    hipLaunchKernelGGL(k_to_time, dim3(grid_for((int64_t)ns * P->nt * P->nphys)), dim3(NT), 0, P->stream,
                       (const float2*)xbar, P->dft_tw, (int)P->dft_freqs.size(), P->nt, P->nphys, ns,
                       (float)(1.0 / P->nt), q);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

extern "C" esi_status_t esi_dtft_gradient(esi_plan_t plan, int32_t shot0, int32_t ns, const float* xbar,
                                          float* grad_m) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    ESI_TRY(need_freqs(P));
    if (!xbar || !grad_m) return fail(ESI_ERR_ARG, "null pointer");
    TileLists* L;
    ESI_TRY(lists_for(P, &L));
    ESI_TRY(grow_t(&P->gshot, &P->gshot_cap, (int64_t)ns * P->nphys, P->stream));
    ESI_TRY(launch_fill(P, P->gshot, (int64_t)ns * P->nphys, 0.f));
    ESI_TRY(ring_for(P, &P->ring, &P->ring_cap, ns));
    StepArgs a = dft_args(P, L, shot0, ns);
    a.gacc = P->gshot;
    int cs = 0;
    ESI_TRY(dtft_forward(P, a, F_PENALTY, (const float2*)xbar, ns, &cs));
    return launch_sum_shots(P, P->gshot, ns, P->nphys, 1.f, grad_m);
}

extern "C" esi_status_t esi_dtft_cg_solve(esi_plan_t plan, int32_t shot0, int32_t ns, const float* d_obs,
                                          float* xbar, float* work, int32_t max_iter, double rtol,
                                          esi_cg_report_t* rep) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, ns));
    ESI_TRY(need_freqs(P));
    if (!xbar || !work || (!d_obs && data_len(P, shot0, ns) > 0)) return fail(ESI_ERR_ARG, "null pointer");
    if (max_iter < 1) return fail(ESI_ERR_ARG, "max_iter must be >= 1");
    if (!(rtol >= 0)) return fail(ESI_ERR_ARG, "rtol must be >= 0");
    const int nf = (int)P->dft_freqs.size();
    const int64_t len = 2LL * nf * P->nphys;          // floats per shot
    float* r = work;
    float* p = work + ns * len;
    float* Ap = work + 2 * ns * len;
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
    ESI_TRY(grow_t(&P->cg_hist, &P->cg_hist_cap, (int64_t)ns * (max_iter + 1), P->stream));
    ESI_TRY(dtft_rhs(P, shot0, ns, d_obs, (float2*)r));
    ESI_TRY(launch_copy(P, p, r, ns * len));
    ESI_TRY(launch_fill(P, xbar, ns * len, 0.f));
    ESI_TRY(launch_dot(P, r, r, ns, len, rr));
    ESI_HIP_TRY(hipMemcpyAsync(rr0, rr, ns * sizeof(double), hipMemcpyDeviceToDevice, P->stream));
    ESI_TRY(launch_cg_init(P, rr0, active, finish, iters, status, P->cg_hist, max_iter + 1, ctl, ns));
    ESI_HIP_TRY(hipMemcpyAsync(P->h_ctl, ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
    ESI_HIP_TRY(hipStreamSynchronize(P->stream));
    int done = 0;
    const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((len + NT - 1) / NT, 2048));
    for (int k = 0; k < max_iter && P->h_ctl[1] > 0; ++k) {
        ESI_TRY(dtft_normal(P, shot0, ns, (const float2*)p, (float2*)Ap, pAp, active));
        ESI_TRY(launch_cg_alpha(P, rr, pAp, alpha, ns));
        ESI_TRY(launch_r_update(P, r, Ap, alpha, active, ns, len, rr_new));
        ESI_TRY(launch_cg_control(P, rr0, rr_new, pAp, active, finish, iters, status, P->cg_hist, max_iter + 1,
                                  ctl, rtol, max_iter, ns));
        ESI_TRY(launch_cg_beta(P, rr_new, rr, beta, ns));
        hipLaunchKernelGGL(k_xp, dim3(gx, ns), dim3(NT), 0, P->stream, xbar, p, r, alpha, beta, active, finish, len);
        ESI_HIP_TRY(hipGetLastError());
        ESI_HIP_TRY(hipMemcpyAsync(P->h_ctl, ctl, 2 * sizeof(int), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipStreamSynchronize(P->stream));
        done = k + 1;
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
        if (hs[s] == ESI_ERR_NONFINITE) return fail(ESI_ERR_NONFINITE, "DTFT CG: non-finite scalar");
    for (int s = 0; s < ns; ++s)
        if (hs[s] == ESI_ERR_BREAKDOWN) return fail(ESI_ERR_BREAKDOWN, "DTFT CG breakdown: p.Mp <= 0");
    return ESI_OK;
}
