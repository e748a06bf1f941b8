// Kernels of the flexible CG with the learned preconditioner: per-cell residual
// energy, network features, the scale z = s r, the products z.r and z.Np,
// the stopping / stall / fallback bookkeeping of FCG(1) (Notay 2000), and the
// (a, c) maps that make the network's training pairs.
#include <cmath>

#include "esi_internal.h"

namespace esi {
namespace {

constexpr int NT = 256;

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 16384)); }

// blocks per shot for reductions over the cells of one shot
int cell_blocks(int64_t nphys) { return (int)std::max<int64_t>(1, std::min<int64_t>(64, (nphys + 4095) / 4096)); }

__device__ __forceinline__ double block_sum_d(double v, double* sm) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < NT / 64; ++k) t += sm[k];
    return t;
}

// a[s][x] = sum_t r[s][t][x]^2 for the shots still iterating.
__global__ void k_energy(const float* __restrict__ r, const int* __restrict__ active, float* __restrict__ a,
                         int ns, int nt, int64_t nphys) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < ns * nphys; i += (int64_t)gridDim.x * NT) {
        const int s = (int)(i / nphys);
        if (active && !active[s]) continue;
        const int64_t x = i % nphys;
        const float* rs = r + (int64_t)s * nt * nphys + x;
        float acc = 0.f;
        for (int t = 0; t < nt; ++t) {
            const float v = rs[(int64_t)t * nphys];
            acc = fmaf(v, v, acc);
        }
        a[i] = acc;
    }
}

// Training maps of the shots that did iteration `k` (iters[s] == k; k = 0:
// every shot): out[s][0][x] = sum_t r^2, out[s][1][x] = sum_t r (xref - xk)
// with xk = x + alpha p (the update the shot has not applied yet; none at k = 0).
__global__ void k_stats(const float* __restrict__ r, const float* __restrict__ x, const float* __restrict__ p,
                        const double* __restrict__ alpha, const float* __restrict__ xref,
                        const int* __restrict__ iters, int k, float* __restrict__ out, int ns, int nt,
                        int64_t nphys) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < ns * nphys; i += (int64_t)gridDim.x * NT) {
        const int s = (int)(i / nphys);
        if (k > 0 && iters[s] != k) continue;
        const int64_t c = i % nphys;
        const int64_t base = (int64_t)s * nt * nphys + c;
        const float al = p ? (float)alpha[s] : 0.f;
        float aa = 0.f, cc = 0.f;
        for (int t = 0; t < nt; ++t) {
            const int64_t j = base + (int64_t)t * nphys;
            const float rv = r[j];
            const float xk = p ? fmaf(al, p[j], x[j]) : x[j];
            aa = fmaf(rv, rv, aa);
            cc = fmaf(rv, xref[j] - xk, cc);
        }
        out[((int64_t)s * 2) * nphys + c] = aa;
        out[((int64_t)s * 2 + 1) * nphys + c] = cc;
    }
}

// mean[s] = mean over cells of sqrt(a / nt).  One workgroup per shot.
__global__ __launch_bounds__(NT) void k_feat_mean(const float* __restrict__ a, int64_t nphys, int nt,
                                                  double* __restrict__ mean) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.x;
    double acc = 0.0;
    for (int64_t x = threadIdx.x; x < nphys; x += NT) acc += sqrt((double)a[(int64_t)s * nphys + x] / nt);
    const double t = block_sum_d(acc, sm);
    if (threadIdx.x == 0) mean[s] = t / (double)nphys;
}

// Network input on the image padded to Hp x Wp (zero outside the grid):
// [log(1 + rms / mean(rms)), v / 3000, log(B) / 4] with rms = sqrt(a / nt) and B the
// annihilator weight |x - x_s| / dx + eps (in cells); also the padded copies
// of a and c when asked for, as a s0^2 and c s0 for a base scale s0 (the
// training maps of the correction exp(o) on top of s0).
__global__ void k_features(const float* __restrict__ a, const float* __restrict__ c,
                           const double* __restrict__ mean, const float* __restrict__ v,
                           const int32_t* __restrict__ src, int shot0, float b_eps, int ns, int nz, int nx,
                           int Hp, int Wp, int nt, const float* __restrict__ base, float* __restrict__ xin,
                           float* __restrict__ apad, float* __restrict__ cpad) {
    const int64_t img = (int64_t)Hp * Wp;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < ns * img; i += (int64_t)gridDim.x * NT) {
        const int s = (int)(i / img);
        const int64_t q = i % img;
        const int iz = (int)(q / Wp), ix = (int)(q % Wp);
        float f0 = 0.f, f1 = 0.f, f2 = 0.f, av = 0.f, cv = 0.f, av_out = 0.f, cv_out = 0.f;
        if (iz < nz && ix < nx) {
            const int64_t cell = (int64_t)iz * nx + ix;
            av = a[(int64_t)s * nz * nx + cell];
            if (c) cv = c[(int64_t)s * nz * nx + cell];
            const float b0 = base ? base[(int64_t)s * nz * nx + cell] : 1.f;
            const double m = mean[s];
            const float rms = sqrtf(av / (float)nt);
            f0 = log1pf(m > 0.0 ? (float)(rms / m) : rms);
            f1 = v[cell] / 3000.f;
            const float dx = (float)(ix - src[3 * (shot0 + s)]), dz = (float)(iz - src[3 * (shot0 + s) + 1]);
            f2 = logf(sqrtf(dx * dx + dz * dz) + b_eps) * 0.25f;
            av_out = av * b0 * b0;
            cv_out = cv * b0;
        }
        float* xs = xin + (int64_t)s * 3 * img;
        xs[q] = f0;
        xs[img + q] = f1;
        xs[2 * img + q] = f2;
        if (apad) apad[i] = av_out;
        if (cpad) cpad[i] = cv_out;
    }
}

// Preconditioner stages of a shot: 0 = the full scale s0 exp(o) (s0 = the
// fixed scale or 1, exp(o) only when the network runs), 1 = s0 alone (only
// when the network runs), 2 = plain CG (1).  A shot moves down the stages
// when its preconditioner is given up.
__device__ __forceinline__ int next_stage(int st, bool has_net) { return (st == 0 && has_net) ? 1 : 2; }

__device__ __forceinline__ float stage_scale(int st, const float* o, const float* fixed, int s, int iz, int ix,
                                             int nz, int nx, int Hp, int Wp) {
    if (st == 2) return 1.f;
    const float f = fixed ? fixed[((int64_t)s * nz + iz) * nx + ix] : 1.f;
    return (st == 0 && o) ? f * expf(o[((int64_t)s * Hp + iz) * Wp + ix]) : f;
}

// zr[3 s + st] = sum_x scale_st(x) a(x) = z.r for each stage st.
__global__ __launch_bounds__(NT) void k_fcg_zr(const float* __restrict__ o, const float* __restrict__ fixed,
                                               const float* __restrict__ a, int nz, int nx, int Hp, int Wp,
                                               double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.y, b = blockIdx.x, bps = gridDim.x;
    const int64_t n = (int64_t)nz * nx;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t x = (int64_t)b * NT + threadIdx.x; x < n; x += (int64_t)bps * NT) {
        const int iz = (int)(x / nx), ix = (int)(x % nx);
        const double av = a[(int64_t)s * n + x];
        for (int st = 0; st < 3; ++st) acc[st] += (double)stage_scale(st, o, fixed, s, iz, ix, nz, nx, Hp, Wp) * av;
    }
    for (int st = 0; st < 3; ++st) {
        const double t = block_sum_d(acc[st], sm);
        if (threadIdx.x == 0) part[(int64_t)(3 * s + st) * bps + b] = t;
    }
}

__device__ __forceinline__ void leave_stage(int s, int k, bool has_net, int* mode, int* restart, int* fallback,
                                            int* cg_at) {
    const int st = next_stage(mode[s], has_net);
    if (fallback[s] < 0) fallback[s] = k;
    if (st == 2) cg_at[s] = k;
    mode[s] = st;
    restart[s] = 1;
}

// A shot whose preconditioned residual is not a descent direction (z.r <= 0
// or not finite) gives up that preconditioner after iteration k, moving down
// the stages until one is usable (plain CG always is); a switch restarts the
// direction and the stall window.
__global__ void k_fcg_check(const double* __restrict__ zr, const int* __restrict__ active, int* __restrict__ mode,
                            int* __restrict__ restart, int* __restrict__ fallback, int* __restrict__ cg_at,
                            double* __restrict__ best, int* __restrict__ kbest, const double* __restrict__ hist,
                            int hstride, int k, int has_net, int n) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || !active[s]) return;
    bool moved = false;
    while (mode[s] < 2) {
        const double z = zr[3 * s + mode[s]];
        if (isfinite(z) && z > 0.0) break;
        leave_stage(s, k, has_net != 0, mode, restart, fallback, cg_at);
        moved = true;
    }
    if (moved && k > 0) {
        kbest[s] = k;
        best[s] = hist[(int64_t)s * hstride + k];
    }
}

// S[s][x] = the scale of the shot's current stage.
__global__ void k_fcg_scale(const float* __restrict__ o, const float* __restrict__ fixed,
                            const int* __restrict__ mode, float* __restrict__ S, int ns, int nz, int nx, int Hp,
                            int Wp) {
    const int64_t n = (int64_t)nz * nx;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < ns * n; i += (int64_t)gridDim.x * NT) {
        const int s = (int)(i / n);
        const int64_t x = i % n;
        S[i] = stage_scale(mode[s], o, fixed, s, (int)(x / nx), (int)(x % nx), nz, nx, Hp, Wp);
    }
}

// p[s][t][x] = S[s][x] r[s][t][x]
__global__ void k_scale_vec(float* __restrict__ p, const float* __restrict__ r, const float* __restrict__ S,
                            int ns, int nt, int64_t nphys) {
    const int64_t len = (int64_t)nt * nphys;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < ns * len; i += (int64_t)gridDim.x * NT) {
        const int s = (int)(i / len);
        p[i] = r[i] * S[(int64_t)s * nphys + (i % len) % nphys];
    }
}

// The residual update of a flexible CG iteration, one thread per cell walking
// the time axis: r -= alpha Np, and per cell the FP64 sums over t of r^2 (for
// z.r and the network's input) and of r Np (for z.Np, since z = s r with s
// constant in time).  part[s][b] = block sums of r^2.  A thread owns CPT cells
// 64 apart, so that a wave reads and writes 64 * CPT consecutive floats of a
// time step (1 KB runs of each vector instead of 256 B ones).
constexpr int CPT = 4;
__global__ __launch_bounds__(NT) void k_r_update_cells(float* __restrict__ r, const float* __restrict__ Np,
                                                       const double* __restrict__ alpha,
                                                       const int* __restrict__ active, int nt, int64_t nphys,
                                                       float* __restrict__ en, double* __restrict__ rnp,
                                                       double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.y, b = blockIdx.x, bps = gridDim.x;
    if (active && !active[s]) {   // uniform over the block
        if (threadIdx.x == 0) part[(int64_t)s * bps + b] = 0.0;
        return;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t c0 = ((int64_t)b * (NT / 64) + wv) * 64 * CPT + lane;   // cells c0 + 64 j
    const float al = (float)alpha[s];
    float* rs = r + (int64_t)s * nt * nphys;
    const float* as = Np + (int64_t)s * nt * nphys;
    double e[CPT], g[CPT];
    bool on[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        e[j] = 0.0;
        g[j] = 0.0;
        on[j] = c0 + 64 * j < nphys;
    }
    // U steps at a time: every load of the chunk is issued before its stores
    constexpr int U = 4;
    for (int t0 = 0; t0 < nt; t0 += U) {
        float rv[U][CPT], av[U][CPT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t o = (int64_t)(t0 + u) * nphys + c0;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const bool ld = on[j] && t0 + u < nt;
                rv[u][j] = ld ? rs[o + 64 * j] : 0.f;
                av[u][j] = ld ? as[o + 64 * j] : 0.f;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t o = (int64_t)(t0 + u) * nphys + c0;
#pragma unroll
            for (int j = 0; j < CPT; ++j) {
                const float v = fmaf(-al, av[u][j], rv[u][j]);
                if (on[j] && t0 + u < nt) rs[o + 64 * j] = v;
                e[j] += (double)v * (double)v;
                g[j] += (double)v * (double)av[u][j];
            }
        }
    }
    double tot = 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        if (on[j]) {
            en[(int64_t)s * nphys + c0 + 64 * j] = (float)e[j];
            rnp[(int64_t)s * nphys + c0 + 64 * j] = g[j];
        }
        tot += e[j];
    }
    tot = block_sum_d(tot, sm);
    if (threadIdx.x == 0) part[(int64_t)s * bps + b] = tot;
}

// part[s][b] = block sums of S[s][x] g[s][x].
__global__ __launch_bounds__(NT) void k_dot_cells(const float* __restrict__ S, const double* __restrict__ g,
                                                  int64_t nphys, double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.y, b = blockIdx.x, bps = gridDim.x;
    double acc = 0.0;
    for (int64_t x = (int64_t)b * NT + threadIdx.x; x < nphys; x += (int64_t)bps * NT)
        acc += (double)S[(int64_t)s * nphys + x] * g[(int64_t)s * nphys + x];
    const double tot = block_sum_d(acc, sm);
    if (threadIdx.x == 0) part[(int64_t)s * bps + b] = tot;
}

// beta = -z.Np / p.Np, or 0 when the direction restarts.
__global__ void k_fcg_beta(const double* __restrict__ zAp, const double* __restrict__ pAp,
                           const int* __restrict__ restart, double* __restrict__ beta, int n) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) beta[s] = restart[s] ? 0.0 : -zAp[s] / pAp[s];
}

__global__ void k_fcg_init(int* __restrict__ mode, int* __restrict__ restart, int* __restrict__ fallback,
                           int* __restrict__ cg_at, double* __restrict__ best, int* __restrict__ kbest, int n) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) {
        mode[s] = 0;
        restart[s] = 0;
        fallback[s] = -1;
        cg_at[s] = -1;
        best[s] = 1.0;
        kbest[s] = 0;
    }
}

// After iteration k of every active shot: the stopping test of k_cg_control,
// then the stall test of the flexible iteration (no new best ||r|| by the
// factor `stall` for `window` iterations: plain CG takes over, the direction
// restarts).  best / kbest: best relative residual so far and its iteration.
__global__ void k_fcg_control(const double* __restrict__ rr0, const double* __restrict__ rr_new,
                              const double* __restrict__ pAp, int* __restrict__ active, int* __restrict__ finish,
                              int* __restrict__ iters, int* __restrict__ status, double* __restrict__ hist,
                              int hstride, int* __restrict__ ctl, double rtol, int max_iter, int* __restrict__ mode,
                              int* __restrict__ restart, int* __restrict__ fallback, int* __restrict__ cg_at,
                              double stall, int window, double* __restrict__ best, int* __restrict__ kbest,
                              int has_net, int n) {
    __shared__ int cnt;
    const int k = ctl[0];
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        int f = 0;
        restart[s] = 0;
        if (active[s]) {
            iters[s] = k + 1;
            const double a = pAp[s], b = rr_new[s];
            const double rel = sqrt(b / rr0[s]);
            double* h = hist + (int64_t)s * hstride;
            h[k + 1] = rel;
            if (!isfinite(a) || !isfinite(b)) {
                status[s] = (int)ESI_ERR_NONFINITE;
                f = 2;
            } else if (a <= 0.0) {
                status[s] = (int)ESI_ERR_BREAKDOWN;
                f = 2;
            } else if (rel < rtol || k == max_iter - 1) {
                f = 1;
            } else {
                if (rel < stall * best[s]) {
                    best[s] = rel;
                    kbest[s] = k + 1;
                }
                if (mode[s] < 2 && k + 1 - kbest[s] >= window) {
                    leave_stage(s, k + 1, has_net != 0, mode, restart, fallback, cg_at);
                    kbest[s] = k + 1;
                    best[s] = rel;
                }
            }
            if (f) active[s] = 0;
            else atomicAdd(&cnt, 1);
        }
        finish[s] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ctl[0] = k + 1;
        ctl[1] = cnt;
    }
}

}  // namespace

esi_status_t launch_energy(Plan* P, const float* r, const int* active, float* a, int ns) {
    hipLaunchKernelGGL(k_energy, dim3(grid_for((int64_t)ns * P->nphys)), dim3(NT), 0, P->stream, r, active, a, ns,
                       P->nt, P->nphys);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_stats(Plan* P, const float* r, const float* x, const float* p, const double* alpha,
                          const float* xref, const int* iters, int k, float* out, int ns) {
    hipLaunchKernelGGL(k_stats, dim3(grid_for((int64_t)ns * P->nphys)), dim3(NT), 0, P->stream, r, x, p, alpha,
                       xref, iters, k, out, ns, P->nt, P->nphys);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_features(Plan* P, int shot0, int ns, const float* a, const float* c, double* mean, int Hp,
                             int Wp, const float* base, float* xin, float* apad, float* cpad) {
    hipLaunchKernelGGL(k_feat_mean, dim3(ns), dim3(NT), 0, P->stream, a, P->nphys, P->nt, mean);
    hipLaunchKernelGGL(k_features, dim3(grid_for((int64_t)ns * Hp * Wp)), dim3(NT), 0, P->stream, a, c, mean,
                       P->vphys, P->d_src, shot0, (float)P->b_eps, ns, P->nz, P->nx, Hp, Wp, P->nt, base, xin,
                       apad, cpad);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_fcg_zr_check_scale(Plan* P, const float* o, const float* fixed, const float* a,
                                       const int* active, int* mode, int* restart, int* fallback, int* cg_at,
                                       double* best, int* kbest, const double* hist, int hstride, int k,
                                       int Hp, int Wp, double* zr, float* S, int ns) {
    const int bps = cell_blocks(P->nphys);
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)3 * bps * ns, P->stream));
    hipLaunchKernelGGL(k_fcg_zr, dim3(bps, ns), dim3(NT), 0, P->stream, o, fixed, a, P->nz, P->nx, Hp, Wp, P->part);
    ESI_TRY(launch_reduce_parts(P, P->part, bps, 3 * ns, zr));      // zr[s][stage]
    hipLaunchKernelGGL(k_fcg_check, dim3((ns + 63) / 64), dim3(64), 0, P->stream, zr, active, mode, restart,
                       fallback, cg_at, best, kbest, hist, hstride, k, o ? 1 : 0, ns);
    hipLaunchKernelGGL(k_fcg_scale, dim3(grid_for((int64_t)ns * P->nphys)), dim3(NT), 0, P->stream, o, fixed,
                       mode, S, ns, P->nz, P->nx, Hp, Wp);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_scale_vec(Plan* P, float* p, const float* r, const float* S, int ns) {
    hipLaunchKernelGGL(k_scale_vec, dim3(grid_for((int64_t)ns * P->nt * P->nphys)), dim3(NT), 0, P->stream, p, r,
                       S, ns, P->nt, P->nphys);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_r_update_cells(Plan* P, float* r, const float* Np, const double* alpha, const int* active,
                                   int ns, float* en, double* rnp, double* rr_out) {
    const int bps = (int)((P->nphys + NT * CPT - 1) / (NT * CPT));
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)bps * ns, P->stream));
    hipLaunchKernelGGL(k_r_update_cells, dim3(bps, ns), dim3(NT), 0, P->stream, r, Np, alpha, active, P->nt,
                       P->nphys, en, rnp, P->part);
    ESI_HIP_TRY(hipGetLastError());
    return launch_reduce_parts(P, P->part, bps, ns, rr_out);
}

esi_status_t launch_dot_cells(Plan* P, const float* S, const double* g, int ns, double* out) {
    const int bps = cell_blocks(P->nphys);
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)bps * ns, P->stream));
    hipLaunchKernelGGL(k_dot_cells, dim3(bps, ns), dim3(NT), 0, P->stream, S, g, P->nphys, P->part);
    ESI_HIP_TRY(hipGetLastError());
    return launch_reduce_parts(P, P->part, bps, ns, out);
}

esi_status_t launch_fcg_beta(Plan* P, const double* zAp, const double* pAp, const int* restart, double* beta,
                             int ns) {
    hipLaunchKernelGGL(k_fcg_beta, dim3((ns + 63) / 64), dim3(64), 0, P->stream, zAp, pAp, restart, beta, ns);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_fcg_init(Plan* P, int* mode, int* restart, int* fallback, int* cg_at, double* best, int* kbest,
                             int ns) {
    hipLaunchKernelGGL(k_fcg_init, dim3((ns + 63) / 64), dim3(64), 0, P->stream, mode, restart, fallback, cg_at,
                       best, kbest, ns);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_fcg_control(Plan* P, const double* rr0, const double* rr_new, const double* pAp, int* active,
                                int* finish, int* iters, int* status, double* hist, int hstride, int* ctl,
                                double rtol, int max_iter, int* mode, int* restart, int* fallback, int* cg_at,
                                double stall, int window, double* best, int* kbest, bool has_net, int ns) {
    hipLaunchKernelGGL(k_fcg_control, dim3(1), dim3(256), 0, P->stream, rr0, rr_new, pAp, active, finish, iters,
                       status, hist, hstride, ctl, rtol, max_iter, mode, restart, fallback, cg_at, stall, window,
                       best, kbest, has_net ? 1 : 0, ns);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

}  // namespace esi
