// CG vector kernels (Algorithm 1): fills, copies, the fused residual update
// with its float64 squared-norm partials, fixed-order float64 reductions, the
// per-shot step lengths, and the shot-sum of gradient accumulators.
//
// Every reduction is two-pass with a fixed summation order (per-block partials
// in float64, then one block per shot), so results are bitwise reproducible.
#include <algorithm>

#include "esi_internal.h"

namespace esi {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ double block_sum(double v, double* sm) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sm[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sm[i];
    __syncthreads();
    return s;   // valid in thread 0
}

__global__ void k_fill(float* __restrict__ p, int64_t n, float v) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        p[i] = v;
}

__global__ void k_fill_d(double* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        p[i] = 0.0;
}

__global__ void k_copy(float* __restrict__ d, const float* __restrict__ s, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        d[i] = s[i];
}

__global__ void k_sub(float* __restrict__ d, const float* __restrict__ a, const float* __restrict__ b,
                      int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        d[i] = a[i] - b[i];
}

// grid: (bps, nshots).  r -= alpha_s Ap; part[s][b] = sum r^2 over the block's chunk.
// Chunks are multiples of 4 elements so the body runs on float4 when the
// shot's slice is 16-byte aligned.
__global__ __launch_bounds__(NT) void k_r_update(float* __restrict__ r, const float* __restrict__ Ap,
                                                 const double* __restrict__ alpha,
                                                 const int* __restrict__ active, int64_t len,
                                                 double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.y, b = blockIdx.x, bps = gridDim.x;
    if (active && !active[s]) {
        if (threadIdx.x == 0) part[(int64_t)s * bps + b] = 0.0;
        return;
    }
    const float al = (float)alpha[s];
    const int64_t chunk = ((len + bps - 1) / bps + 3) & ~(int64_t)3;
    const int64_t beg = min(len, (int64_t)b * chunk), end = min(len, beg + chunk);
    float* rs = r + (int64_t)s * len;
    const float* as = Ap + (int64_t)s * len;
    double acc = 0.0;
    const bool vec = ((reinterpret_cast<uintptr_t>(rs) | reinterpret_cast<uintptr_t>(as)) & 15) == 0;
    int64_t i0 = beg;
    if (vec) {
        const int64_t nv = (end - beg) >> 2;
        float4* r4 = reinterpret_cast<float4*>(rs + beg);
        const float4* a4 = reinterpret_cast<const float4*>(as + beg);
        for (int64_t k = threadIdx.x; k < nv; k += NT) {
            float4 v = r4[k];
            const float4 w = a4[k];
            v.x = fmaf(-al, w.x, v.x); v.y = fmaf(-al, w.y, v.y);
            v.z = fmaf(-al, w.z, v.z); v.w = fmaf(-al, w.w, v.w);
            r4[k] = v;
            acc += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
        }
        i0 = beg + 4 * nv;
    }
    for (int64_t i = i0 + threadIdx.x; i < end; i += NT) {
        const float v = fmaf(-al, as[i], rs[i]);
        rs[i] = v;
        acc += (double)v * (double)v;
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[(int64_t)s * bps + b] = t;
}

// grid: (bps, nshots).  part[s][b] = sum a.b over the block's chunk.
__global__ __launch_bounds__(NT) void k_dot(const float* __restrict__ x, const float* __restrict__ y,
                                            int64_t len, double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.y, b = blockIdx.x, bps = gridDim.x;
    const int64_t chunk = (len + bps - 1) / bps;
    const int64_t beg = (int64_t)b * chunk, end = min(len, beg + chunk);
    const float* xs = x + (int64_t)s * len;
    const float* ys = y + (int64_t)s * len;
    double acc = 0.0;
    for (int64_t i = beg + threadIdx.x; i < end; i += NT) acc += (double)xs[i] * (double)ys[i];
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[(int64_t)s * bps + b] = t;
}

// one block per shot: out[s] = sum_b part[s][b] in a fixed order
__global__ __launch_bounds__(NT) void k_reduce(const double* __restrict__ part, int64_t n,
                                               double* __restrict__ out) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += NT) acc += part[(int64_t)s * n + i];
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) out[s] = t;
}

__global__ void k_axpy_flag(float* __restrict__ x, const float* __restrict__ p,
                            const double* __restrict__ alpha, const int* __restrict__ flag, int which,
                            int64_t len) {
    const int s = blockIdx.y;
    if (flag[s] != which) return;
    const float al = (float)alpha[s];
    float* xs = x + (int64_t)s * len;
    const float* ps = p + (int64_t)s * len;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < len; i += (int64_t)gridDim.x * NT)
        xs[i] = fmaf(al, ps[i], xs[i]);
}

__global__ void k_cg_alpha(const double* rr, const double* pAp, double* alpha, int n) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) alpha[s] = rr[s] / pAp[s];
}

// grid (DATA_BLOCKS, nshots): part[s][b] = block sums of d^2 over shot s's
// traces (the data of shots shot0.. back to back, nt samples per receiver)
__global__ __launch_bounds__(NT) void k_data_sq(const float* __restrict__ d, const int64_t* __restrict__ rec_ptr,
                                                int shot0, int nt, const int* __restrict__ active,
                                                double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    const int s = blockIdx.y;
    double acc = 0.0;
    if (!active || active[s]) {   // uniform over the block
        const int64_t base = rec_ptr[shot0];
        const int64_t beg = (int64_t)nt * (rec_ptr[shot0 + s] - base);
        const int64_t end = (int64_t)nt * (rec_ptr[shot0 + s + 1] - base);
        for (int64_t i = beg + blockIdx.x * (int64_t)NT + threadIdx.x; i < end; i += (int64_t)gridDim.x * NT)
            acc += (double)d[i] * (double)d[i];
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[(int64_t)s * gridDim.x + blockIdx.x] = t;
}

// pAp = beta B^2 p.p (in pAp) + ||S p||^2 (in dsq); alpha = rr / pAp
__global__ void k_cg_alpha_data(const double* rr, double* pAp, const double* dsq, double* alpha, int n) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) {
        const double v = pAp[s] + dsq[s];
        pAp[s] = v;
        alpha[s] = rr[s] / v;
    }
}

__global__ void k_cg_beta(const double* rr_new, double* rr, double* beta, int n) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) {
        beta[s] = rr_new[s] / rr[s];
        rr[s] = rr_new[s];
    }
}

// Device-side bookkeeping of Algorithm 1's stopping test, so that an iteration
// needs no host decision and can be replayed from a captured graph.
// ctl[0] = iterations done, ctl[1] = shots still iterating.  One workgroup.
__global__ void k_cg_init(const double* __restrict__ rr0, int* __restrict__ active,
                          int* __restrict__ finish, int* __restrict__ iters,
                          int* __restrict__ status, double* __restrict__ hist, int hstride,
                          int* __restrict__ ctl, int n) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        const double v = rr0[s];
        const bool ok = isfinite(v);
        const int a = (ok && v > 0.0) ? 1 : 0;   // b = 0: x = 0 is exact
        active[s] = a;
        finish[s] = 0;
        iters[s] = 0;
        status[s] = ok ? 0 : (int)ESI_ERR_NONFINITE;
        hist[(int64_t)s * hstride] = 1.0;
        for (int k = 1; k < hstride; ++k) hist[(int64_t)s * hstride + k] = -1.0;
        if (a) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ctl[0] = 0;
        ctl[1] = cnt;
    }
}

// After iteration k (= ctl[0]) of every active shot: record ||r_{k+1}|| / ||r_0||,
// flag shots that converged or reached max_iter (finish = 1: they take their
// last update x += alpha p) or broke down (finish = 2: x stays at x_k), and
// retire them.
__global__ void k_cg_control(const double* __restrict__ rr0, const double* __restrict__ rr_new,
                             const double* __restrict__ pAp, int* __restrict__ active,
                             int* __restrict__ finish, int* __restrict__ iters,
                             int* __restrict__ status, double* __restrict__ hist, int hstride,
                             int* __restrict__ ctl, double rtol, int max_iter, int n) {
    __shared__ int cnt;
    const int k = ctl[0];
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < n; s += blockDim.x) {
        int f = 0;
        if (active[s]) {
            iters[s] = k + 1;
            const double a = pAp[s], b = rr_new[s];
            const double rel = sqrt(b / rr0[s]);
            hist[(int64_t)s * hstride + k + 1] = rel;
            if (!isfinite(a) || !isfinite(b)) {
                status[s] = (int)ESI_ERR_NONFINITE;
                f = 2;
            } else if (a <= 0.0) {
                status[s] = (int)ESI_ERR_BREAKDOWN;
                f = 2;
            } else if (rel < rtol || k == max_iter - 1) {
                f = 1;
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

__global__ void k_sum_shots(const float* __restrict__ g, int nshots, int64_t len, float sign,
                            float* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < len; i += (int64_t)gridDim.x * NT) {
        float acc = 0.f;
        for (int s = 0; s < nshots; ++s) acc += g[(int64_t)s * len + i];
        out[i] += sign * acc;
    }
}

// out[s][n] = dense[s][n][cell of shot s's source]
__global__ void k_trace_at_src(const float* __restrict__ dense, const int32_t* __restrict__ src,
                               int shot0, int nshots, int nt, int nz, int ny, int nx, int ndim,
                               float* __restrict__ out) {
    const int64_t nphys = (int64_t)nz * ny * nx;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < (int64_t)nshots * nt;
         i += (int64_t)gridDim.x * NT) {
        const int s = (int)(i / nt), n = (int)(i - (int64_t)s * nt);
        const int32_t* ps = src + (shot0 + s) * 3;
        const int64_t cell = ((int64_t)ps[1] * ny + (ndim == 3 ? ps[2] : 0)) * nx + ps[0];
        out[i] = dense[((int64_t)s * nt + n) * nphys + cell];
    }
}

// grid: (blocks, nshots): dst[s*ds + i] = src[s*ss + i], i < n
__global__ void k_copy_shots(float* __restrict__ d, int64_t ds, const float* __restrict__ src,
                             int64_t ss, int64_t n) {
    const int s = blockIdx.y;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        d[s * ds + i] = src[s * ss + i];
}

// grid: (blocks, nshots): the part of shot s's field that a shot with an
// aperture ever makes non-zero, rows [row0, row0 + nrows) of storage columns
// [win[2 gs] + clo, win[2 gs + 1] + chi), gs = shot0 + s; the rest of its
// fields stays zero (no velocity outside the window and its absorbing layer)
__global__ void k_copy_shots_win(float* __restrict__ d, int64_t ds, const float* __restrict__ src, int64_t ss,
                                 int XS, int row0, int nrows, const int32_t* __restrict__ win, int shot0,
                                 int clo, int chi) {
    const int s = blockIdx.y;
    const int c0 = win[2 * (shot0 + s)] + clo, w = win[2 * (shot0 + s) + 1] + chi - c0;
    const int n = nrows * w;
    for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) {
        const int r = i / w;
        const int64_t o = (int64_t)(row0 + r) * XS + c0 + (i - r * w);
        d[s * ds + o] = src[s * ss + o];
    }
}

__global__ void k_grad_velocity(const float* __restrict__ v, const float* gm, float* gv, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const float vi = v[i];
        gv[i] = -2.f * gm[i] / (vi * vi * vi);
    }
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 8192)); }

int bps_for(int64_t len) { return (int)std::max<int64_t>(1, std::min<int64_t>(512, (len + 4095) / 4096)); }

}  // namespace

esi_status_t launch_fill(Plan* P, float* p, int64_t n, float v) {
    if (n <= 0) return ESI_OK;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(NT), 0, P->stream, p, n, v);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

// zero a float64 array with a kernel (no memset nodes: calls may be captured)
esi_status_t launch_fill_d(Plan* P, double* p, int64_t n) {
    if (n <= 0) return ESI_OK;
    hipLaunchKernelGGL(k_fill_d, dim3(grid_for(n)), dim3(NT), 0, P->stream, p, n);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_copy(Plan* P, float* dst, const float* src, int64_t n) {
    if (n <= 0) return ESI_OK;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(NT), 0, P->stream, dst, src, n);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_copy_shots(Plan* P, float* dst, int64_t dst_stride, const float* src,
                               int64_t src_stride, int64_t n, int nshots) {
    if (n <= 0) return ESI_OK;
    const int g = (int)std::min<int64_t>(std::max<int64_t>(1, (n + NT - 1) / NT), 2048);
    hipLaunchKernelGGL(k_copy_shots, dim3(g, nshots), dim3(NT), 0, P->stream, dst, dst_stride, src,
                       src_stride, n);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_copy_fields(Plan* P, float* dst, int64_t dst_stride, const float* src, int64_t src_stride,
                                int shot0, int nshots) {
    if (!P->d_win || P->ndim != 2)
        return launch_copy_shots(P, dst, dst_stride, src, src_stride, P->fsize, nshots);
    // padded columns [lo, hi + 2 nb) of the window, storage column = padded + GH
    const int64_t n = (int64_t)P->nzp * P->nxp;   // bound of a window's cells
    const int g = (int)std::min<int64_t>(std::max<int64_t>(1, (n + NT - 1) / NT), 2048);
    hipLaunchKernelGGL(k_copy_shots_win, dim3(g, nshots), dim3(NT), 0, P->stream, dst, dst_stride, src,
                       src_stride, P->XS, GH, P->nzp, (const int32_t*)P->d_win, shot0, GH, 2 * P->nb + GH);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_sub(Plan* P, float* out, const float* a, const float* b, int64_t n) {
    if (n <= 0) return ESI_OK;
    hipLaunchKernelGGL(k_sub, dim3(grid_for(n)), dim3(NT), 0, P->stream, out, a, b, n);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_reduce_parts(Plan* P, const double* part, int64_t n, int nshots, double* out) {
    hipLaunchKernelGGL(k_reduce, dim3(nshots), dim3(NT), 0, P->stream, part, n, out);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_r_update(Plan* P, float* r, const float* Ap, const double* alpha,
                             const int* active, int nshots, int64_t len, double* rr_out) {
    const int bps = bps_for(len);
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)bps * nshots, P->stream));
    hipLaunchKernelGGL(k_r_update, dim3(bps, nshots), dim3(NT), 0, P->stream, r, Ap, alpha, active,
                       len, P->part);
    ESI_HIP_TRY(hipGetLastError());
    return launch_reduce_parts(P, P->part, bps, nshots, rr_out);
}

esi_status_t launch_dot(Plan* P, const float* x, const float* y, int nshots, int64_t len,
                        double* out) {
    const int bps = bps_for(len);
    ESI_TRY(grow_t(&P->part, &P->part_cap, (int64_t)bps * nshots, P->stream));
    hipLaunchKernelGGL(k_dot, dim3(bps, nshots), dim3(NT), 0, P->stream, x, y, len, P->part);
    ESI_HIP_TRY(hipGetLastError());
    return launch_reduce_parts(P, P->part, bps, nshots, out);
}

esi_status_t launch_axpy_flag(Plan* P, float* x, const float* p, const double* alpha,
                              const int* flag, int which, int nshots, int64_t len) {
    // about 8192 workgroups over all shots: enough to stream the shots that
    // do update, few enough that the launch costs little when none does
    // (most iterations: the blocks of the other shots return at once)
    const int per = std::max(64, 8192 / std::max(1, nshots));
    const int g = (int)std::min<int64_t>(std::max<int64_t>(1, (len + NT - 1) / NT), per);
    hipLaunchKernelGGL(k_axpy_flag, dim3(g, nshots), dim3(NT), 0, P->stream, x, p, alpha, flag, which,
                       len);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_cg_alpha(Plan* P, const double* rr, const double* pAp, double* alpha,
                             int nshots) {
    hipLaunchKernelGGL(k_cg_alpha, dim3((nshots + 63) / 64), dim3(64), 0, P->stream, rr, pAp, alpha,
                       nshots);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_cg_alpha_data(Plan* P, int shot0, int nshots, const float* data, const int* active,
                                  const double* rr, double* pAp, double* tmp, double* alpha) {
    if (P->part_cap < (int64_t)DATA_BLOCKS * nshots) return fail(ESI_ERR_ARG, "internal: partials too small");
    hipLaunchKernelGGL(k_data_sq, dim3(DATA_BLOCKS, nshots), dim3(NT), 0, P->stream, data, P->d_rec_ptr, shot0,
                       P->nt, active, P->part);
    ESI_HIP_TRY(hipGetLastError());
    ESI_TRY(launch_reduce_parts(P, P->part, DATA_BLOCKS, nshots, tmp));
    hipLaunchKernelGGL(k_cg_alpha_data, dim3((nshots + 63) / 64), dim3(64), 0, P->stream, rr, pAp, tmp, alpha,
                       nshots);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_cg_beta(Plan* P, const double* rr_new, double* rr, double* beta, int nshots) {
    hipLaunchKernelGGL(k_cg_beta, dim3((nshots + 63) / 64), dim3(64), 0, P->stream, rr_new, rr, beta,
                       nshots);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_cg_init(Plan* P, const double* rr0, int* active, int* finish, int* iters,
                            int* status, double* hist, int hstride, int* ctl, int nshots) {
    hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(256), 0, P->stream, rr0, active, finish, iters,
                       status, hist, hstride, ctl, nshots);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_cg_control(Plan* P, const double* rr0, const double* rr_new, const double* pAp,
                               int* active, int* finish, int* iters, int* status, double* hist,
                               int hstride, int* ctl, double rtol, int max_iter, int nshots) {
    hipLaunchKernelGGL(k_cg_control, dim3(1), dim3(256), 0, P->stream, rr0, rr_new, pAp, active,
                       finish, iters, status, hist, hstride, ctl, rtol, max_iter, nshots);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_sum_shots(Plan* P, const float* gacc, int nshots, int64_t len, float sign,
                              float* grad) {
    hipLaunchKernelGGL(k_sum_shots, dim3(grid_for(len)), dim3(NT), 0, P->stream, gacc, nshots, len,
                       sign, grad);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_grad_velocity(Plan* P, const float* vel, const float* gm, float* gv, int64_t n) {
    if (n <= 0) return ESI_OK;
    hipLaunchKernelGGL(k_grad_velocity, dim3(grid_for(n)), dim3(NT), 0, P->stream, vel, gm, gv, n);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t launch_trace_at_src(Plan* P, const float* dense, int shot0, int nshots, float* out) {
    hipLaunchKernelGGL(k_trace_at_src, dim3(grid_for((int64_t)nshots * P->nt)), dim3(NT), 0,
                       P->stream, dense, P->d_src, shot0, nshots, P->nt, P->nz, P->ny, P->nx,
                       P->ndim, out);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

}  // namespace esi
