// The outer loop of Algorithm 2 (nested loops for variable projection between
// m = 1/v^2 and the extended source q): per outer iteration the inner CG solve
// of every shot, the PENALTY gradient, an L-BFGS direction (two-loop
// recursion, Nocedal & Wright Algorithm 7.4) and a backtracking Armijo line
// search on the model clipped to velocity bounds; the penalty beta can follow
// the discrepancy principle (Sec. 2.4).  The model-space vectors are FP64 on
// the device; every reduction runs in a fixed order, so a run is reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "esi_internal.h"

namespace esi {
namespace {

constexpr int NT = 256;
constexpr int RB = 256;   // blocks of a reduction; partials summed on the host in order

__device__ __forceinline__ double block_sum(double v, double* sm) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < NT / 64; ++k) t += sm[k];
    return t;
}

// part[b] = block sums of a[i] * (b1[i] - b0[i]) (b0 may be null).
template <class TA, class TB>
__global__ __launch_bounds__(NT) void k_dot_diff(const TA* __restrict__ a, const TB* __restrict__ b1,
                                                 const TB* __restrict__ b0, int64_t n, double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double d = b0 ? (double)b1[i] - (double)b0[i] : (double)b1[i];
        acc += (double)a[i] * d;
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// part[b] = block sums of (a[i] - b[i])^2 (b may be null).
__global__ __launch_bounds__(NT) void k_sqdiff(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                                               double* __restrict__ part) {
    __shared__ double sm[NT / 64];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double d = b ? (double)a[i] - (double)b[i] : (double)a[i];
        acc += d * d;
    }
    const double t = block_sum(acc, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// part[b] = block maxima of |a[i]| (absolute) or a[i] (signed).
__global__ __launch_bounds__(NT) void k_max_d(const double* __restrict__ a, int64_t n, int absolute,
                                              double* __restrict__ part) {
    __shared__ double sm[NT];
    double m = -INFINITY;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        m = fmax(m, absolute ? fabs(a[i]) : a[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// m = clip(1 / v^2)
__global__ void k_m_from_vel(const float* __restrict__ v, double lo, double hi, double* __restrict__ m, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const double vv = (double)v[i];
        m[i] = fmin(fmax(1.0 / (vv * vv), lo), hi);
    }
}

__global__ void k_vel_from_m(const double* __restrict__ m, float* __restrict__ v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        v[i] = (float)(1.0 / sqrt(m[i]));
}

// mt = clip(m + alpha d)
__global__ void k_trial(const double* __restrict__ m, const double* __restrict__ d, double alpha, double lo,
                        double hi, double* __restrict__ mt, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        mt[i] = fmin(fmax(m[i] + alpha * d[i], lo), hi);
}

// s[k][x] = 1 / (beta B^2 + gamma), B = |x - x_s| + b_eps in cells, for shots s0 + k
__global__ void k_cell_scale(const int32_t* __restrict__ src, int s0, int ns, int nz, int nx, double beta,
                             double b_eps, double gamma, float* __restrict__ out) {
    const int64_t n = (int64_t)nz * nx;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < ns * n; i += (int64_t)gridDim.x * NT) {
        const int k = (int)(i / n);
        const int64_t c = i - k * n;
        const int iz = (int)(c / nx), ix = (int)(c - (int64_t)iz * nx);
        const double dx = ix - src[(s0 + k) * 3 + 0], dz = iz - src[(s0 + k) * 3 + 1];
        const double b = sqrt(dx * dx + dz * dz) + b_eps;
        out[i] = (float)(1.0 / (beta * b * b + gamma));
    }
}

// g = gm (* mask)
__global__ void k_grad_d(const float* __restrict__ gm, const float* __restrict__ mask, double* __restrict__ g,
                         int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        g[i] = mask ? (double)gm[i] * (double)mask[i] : (double)gm[i];
}

// out = a * x + b * y
__global__ void k_axpby_d(double* __restrict__ out, double a, const double* __restrict__ x, double b,
                          const double* __restrict__ y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        out[i] = y ? a * x[i] + b * y[i] : a * x[i];
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 4096)); }

// Device buffers of one call, freed when it returns.
struct Scratch {
    std::vector<void*> bufs;
    hipStream_t stream = nullptr;
    ~Scratch() {
        if (stream) hipStreamSynchronize(stream);
        for (void* b : bufs) hipFree(b);
    }
    template <class T>
    esi_status_t alloc(T** p, int64_t n) {
        *p = nullptr;
        ESI_HIP_TRY(hipMalloc((void**)p, std::max<int64_t>(n, 1) * sizeof(T)));
        bufs.push_back(*p);
        return ESI_OK;
    }
};

struct Outer {
    Plan* P;
    esi_plan_t plan;
    int shot0, ns, G;
    const float* d_obs;
    const float* wavelet;
    const float* mask;
    float* x;
    float* work;
    const esi_invert_opts_t* o;
    int64_t n;            // physical cells
    double* red;          // [RB] reduction partials
    float* vt;            // trial velocity
    float* gm;            // summed gradient (float)
    float* dsyn;          // synthetic data of a group
    float* dres;          // WRI right-hand side data of a group
    float* scale;         // inner FCG cell scale of a group [G][phys]
    float* dw;            // data-space inner solve: synthetic data of a group
    double* pen;          // [G] per-shot penalty sums
    double dd = 0.0;      // ||d_obs||^2

    esi_status_t host_sum(double* out) {
        std::vector<double> h(RB);
        ESI_HIP_TRY(hipMemcpyAsync(h.data(), red, RB * sizeof(double), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipStreamSynchronize(P->stream));
        double s = 0.0;
        for (double v : h) s += v;
        *out = s;
        return ESI_OK;
    }
    esi_status_t host_max(double* out) {
        std::vector<double> h(RB);
        ESI_HIP_TRY(hipMemcpyAsync(h.data(), red, RB * sizeof(double), hipMemcpyDeviceToHost, P->stream));
        ESI_HIP_TRY(hipStreamSynchronize(P->stream));
        double m = -INFINITY;
        for (double v : h) m = std::max(m, v);
        *out = m;
        return ESI_OK;
    }
    // a . (b1 - b0) over the model vector (b0 may be null)
    esi_status_t dot(const double* a, const double* b1, const double* b0, double* out) {
        hipLaunchKernelGGL((k_dot_diff<double, double>), dim3(RB), dim3(NT), 0, P->stream, a, b1, b0, n, red);
        ESI_HIP_TRY(hipGetLastError());
        return host_sum(out);
    }
    esi_status_t vmax(const double* a, bool absolute, double* out) {
        hipLaunchKernelGGL(k_max_d, dim3(RB), dim3(NT), 0, P->stream, a, n, absolute ? 1 : 0, red);
        ESI_HIP_TRY(hipGetLastError());
        return host_max(out);
    }
    esi_status_t sqdiff(const float* a, const float* b, int64_t len, double* out) {
        if (len == 0) {
            *out = 0.0;
            return ESI_OK;
        }
        hipLaunchKernelGGL(k_sqdiff, dim3(RB), dim3(NT), 0, P->stream, a, b, len, red);
        ESI_HIP_TRY(hipGetLastError());
        return host_sum(out);
    }
    esi_status_t axpby(double* out, double a, const double* xv, double b, const double* yv) {
        hipLaunchKernelGGL(k_axpby_d, dim3(grid_for(n)), dim3(NT), 0, P->stream, out, a, xv, b, yv, n);
        ESI_HIP_TRY(hipGetLastError());
        return ESI_OK;
    }
    int64_t doff(int s) const { return (int64_t)P->nt * (P->h_rec_ptr[s] - P->h_rec_ptr[shot0]); }

    // J, gradient g (FP64, masked) and relative data misfit at model m
    esi_status_t evaluate(const double* m, double beta, double* J, double* g, double* e) {
        P->beta = beta;
        hipLaunchKernelGGL(k_vel_from_m, dim3(grid_for(n)), dim3(NT), 0, P->stream, m, vt, n);
        ESI_HIP_TRY(hipGetLastError());
        ESI_TRY(esi_plan_set_model(plan, vt));
        ESI_TRY(launch_fill(P, gm, n, 0.f));
        double Jsum = 0.0, r2 = 0.0;
        for (int s0 = shot0; s0 < shot0 + ns; s0 += G) {
            const int k = std::min(G, shot0 + ns - s0);
            const float* dg = d_obs + doff(s0);
            const int64_t dl = doff(s0 + k) - doff(s0);
            const float* f = wavelet ? wavelet + (int64_t)(s0 - shot0) * P->nt : nullptr;
            const float* rhs = dg;
            if (f) {
                ESI_TRY(esi_data_residual(plan, s0, k, f, dg, dres));
                rhs = dres;
            }
            esi_cg_report_t rep;
            std::memset(&rep, 0, sizeof rep);
            if (o->inner == ESI_INNER_DATASPACE) {
                ESI_TRY(esi_ds_cg_solve(plan, s0, k, rhs, dw, x, work, o->cg_iters, o->cg_rtol, &rep));
            } else if (o->inner == ESI_INNER_FCG_SCALE) {
                hipLaunchKernelGGL(k_cell_scale, dim3(grid_for((int64_t)k * n)), dim3(NT), 0, P->stream, P->d_src,
                                   s0, k, P->nz, P->nx, beta, P->b_eps, o->inner_gamma, scale);
                ESI_HIP_TRY(hipGetLastError());
                ESI_TRY(esi_fpcg_solve(plan, s0, k, rhs, x, work, o->cg_iters, o->cg_rtol, nullptr, 0, scale, &rep));
            } else {
                ESI_TRY(esi_cg_solve(plan, s0, k, rhs, x, work, o->cg_iters, o->cg_rtol, &rep));
            }
            ESI_TRY(grow_t(&P->gshot, &P->gshot_cap, (int64_t)k * n, P->stream));
            ESI_TRY(launch_fill(P, P->gshot, (int64_t)k * n, 0.f));
            ESI_TRY(penalty_eval(P, s0, k, x, f, P->gshot, dsyn, pen));
            ESI_TRY(launch_sum_shots(P, P->gshot, k, n, 1.f, gm));
            double rg;
            ESI_TRY(sqdiff(dsyn, dg, dl, &rg));
            std::vector<double> hp(k);
            ESI_HIP_TRY(hipMemcpyAsync(hp.data(), pen, k * sizeof(double), hipMemcpyDeviceToHost, P->stream));
            ESI_HIP_TRY(hipStreamSynchronize(P->stream));
            double ps = 0.0;
            for (double v : hp) ps += v;
            Jsum += 0.5 * rg + 0.5 * ps;
            r2 += rg;
        }
        hipLaunchKernelGGL(k_grad_d, dim3(grid_for(n)), dim3(NT), 0, P->stream, gm, mask, g, n);
        ESI_HIP_TRY(hipGetLastError());
        *J = Jsum;
        *e = dd > 0 ? std::sqrt(r2 / dd) : 0.0;
        if (!std::isfinite(Jsum)) return fail(ESI_ERR_NONFINITE, "outer loop: non-finite objective");
        return ESI_OK;
    }
};

esi_status_t check_opts(const esi_invert_opts_t* o, int ns) {
    if (!o) return fail(ESI_ERR_ARG, "null options");
    if (o->outer_iters < 0 || o->cg_iters < 1 || !(o->cg_rtol >= 0) || o->shot_group < 1 || o->shot_group > ns ||
        o->lbfgs_mem < 1 || o->ls_max < 1 || !(o->armijo_c1 > 0 && o->armijo_c1 < 1) || !(o->first_step > 0) ||
        !(o->v_min > 0 && o->v_max > o->v_min) || (o->beta_rule != ESI_BETA_FIXED && o->beta_rule != ESI_BETA_DISCREPANCY) ||
        !(o->misfit_lo >= 0 && o->misfit_hi >= o->misfit_lo) || !(o->beta_factor > 1) || o->beta_tries < 0 ||
        (o->inner != ESI_INNER_CG && o->inner != ESI_INNER_FCG_SCALE && o->inner != ESI_INNER_DATASPACE) ||
        !(o->inner_gamma > 0))
        return fail(ESI_ERR_ARG, "invalid outer-loop options");
    return ESI_OK;
}

}  // namespace
}  // namespace esi

using namespace esi;

extern "C" esi_status_t esi_invert(esi_plan_t plan, int32_t shot0, int32_t ns, const float* d_obs,
                                   const float* wavelet, float* vel, const float* grad_mask, float* x,
                                   float* work, const esi_invert_opts_t* opts, esi_invert_report_t* rep) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    if (ns < 1 || shot0 < 0 || shot0 + ns > P->nshots) return fail(ESI_ERR_ARG, "bad shot range");
    ESI_TRY(check_opts(opts, ns));
    const int64_t dl = (int64_t)P->nt * (P->h_rec_ptr[shot0 + ns] - P->h_rec_ptr[shot0]);
    if (!vel || !x || !work || (dl > 0 && !d_obs)) return fail(ESI_ERR_ARG, "null pointer");
    if (opts->inner == ESI_INNER_FCG_SCALE && (wavelet || P->ndim != 2))
        return fail(ESI_ERR_ARG, "the scaled inner solver is for 2D ESI");
    const esi_invert_opts_t& o = *opts;
    Outer S;
    S.P = P; S.plan = plan; S.shot0 = shot0; S.ns = ns; S.G = o.shot_group;
    S.d_obs = d_obs; S.wavelet = wavelet; S.mask = grad_mask; S.x = x; S.work = work; S.o = opts;
    S.n = P->nphys;
    const int64_t n = S.n;
    int64_t gdl = 0;   // largest data length of a group
    for (int s0 = shot0; s0 < shot0 + ns; s0 += S.G) {
        const int k = std::min(S.G, shot0 + ns - s0);
        gdl = std::max<int64_t>(gdl, S.doff(s0 + k) - S.doff(s0));
    }
    const int mem = o.lbfgs_mem;
    Scratch sc;
    sc.stream = P->stream;
    double *m, *g, *mt, *gt, *d, *q;
    ESI_TRY(sc.alloc(&m, n)); ESI_TRY(sc.alloc(&g, n)); ESI_TRY(sc.alloc(&mt, n)); ESI_TRY(sc.alloc(&gt, n));
    ESI_TRY(sc.alloc(&d, n)); ESI_TRY(sc.alloc(&q, n));
    std::vector<double*> sv(mem + 1), yv(mem + 1);   // one spare slot for the candidate pair
    for (int i = 0; i <= mem; ++i) {
        ESI_TRY(sc.alloc(&sv[i], n));
        ESI_TRY(sc.alloc(&yv[i], n));
    }
    ESI_TRY(sc.alloc(&S.red, RB)); ESI_TRY(sc.alloc(&S.vt, n)); ESI_TRY(sc.alloc(&S.gm, n));
    ESI_TRY(sc.alloc(&S.dsyn, gdl)); ESI_TRY(sc.alloc(&S.dres, wavelet ? gdl : 1)); ESI_TRY(sc.alloc(&S.pen, S.G));
    ESI_TRY(sc.alloc(&S.scale, o.inner == ESI_INNER_FCG_SCALE ? (int64_t)S.G * n : 1));
    ESI_TRY(sc.alloc(&S.dw, o.inner == ESI_INNER_DATASPACE ? gdl : 1));
    if (o.inner == ESI_INNER_DATASPACE && P->ndim != 2) return fail(ESI_ERR_ARG, "the data-space inner solver is 2D");

    const double lo = 1.0 / (o.v_max * o.v_max), hi = 1.0 / (o.v_min * o.v_min);
    hipLaunchKernelGGL(k_m_from_vel, dim3(grid_for(n)), dim3(NT), 0, P->stream, vel, lo, hi, m, n);
    ESI_HIP_TRY(hipGetLastError());
    ESI_TRY(S.sqdiff(d_obs, nullptr, dl, &S.dd));

    std::vector<double> hJ, hmis, hbeta, hbeta_it, hstep;
    std::vector<int32_t> htr;
    double beta = P->beta, J, e;
    int evals = 0, status = 0;
    ESI_TRY(S.evaluate(m, beta, &J, g, &e));
    ++evals;
    hJ.push_back(J); hmis.push_back(e); hbeta.push_back(beta);
    std::vector<int> pairs;          // slots, oldest first
    std::vector<double> rho(mem + 1, 0.0);
    for (int it = 0; it < o.outer_iters; ++it) {
        if (o.beta_rule == ESI_BETA_DISCREPANCY) {
            for (int tries = 0; tries < o.beta_tries && (e < o.misfit_lo || e > o.misfit_hi); ++tries) {
                beta = e < o.misfit_lo ? beta * o.beta_factor : beta / o.beta_factor;
                ESI_TRY(S.evaluate(m, beta, &J, g, &e));
                ++evals;
                pairs.clear();
            }
        }
        hbeta_it.push_back(beta);
        // d = -H g (two-loop recursion)
        ESI_TRY(S.axpby(q, 1.0, g, 0.0, nullptr));
        std::vector<double> al(pairs.size());
        for (int j = (int)pairs.size() - 1; j >= 0; --j) {
            const int sl = pairs[j];
            double sq;
            ESI_TRY(S.dot(sv[sl], q, nullptr, &sq));
            al[j] = rho[sl] * sq;
            ESI_TRY(S.axpby(q, 1.0, q, -al[j], yv[sl]));
        }
        if (!pairs.empty()) {
            const int sl = pairs.back();
            double sy, yy;
            ESI_TRY(S.dot(sv[sl], yv[sl], nullptr, &sy));
            ESI_TRY(S.dot(yv[sl], yv[sl], nullptr, &yy));
            ESI_TRY(S.axpby(q, sy / yy, q, 0.0, nullptr));
        }
        for (size_t j = 0; j < pairs.size(); ++j) {
            const int sl = pairs[j];
            double yq;
            ESI_TRY(S.dot(yv[sl], q, nullptr, &yq));
            ESI_TRY(S.axpby(q, 1.0, q, al[j] - rho[sl] * yq, sv[sl]));
        }
        ESI_TRY(S.axpby(d, -1.0, q, 0.0, nullptr));
        if (!pairs.empty()) {
            double gd;
            ESI_TRY(S.dot(g, d, nullptr, &gd));
            if (gd >= 0.0) {
                pairs.clear();
                ESI_TRY(S.axpby(d, -1.0, g, 0.0, nullptr));
            }
        }
        double alpha = 1.0;
        if (pairs.empty()) {
            double mmax, gmax;
            ESI_TRY(S.vmax(m, false, &mmax));
            ESI_TRY(S.vmax(g, true, &gmax));
            if (!(gmax > 0.0)) break;            // stationary: nothing to do
            alpha = o.first_step * mmax / gmax;
        }
        bool accepted = false;
        double Jt = 0.0, et = 0.0;
        int t = 0;
        for (t = 0; t < o.ls_max; ++t) {
            hipLaunchKernelGGL(k_trial, dim3(grid_for(n)), dim3(NT), 0, P->stream, m, d, alpha, lo, hi, mt, n);
            ESI_HIP_TRY(hipGetLastError());
            ESI_TRY(S.evaluate(mt, beta, &Jt, gt, &et));
            ++evals;
            double gs;
            ESI_TRY(S.dot(g, mt, m, &gs));
            if (Jt <= J + o.armijo_c1 * gs) {
                accepted = true;
                break;
            }
            alpha *= 0.5;
        }
        htr.push_back(std::min(t + 1, o.ls_max));
        if (!accepted) {
            status = 1;
            break;
        }
        // candidate pair in the free slot
        int free_sl = 0;
        while (std::find(pairs.begin(), pairs.end(), free_sl) != pairs.end()) ++free_sl;
        ESI_TRY(S.axpby(sv[free_sl], 1.0, mt, -1.0, m));
        ESI_TRY(S.axpby(yv[free_sl], 1.0, gt, -1.0, g));
        double sy;
        ESI_TRY(S.dot(sv[free_sl], yv[free_sl], nullptr, &sy));
        if (sy > 0.0) {
            rho[free_sl] = 1.0 / sy;
            pairs.push_back(free_sl);
            if ((int)pairs.size() > mem) pairs.erase(pairs.begin());
        }
        std::swap(m, mt);
        std::swap(g, gt);
        J = Jt;
        e = et;
        hstep.push_back(alpha); hJ.push_back(J); hmis.push_back(e); hbeta.push_back(beta);
    }
    // leave the plan and vel at the last accepted model
    hipLaunchKernelGGL(k_vel_from_m, dim3(grid_for(n)), dim3(NT), 0, P->stream, m, vel, n);
    ESI_HIP_TRY(hipGetLastError());
    ESI_TRY(esi_plan_set_model(plan, vel));
    P->beta = beta;
    ESI_HIP_TRY(hipStreamSynchronize(P->stream));
    if (rep) {
        rep->outer_done = (int32_t)hstep.size();
        rep->evals = evals;
        rep->status = status;
        rep->beta_final = beta;
        auto put = [](double* dst, const std::vector<double>& v) {
            if (dst) std::copy(v.begin(), v.end(), dst);
        };
        put(rep->J, hJ); put(rep->misfit, hmis); put(rep->beta, hbeta); put(rep->beta_iter, hbeta_it);
        put(rep->step, hstep);
        if (rep->trials) std::copy(htr.begin(), htr.end(), rep->trials);
    }
    return ESI_OK;
}

extern "C" esi_status_t esi_precond_scale(esi_plan_t plan, int32_t shot0, int32_t nshots, double gamma,
                                          float* out) {
    set_error("");
    if (!plan) return fail(ESI_ERR_ARG, "null plan");
    Plan* P = (Plan*)plan;
    ESI_TRY(check_shots(P, shot0, nshots));
    if (P->ndim != 2) return fail(ESI_ERR_ARG, "the cell scale is for 2D plans");
    if (P->w_identity) return fail(ESI_ERR_ARG, "the cell scale models the annihilator weight, not B = I");
    if (!out) return fail(ESI_ERR_ARG, "null out");
    if (!(gamma > 0) || !std::isfinite(gamma)) return fail(ESI_ERR_ARG, "gamma must be finite and > 0");
    const int64_t n = (int64_t)nshots * P->nphys;
    hipLaunchKernelGGL(k_cell_scale, dim3(grid_for(n)), dim3(NT), 0, P->stream, P->d_src, shot0, nshots, P->nz,
                       P->nx, P->beta, P->b_eps, gamma, out);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}
