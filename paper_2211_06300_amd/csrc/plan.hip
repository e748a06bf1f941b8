// Plan creation: grid validation, CFL check, model coefficients, absorbing
// profile, geometry, per-tile sparse lists, scratch management and errors.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>

#include "esi_internal.h"

namespace esi {

void step3d_tile_shape(int* tx, int* ty, int* tz);   // step3d.hip

static thread_local std::string g_err;

void set_error(const std::string& s) { g_err = s; }

esi_status_t fail(esi_status_t code, const std::string& s) {
    g_err = s;
    return code;
}

esi_status_t grow(void** p, int64_t* cap, int64_t need, hipStream_t stream) {
    if (need <= *cap && *p) return ESI_OK;
    if (*p) {
        // queued kernels may still use the old buffer
        hipError_t se = hipStreamSynchronize(stream);
        if (se != hipSuccess) return fail(ESI_ERR_HIP, std::string("sync: ") + hipGetErrorString(se));
        hipError_t e = hipFree(*p);
        *p = nullptr;
        *cap = 0;
        if (e != hipSuccess) return fail(ESI_ERR_HIP, std::string("hipFree: ") + hipGetErrorString(e));
    }
    if (need <= 0) return ESI_OK;
    hipError_t e = hipMalloc(p, (size_t)need);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ESI_ERR_OOM, "hipMalloc of " + std::to_string(need) + " bytes failed: " +
                                     hipGetErrorString(e));
    }
    *cap = need;
    return ESI_OK;
}

// Centred second-difference weights of order 2M from the closed form
// a_k = 2 (-1)^{k+1} (M!)^2 / (k^2 (M-k)! (M+k)!), a_0 = -2 sum_k a_k.
static void lap_weights(double w[5]) {
    const int M = 4;
    auto fact = [](int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; };
    double s = 0;
    for (int k = 1; k <= M; ++k) {
        w[k] = 2.0 * ((k & 1) ? 1.0 : -1.0) * fact(M) * fact(M) /
               ((double)k * k * fact(M - k) * fact(M + k));
        s += w[k];
    }
    w[0] = -2.0 * s;
}

// Largest stable v dt / dx of leapfrog with this Laplacian in `ndim` dimensions:
// c |lambda_max| <= 4 with |lambda_max| dx^2 = ndim |a_0 + 2 sum_k (-1)^k a_k|.
static double cfl_limit(int ndim) {
    double w[5];
    lap_weights(w);
    double sym = w[0];
    for (int k = 1; k <= 4; ++k) sym += 2.0 * w[k] * ((k & 1) ? -1.0 : 1.0);
    return 2.0 / std::sqrt(ndim * std::fabs(sym));
}

static int round_up(int a, int b) { return (a + b - 1) / b * b; }

// ---- model kernels ----------------------------------------------------------
// c2 on the storage grid: v^2 dt^2 / dx^2 of the nearest physical cell inside
// the padded grid (edge extension into the absorbing layer), 0 in the ghost halo.
__global__ void k_model_c2(float* __restrict__ c2, const float* __restrict__ vel, int nz, int ny,
                           int nx, int nb, int nzp, int nyp, int nxp, int ZS, int YS, int XS,
                           double dt2_dx2, int ndim) {
    int64_t n = (int64_t)ZS * YS * XS;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int sx = (int)(i % XS);
        int64_t rest = i / XS;
        int sy = (int)(rest % YS);
        int sz = (int)(rest / YS);
        int x = sx - GH, z = sz - GH, y = ndim == 3 ? sy - GH : sy;
        float out = 0.f;
        if (x >= 0 && x < nxp && z >= 0 && z < nzp && y >= 0 && y < nyp) {
            int jx = min(max(x - nb, 0), nx - 1);
            int jz = min(max(z - nb, 0), nz - 1);
            int jy = ndim == 3 ? min(max(y - nb, 0), ny - 1) : 0;
            double v = vel[((int64_t)jz * ny + jy) * nx + jx];
            out = (float)(v * v * dt2_dx2);
        }
        c2[i] = out;
    }
}

// Block-wise maximum of a positive float array (exact: max is order-free).
__global__ void k_max(const float* __restrict__ v, int64_t n, float* __restrict__ out) {
    __shared__ float sm[256];
    float m = 0.f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, v[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sm[0];
}

static esi_status_t set_model(Plan* P, const float* vel, bool first, double eta_req) {
    // v_max (device reduction, 256 partial maxima, final max on host)
    float* part = nullptr;
    ESI_HIP_TRY(hipMalloc(&part, 256 * sizeof(float)));
    hipLaunchKernelGGL(k_max, dim3(256), dim3(256), 0, P->stream, vel, P->nphys, part);
    float hpart[256];
    hipError_t e = hipMemcpyAsync(hpart, part, sizeof(hpart), hipMemcpyDeviceToHost, P->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    hipFree(part);
    if (e != hipSuccess) return fail(ESI_ERR_HIP, std::string("v_max: ") + hipGetErrorString(e));
    float vmax = 0.f;
    for (int i = 0; i < 256; ++i) vmax = std::max(vmax, hpart[i]);
    if (!(vmax > 0.f) || !std::isfinite(vmax))
        return fail(ESI_ERR_ARG, "velocity model must be positive and finite");
    double lim = cfl_limit(P->ndim);
    double cfl = (double)vmax * P->dt / P->dx;
    if (cfl > lim) {
        char buf[200];
        snprintf(buf, sizeof buf, "CFL: v_max dt/dx = %.4f exceeds %.4f for the %dD 8th-order scheme",
                 cfl, lim, P->ndim);
        return fail(ESI_ERR_CFL, buf);
    }
    P->vmax = vmax;
    if (first) {
        P->eta_max = eta_req < 0 ? 3.0 * vmax * std::log(1000.0) / (2.0 * P->nb * P->dx) : eta_req;
        // damping kappa = eta dt / 2 split per axis: eta_max (delta_d / nb)^2
        auto prof = [&](int n, float** dst) -> esi_status_t {
            std::vector<float> h(n + 2 * P->nb);
            for (int i = 0; i < (int)h.size(); ++i) {
                int d = std::max(std::max(P->nb - i, i - (n + P->nb - 1)), 0);
                double r = (double)d / P->nb;
                h[i] = (float)(P->eta_max * r * r * P->dt / 2.0);
            }
            ESI_HIP_TRY(hipMalloc(dst, h.size() * sizeof(float)));
            ESI_HIP_TRY(hipMemcpy(*dst, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
            return ESI_OK;
        };
        if (P->h_win.empty()) {
            ESI_TRY(prof(P->nx, &P->kx));
        } else {
            // one profile per shot, around its window [x0, x1) (padded x0 .. x1 + 2 nb)
            std::vector<float> h((size_t)P->nshots * P->nxp);
            for (int s = 0; s < P->nshots; ++s) {
                const int x0 = P->h_win[2 * s], x1 = P->h_win[2 * s + 1];
                for (int i = 0; i < P->nxp; ++i) {
                    int d = std::max(std::max(x0 + P->nb - i, i - (x1 + P->nb - 1)), 0);
                    double r = (double)d / P->nb;
                    h[(size_t)s * P->nxp + i] = (float)(P->eta_max * r * r * P->dt / 2.0);
                }
            }
            ESI_HIP_TRY(hipMalloc(&P->kx, h.size() * sizeof(float)));
            ESI_HIP_TRY(hipMemcpy(P->kx, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
        }
        ESI_TRY(prof(P->nz, &P->kz));
        if (P->ndim == 3) {
            ESI_TRY(prof(P->ny, &P->ky));
        } else {
            ESI_HIP_TRY(hipMalloc(&P->ky, sizeof(float)));
            ESI_HIP_TRY(hipMemset(P->ky, 0, sizeof(float)));
        }
        ESI_HIP_TRY(hipMalloc(&P->c2, P->fsize * sizeof(float)));
    }
    if (first) ESI_HIP_TRY(hipMalloc(&P->vphys, P->nphys * sizeof(float)));
    ESI_HIP_TRY(hipMemcpyAsync(P->vphys, vel, P->nphys * sizeof(float), hipMemcpyDeviceToDevice, P->stream));
    int64_t n = P->fsize;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_model_c2, dim3(blocks), dim3(256), 0, P->stream, P->c2, vel, P->nz, P->ny,
                       P->nx, P->nb, P->nzp, P->nyp, P->nxp, P->ZS, P->YS, P->XS,
                       P->dt * P->dt / (P->dx * P->dx), P->ndim);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

// ---- per-tile lists -------------------------------------------------------------
esi_status_t get_lists(Plan* P, int tx, int tz, int ty, TileLists** out) {
    for (TileLists* L : P->lists)
        if (L->tx == tx && L->tz == tz && L->ty == ty) { *out = L; return ESI_OK; }
    TileLists* L = new (std::nothrow) TileLists();
    if (!L) return fail(ESI_ERR_OOM, "host allocation failed");
    L->tx = tx; L->tz = tz; L->ty = ty;
    L->tiles_x = (P->nxp + tx - 1) / tx;
    L->tiles_z = (P->nzp + tz - 1) / tz;
    L->tiles_y = P->ndim == 3 ? (P->nyp + ty - 1) / ty : 1;
    L->tiles = L->tiles_x * L->tiles_y * L->tiles_z;
    const int nd = P->ndim;
    // tile id and tile-local cell of a padded cell.  2D tiles are (z, x) blocks;
    // 3D tiles are (y, x) columns spanning tz planes of z.
    auto locate = [&](int x, int z, int y, int* tile, int* cell) {
        int txi = x / tx, tzi = z / tz, tyi = nd == 3 ? y / ty : 0;
        *tile = (tzi * L->tiles_y + tyi) * L->tiles_x + txi;
        int lx = x - txi * tx, lz = z - tzi * tz, ly = nd == 3 ? y - tyi * ty : 0;
        *cell = nd == 3 ? ((lz * ty + ly) * tx + lx) : (lz * tx + lx);
    };
    const int T = L->tiles, S = P->nshots;
    std::vector<int32_t> inj_ptr((size_t)S * (T + 1)), gat_ptr((size_t)S * (T + 1));
    std::vector<int32_t> inj_cell, inj_rptr{0}, inj_rid, gat_cell, gat_rid;
    std::vector<int32_t> src_tile(S), src_cell(S);
    // grown-tile injection lists: a receiver belongs to every tile whose region
    // grown by one stencil radius, [x0-4, x0+tx+4) x [z0-4, z0+tz+4)
    // (x [y0-4, y0+ty+4) in 3D), holds it; cells are indexed on the grown tile
    std::vector<int32_t> inj2_ptr((size_t)S * (T + 1)), inj2_cell, inj2_rptr{0}, inj2_rid;
    const int gw = tx + 2 * HALO, gh = tz + 2 * HALO, gy3 = ty + 2 * HALO;
    for (int s = 0; s < S; ++s) {
        int64_t r0 = P->h_rec_ptr[s], r1 = P->h_rec_ptr[s + 1];
        // (tile, cell, rid) for every receiver of this shot, sorted
        std::vector<std::array<int32_t, 3>> e;
        e.reserve(r1 - r0);
        for (int64_t r = r0; r < r1; ++r) {
            const int32_t* pr = &P->h_rec[r * nd];
            int tile, cell;
            locate(pr[0] + P->nb, pr[1] + P->nb, nd == 3 ? pr[2] + P->nb : 0, &tile, &cell);
            e.push_back({tile, cell, (int32_t)(r - r0)});
        }
        std::sort(e.begin(), e.end());
        size_t k = 0;
        int32_t* ip = &inj_ptr[(size_t)s * (T + 1)];
        int32_t* gp = &gat_ptr[(size_t)s * (T + 1)];
        for (int t = 0; t < T; ++t) {
            ip[t] = (int32_t)inj_cell.size();
            gp[t] = (int32_t)gat_cell.size();
            while (k < e.size() && e[k][0] == t) {
                // one unique cell, all its receivers in increasing id order
                int32_t cell = e[k][1];
                inj_cell.push_back(cell);
                while (k < e.size() && e[k][0] == t && e[k][1] == cell) {
                    inj_rid.push_back(e[k][2]);
                    gat_cell.push_back(cell);
                    gat_rid.push_back(e[k][2]);
                    ++k;
                }
                inj_rptr.push_back((int32_t)inj_rid.size());
            }
        }
        ip[T] = (int32_t)inj_cell.size();
        gp[T] = (int32_t)gat_cell.size();
        {
            // (tile, grown cell, rid) for every tile region holding each receiver
            std::vector<std::array<int32_t, 3>> g2;
            for (int64_t r = r0; r < r1; ++r) {
                const int32_t* pr = &P->h_rec[r * nd];
                const int x = pr[0] + P->nb, z = pr[1] + P->nb, y = nd == 3 ? pr[2] + P->nb : 0;
                for (int tzi = 0; tzi < L->tiles_z; ++tzi) {
                    const int gz = z - (tzi * tz - HALO);
                    if (gz < 0 || gz >= gh) continue;
                    for (int tyi = 0; tyi < L->tiles_y; ++tyi) {
                        const int gy = nd == 3 ? y - (tyi * ty - HALO) : 0;
                        if (nd == 3 && (gy < 0 || gy >= gy3)) continue;
                        for (int txi = 0; txi < L->tiles_x; ++txi) {
                            const int gx = x - (txi * tx - HALO);
                            if (gx < 0 || gx >= gw) continue;
                            const int tile = (tzi * L->tiles_y + tyi) * L->tiles_x + txi;
                            const int cell = nd == 3 ? (gz * gy3 + gy) * gw + gx : gz * gw + gx;
                            g2.push_back({tile, cell, (int32_t)(r - r0)});
                        }
                    }
                }
            }
            std::sort(g2.begin(), g2.end());
            size_t q = 0;
            int32_t* ip2 = &inj2_ptr[(size_t)s * (T + 1)];
            for (int t = 0; t < T; ++t) {
                ip2[t] = (int32_t)inj2_cell.size();
                while (q < g2.size() && g2[q][0] == t) {
                    const int32_t cell = g2[q][1];
                    inj2_cell.push_back(cell);
                    while (q < g2.size() && g2[q][0] == t && g2[q][1] == cell) inj2_rid.push_back(g2[q++][2]);
                    inj2_rptr.push_back((int32_t)inj2_rid.size());
                }
            }
            ip2[T] = (int32_t)inj2_cell.size();
        }
        const int32_t* ps = &P->h_src[(size_t)s * nd];
        locate(ps[0] + P->nb, ps[1] + P->nb, nd == 3 ? ps[2] + P->nb : 0, &src_tile[s], &src_cell[s]);
    }
    auto up = [&](std::vector<int32_t>& h, int32_t** d) -> esi_status_t {
        size_t n = std::max<size_t>(h.size(), 1);
        ESI_HIP_TRY(hipMalloc(d, n * sizeof(int32_t)));
        if (!h.empty())
            ESI_HIP_TRY(hipMemcpy(*d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        return ESI_OK;
    };
    ESI_TRY(up(inj_ptr, &L->inj_ptr));
    ESI_TRY(up(inj_cell, &L->inj_cell));
    ESI_TRY(up(inj_rptr, &L->inj_rptr));
    ESI_TRY(up(inj_rid, &L->inj_rid));
    ESI_TRY(up(gat_ptr, &L->gat_ptr));
    ESI_TRY(up(gat_cell, &L->gat_cell));
    ESI_TRY(up(gat_rid, &L->gat_rid));
    ESI_TRY(up(src_tile, &L->src_tile));
    ESI_TRY(up(src_cell, &L->src_cell));
    ESI_TRY(up(inj2_ptr, &L->inj2_ptr));
    ESI_TRY(up(inj2_cell, &L->inj2_cell));
    ESI_TRY(up(inj2_rptr, &L->inj2_rptr));
    ESI_TRY(up(inj2_rid, &L->inj2_rid));
    if (!P->h_win.empty()) {
        // the (shot, tile) items whose tile columns meet the shot's window plus layer
        std::vector<int32_t> work;
        L->work_ptr.assign(P->nshots + 1, 0);
        for (int s = 0; s < P->nshots; ++s) {
            const int lo = P->h_win[2 * s], hi = P->h_win[2 * s + 1] + 2 * P->nb;   // padded [lo, hi)
            for (int t = 0; t < L->tiles; ++t) {
                const int txi = t % L->tiles_x;
                const int a0 = txi * tx, a1 = a0 + tx;
                if (a0 < hi && a1 > lo) work.push_back(s * L->tiles + t);
            }
            L->work_ptr[s + 1] = (int64_t)work.size();
        }
        ESI_TRY(up(work, &L->work));
    }
    P->lists.push_back(L);
    *out = L;
    return ESI_OK;
}

static void free_lists(TileLists* L) {
    hipFree(L->inj_ptr); hipFree(L->inj_cell); hipFree(L->inj_rptr); hipFree(L->inj_rid);
    hipFree(L->gat_ptr); hipFree(L->gat_cell); hipFree(L->gat_rid);
    hipFree(L->src_tile); hipFree(L->src_cell);
    hipFree(L->inj2_ptr); hipFree(L->inj2_cell); hipFree(L->inj2_rptr); hipFree(L->inj2_rid);
    if (L->work) hipFree(L->work);
    delete L;
}

static void free_plan(Plan* P) {
    for (TileLists* L : P->lists) free_lists(L);
    for (int i = 0; i < 2; ++i) {
        if (P->cg_exec[i]) hipGraphExecDestroy(P->cg_exec[i]);
        if (P->cg_g[i]) hipGraphDestroy(P->cg_g[i]);
        if (P->cap_ev[i]) hipEventDestroy(P->cap_ev[i]);
    }
    if (P->cap_stream) hipStreamDestroy(P->cap_stream);
    if (P->h_ctl) hipHostFree(P->h_ctl);
    void* bufs[] = {P->d_src, P->d_rec_ptr, P->c2, P->kx, P->kz, P->ky, P->ring, P->ring2,
                    P->dscr, P->dscr2, P->part, P->scal, P->gshot, P->store, P->ckpt, P->flags,
                    P->d_rec, P->cgi, P->cg_hist, P->vphys, P->d_win, P->fcg_s, P->fcg_a, P->fcg_g,
                    P->fcg_in, P->fcg_o, P->fcg_d, P->fcg_i, P->dft_tw, P->dft_C, P->ds_mu, P->ds_winv,
                    P->ds_seg, P->dft_blk, P->ds_ck};
    for (void* b : bufs)
        if (b) hipFree(b);
    delete P;
}

}  // namespace esi

using namespace esi;

extern "C" const char* esi_last_error(void) { return g_err.c_str(); }

extern "C" esi_status_t esi_plan_create(esi_plan_t* plan, const esi_grid_t* g, const esi_geom_t* geo,
                                        const float* vel, void* stream) {
    set_error("");
    if (!plan || !g || !geo || !vel) return fail(ESI_ERR_ARG, "null argument");
    *plan = nullptr;
    if (g->ndim != 2 && g->ndim != 3) return fail(ESI_ERR_ARG, "ndim must be 2 or 3");
    if (g->nz < 1 || g->nx < 1 || g->ny < 1 || (g->ndim == 2 && g->ny != 1))
        return fail(ESI_ERR_SHAPE, "grid sizes must be >= 1 (ny = 1 in 2D)");
    if (g->nb < HALO) return fail(ESI_ERR_SHAPE, "nb must be >= 4");
    if (g->nt < 1) return fail(ESI_ERR_SHAPE, "nt must be >= 1");
    if (!(g->dx > 0) || !(g->dt > 0)) return fail(ESI_ERR_ARG, "dx and dt must be positive");
    if (!(g->beta >= 0) || !std::isfinite(g->beta)) return fail(ESI_ERR_ARG, "beta must be >= 0");
    if (g->beta > 0 && !(g->b_eps > 0)) return fail(ESI_ERR_ARG, "b_eps must be > 0 when beta > 0");
    if (geo->nshots < 1 || !geo->src || !geo->rec_ptr)
        return fail(ESI_ERR_ARG, "geometry needs nshots >= 1, src and rec_ptr");
    const int nd = g->ndim;
    if (geo->rec_ptr[0] != 0) return fail(ESI_ERR_SHAPE, "rec_ptr[0] must be 0");
    for (int s = 0; s < geo->nshots; ++s)
        if (geo->rec_ptr[s + 1] < geo->rec_ptr[s]) return fail(ESI_ERR_SHAPE, "rec_ptr must be non-decreasing");
    int64_t nrec = geo->rec_ptr[geo->nshots];
    if (nrec > 0 && !geo->rec) return fail(ESI_ERR_ARG, "rec is null");
    auto inside = [&](const int32_t* p) {
        return p[0] >= 0 && p[0] < g->nx && p[1] >= 0 && p[1] < g->nz &&
               (nd == 2 || (p[2] >= 0 && p[2] < g->ny));
    };
    for (int s = 0; s < geo->nshots; ++s)
        if (!inside(geo->src + (size_t)s * nd)) return fail(ESI_ERR_SHAPE, "source " + std::to_string(s) + " outside the grid");
    for (int64_t r = 0; r < nrec; ++r)
        if (!inside(geo->rec + r * nd)) return fail(ESI_ERR_SHAPE, "receiver " + std::to_string(r) + " outside the grid");
    if (geo->window) {
        if (nd != 2) return fail(ESI_ERR_ARG, "shot apertures are supported on 2D grids");
        for (int s = 0; s < geo->nshots; ++s) {
            const int32_t x0 = geo->window[2 * s], x1 = geo->window[2 * s + 1];
            if (!(x0 >= 0 && x0 < x1 && x1 <= g->nx))
                return fail(ESI_ERR_SHAPE, "window of shot " + std::to_string(s) + " outside [0, nx)");
            const int32_t sx = geo->src[(size_t)s * nd];
            if (sx < x0 || sx >= x1) return fail(ESI_ERR_SHAPE, "source " + std::to_string(s) + " outside its window");
            for (int64_t r = geo->rec_ptr[s]; r < geo->rec_ptr[s + 1]; ++r)
                if (geo->rec[r * nd] < x0 || geo->rec[r * nd] >= x1)
                    return fail(ESI_ERR_SHAPE, "receiver " + std::to_string(r) + " outside its shot's window");
        }
    }

    Plan* P = new (std::nothrow) Plan();
    if (!P) return fail(ESI_ERR_OOM, "host allocation failed");
    P->ndim = nd; P->nz = g->nz; P->nx = g->nx; P->ny = g->ny; P->nb = g->nb; P->nt = g->nt;
    P->dx = g->dx; P->dt = g->dt; P->beta = g->beta; P->b_eps = g->b_eps;
    P->stream = (hipStream_t)stream;
    hipGetDevice(&P->device);
    P->nzp = g->nz + 2 * g->nb;
    P->nxp = g->nx + 2 * g->nb;
    P->nyp = nd == 3 ? g->ny + 2 * g->nb : 1;
    // storage: zero ghost halo of HALO cells beyond every tile that may be used
    if (nd == 2) {
        // wide enough for every tile shape used: 64- to 256-wide tiles over
        // round_up(nxp, 256) plus the ghost frame, and 56-wide two-step tiles
        // whose staged region reaches 72 columns past the last tile origin
        P->XS = round_up(std::max(round_up(P->nxp, 256) + 2 * GH, P->nxp + 80), 32);
        // rows: whole tiles of every height in use (64-row one-step tiles,
        // two-step tiles of 24, 32 or 40 rows) plus the ghost frame
        P->ZS = std::max({round_up(P->nzp, 64), round_up(P->nzp, 24), round_up(P->nzp, 40)}) + 2 * GH;
        P->YS = 1;
    } else {
        // the 3D step kernel's column blocks (tx x ty) and z chunks (tz
        // planes) over the padded grid, plus the ghost frame
        int tx, ty, tz;
        step3d_tile_shape(&tx, &ty, &tz);
        P->XS = round_up(round_up(P->nxp, tx) + 2 * GH, 32);
        P->YS = round_up(P->nyp, ty) + 2 * GH;
        P->ZS = round_up(P->nzp, tz) + 2 * GH;
    }
    P->fsize = (int64_t)P->ZS * P->YS * P->XS;
    if (nd == 3) P->tb_fwd = P->tb_adj = LS_ONE;   // two steps per launch on request
    P->nphys = (int64_t)g->nz * g->ny * g->nx;
    double w[5];
    lap_weights(w);
    for (int k = 0; k < 5; ++k) P->lap_w[k] = (float)w[k];
    P->nshots = geo->nshots;
    P->h_src.assign(geo->src, geo->src + (size_t)geo->nshots * nd);
    P->h_rec_ptr.assign(geo->rec_ptr, geo->rec_ptr + geo->nshots + 1);
    if (geo->window) P->h_win.assign(geo->window, geo->window + 2 * (size_t)geo->nshots);
    P->h_rec.assign(geo->rec, geo->rec + nrec * nd);
    for (int s = 0; s < geo->nshots; ++s)
        P->max_nrec = std::max<int>(P->max_nrec, (int)(geo->rec_ptr[s + 1] - geo->rec_ptr[s]));

    auto cleanup = [&](esi_status_t st) { std::string e = esi_last_error(); free_plan(P); set_error(e); return st; };
    {
        std::vector<int32_t> s3((size_t)geo->nshots * 3, 0);
        for (int s = 0; s < geo->nshots; ++s)
            for (int d = 0; d < nd; ++d) s3[(size_t)s * 3 + d] = geo->src[(size_t)s * nd + d];
        std::vector<int32_t> r3((size_t)std::max<int64_t>(nrec, 1) * 3, 0);
        for (int64_t r = 0; r < nrec; ++r)
            for (int d = 0; d < nd; ++d) r3[r * 3 + d] = geo->rec[r * nd + d];
        if (hipMalloc(&P->d_src, s3.size() * 4) != hipSuccess ||
            hipMalloc(&P->d_rec_ptr, (geo->nshots + 1) * 8) != hipSuccess ||
            hipMalloc(&P->d_rec, r3.size() * 4) != hipSuccess ||
            hipMalloc(&P->scal, (size_t)8 * geo->nshots * sizeof(double)) != hipSuccess ||
            hipMalloc(&P->flags, (size_t)2 * geo->nshots * sizeof(int)) != hipSuccess ||
            hipMalloc(&P->cgi, ((size_t)2 * geo->nshots + 2) * sizeof(int)) != hipSuccess ||
            hipHostMalloc((void**)&P->h_ctl, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
            return cleanup(fail(ESI_ERR_OOM, "plan allocation failed"));
        if (hipMemcpy(P->d_src, s3.data(), s3.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(P->d_rec_ptr, geo->rec_ptr, (geo->nshots + 1) * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(P->d_rec, r3.data(), r3.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(ESI_ERR_HIP, "geometry upload failed"));
        if (!P->h_win.empty() &&
            (hipMalloc(&P->d_win, P->h_win.size() * 4) != hipSuccess ||
             hipMemcpy(P->d_win, P->h_win.data(), P->h_win.size() * 4, hipMemcpyHostToDevice) != hipSuccess))
            return cleanup(fail(ESI_ERR_HIP, "aperture upload failed"));
    }
    esi_status_t st = set_model(P, vel, true, g->eta_max);
    if (st != ESI_OK) return cleanup(st);
    // the tilings of the default time loops are built now, so that calls that
    // must not allocate (esi_forward_noalloc) find them
    {
        TileLists* L = nullptr;
        st = lists_for(P, &L);
        if (st == ESI_OK) st = shape_lists(P, loop_shape(P, F_SRC_POINT | F_GATHER, false), &L);
        if (st != ESI_OK) return cleanup(st);
    }
    noalloc_init_device(P->device);
    hipError_t e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) return cleanup(fail(ESI_ERR_HIP, hipGetErrorString(e)));
    *plan = (esi_plan_t)P;
    return ESI_OK;
}

extern "C" esi_status_t esi_plan_set_model(esi_plan_t plan, const float* vel) {
    set_error("");
    if (!plan || !vel) return fail(ESI_ERR_ARG, "null argument");
    ((Plan*)plan)->model_version++;
    ((Plan*)plan)->ck_valid = false;   // checkpoints belong to the old model
    return set_model((Plan*)plan, vel, false, 0.0);
}

extern "C" esi_status_t esi_plan_destroy(esi_plan_t plan) {
    set_error("");
    if (!plan) return ESI_OK;
    Plan* P = (Plan*)plan;
    hipStreamSynchronize(P->stream);
    free_plan(P);
    return ESI_OK;
}
