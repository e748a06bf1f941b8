// One time step of the 2D 8th-order acoustic scheme (Sec. 4.1) with the fused
// work of the hot path: point / dense source injection (Sec. 2.1, eq. newq2),
// receiver recording R and adjoint injection R^T (Sec. 2.1, Sec. 3), the CG
// direction update (Algorithm 1), the normal-operator output N p = mu + beta
// B^2 p with its p.Np partials (eq. axb), and the zero-lag correlations of the
// gradient (eq. gradewi).
//
// Layout: each shot's state is u^n, u^{n+1} (two slots used in turn) and the
// increment d^n = u^n - u^{n-1}, each on a storage grid with a zero ghost halo
// of 4 cells beyond the padded grid, rows XS floats apart, so stencil loads
// need no bounds checks.  A 256-thread workgroup owns a 64 x (4*RZ) tile: the tile
// of u^n plus its halo is staged in LDS with coalesced row loads, each lane
// owns one column and sweeps RZ rows, z neighbours come from registers, x
// neighbours from LDS.  Workgroup ids are remapped so that consecutive tiles
// land on the same XCD (8 XCDs take workgroups round-robin), keeping a
// tile's halo neighbours in the same L2.
#include "esi_internal.h"

namespace esi {

namespace {

constexpr int TX = 64;     // tile width (one wave of lanes)
constexpr int WZ = 4;      // waves stacked along z
constexpr int RZ = 8;      // rows per lane
constexpr int TZ = WZ * RZ;
constexpr int LW = TX + 2 * HALO;
constexpr int LH = TZ + 2 * HALO;

__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int per = nblocks / XCDS, rem = nblocks % XCDS;
    const int xcd = b % XCDS, idx = b / XCDS;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <unsigned FL>
__global__ __launch_bounds__(256) void k_step2d(const StepArgs a) {
    __shared__ float sh[LH * LW];
    __shared__ float sinj[(FL & F_INJ) ? TZ * TX : 1];
    __shared__ double sred[WZ];

    // tile index fastest within a shot: each XCD streams a contiguous stretch
    // of one shot's fields (tried shot-fastest to share c2 in L2: fewer bytes
    // fetched but slower, the scattered streams cost more than they save)
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int s = L / a.tiles;
    const int t = L - s * a.tiles;
    if (a.active && !a.active[s]) return;   // uniform over the workgroup
    const int gs = a.shot0 + s;
    const int tzi = t / a.tiles_x, txi = t - tzi * a.tiles_x;
    const int x0 = txi * TX, z0 = tzi * TZ;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int XS = a.XS;
    // every storage offset of a shot's field fits in 32 bits
    const float* __restrict__ cur = a.cur + s * a.fstride;
    float* __restrict__ nxt = a.nxt + s * a.fstride;
    float* __restrict__ dvel = a.dvel + s * a.fstride;

    // LDS (r, c) <- storage (z0 + r, x0 + c), i.e. padded (z0 + r - 4, x0 + c - 4).
    // Wave w stages rows w, w + 4, ...: 64 lanes take the row body, 8 the halo
    // (the other lanes repeat a halo load so every load is unconditional).
    // All rows are loaded into registers before the first LDS write.
    constexpr int RPW = LH / WZ;
    static_assert(LH % WZ == 0, "tile rows must split evenly over the waves");
    float tb[RPW], th[RPW];
    {
        const float* src = cur + (z0 + wv) * XS + x0;
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
            tb[k] = src[k * WZ * XS + lane];
            th[k] = src[k * WZ * XS + TX + (lane & (2 * HALO - 1))];
        }
    }

    // Per-lane column and rows of this lane: issue every global load first.
    const int x = x0 + lane;
    const bool xin = x < a.nxp;
    const float kxv = a.kx[min(x, a.nxp - 1)];
    const int ix = x - a.nb;
    const bool xphys = ix >= 0 && ix < a.nx;
    const int zb = z0 + wv * RZ;                         // first row of this lane
    const int so0 = (zb + HALO) * XS + x + HALO;         // storage offset of that row
    const int64_t vbase = ((int64_t)s * a.nt + a.step) * a.nphys;
    float c2v[RZ], dv[RZ], kzv[RZ], qv[RZ];
    int pi[RZ];
    bool ph[RZ];
#pragma unroll
    for (int i = 0; i < RZ; ++i) {
        const int z = zb + i;
        c2v[i] = a.c2[so0 + i * XS];
        dv[i] = dvel[so0 + i * XS];
        kzv[i] = a.kz[min(z, a.nzp - 1)];
        const int iz = z - a.nb;
        ph[i] = xphys && iz >= 0 && iz < a.nz;
        pi[i] = ph[i] ? iz * a.nx + ix : 0;             // clamped: loads stay unconditional
        qv[i] = 0.f;
    }
    float po[RZ], pn[RZ], pv[RZ];
    if constexpr ((FL & F_SRC_DENSE) != 0) {
        const float* __restrict__ q = a.dsrc + vbase;
#pragma unroll
        for (int i = 0; i < RZ; ++i) qv[i] = ph[i] ? q[pi[i]] : 0.f;
    }
    if constexpr ((FL & F_CG_FUSE) != 0) {
        const float alp = (float)a.cg_alpha[s];
        const float bet = (float)a.cg_beta[s];
        float* __restrict__ p = a.cg_p + vbase;
        const float* __restrict__ r = a.cg_r + vbase;
        float* __restrict__ xv = a.cg_x + vbase;
        float rv[RZ], xo[RZ];
#pragma unroll
        for (int i = 0; i < RZ; ++i) { po[i] = p[pi[i]]; rv[i] = r[pi[i]]; xo[i] = xv[pi[i]]; }
#pragma unroll
        for (int i = 0; i < RZ; ++i) {
            pn[i] = fmaf(bet, po[i], rv[i]);
            if (ph[i]) {
                p[pi[i]] = pn[i];
                if (alp != 0.f) xv[pi[i]] = fmaf(alp, po[i], xo[i]);
            }
            qv[i] = ph[i] ? pn[i] : 0.f;
        }
    }
    if constexpr ((FL & F_NORMAL) != 0) {
        const float* __restrict__ p = a.dp + vbase;
#pragma unroll
        for (int i = 0; i < RZ; ++i) pv[i] = p[pi[i]];
    }
    float stv[RZ];
    if constexpr ((FL & F_CORR) != 0) {
        const float* __restrict__ st = a.store + s * a.store_stride + (int64_t)a.store_slot * a.nphys;
#pragma unroll
        for (int i = 0; i < RZ; ++i) stv[i] = st[pi[i]];
    }

#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wv + k * WZ;
        sh[r * LW + lane] = tb[k];
        if (lane < 2 * HALO) sh[r * LW + TX + lane] = th[k];
    }

    const int64_t nrec_s = (FL & (F_INJ | F_GATHER)) ? a.rec_ptr[gs + 1] - a.rec_ptr[gs] : 0;
    const int64_t doff = (FL & (F_INJ | F_GATHER)) ? (int64_t)a.nt * (a.rec_ptr[gs] - a.rec_ptr[a.shot0]) : 0;
    bool has_inj = false;
    if constexpr ((FL & F_INJ) != 0) {
        const int32_t* ip = a.inj_ptr + (int64_t)gs * (a.tiles + 1);
        const int beg = ip[t], end = ip[t + 1];
        has_inj = end > beg;
        if (has_inj) {
            for (int i = tid; i < TZ * TX; i += 256) sinj[i] = 0.f;
            __syncthreads();
            const float* dj = a.inj_data + doff + (int64_t)a.step * nrec_s;
            for (int e = beg + tid; e < end; e += 256) {
                float v = 0.f;
                for (int k = a.inj_rptr[e]; k < a.inj_rptr[e + 1]; ++k) v += dj[a.inj_rid[k]];
                sinj[a.inj_cell[e]] = v;
            }
        }
    }
    __syncthreads();

    if constexpr ((FL & F_GATHER) != 0) {
        if (a.step > 0) {
            const int32_t* gp = a.gat_ptr + (int64_t)gs * (a.tiles + 1);
            float* dn = a.gat_data + doff + (int64_t)(a.step - 1) * nrec_s;
            for (int e = gp[t] + tid; e < gp[t + 1]; e += 256) {
                const int cell = a.gat_cell[e];
                const int r = cell / TX, c = cell - r * TX;
                dn[a.gat_rid[e]] = sh[(r + HALO) * LW + c + HALO];
            }
        }
    }

    int src_cell = -1;
    float src_val = 0.f;
    if constexpr ((FL & (F_SRC_POINT | F_SRC_REC)) != 0) {
        if (a.src_tile[gs] == t) {
            src_cell = a.src_cell[gs];
            if constexpr ((FL & F_SRC_POINT) != 0) src_val = a.wavelet[(int64_t)s * a.nt + a.step];
        }
    }
    float sx = 0.f, sz = 0.f;
    if constexpr ((FL & (F_NORMAL | F_PENALTY)) != 0) {
        sx = (float)a.src_pos[gs * 3 + 0];
        sz = (float)a.src_pos[gs * 3 + 1];
    }

    float col[RZ + 2 * HALO];
#pragma unroll
    for (int k = 0; k < RZ + 2 * HALO; ++k) col[k] = sh[(wv * RZ + k) * LW + lane + HALO];

    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < RZ; ++i) {
        const int zl = wv * RZ + i;
        const int z = z0 + zl;
        const bool valid = xin && z < a.nzp;
        const float* row = sh + (zl + HALO) * LW + lane + HALO;
        const float cv = col[i + HALO];
        // Laplacian from neighbour differences: the centre weight is -2 sum_k a_k,
        // and for a smooth field each u_{+-k} - u is exact in float32, so the
        // weighted sum carries no cancellation error.
        float lx = a.w1 * ((row[-1] - cv) + (row[1] - cv));
        lx = fmaf(a.w2, (row[-2] - cv) + (row[2] - cv), lx);
        lx = fmaf(a.w3, (row[-3] - cv) + (row[3] - cv), lx);
        lx = fmaf(a.w4, (row[-4] - cv) + (row[4] - cv), lx);
        float lz = a.w1 * ((col[i + 3] - cv) + (col[i + 5] - cv));
        lz = fmaf(a.w2, (col[i + 2] - cv) + (col[i + 6] - cv), lz);
        lz = fmaf(a.w3, (col[i + 1] - cv) + (col[i + 7] - cv), lz);
        lz = fmaf(a.w4, (col[i + 0] - cv) + (col[i + 8] - cv), lz);
        const float lap = lx + lz;

        float q = qv[i];
        if constexpr ((FL & F_SRC_POINT) != 0) {
            if (zl * TX + lane == src_cell) q += src_val;
        }
        if constexpr ((FL & F_INJ) != 0) {
            if (has_inj) q += sinj[zl * TX + lane];
        }
        const float kap = kxv + kzv[i];
        const float lq = fmaf(a.dx2, q, lap);
        // (1+k) u^{n+1} = 2u^n - (1-k) u^{n-1} + c lq advanced through the
        // increment d^n = u^n - u^{n-1}: (1+k) d^{n+1} = (1-k) d^n + c lq and
        // u^{n+1} = u^n + d^{n+1}.  Keeping d in its own array stops the rounding
        // of u from leaking into the velocity, where it would persist.
        const float dn = fmaf(c2v[i], lq, (1.f - kap) * dv[i]) / (1.f + kap);
        const float un = cv + dn;
        if (valid) {
            dvel[so0 + i * XS] = dn;
            nxt[so0 + i * XS] = un;
        }
        if (!ph[i]) continue;
        if constexpr ((FL & F_OUT) != 0) a.dout[vbase + pi[i]] = un;
        if constexpr ((FL & F_SRC_REC) != 0) {
            if (zl * TX + lane == src_cell) a.src_rec[(int64_t)s * a.nt + a.step] = un;
        }
        if constexpr ((FL & (F_NORMAL | F_PENALTY)) != 0) {
            const float ddx = (float)ix - sx, ddz = (float)(z - a.nb) - sz;
            const float bb = sqrtf(ddx * ddx + ddz * ddz) + a.b_eps;
            const float wb = a.beta * (bb * bb);
            if constexpr ((FL & F_NORMAL) != 0) {
                const float np = fmaf(wb, pv[i], un);
                a.dout[vbase + pi[i]] = np;
                acc += (double)pv[i] * (double)np;
            }
            if constexpr ((FL & F_PENALTY) != 0) {
                float* g = a.gacc + (int64_t)s * a.nphys + pi[i];
                *g = fmaf(wb * q, c2v[i] * a.inv_dt2 * lq, *g);
            }
        }
        if constexpr ((FL & F_STORE) != 0)
            a.store[s * a.store_stride + (int64_t)a.store_slot * a.nphys + pi[i]] = c2v[i] * a.inv_dt2 * lq;
        if constexpr ((FL & F_CORR) != 0) {
            float* g = a.gacc + (int64_t)s * a.nphys + pi[i];
            *g = fmaf(un, stv[i], *g);
        }
    }

    if constexpr ((FL & F_NORMAL) != 0) {
        acc = wave_sum(acc);
        if (lane == 0) sred[wv] = acc;
        __syncthreads();
        if (tid == 0) {
            double sum = 0.0;
            for (int w = 0; w < WZ; ++w) sum += sred[w];
            a.part[(int64_t)s * a.tiles + t] += sum;
        }
    }
}

// Record d^{nt-1} = R u^{nt} after the last step (one thread per receiver).
__global__ void k_final_gather(const float* __restrict__ field, int64_t fstride,
                               const int32_t* __restrict__ rec, const int64_t* __restrict__ rec_ptr,
                               int shot0, int nshots, int nt, int nb, int XS, int YS, int ndim,
                               float* __restrict__ data) {
    const int64_t base = rec_ptr[shot0];
    const int64_t n = rec_ptr[shot0 + nshots] - base;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = base + i;
        int s = 0;
        while (rec_ptr[shot0 + s + 1] <= r) ++s;   // shots per call are few
        const int64_t nrec_s = rec_ptr[shot0 + s + 1] - rec_ptr[shot0 + s];
        const int64_t rid = r - rec_ptr[shot0 + s];
        const int x = rec[r * 3 + 0] + nb + HALO, z = rec[r * 3 + 1] + nb + HALO;
        const int y = ndim == 3 ? rec[r * 3 + 2] + nb + HALO : 0;
        const float v = field[s * fstride + ((int64_t)z * YS + y) * XS + x];
        data[(int64_t)nt * (rec_ptr[shot0 + s] - base) + (int64_t)(nt - 1) * nrec_s + rid] = v;
    }
}

template <unsigned FL>
esi_status_t launch2d(Plan* P, const StepArgs& a) {
    const int blocks = a.tiles * a.nshots;
    hipLaunchKernelGGL(k_step2d<FL>, dim3(blocks), dim3(256), 0, P->stream, a);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

}  // namespace

esi_status_t launch_step2d(Plan* P, unsigned flags, const StepArgs& a) {
    switch (flags) {
        case F_SRC_POINT | F_GATHER: return launch2d<F_SRC_POINT | F_GATHER>(P, a);
        case F_SRC_POINT | F_GATHER | F_STORE: return launch2d<F_SRC_POINT | F_GATHER | F_STORE>(P, a);
        case F_SRC_POINT | F_STORE: return launch2d<F_SRC_POINT | F_STORE>(P, a);
        case F_SRC_POINT: return launch2d<F_SRC_POINT>(P, a);
        case F_SRC_DENSE | F_GATHER: return launch2d<F_SRC_DENSE | F_GATHER>(P, a);
        case F_SRC_DENSE | F_GATHER | F_STORE: return launch2d<F_SRC_DENSE | F_GATHER | F_STORE>(P, a);
        case F_SRC_DENSE | F_STORE: return launch2d<F_SRC_DENSE | F_STORE>(P, a);
        case F_SRC_DENSE | F_PENALTY: return launch2d<F_SRC_DENSE | F_PENALTY>(P, a);
        case F_CG_FUSE | F_GATHER: return launch2d<F_CG_FUSE | F_GATHER>(P, a);
        case F_INJ | F_OUT: return launch2d<F_INJ | F_OUT>(P, a);
        case F_INJ | F_NORMAL: return launch2d<F_INJ | F_NORMAL>(P, a);
        case F_INJ | F_CORR: return launch2d<F_INJ | F_CORR>(P, a);
        case F_INJ | F_CORR | F_OUT: return launch2d<F_INJ | F_CORR | F_OUT>(P, a);
        case F_INJ | F_CORR | F_SRC_REC: return launch2d<F_INJ | F_CORR | F_SRC_REC>(P, a);
        default: return fail(ESI_ERR_ARG, "internal: unsupported 2D step flags " + std::to_string(flags));
    }
}

void step2d_tile_shape(int* tx, int* tz) { *tx = TX; *tz = TZ; }

esi_status_t launch_final_gather(Plan* P, const float* field, int64_t fstride, float* data,
                                 int shot0, int nshots) {
    int64_t n = P->h_rec_ptr[shot0 + nshots] - P->h_rec_ptr[shot0];
    if (n == 0) return ESI_OK;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_final_gather, dim3(blocks), dim3(256), 0, P->stream, field, fstride,
                       P->d_rec, P->d_rec_ptr, shot0, nshots, P->nt, P->nb, P->XS, P->YS,
                       P->ndim, data);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

}  // namespace esi
