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

    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int s = L / a.tiles;
    const int t = L - s * a.tiles;
    if (a.active && !a.active[s]) return;   // uniform over the workgroup
    const int gs = a.shot0 + s;
    const int tzi = t / a.tiles_x, txi = t - tzi * a.tiles_x;
    const int x0 = txi * TX, z0 = tzi * TZ;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const float* __restrict__ cur = a.cur + s * a.fstride;
    float* __restrict__ nxt = a.nxt + s * a.fstride;
    float* __restrict__ dvel = a.dvel + s * a.fstride;

    // LDS (r, c) <- storage (z0 + r, x0 + c), i.e. padded (z0 + r - 4, x0 + c - 4)
    for (int i = tid; i < LH * LW; i += 256) {
        const int r = i / LW, c = i - r * LW;
        sh[i] = cur[(int64_t)(z0 + r) * a.XS + x0 + c];
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
    float alp = 0.f, bet = 0.f;
    if constexpr ((FL & F_CG_FUSE) != 0) {
        alp = (float)a.cg_alpha[s];
        bet = (float)a.cg_beta[s];
    }
    float sx = 0.f, sz = 0.f;
    if constexpr ((FL & (F_NORMAL | F_PENALTY)) != 0) {
        sx = (float)a.src_pos[gs * 3 + 0];
        sz = (float)a.src_pos[gs * 3 + 1];
    }

    float col[RZ + 2 * HALO];
#pragma unroll
    for (int k = 0; k < RZ + 2 * HALO; ++k) col[k] = sh[(wv * RZ + k) * LW + lane + HALO];

    const int x = x0 + lane;
    const bool xin = x < a.nxp;
    const float kxv = xin ? a.kx[x] : 0.f;
    const int ix = x - a.nb;
    const bool xphys = ix >= 0 && ix < a.nx;
    const int64_t vbase = ((int64_t)s * a.nt + a.step) * a.nphys;
    double acc = 0.0;

#pragma unroll
    for (int i = 0; i < RZ; ++i) {
        const int zl = wv * RZ + i;
        const int z = z0 + zl;
        if (!xin || z >= a.nzp) continue;
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

        const int64_t si = (int64_t)(z + HALO) * a.XS + x + HALO;
        const float c2v = a.c2[si];
        const float dv = dvel[si];
        const int iz = z - a.nb;
        const bool phys = xphys && iz >= 0 && iz < a.nz;
        const int64_t pi = (int64_t)iz * a.nx + ix;

        float q = 0.f;
        if constexpr ((FL & F_SRC_DENSE) != 0) {
            if (phys) q = a.dsrc[vbase + pi];
        }
        if constexpr ((FL & F_CG_FUSE) != 0) {
            if (phys) {
                const float po = a.cg_p[vbase + pi];
                const float pn = fmaf(bet, po, a.cg_r[vbase + pi]);
                a.cg_p[vbase + pi] = pn;
                if (alp != 0.f) a.cg_x[vbase + pi] = fmaf(alp, po, a.cg_x[vbase + pi]);
                q = pn;
            }
        }
        if constexpr ((FL & F_SRC_POINT) != 0) {
            if (zl * TX + lane == src_cell) q += src_val;
        }
        if constexpr ((FL & F_INJ) != 0) {
            if (has_inj) q += sinj[zl * TX + lane];
        }
        const float kap = kxv + a.kz[z];
        const float lq = fmaf(a.dx2, q, lap);
        // (1+k) u^{n+1} = 2u^n - (1-k) u^{n-1} + c lq advanced through the
        // increment d^n = u^n - u^{n-1}: (1+k) d^{n+1} = (1-k) d^n + c lq and
        // u^{n+1} = u^n + d^{n+1}.  Keeping d in its own array stops the rounding
        // of u from leaking into the velocity, where it would persist.
        const float dn = fmaf(c2v, lq, (1.f - kap) * dv) / (1.f + kap);
        const float un = cv + dn;
        dvel[si] = dn;
        nxt[si] = un;

        if constexpr ((FL & F_OUT) != 0) {
            if (phys) a.dout[vbase + pi] = un;
        }
        if constexpr ((FL & F_SRC_REC) != 0) {
            if (zl * TX + lane == src_cell) a.src_rec[(int64_t)s * a.nt + a.step] = un;
        }
        if constexpr ((FL & (F_NORMAL | F_PENALTY)) != 0) {
            if (phys) {
                const float ddx = (float)ix - sx, ddz = (float)iz - sz;
                const float bb = sqrtf(ddx * ddx + ddz * ddz) + a.b_eps;
                const float wb = a.beta * (bb * bb);
                if constexpr ((FL & F_NORMAL) != 0) {
                    const float pv = a.dp[vbase + pi];
                    const float np = fmaf(wb, pv, un);
                    a.dout[vbase + pi] = np;
                    acc += (double)pv * (double)np;
                }
                if constexpr ((FL & F_PENALTY) != 0) {
                    float* g = a.gacc + (int64_t)s * a.nphys + pi;
                    *g = fmaf(wb * q, c2v * a.inv_dt2 * lq, *g);
                }
            }
        }
        if constexpr ((FL & F_STORE) != 0) {
            if (phys) a.store[s * a.store_stride + (int64_t)a.store_slot * a.nphys + pi] =
                c2v * a.inv_dt2 * lq;
        }
        if constexpr ((FL & F_CORR) != 0) {
            if (phys) {
                float* g = a.gacc + (int64_t)s * a.nphys + pi;
                *g = fmaf(un, a.store[s * a.store_stride + (int64_t)a.store_slot * a.nphys + pi], *g);
            }
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
