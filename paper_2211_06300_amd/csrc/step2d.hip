// Time steps of the 2D 8th-order acoustic scheme (Sec. 4.1) with the fused
// work of the hot path: point / dense source injection (Sec. 2.1, eq. newq2),
// receiver recording R and adjoint injection R^T (Sec. 2.1, Sec. 3), the CG
// direction update (Algorithm 1), the normal-operator output N p = mu + beta
// B^2 p with its p.Np partials (eq. axb), and the zero-lag correlations of the
// gradient (eq. gradewi).
//
// State per shot: u (two slots) and the increment d = u^n - u^{n-1} (two
// slots), each on a storage grid with a zero ghost frame of GH = 8 cells
// around the padded grid (rows XS floats apart), so stencil loads of a tile
// grown by two stencil radii never need bounds checks.  A launch reads the
// current slots and writes the other ones.
//
// k_step2d<FL>:    one step; a 256-thread workgroup owns a 64 x 32 tile.  The
//                  tile of u^n plus a 4-cell halo is staged in LDS, each lane
//                  owns a column and 8 rows, z neighbours from registers, x
//                  neighbours from LDS.
// k_step2d_t2<FL>: two steps per launch (time blocking) on 56 x 32 tiles.
//                  u^n is staged on the tile grown by 8 cells, the first step
//                  is computed on the tile grown by 4 cells (64 columns: one
//                  wave across) into LDS, the second on the tile.  The
//                  wavefield state crosses HBM once per two steps.
//
// Workgroup ids are remapped so that consecutive tiles land on the same XCD
// (8 XCDs take workgroups round-robin), keeping halo neighbours in one L2.
#include "esi_internal.h"

namespace esi {

namespace {

#ifndef ESI_RZ
#define ESI_RZ 8
#endif
#ifndef ESI_TX
#define ESI_TX 64
#endif
#ifndef ESI_MINW
#define ESI_MINW 1
#endif
constexpr int TX = ESI_TX;   // tile width: WX waves of 64 lanes side by side
constexpr int WX = TX / 64;
constexpr int WZ = 4 / WX;   // waves stacked along z (4 waves per workgroup)
constexpr int RZ = ESI_RZ;   // rows per lane
static_assert(TX % 64 == 0 && 4 % WX == 0, "tile width must be 64, 128 or 256");
constexpr int TZ = WZ * RZ;
// one-step kernel: tile + one radius
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

// Laplacian (times dx^2) at an LDS cell from neighbour differences: the centre
// weight is -2 sum_k a_k, and for a smooth field each u_{+-k} - u is exact in
// float32, so the weighted sum carries no cancellation error.  `p` points at
// the cell, `stride` is the LDS row pitch.
__device__ __forceinline__ float lap_lds(const StepArgs& a, const float* p, int stride) {
    const float cv = p[0];
    float lx = a.w1 * ((p[-1] - cv) + (p[1] - cv));
    lx = fmaf(a.w2, (p[-2] - cv) + (p[2] - cv), lx);
    lx = fmaf(a.w3, (p[-3] - cv) + (p[3] - cv), lx);
    lx = fmaf(a.w4, (p[-4] - cv) + (p[4] - cv), lx);
    float lz = a.w1 * ((p[-stride] - cv) + (p[stride] - cv));
    lz = fmaf(a.w2, (p[-2 * stride] - cv) + (p[2 * stride] - cv), lz);
    lz = fmaf(a.w3, (p[-3 * stride] - cv) + (p[3 * stride] - cv), lz);
    lz = fmaf(a.w4, (p[-4 * stride] - cv) + (p[4 * stride] - cv), lz);
    return lx + lz;
}

// (1+k) u^{n+1} = 2u^n - (1-k) u^{n-1} + c lq advanced through the increment
// d^n = u^n - u^{n-1}: (1+k) d^{n+1} = (1-k) d^n + c lq, u^{n+1} = u^n + d^{n+1}.
// Keeping d in its own array stops the rounding of u from leaking into the
// velocity, where it would persist.
// The division by 1 + k uses the hardware reciprocal (within 1 ulp): k = 0 on
// every physical cell, where rcp(1) = 1 exactly and the update is unchanged.
__device__ __forceinline__ float incr(float c2v, float lq, float dv, float kap) {
    return fmaf(c2v, lq, (1.f - kap) * dv) * __builtin_amdgcn_rcpf(1.f + kap);
}

// Element access through a uniform base and a 32-bit byte offset, so that the
// compiler can use scalar-base + 32-bit-offset addressing (every array a
// kernel indexes this way is below 4 GiB from its base).
template <class T>
__device__ __forceinline__ T& at(T* base, uint32_t i) {
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ const T& at(const T* base, uint32_t i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}

// Base pointers of one step's dense streams (uniform: shot and step fixed).
struct StepPtrs {
    float* dout;         // adjoint output or N p, this step's slice
    float* gacc;         // this shot's gradient accumulator
    float* store;        // this step's (dA/dm)u slot
    const float* stin;   // stored (dA/dm)u of this step (CORR)
    float* r;            // this step's slice of r (RUPD with NORMAL)
    float al;            // the shot's CG step length (RUPD with NORMAL)
};

// Shot and tile of workgroup L: from the batch's work list when shots have
// apertures, else tile fastest within a shot.
__device__ __forceinline__ void work_item(const StepArgs& a, int L, int* s, int* t) {
    if (a.work) {
        const int w = a.work[L];
        const int gs = w / a.tiles;
        *s = gs - a.shot0;
        *t = w - gs * a.tiles;
    } else {
        *s = L / a.tiles;
        *t = L - *s * a.tiles;
    }
}

// Physical columns [lo, hi) of global shot gs and its damping table.  Cells
// outside the aperture plus its absorbing layer see c2 = 0, so their zero
// state stays zero: the shot propagates on its window alone.
struct Aperture {
    int lo, hi;
    const float* kx;
};
__device__ __forceinline__ Aperture aperture(const StepArgs& a, int gs) {
    Aperture ap;
    ap.lo = a.win ? a.win[2 * gs] : 0;
    ap.hi = a.win ? a.win[2 * gs + 1] : a.nx;
    ap.kx = a.kx + (int64_t)a.kx_stride * gs;
    return ap;
}

// Offset of step `step` of shot s in dsrc / dout: vbase on the whole time
// axis, slot step % blk_T of the shot's block otherwise.
__device__ __forceinline__ int64_t blk_off(const StepArgs& a, int s, int step, int64_t vbase) {
    return a.blk_T ? ((int64_t)s * a.blk_T + step % a.blk_T) * a.nphys : vbase;
}

__device__ __forceinline__ StepPtrs step_ptrs(const StepArgs& a, int s, int step, int64_t vbase, int slot) {
    StepPtrs q;
    q.dout = a.dout ? a.dout + blk_off(a, s, step, vbase) : nullptr;
    q.gacc = a.gacc ? a.gacc + (int64_t)s * a.nphys : nullptr;
    q.store = a.store ? a.store + s * a.store_stride + (int64_t)slot * a.nphys : nullptr;
    q.stin = q.store;
    q.r = a.cg_rw ? a.cg_rw + vbase : nullptr;
    q.al = a.cg_rw ? (float)a.cg_alpha[s] : 0.f;
    return q;
}

// Fused per-cell outputs of one step at a physical cell of the tile.
//  un: new field, q: source term, lq: lap + dx^2 q, c2v: c / dx^2,
//  pv: p^t (NORMAL), stv: stored (dA/dm)u (CORR), rv: r^t (NORMAL with RUPD).
//
// (The DTFT helpers below: the source of step n from the frequency slices,
// q = inv_nt sum_m (re_m cos w_m t_n + im_m sin w_m t_n), and the update of a
// cell's accumulators acc_m += mu (cos, sin)(w_m t), for the earlier step tA
// first when a two-step launch passes its output muA.)
template <int R>
__device__ __forceinline__ void dtft_source(const StepArgs& a, int s, int step, const uint32_t* pi, const bool* ph,
                                            float* q) {
    const float2* __restrict__ tw = a.dft_tw + (int64_t)step * a.dft_nf;
    const float2* __restrict__ sb = a.dft_src + (int64_t)s * a.dft_nf * a.nphys;
    float acc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = 0.f;
    for (int m = 0; m < a.dft_nf; ++m) {
        const float2 w = tw[m];
        const float2* __restrict__ sm = sb + (int64_t)m * a.nphys;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const float2 v = sm[pi[i]];
            acc[i] = fmaf(v.y, w.y, fmaf(v.x, w.x, acc[i]));
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) q[i] = ph[i] ? acc[i] * a.inv_nt : 0.f;
}

// Frequencies go in chunks whose loads are all issued before any store, so a
// cell's read-modify-writes overlap instead of waiting one on another.
__device__ __forceinline__ void dtft_accumulate(const StepArgs& a, int s, uint32_t pi, int step, float mu, int stepA,
                                                float muA) {
    constexpr int CH = 8;
    float2* __restrict__ acc = a.dft_acc + (int64_t)s * a.dft_nf * a.nphys + pi;
    const float2* __restrict__ tw = a.dft_tw + (int64_t)step * a.dft_nf;
    const float2* __restrict__ twA = a.dft_tw + (int64_t)(stepA < 0 ? 0 : stepA) * a.dft_nf;
    for (int m0 = 0; m0 < a.dft_nf; m0 += CH) {
        float2 v[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k)
            if (m0 + k < a.dft_nf) v[k] = acc[(int64_t)(m0 + k) * a.nphys];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if (m0 + k < a.dft_nf) {
                if (stepA >= 0) {
                    v[k].x = fmaf(muA, twA[m0 + k].x, v[k].x);
                    v[k].y = fmaf(muA, twA[m0 + k].y, v[k].y);
                }
                v[k].x = fmaf(mu, tw[m0 + k].x, v[k].x);
                v[k].y = fmaf(mu, tw[m0 + k].y, v[k].y);
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k)
            if (m0 + k < a.dft_nf) acc[(int64_t)(m0 + k) * a.nphys] = v[k];
    }
}

template <unsigned FL>
__device__ __forceinline__ void cell_outputs(const StepArgs& a, const StepPtrs& o, uint32_t pi,
                                             float un, float q, float lq, float c2v, float pv,
                                             float stv, float rv, float wb, double& acc) {
    if constexpr ((FL & F_OUT) != 0) at(o.dout, pi) = un;
    if constexpr ((FL & F_NORMAL) != 0) {
        const float np = fmaf(wb, pv, un);
        if constexpr ((FL & F_RUPD) != 0) {   // r -= alpha N p, as a separate pass would
            const float rn = fmaf(-o.al, np, rv);
            at(o.r, pi) = rn;
            acc += (double)(rn * rn);
        } else {
            at(o.dout, pi) = np;
            acc += (double)pv * (double)np;
        }
    }
    if constexpr ((FL & (F_CG_FUSE | F_SRC_DENSE)) != 0 && (FL & F_RUPD) != 0)
        acc += (double)(q * (wb * q));   // beta B^2 p.p of the direction (dense source)
    if constexpr ((FL & F_PENALTY) != 0) {
        at(o.gacc, pi) = fmaf(wb * q, c2v * a.inv_dt2 * lq, at(o.gacc, pi));
        acc += (double)(wb * q) * (double)q;   // penalty term beta W q^2 (kept when a.part is set)
    }
    if constexpr ((FL & F_STORE) != 0) at(o.store, pi) = c2v * a.inv_dt2 * lq;
    if constexpr ((FL & F_CORR) != 0) at(o.gacc, pi) = fmaf(un, stv, at(o.gacc, pi));
}

__device__ __forceinline__ float annih_w(const StepArgs& a, int ix, int iz, float sx, float sz) {
    if (a.w_identity) return a.beta;   // uniform over the launch
    const float ddx = (float)ix - sx, ddz = (float)iz - sz;
    // the hardware square root (within 1 ulp; the argument is a sum of squared
    // integers, never denormal) instead of the correctly rounded sequence
    const float bb = __builtin_amdgcn_sqrtf(ddx * ddx + ddz * ddz) + a.b_eps;
    return a.beta * (bb * bb);
}

// ---------------------------------------------------------------------------
template <unsigned FL>
__global__ __launch_bounds__(256, ESI_MINW) void k_step2d(const StepArgs a) {
    __shared__ float sh[LH * LW];
    __shared__ float sinj[(FL & F_INJ) ? TZ * TX : 1];
    __shared__ double sred[4];

    // tile index fastest within a shot: each XCD streams a contiguous stretch
    // of one shot's fields (shot-fastest, to share c2 in L2, fetched fewer
    // bytes but ran slower: the scattered streams cost more than they save)
    int s, t;
    work_item(a, xcd_remap(blockIdx.x, gridDim.x), &s, &t);
    if (a.active && !a.active[s]) return;   // uniform over the workgroup
    const int gs = a.shot0 + s;
    const Aperture ap = aperture(a, gs);
    const int tzi = t / a.tiles_x, txi = t - tzi * a.tiles_x;
    const int x0 = txi * TX, z0 = tzi * TZ;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index: uniform
    const int XS = a.XS;
    // every storage offset of a shot's field fits in 32 bits
    const float* __restrict__ cur = a.cur + s * a.fstride;
    float* __restrict__ nxt = a.nxt + s * a.fstride;
    const float* __restrict__ din = a.din + s * a.fstride;
    float* __restrict__ dnx = a.dnx + s * a.fstride;

    // LDS (r, c) <- padded (z0 + r - 4, x0 + c - 4).  Wave w stages rows w,
    // w + 4, ...: 64 lanes take the row body, 8 the halo (the other lanes
    // repeat a halo load so every load is unconditional).  All rows are loaded
    // into registers before the first LDS write.
    constexpr int RPW = LH / 4;
    static_assert(LH % 4 == 0, "tile rows must split evenly over the waves");
    float tb[RPW][WX], th[RPW];
    {
        const float* src = cur + (z0 + GH - HALO + wv) * XS + x0 + GH - HALO;
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
#pragma unroll
            for (int j = 0; j < WX; ++j) tb[k][j] = at(src, (uint32_t)(k * 4 * XS + 64 * j) + (uint32_t)lane);
            th[k] = at(src, (uint32_t)(k * 4 * XS + TX) + (uint32_t)(lane & (2 * HALO - 1)));
        }
    }
    const int wx = wv % WX, wz = wv / WX;

    // this lane's column and rows: issue every global load first
    const int xl = wx * 64 + lane;                       // tile-local column
    const int x = x0 + xl;
    const float kxv = at(ap.kx, (uint32_t)min(x, a.nxp - 1));
    const int ix = x - a.nb;
    const bool xphys = ix >= ap.lo && ix < ap.hi;
    const bool xwin = x >= ap.lo && x < ap.hi + 2 * a.nb;
    const int zb = z0 + wz * RZ;
    const uint32_t so0 = (uint32_t)((zb + GH) * XS + x + GH);
    const int64_t vbase = ((int64_t)s * a.nt + a.step) * a.nphys;
    const StepPtrs o1 = step_ptrs(a, s, a.step, vbase, a.store_slot);
    float c2v[RZ], dv[RZ], kzv[RZ], qv[RZ];
    uint32_t pi[RZ];
    bool ph[RZ];
#pragma unroll
    for (int i = 0; i < RZ; ++i) {
        const int z = zb + i;
        c2v[i] = xwin ? at(a.c2, so0 + (uint32_t)(i * XS)) : 0.f;
        dv[i] = at(din, so0 + (uint32_t)(i * XS));
        kzv[i] = at(a.kz, (uint32_t)min(z, a.nzp - 1));
        const int iz = z - a.nb;
        ph[i] = xphys && iz >= 0 && iz < a.nz;
        pi[i] = ph[i] ? (uint32_t)(iz * a.nx + ix) : 0u;   // clamped: loads stay unconditional
        qv[i] = 0.f;
    }
    if constexpr ((FL & F_SRC_DENSE) != 0) {
        const float* __restrict__ q = a.dsrc + blk_off(a, s, a.step, vbase);
#pragma unroll
        for (int i = 0; i < RZ; ++i) qv[i] = ph[i] ? at(q, pi[i]) : 0.f;
        if constexpr ((FL & F_SCALE) != 0) {   // cell-scaled dense source
            const float* __restrict__ sc = a.cg_s + (int64_t)s * a.nphys;
#pragma unroll
            for (int i = 0; i < RZ; ++i) qv[i] = qv[i] * at(sc, pi[i]);
        }
    }
    if constexpr ((FL & F_DTFT_SRC) != 0) dtft_source<RZ>(a, s, a.step, pi, ph, qv);
    double pr_acc = 0.0;   // p_new . r partial (F_SCALE)
    if constexpr ((FL & F_CG_FUSE) != 0) {
        const float alp = (float)a.cg_alpha[s];
        const float bet = (float)a.cg_beta[s];
        const float* __restrict__ p = a.cg_p + vbase;
        float* __restrict__ pnew = a.cg_pn + vbase;
        const float* __restrict__ r = a.cg_r + vbase;
        float* __restrict__ xv = a.cg_x + vbase;
        float po[RZ], rv[RZ], xo[RZ], rraw[RZ];
#pragma unroll
        for (int i = 0; i < RZ; ++i) { po[i] = at(p, pi[i]); rv[i] = at(r, pi[i]); xo[i] = at(xv, pi[i]); }
        if constexpr ((FL & F_SCALE) != 0) {
            const float* __restrict__ sc = a.cg_s + (int64_t)s * a.nphys;
#pragma unroll
            for (int i = 0; i < RZ; ++i) { rraw[i] = rv[i]; rv[i] = rv[i] * at(sc, pi[i]); }
        }
#pragma unroll
        for (int i = 0; i < RZ; ++i) {
            const float pn = fmaf(bet, po[i], rv[i]);
            if (ph[i]) {
                at(pnew, pi[i]) = pn;
                if (alp != 0.f) at(xv, pi[i]) = fmaf(alp, po[i], xo[i]);
                if constexpr ((FL & F_SCALE) != 0) pr_acc += (double)pn * (double)rraw[i];
            }
            qv[i] = ph[i] ? pn : 0.f;
        }
    }
    float pv[RZ], stv[RZ], rw[RZ];
#pragma unroll
    for (int i = 0; i < RZ; ++i) { pv[i] = 0.f; stv[i] = 0.f; rw[i] = 0.f; }
    if constexpr ((FL & F_NORMAL) != 0) {
        const float* __restrict__ p = a.dp + vbase;
#pragma unroll
        for (int i = 0; i < RZ; ++i) pv[i] = at(p, pi[i]);
        if constexpr ((FL & F_RUPD) != 0) {
#pragma unroll
            for (int i = 0; i < RZ; ++i) rw[i] = at(o1.r, pi[i]);
        }
    }
    if constexpr ((FL & F_CORR) != 0) {
#pragma unroll
        for (int i = 0; i < RZ; ++i) stv[i] = at(o1.stin, pi[i]);
    }

#pragma unroll
    for (int k = 0; k < RPW; ++k) {
        const int r = wv + k * 4;
#pragma unroll
        for (int j = 0; j < WX; ++j) sh[r * LW + 64 * j + lane] = tb[k][j];
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
    if constexpr ((FL & (F_NORMAL | F_PENALTY | F_RUPD)) != 0) {
        sx = (float)a.src_pos[gs * 3 + 0];
        sz = (float)a.src_pos[gs * 3 + 1];
    }

    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < RZ; ++i) {
        const int zl = wz * RZ + i;
        const int z = z0 + zl;
        const float* cp = sh + (zl + HALO) * LW + xl + HALO;
        const float lap = lap_lds(a, cp, LW);
        float q = qv[i];
        const float qd = q;   // the extended (dense) part of the source
        if constexpr ((FL & F_SRC_POINT) != 0) {
            if (zl * TX + xl == src_cell) q += src_val;
        }
        if constexpr ((FL & F_INJ) != 0) {
            if (has_inj) q += sinj[zl * TX + xl];
        }
        const float kap = kxv + kzv[i];
        const float lq = fmaf(a.dx2, q, lap);
        const float dn = incr(c2v[i], lq, dv[i], kap);
        const float un = cp[0] + dn;
        // cells past the padded grid sit in the zero ghost frame (c2 = u = d = 0)
        // and compute exactly 0, so the stores need no mask
        at(dnx, so0 + (uint32_t)(i * XS)) = dn;
        at(nxt, so0 + (uint32_t)(i * XS)) = un;
        if (!ph[i]) continue;
        if constexpr ((FL & F_SRC_REC) != 0) {
            if (zl * TX + xl == src_cell) a.src_rec[(int64_t)s * a.nt + a.step] = un;
        }
        if constexpr ((FL & F_DTFT_ACC) != 0) dtft_accumulate(a, s, pi[i], a.step, un, -1, 0.f);
        float wb = 0.f;
        if constexpr ((FL & (F_NORMAL | F_PENALTY | F_RUPD)) != 0) wb = annih_w(a, ix, z - a.nb, sx, sz);
        cell_outputs<FL>(a, o1, pi[i], un, qd, lq, c2v[i], pv[i], stv[i], rw[i], wb, acc);
    }

    if constexpr ((FL & (F_NORMAL | F_SCALE | F_PENALTY | F_RUPD)) != 0) {
        if (a.part) {   // uniform over the launch
            acc = wave_sum(acc + pr_acc);
            if (lane == 0) sred[wv] = acc;
            __syncthreads();
            if (tid == 0) {
                double sum = 0.0;
                for (int w = 0; w < 4; ++w) sum += sred[w];
                a.part[(int64_t)s * a.part_stride + t] += sum;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Two steps, tA = a.step and tB = a.step + a.dir, in one launch, on 56 x 32
// output tiles.  The first step runs on the tile grown by 4 cells, 64 x 40:
// one lane per column (a wave spans it exactly), 10 rows per wave, z
// neighbours from a register window.  The second step runs on the tile, one
// lane per column (lanes 56..63 idle), 8 rows per wave.
// The tile height TH (24, 32 or 40 rows) is a template parameter: the
// autotuner's candidates.  Every height computes the same bits per cell.
constexpr int T2W = 56;                           // output tile width
constexpr int A_W = T2W + 2 * HALO;               // 64: first-step region width
constexpr int U0W = T2W + 4 * HALO;               // 72
static_assert(A_W == 64, "two-step tile geometry");

// Occupancy targets: five waves per SIMD for the injecting (adjoint)
// variants, whose registers and LDS allow it without spilling, and at least
// four for the others (the flexible-CG direction update would otherwise take
// 129 VGPRs and drop to three).
template <unsigned FL, int TH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(((FL & F_INJ) != 0 && TH <= 32) ? 5 : 4)))
void k_step2d_t2(const StepArgs a) {
    constexpr int T2Z = TH;                       // output tile rows
    constexpr int A_H = T2Z + 2 * HALO;           // first-step region rows
    constexpr int A_RZ = A_H / 4;                 // first-step rows per wave
    constexpr int B_RZ = T2Z / 4;                 // second-step rows per wave
    constexpr int U0H = T2Z + 4 * HALO;
    static_assert(T2Z % 4 == 0 && A_H % 4 == 0 && U0H % 4 == 0, "two-step tile geometry");
    // LDS (31 KB, five workgroups per CU): u^{tA} on the tile + 8 (dead after
    // the first step, then holding the second step's injection), u after the
    // first step on the tile + 4, d after the first step on the tile.  The
    // first step's injection goes to registers.
    __shared__ float U0[U0H * U0W];
    __shared__ float U1[A_H * A_W];
    __shared__ float D1[T2Z * T2W];
    __shared__ double sred[4];
    float* const sinjB = U0;
    static_assert(U0H * U0W >= A_H * A_W, "the second step's injection fits the u^{tA} buffer");
    // Gradient accumulators are read and written once per launch: both steps'
    // products are chained per cell in the second step, g = fmaf(B, fmaf(A, g))
    // as two one-step launches would add them.  CORR takes the first step's
    // field from U1 and reloads its stored (dA/dm)u there; PENALTY recomputes
    // the first step's (dA/dm)u from u^{tA}, which U0 still holds (no
    // injection reuses it in forward variants).  The DTFT source is not
    // recomputed: that variant keeps one update per step.
    constexpr bool CHAIN_CORR = (FL & F_CORR) != 0;
    constexpr bool CHAIN_PEN = (FL & F_PENALTY) != 0 && (FL & (F_DTFT_SRC | F_INJ)) == 0;
    constexpr unsigned FL_A = FL & ~((CHAIN_CORR ? F_CORR : 0u) | (CHAIN_PEN ? F_PENALTY : 0u));

    int s, t;
    work_item(a, xcd_remap(blockIdx.x, gridDim.x), &s, &t);
    if (a.active && !a.active[s]) return;   // uniform over the workgroup
    const int gs = a.shot0 + s;
    const Aperture ap = aperture(a, gs);
    const int tzi = t / a.tiles_x, txi = t - tzi * a.tiles_x;
    const int x0 = txi * T2W, z0 = tzi * T2Z;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index: uniform
    const int XS = a.XS;
    const int tA = a.step, tB = a.step + a.dir;
    const float* __restrict__ cur = a.cur + s * a.fstride;
    float* __restrict__ nxt = a.nxt + s * a.fstride;
    const float* __restrict__ din = a.din + s * a.fstride;
    float* __restrict__ dnx = a.dnx + s * a.fstride;
    const int64_t vA = ((int64_t)s * a.nt + tA) * a.nphys;
    const int64_t vB = ((int64_t)s * a.nt + tB) * a.nphys;
    const StepPtrs oA = step_ptrs(a, s, tA, vA, a.store_slot);
    const StepPtrs oB = step_ptrs(a, s, tB, vB, a.store_slot2);

    // U0 (r, c) <- padded (z0 - 8 + r, x0 - 8 + c) = storage (z0 + r, x0 + c).
    // Cells off the padded grid sit in the zero ghost frame: they take 0
    // without a load (the last tile column and row reach well into it).
    constexpr int RPW0 = U0H / 4;
    float tb[RPW0], th[RPW0];
    {
        const float* src = cur + (z0 + GH - 2 * HALO + wv) * XS + x0 + GH - 2 * HALO;
        const int xb = x0 - 2 * HALO + lane, xh = x0 - 2 * HALO + 64 + (lane & 7);
        const bool xbin = xb >= 0 && xb < a.nxp, xhin = xh >= 0 && xh < a.nxp;
#pragma unroll
        for (int k = 0; k < RPW0; ++k) {
            const int z = z0 - 2 * HALO + wv + 4 * k;
            const bool zin = z >= 0 && z < a.nzp;
            tb[k] = (zin && xbin) ? at(src, (uint32_t)(k * 4 * XS) + (uint32_t)lane) : 0.f;
            th[k] = (zin && xhin) ? at(src, (uint32_t)(k * 4 * XS + 64) + (uint32_t)(lane & 7)) : 0.f;
        }
    }

    // ---- first-step loads: lane = region column, rows wv*A_RZ + i of the region
    const int xa = x0 - HALO + lane;                      // padded column
    const bool xa_in = xa >= 0 && xa < a.nxp;
    const float kxa = at(ap.kx, (uint32_t)min(max(xa, 0), a.nxp - 1));
    const int ixa = xa - a.nb;
    const bool xa_phys = ixa >= ap.lo && ixa < ap.hi;
    const bool xa_win = xa >= ap.lo && xa < ap.hi + 2 * a.nb;
    const bool xa_tile = lane >= HALO && lane < HALO + T2W;
    const int zra = wv * A_RZ;                            // first region row of this wave
    const uint32_t soA = (uint32_t)((z0 - HALO + zra + GH) * XS + xa + GH);
    float cA[A_RZ], dA[A_RZ], kA[A_RZ], qA[A_RZ], pvA[A_RZ], stA[A_RZ], poA[A_RZ], xoA[A_RZ], rA[A_RZ];
    uint32_t piA[A_RZ];
    bool inA[A_RZ], phA[A_RZ], tlA[A_RZ];   // tlA: physical cell of the output tile
#pragma unroll
    for (int i = 0; i < A_RZ; ++i) {
        const int z = z0 - HALO + zra + i;
        inA[i] = xa_in && z >= 0 && z < a.nzp;
        cA[i] = xa_win ? at(a.c2, soA + (uint32_t)(i * XS)) : 0.f;
        // (the injecting variants load the ghost frame's zeros: the test would
        // cost them their fifth wave's registers)
        if constexpr ((FL & F_INJ) != 0) dA[i] = at(din, soA + (uint32_t)(i * XS));
        else dA[i] = inA[i] ? at(din, soA + (uint32_t)(i * XS)) : 0.f;
        kA[i] = kxa + at(a.kz, (uint32_t)min(max(z, 0), a.nzp - 1));
        const int iz = z - a.nb;
        phA[i] = xa_phys && iz >= 0 && iz < a.nz;
        piA[i] = phA[i] ? (uint32_t)(iz * a.nx + ixa) : 0u;
        tlA[i] = phA[i] && xa_tile && zra + i >= HALO && zra + i < HALO + T2Z;
        qA[i] = 0.f; pvA[i] = 0.f; stA[i] = 0.f; poA[i] = 0.f; xoA[i] = 0.f; rA[i] = 0.f;
    }
    // (values that only the output tile uses, x, p, r of N p and the stored
    // (dA/dm)u, are loaded there alone: the grown region's ring is the
    // neighbours' tiles)
    if constexpr ((FL & F_SRC_DENSE) != 0) {
        const float* __restrict__ q = a.dsrc + blk_off(a, s, tA, vA);
#pragma unroll
        for (int i = 0; i < A_RZ; ++i) qA[i] = phA[i] ? at(q, piA[i]) : 0.f;
        if constexpr ((FL & F_SCALE) != 0) {
            const float* __restrict__ sc = a.cg_s + (int64_t)s * a.nphys;
#pragma unroll
            for (int i = 0; i < A_RZ; ++i) qA[i] = qA[i] * at(sc, piA[i]);
        }
    }
    if constexpr ((FL & F_DTFT_SRC) != 0) dtft_source<A_RZ>(a, s, tA, piA, phA, qA);
    float alp = 0.f, bet = 0.f;
    if constexpr ((FL & F_CG_FUSE) != 0) {
        alp = (float)a.cg_alpha[s];
        bet = (float)a.cg_beta[s];
        const float* __restrict__ p = a.cg_p + vA;
        const float* __restrict__ r = a.cg_r + vA;
        const float* __restrict__ xv = a.cg_x + vA;
#pragma unroll
        for (int i = 0; i < A_RZ; ++i) {
            poA[i] = at(p, piA[i]);
            qA[i] = at(r, piA[i]);
            xoA[i] = tlA[i] ? at(xv, piA[i]) : 0.f;
        }
        if constexpr ((FL & F_SCALE) != 0) {
            const float* __restrict__ sc = a.cg_s + (int64_t)s * a.nphys;
#pragma unroll
            for (int i = 0; i < A_RZ; ++i) { rA[i] = qA[i]; qA[i] = qA[i] * at(sc, piA[i]); }
        }
    }
    if constexpr ((FL & F_NORMAL) != 0) {
        const float* __restrict__ p = a.dp + vA;
#pragma unroll
        for (int i = 0; i < A_RZ; ++i) pvA[i] = tlA[i] ? at(p, piA[i]) : 0.f;
        if constexpr ((FL & F_RUPD) != 0) {   // r^tA into rA (no F_SCALE here)
#pragma unroll
            for (int i = 0; i < A_RZ; ++i) rA[i] = tlA[i] ? at(oA.r, piA[i]) : 0.f;
        }
    }

#pragma unroll
    for (int k = 0; k < RPW0; ++k) {
        const int r = wv + k * 4;
        U0[r * U0W + lane] = tb[k];
        if (lane < 2 * HALO) U0[r * U0W + 64 + lane] = th[k];
    }

    const int64_t nrec_s = (FL & (F_INJ | F_GATHER)) ? a.rec_ptr[gs + 1] - a.rec_ptr[gs] : 0;
    const int64_t doff = (FL & (F_INJ | F_GATHER)) ? (int64_t)a.nt * (a.rec_ptr[gs] - a.rec_ptr[a.shot0]) : 0;
    int ibeg = 0, iend = 0;
    if constexpr ((FL & F_INJ) != 0) {
        const int32_t* ip = a.inj2_ptr + (int64_t)gs * (a.tiles + 1);
        ibeg = ip[t];
        iend = ip[t + 1];
    }
    __syncthreads();

    const int32_t* gp = (FL & F_GATHER) ? a.gat_ptr + (int64_t)gs * (a.tiles + 1) : nullptr;
    if constexpr ((FL & F_GATHER) != 0) {
        // d^{tA-1} = R u^{tA} (forward only)
        if (tA > 0) {
            float* dn = a.gat_data + doff + (int64_t)(tA - 1) * nrec_s;
            for (int e = gp[t] + tid; e < gp[t + 1]; e += 256) {
                const int cell = a.gat_cell[e];
                const int r = cell / T2W, c = cell - r * T2W;
                dn[a.gat_rid[e]] = U0[(r + 2 * HALO) * U0W + c + 2 * HALO];
            }
        }
    }

    // the point source and the source-cell record
    int srcA = -1, srcB = -1;
    float sx = 0.f, sz = 0.f;
    if constexpr ((FL & (F_SRC_POINT | F_SRC_REC | F_NORMAL | F_PENALTY | F_RUPD)) != 0) {
        sx = (float)a.src_pos[gs * 3 + 0];
        sz = (float)a.src_pos[gs * 3 + 1];
        const int gz = a.src_pos[gs * 3 + 1] + a.nb - (z0 - HALO);
        const int gx = a.src_pos[gs * 3 + 0] + a.nb - (x0 - HALO);
        if (gz >= 0 && gz < A_H && gx >= 0 && gx < A_W) srcA = gz * A_W + gx;
        const int lz = gz - HALO, lx = gx - HALO;
        if (lz >= 0 && lz < T2Z && lx >= 0 && lx < T2W) srcB = lz * T2W + lx;
    }

    // the first step's injection straight into registers: every lane walks the
    // tile's entries (uniform loads) and keeps those of its own column, so the
    // injecting variants need no LDS plane for it
    float injA[(FL & F_INJ) ? A_RZ : 1];
    if constexpr ((FL & F_INJ) != 0) {
#pragma unroll
        for (int i = 0; i < A_RZ; ++i) injA[i] = 0.f;
        if (iend > ibeg) {   // uniform over the workgroup
            const float* dj = a.inj_data + doff + (int64_t)tA * nrec_s;
            for (int e = ibeg; e < iend; ++e) {
                const int cell = a.inj2_cell[e];
                const int zr = cell / A_W, col = cell - zr * A_W;
                float v = 0.f;
                for (int k = a.inj2_rptr[e]; k < a.inj2_rptr[e + 1]; ++k) v += dj[a.inj2_rid[k]];
                if (col == lane) {
#pragma unroll
                    for (int i = 0; i < A_RZ; ++i)
                        if (zr == zra + i) injA[i] = v;
                }
            }
        }
    }

    // ---- first step
    float colA[A_RZ + 2 * HALO];
#pragma unroll
    for (int k = 0; k < A_RZ + 2 * HALO; ++k) colA[k] = U0[(zra + k) * U0W + lane + HALO];
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < A_RZ; ++i) {
        const int zr = zra + i;
        const float* cp = U0 + (zr + HALO) * U0W + lane + HALO;
        const float lap = lap_lds(a, cp, U0W);
        float q = qA[i];
        if constexpr ((FL & F_CG_FUSE) != 0) q = phA[i] ? fmaf(bet, poA[i], qA[i]) : 0.f;
        const float qd = q;   // the extended (dense) part of the source
        if constexpr ((FL & F_SRC_POINT) != 0) {
            if (zr * A_W + lane == srcA) q += a.wavelet[(int64_t)s * a.nt + tA];
        }
        if constexpr ((FL & F_INJ) != 0) {
            if (iend > ibeg) q += injA[i];
        }
        const float lq = fmaf(a.dx2, q, lap);
        const float dn = incr(cA[i], lq, dA[i], kA[i]);
        const float un = colA[i + HALO] + dn;
        U1[zr * A_W + lane] = inA[i] ? un : 0.f;
        const bool tile = xa_tile && zr >= HALO && zr < HALO + T2Z;
        if (tile) {
            D1[(zr - HALO) * T2W + lane - HALO] = dn;
            if (phA[i]) {
                if constexpr ((FL & F_CG_FUSE) != 0) {
                    at(a.cg_pn + vA, piA[i]) = qd;
                    if (alp != 0.f) at(a.cg_x + vA, piA[i]) = fmaf(alp, poA[i], xoA[i]);
                    if constexpr ((FL & F_SCALE) != 0) acc += (double)qd * (double)rA[i];
                }
                if constexpr ((FL & F_SRC_REC) != 0) {
                    if (zr * A_W + lane == srcA) a.src_rec[(int64_t)s * a.nt + tA] = un;
                }
                float wb = 0.f;
                if constexpr ((FL & (F_NORMAL | F_PENALTY | F_RUPD)) != 0)
                    wb = annih_w(a, ixa, z0 - HALO + zr - a.nb, sx, sz);
                cell_outputs<FL_A>(a, oA, piA[i], un, qd, lq, cA[i], pvA[i], stA[i], rA[i], wb, acc);
                if constexpr (CHAIN_PEN) acc += (double)(wb * qd) * (double)qd;   // penalty term
            }
        }
    }
    __syncthreads();

    if constexpr ((FL & F_GATHER) != 0) {
        // d^{tA} = R u^{tA+1}
        float* dn = a.gat_data + doff + (int64_t)tA * nrec_s;
        for (int e = gp[t] + tid; e < gp[t + 1]; e += 256) {
            const int cell = a.gat_cell[e];
            const int r = cell / T2W, c = cell - r * T2W;
            dn[a.gat_rid[e]] = U1[(r + HALO) * A_W + c + HALO];
        }
    }
    if constexpr ((FL & F_INJ) != 0) {
        if (iend > ibeg) {   // U0 is dead since the barrier after the first step
            for (int i = tid; i < A_H * A_W; i += 256) sinjB[i] = 0.f;
            __syncthreads();
            const float* dj = a.inj_data + doff + (int64_t)tB * nrec_s;
            for (int e = ibeg + tid; e < iend; e += 256) {
                float v = 0.f;
                for (int k = a.inj2_rptr[e]; k < a.inj2_rptr[e + 1]; ++k) v += dj[a.inj2_rid[k]];
                sinjB[a.inj2_cell[e]] = v;
            }
            __syncthreads();
        }
    }

    // ---- second step on the tile: lane = column (lanes >= 56 idle), 8 rows per wave
    const int lc = min(lane, T2W - 1);
    const bool lane_on = lane < T2W;
    const int x = x0 + lc;
    const float kxv = at(ap.kx, (uint32_t)min(x, a.nxp - 1));
    const int ix = x - a.nb;
    const bool xphys = lane_on && ix >= ap.lo && ix < ap.hi;
    const bool xwin = x >= ap.lo && x < ap.hi + 2 * a.nb;
    const int zb = z0 + wv * B_RZ;
    const uint32_t so0 = (uint32_t)((zb + GH) * XS + x + GH);
    float c2v[B_RZ], kzv[B_RZ], qv[B_RZ], pvB[B_RZ], stB[B_RZ], poB[B_RZ], xoB[B_RZ], rB[B_RZ];
    uint32_t pi[B_RZ];
    bool ph[B_RZ];
#pragma unroll
    for (int i = 0; i < B_RZ; ++i) {
        const int z = zb + i;
        c2v[i] = xwin ? at(a.c2, so0 + (uint32_t)(i * XS)) : 0.f;
        kzv[i] = at(a.kz, (uint32_t)min(z, a.nzp - 1));
        const int iz = z - a.nb;
        ph[i] = xphys && iz >= 0 && iz < a.nz;
        pi[i] = ph[i] ? (uint32_t)(iz * a.nx + ix) : 0u;
        qv[i] = 0.f; pvB[i] = 0.f; stB[i] = 0.f; poB[i] = 0.f; xoB[i] = 0.f; rB[i] = 0.f;
    }
    if constexpr ((FL & F_SRC_DENSE) != 0) {
        const float* __restrict__ q = a.dsrc + blk_off(a, s, tB, vB);
#pragma unroll
        for (int i = 0; i < B_RZ; ++i) qv[i] = ph[i] ? at(q, pi[i]) : 0.f;
        if constexpr ((FL & F_SCALE) != 0) {
            const float* __restrict__ sc = a.cg_s + (int64_t)s * a.nphys;
#pragma unroll
            for (int i = 0; i < B_RZ; ++i) qv[i] = qv[i] * at(sc, pi[i]);
        }
    }
    if constexpr ((FL & F_DTFT_SRC) != 0) dtft_source<B_RZ>(a, s, tB, pi, ph, qv);
    if constexpr ((FL & F_CG_FUSE) != 0) {
        const float* __restrict__ p = a.cg_p + vB;
        const float* __restrict__ r = a.cg_r + vB;
        const float* __restrict__ xv = a.cg_x + vB;
#pragma unroll
        for (int i = 0; i < B_RZ; ++i) { poB[i] = at(p, pi[i]); qv[i] = at(r, pi[i]); xoB[i] = at(xv, pi[i]); }
        if constexpr ((FL & F_SCALE) != 0) {
            const float* __restrict__ sc = a.cg_s + (int64_t)s * a.nphys;
#pragma unroll
            for (int i = 0; i < B_RZ; ++i) { rB[i] = qv[i]; qv[i] = qv[i] * at(sc, pi[i]); }
        }
    }
    if constexpr ((FL & F_NORMAL) != 0) {
        const float* __restrict__ p = a.dp + vB;
#pragma unroll
        for (int i = 0; i < B_RZ; ++i) pvB[i] = at(p, pi[i]);
        if constexpr ((FL & F_RUPD) != 0) {   // r^tB into rB (no F_SCALE here)
#pragma unroll
            for (int i = 0; i < B_RZ; ++i) rB[i] = at(oB.r, pi[i]);
        }
    }
    if constexpr ((FL & F_CORR) != 0) {
#pragma unroll
        for (int i = 0; i < B_RZ; ++i) stB[i] = at(oB.stin, pi[i]);
    }
    // the first step's stored (dA/dm)u (CORR) or dense source (PENALTY) on the tile
    // and the accumulator, read here so that its latency overlaps the stencil
    // (in the variants with a dense output too it would spill: read in place)
    constexpr bool G_EARLY = (CHAIN_CORR || CHAIN_PEN) && (FL & F_OUT) == 0;
    float chA[(CHAIN_CORR || CHAIN_PEN) ? B_RZ : 1], gv[G_EARLY ? B_RZ : 1];
    if constexpr (CHAIN_CORR) {
#pragma unroll
        for (int i = 0; i < B_RZ; ++i) chA[i] = at(oA.stin, pi[i]);
    }
    if constexpr (CHAIN_PEN) {
        const float* __restrict__ q = a.dsrc + blk_off(a, s, tA, vA);
#pragma unroll
        for (int i = 0; i < B_RZ; ++i) chA[i] = ph[i] ? at(q, pi[i]) : 0.f;
    }
    if constexpr (G_EARLY) {
#pragma unroll
        for (int i = 0; i < B_RZ; ++i) gv[i] = at(oB.gacc, pi[i]);
    }

    float colB[B_RZ + 2 * HALO];
#pragma unroll
    for (int k = 0; k < B_RZ + 2 * HALO; ++k) colB[k] = U1[(wv * B_RZ + k) * A_W + lc + HALO];
#pragma unroll
    for (int i = 0; i < B_RZ; ++i) {
        const int zl = wv * B_RZ + i;
        const int z = z0 + zl;
        const float* cp = U1 + (zl + HALO) * A_W + lc + HALO;
        const float lap = lap_lds(a, cp, A_W);
        float q = qv[i];
        if constexpr ((FL & F_CG_FUSE) != 0) q = ph[i] ? fmaf(bet, poB[i], qv[i]) : 0.f;
        const float qd = q;   // the extended (dense) part of the source
        if constexpr ((FL & F_SRC_POINT) != 0) {
            if (lane_on && zl * T2W + lc == srcB) q += a.wavelet[(int64_t)s * a.nt + tB];
        }
        if constexpr ((FL & F_INJ) != 0) {
            if (iend > ibeg) q += sinjB[(zl + HALO) * A_W + lc + HALO];
        }
        const float kap = kxv + kzv[i];
        const float lq = fmaf(a.dx2, q, lap);
        const float dn = incr(c2v[i], lq, D1[zl * T2W + lc], kap);
        const float un = colB[i + HALO] + dn;
        // cells past the padded grid sit in the zero ghost frame (they would
        // compute 0): not stored
        if (lane_on && x < a.nxp && zb + i < a.nzp) {
            at(dnx, so0 + (uint32_t)(i * XS)) = dn;
            at(nxt, so0 + (uint32_t)(i * XS)) = un;
        }
        if (!ph[i]) continue;
        if constexpr ((FL & F_DTFT_ACC) != 0)
            dtft_accumulate(a, s, pi[i], tB, un, tA, U1[(zl + HALO) * A_W + lc + HALO]);
        if constexpr ((FL & F_CG_FUSE) != 0) {
            at(a.cg_pn + vB, pi[i]) = qd;
            if (alp != 0.f) at(a.cg_x + vB, pi[i]) = fmaf(alp, poB[i], xoB[i]);
            if constexpr ((FL & F_SCALE) != 0) acc += (double)qd * (double)rB[i];
        }
        if constexpr ((FL & F_SRC_REC) != 0) {
            if (zl * T2W + lc == srcB) a.src_rec[(int64_t)s * a.nt + tB] = un;
        }
        float wb = 0.f;
        if constexpr ((FL & (F_NORMAL | F_PENALTY | F_RUPD)) != 0) wb = annih_w(a, ix, z - a.nb, sx, sz);
        cell_outputs<FL_A>(a, oB, pi[i], un, qd, lq, c2v[i], pvB[i], stB[i], rB[i], wb, acc);
        if constexpr (CHAIN_CORR) {
            const float uA = U1[(zl + HALO) * A_W + lc + HALO];
            const float gA = fmaf(uA, chA[i], G_EARLY ? gv[G_EARLY ? i : 0] : at(oB.gacc, pi[i]));
            at(oB.gacc, pi[i]) = fmaf(un, stB[i], gA);
        }
        if constexpr (CHAIN_PEN) {
            // the first step's lap + dx^2 q at this cell, as that step formed it
            float qa = chA[i];
            if constexpr ((FL & F_SRC_POINT) != 0) {
                if ((zl + HALO) * A_W + lc + HALO == srcA) qa += a.wavelet[(int64_t)s * a.nt + tA];
            }
            const float lapA = lap_lds(a, U0 + (zl + 2 * HALO) * U0W + lc + 2 * HALO, U0W);
            const float lqA = fmaf(a.dx2, qa, lapA);
            const float gA = fmaf(wb * chA[i], c2v[i] * a.inv_dt2 * lqA, G_EARLY ? gv[G_EARLY ? i : 0] : at(oB.gacc, pi[i]));
            at(oB.gacc, pi[i]) = fmaf(wb * qd, c2v[i] * a.inv_dt2 * lq, gA);
            acc += (double)(wb * qd) * (double)qd;   // penalty term (kept when a.part is set)
        }
    }

    if constexpr ((FL & (F_NORMAL | F_SCALE | F_PENALTY | F_RUPD)) != 0) {
        if (a.part) {   // uniform over the launch
            acc = wave_sum(acc);
            if (lane == 0) sred[wv] = acc;
            __syncthreads();
            if (tid == 0) {
                double sum = 0.0;
                for (int w = 0; w < 4; ++w) sum += sred[w];
                a.part[(int64_t)s * a.part_stride + t] += sum;
            }
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
        const int x = rec[r * 3 + 0] + nb + GH, z = rec[r * 3 + 1] + nb + GH;
        const int y = ndim == 3 ? rec[r * 3 + 2] + nb + GH : 0;
        const float v = field[s * fstride + ((int64_t)z * YS + y) * XS + x];
        data[(int64_t)nt * (rec_ptr[shot0 + s] - base) + (int64_t)(nt - 1) * nrec_s + rid] = v;
    }
}

// TH = 0: the one-step kernel; else the two-step kernel with TH-row tiles
template <unsigned FL, int TH>
esi_status_t launch2d(Plan* P, const StepArgs& a) {
    const int blocks = a.work ? a.nwork : a.tiles * a.nshots;
    if (blocks == 0) return ESI_OK;
    if constexpr (TH > 0)
        hipLaunchKernelGGL((k_step2d_t2<FL, TH>), dim3(blocks), dim3(256), 0, P->stream, a);
    else
        hipLaunchKernelGGL(k_step2d<FL>, dim3(blocks), dim3(256), 0, P->stream, a);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

// The variants the autotuner may give other tile heights: those of the CG,
// modelling and gradient loops.  Other variants run on 32-row tiles.
template <int TH>
esi_status_t dispatch2d_tuned(Plan* P, unsigned flags, const StepArgs& a) {
    switch (flags) {
#define ESI_CASE(F) case (F): return launch2d<(F), TH>(P, a);
        ESI_CASE(F_SRC_POINT | F_GATHER)
        ESI_CASE(F_SRC_POINT | F_STORE)
        ESI_CASE(F_SRC_DENSE | F_GATHER)
        ESI_CASE(F_SRC_DENSE | F_PENALTY)
        ESI_CASE(F_CG_FUSE | F_GATHER | F_RUPD)
        ESI_CASE(F_SRC_DENSE | F_GATHER | F_RUPD)
        ESI_CASE(F_CG_FUSE | F_GATHER | F_SCALE)
        ESI_CASE(F_SRC_DENSE | F_SCALE | F_GATHER)
        ESI_CASE(F_INJ)
        ESI_CASE(F_INJ | F_OUT)
        ESI_CASE(F_INJ | F_NORMAL)
        ESI_CASE(F_INJ | F_NORMAL | F_RUPD)
        ESI_CASE(F_INJ | F_CORR)
#undef ESI_CASE
        default: return fail(ESI_ERR_ARG, "internal: 2D step flags " + std::to_string(flags) +
                                              " have no " + std::to_string(TH) + "-row tiles");
    }
}

bool tuned_variant(unsigned flags) {
    switch (flags) {
        case F_SRC_POINT | F_GATHER: case F_SRC_POINT | F_STORE: case F_SRC_DENSE | F_GATHER:
        case F_SRC_DENSE | F_PENALTY: case F_CG_FUSE | F_GATHER | F_RUPD: case F_SRC_DENSE | F_GATHER | F_RUPD:
        case F_CG_FUSE | F_GATHER | F_SCALE: case F_SRC_DENSE | F_SCALE | F_GATHER: case F_INJ:
        case F_INJ | F_OUT: case F_INJ | F_NORMAL: case F_INJ | F_NORMAL | F_RUPD: case F_INJ | F_CORR:
            return true;
        default:
            return false;
    }
}

template <int TH>
esi_status_t dispatch2d(Plan* P, unsigned flags, const StepArgs& a) {
    switch (flags) {
#define ESI_CASE(F) case (F): return launch2d<(F), TH>(P, a);
        ESI_CASE(F_SRC_POINT | F_GATHER)
        ESI_CASE(F_SRC_POINT | F_GATHER | F_STORE)
        ESI_CASE(F_SRC_POINT | F_STORE)
        ESI_CASE(F_SRC_POINT)
        ESI_CASE(F_SRC_DENSE | F_GATHER)
        ESI_CASE(F_SRC_DENSE | F_GATHER | F_STORE)
        ESI_CASE(F_SRC_DENSE | F_STORE)
        ESI_CASE(F_SRC_DENSE)
        ESI_CASE(F_SRC_DENSE | F_PENALTY)
        ESI_CASE(F_SRC_POINT | F_SRC_DENSE | F_PENALTY)
        ESI_CASE(F_SRC_DENSE | F_PENALTY | F_GATHER)
        ESI_CASE(F_SRC_POINT | F_SRC_DENSE | F_PENALTY | F_GATHER)
        ESI_CASE(F_SRC_POINT | F_SRC_DENSE | F_GATHER)
        ESI_CASE(F_SRC_POINT | F_SRC_DENSE | F_GATHER | F_STORE)
        ESI_CASE(F_SRC_POINT | F_SRC_DENSE | F_STORE)
        ESI_CASE(F_CG_FUSE | F_GATHER)
        ESI_CASE(F_CG_FUSE | F_GATHER | F_SCALE)
        ESI_CASE(F_CG_FUSE | F_GATHER | F_RUPD)
        ESI_CASE(F_SRC_DENSE | F_GATHER | F_RUPD)
        ESI_CASE(F_DTFT_SRC | F_GATHER)
        ESI_CASE(F_SRC_DENSE | F_SCALE | F_GATHER)
        ESI_CASE(F_DTFT_SRC | F_PENALTY)
        ESI_CASE(F_INJ | F_DTFT_ACC)
        ESI_CASE(F_INJ)
        ESI_CASE(F_INJ | F_OUT)
        ESI_CASE(F_INJ | F_NORMAL)
        ESI_CASE(F_INJ | F_NORMAL | F_RUPD)
        ESI_CASE(F_INJ | F_CORR)
        ESI_CASE(F_INJ | F_CORR | F_OUT)
        ESI_CASE(F_INJ | F_CORR | F_SRC_REC)
#undef ESI_CASE
        default: return fail(ESI_ERR_ARG, "internal: unsupported 2D step flags " + std::to_string(flags));
    }
}

}  // namespace

esi_status_t launch_step2d(Plan* P, unsigned flags, const StepArgs& a, int shape) {
    switch (shape) {
        case LS_ONE: return dispatch2d<0>(P, flags, a);
        case LS_T2_32: return dispatch2d<32>(P, flags, a);
        case LS_T2_24: return dispatch2d_tuned<24>(P, flags, a);
        case LS_T2_40: return dispatch2d_tuned<40>(P, flags, a);
        default: return fail(ESI_ERR_ARG, "internal: launch shape " + std::to_string(shape));
    }
}

int step2d_loop_shape(unsigned flags, int shape) {
    return (shape == LS_T2_24 || shape == LS_T2_40) && !tuned_variant(flags) ? LS_T2_32 : shape;
}

void step2d_tile_shape(int* tx, int* tz) { *tx = TX; *tz = TZ; }
void step2d_shape_tile(int shape, int* tx, int* tz) {
    *tx = shape == LS_ONE ? TX : T2W;
    *tz = shape == LS_ONE ? TZ : shape == LS_T2_24 ? 24 : shape == LS_T2_40 ? 40 : 32;
}

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
