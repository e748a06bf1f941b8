// Two time steps per launch of the 3D 8th-order scheme (Sec. 4.1): time
// blocking on top of the 2.5D z-march, with the fused work of the one-step
// kernel (point / dense sources, receiver recording and injection, dense
// outputs, the normal operator with its p.Np partials, the CG direction update
// and the gradient correlation).
//
// A 1024-thread workgroup owns a block of 56 (x) x 24 (y) output columns and
// a chunk of 64 z-planes.  The first step runs on the block grown by one
// stencil radius, 64 x 32 columns: one wave spans its width and each of the 16
// waves owns two of its rows.  The first step marches four planes ahead of
// the second: in iteration i it computes u^{n+1} on plane z1 = zc0 - 4 + i,
// and the second step computes u^{n+2} on plane z2 = z1 - 4 from the thread's
// own register window of u^{n+1} (z neighbours) and a double-buffered LDS
// plane of it (x, y neighbours).  u^n comes from a register window (z) and a
// double-buffered LDS plane with a 4-cell halo (x, y).  The wavefield state
// crosses HBM once per two steps: per output cell, u^n, d^n and c are read
// (with the grown block's ring and the chunk's 8-plane prologue) and u^{n+2},
// d^{n+2} written.
//
// The update of a cell is the one-step kernel's, operation for operation, so
// one- and two-step launches give the same bits.
#include "esi_internal.h"

namespace esi {
namespace {

#ifndef ESI3_BZ
#define ESI3_BZ 64
#endif
#ifndef ESI3_PF
#define ESI3_PF 1
#endif
constexpr int BX = 56, BY = 24, BZ = ESI3_BZ;            // output block and z chunk
constexpr int PF = ESI3_PF;                              // planes of state loads in flight ahead
constexpr int RX = BX + 2 * HALO, RY = BY + 2 * HALO;    // first-step region: 64 x 32
constexpr int NW = 16, NTH = 64 * NW;                    // 16 waves of 64 lanes
constexpr int RPT = RY / NW;                             // region rows per thread: 2
constexpr int AW = RX + 2 * HALO, AH = RY + 2 * HALO;    // u^n plane with halo: 72 x 40
constexpr int NHALO = AW * AH - RX * RY;                 // 832 halo cells per plane
constexpr int WIN = 2 * HALO + 1;                        // z window
static_assert(RX == 64 && RY % NW == 0 && NHALO <= NTH, "3D two-step geometry");

__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int per = nblocks / XCDS, rem = nblocks % XCDS;
    const int xcd = b % XCDS, idx = b / XCDS;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

template <class T>
__device__ __forceinline__ T& at(T* base, uint32_t i) {
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ const T& at(const T* base, uint32_t i) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}

// Laplacian (times dx^2) from neighbour differences, as the one-step kernel
// forms it: x and y arms from an LDS plane (row pitch `pw`), z arms from the
// register window w (centre w[4]).
__device__ __forceinline__ float lap3(const StepArgs& a, const float* cp, int pw, const float* w) {
    const float cv = w[HALO];
    float lx = a.w1 * ((cp[-1] - cv) + (cp[1] - cv));
    lx = fmaf(a.w2, (cp[-2] - cv) + (cp[2] - cv), lx);
    lx = fmaf(a.w3, (cp[-3] - cv) + (cp[3] - cv), lx);
    lx = fmaf(a.w4, (cp[-4] - cv) + (cp[4] - cv), lx);
    float ly = a.w1 * ((cp[-pw] - cv) + (cp[pw] - cv));
    ly = fmaf(a.w2, (cp[-2 * pw] - cv) + (cp[2 * pw] - cv), ly);
    ly = fmaf(a.w3, (cp[-3 * pw] - cv) + (cp[3 * pw] - cv), ly);
    ly = fmaf(a.w4, (cp[-4 * pw] - cv) + (cp[4 * pw] - cv), ly);
    float lz = a.w1 * ((w[3] - cv) + (w[5] - cv));
    lz = fmaf(a.w2, (w[2] - cv) + (w[6] - cv), lz);
    lz = fmaf(a.w3, (w[1] - cv) + (w[7] - cv), lz);
    lz = fmaf(a.w4, (w[0] - cv) + (w[8] - cv), lz);
    return (lx + ly) + lz;
}

__device__ __forceinline__ float incr3(float c2v, float lq, float dv, float kap) {
    return fmaf(c2v, lq, (1.f - kap) * dv) * __builtin_amdgcn_rcpf(1.f + kap);
}

__device__ __forceinline__ float annih3(const StepArgs& a, int ix, int iy, int iz, float sx, float sy, float sz) {
    if (a.w_identity) return a.beta;
    // the hardware square root (within 1 ulp; the argument is a sum of
    // squared integers, never denormal), as the one-step kernel takes it
    const float ddx = (float)ix - sx, ddy = (float)iy - sy, ddz = (float)iz - sz;
    const float bb = __builtin_amdgcn_sqrtf(ddx * ddx + ddy * ddy + ddz * ddz) + a.b_eps;
    return a.beta * (bb * bb);
}

// offset of step t of shot s in dsrc / dout (blocks of blk_T steps, or the whole axis)
__device__ __forceinline__ int64_t voff(const StepArgs& a, int s, int t) {
    return a.blk_T ? ((int64_t)s * a.blk_T + t % a.blk_T) * a.nphys : ((int64_t)s * a.nt + t) * a.nphys;
}

// Per-cell outputs of one step at a physical output cell: dense output,
// normal operator (with the fused residual update), the CG direction's
// penalty part, the stored (dA/dm)u and the source-cell record.  The gradient
// correlation (CORR) is chained over both steps by the caller.
template <unsigned FL>
__device__ __forceinline__ void outputs3(const StepArgs& a, int s, int t, uint32_t pi, float un, float qd, float lq,
                                         float c2v, float wb, float pv, float rv, bool at_src, double& acc) {
    const int64_t vb = ((int64_t)s * a.nt + t) * a.nphys;
    if constexpr ((FL & F_OUT) != 0) at(a.dout + voff(a, s, t), pi) = un;
    if constexpr ((FL & F_SRC_REC) != 0) {
        if (at_src) a.src_rec[(int64_t)s * a.nt + t] = un;
    }
    if constexpr ((FL & (F_CG_FUSE | F_SRC_DENSE)) != 0 && (FL & F_RUPD) != 0)
        acc += (double)(qd * (wb * qd));   // beta B^2 p.p of the direction (dense source)
    if constexpr ((FL & F_NORMAL) != 0) {
        const float np = fmaf(wb, pv, un);
        if constexpr ((FL & F_RUPD) != 0) {   // r -= alpha N p, as a separate pass would
            const float rn = fmaf(-(float)a.cg_alpha[s], np, rv);
            at(a.cg_rw + vb, pi) = rn;
            acc += (double)(rn * rn);
        } else {
            at(a.dout + voff(a, s, t), pi) = np;
            acc += (double)pv * (double)np;
        }
    }
    if constexpr ((FL & F_STORE) != 0) {
        const int slot = t == a.step ? a.store_slot : a.store_slot2;
        at(a.store + s * a.store_stride + (int64_t)slot * a.nphys, pi) = c2v * a.inv_dt2 * lq;
    }
}

template <unsigned FL>
__global__ __launch_bounds__(NTH) void k_step3d_t2(const StepArgs a) {
    __shared__ float A[2][AH * AW];                               // u^n planes, 4-cell halo
    __shared__ float B[2][RY * RX];                               // u^{n+1} planes, region
    __shared__ float IA[(FL & F_INJ) ? RY * RX : 1];              // first-step injection plane
    __shared__ float IB[(FL & F_INJ) ? BY * BX : 1];              // second-step injection plane
    __shared__ double sred[NW];

    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int s = L / a.tiles;
    const int t = L - s * a.tiles;
    if (a.active && !a.active[s]) return;   // uniform over the workgroup
    const int gs = a.shot0 + s;
    const int tzi = t / (a.tiles_x * a.tiles_y);
    const int rem = t - tzi * a.tiles_x * a.tiles_y;
    const int tyi = rem / a.tiles_x, txi = rem - tyi * a.tiles_x;
    const int x0 = txi * BX, y0 = tyi * BY, zc0 = tzi * BZ;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int XS = a.XS, YS = a.YS;
    const uint32_t PS = (uint32_t)(YS * XS);
    const int tA = a.step, tB = a.step + a.dir;
    const float* __restrict__ cur = a.cur + s * a.fstride;
    float* __restrict__ nxt = a.nxt + s * a.fstride;
    const float* __restrict__ din = a.din + s * a.fstride;
    float* __restrict__ dnx = a.dnx + s * a.fstride;

    // this thread's region columns: lane = region column, rows wv + r * NW
    const int x = x0 - HALO + lane;
    const int ix = x - a.nb;
    const bool xin = x >= 0 && x < a.nxp;
    const bool xout = lane >= HALO && lane < HALO + BX;
    int ry[RPT], iy[RPT];
    uint32_t col[RPT];
    float kxy[RPT];
    bool cin[RPT], cout[RPT], xyph[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        ry[r] = wv + r * NW;
        const int y = y0 - HALO + ry[r];
        iy[r] = y - a.nb;
        cin[r] = xin && y >= 0 && y < a.nyp;
        col[r] = cin[r] ? (uint32_t)((y + GH) * XS + x + GH) : 0u;
        kxy[r] = at(a.kx, (uint32_t)min(max(x, 0), a.nxp - 1)) + at(a.ky, (uint32_t)min(max(y, 0), a.nyp - 1));
        cout[r] = cin[r] && xout && ry[r] >= HALO && ry[r] < HALO + BY;
        xyph[r] = ix >= 0 && ix < a.nx && iy[r] >= 0 && iy[r] < a.ny;
    }
    // the halo cell of the u^n plane this thread stages (tid < NHALO)
    int hl = -1;
    uint32_t ho = ~0u;
    if (tid < NHALO) {
        int hy, hx, h = tid;
        if (h < 2 * HALO * AW) {                   // y slabs, full width
            hy = h / AW;
            hx = h - hy * AW;
            if (hy >= HALO) hy += RY;
        } else {                                   // x columns beside the region rows
            h -= 2 * HALO * AW;
            hy = HALO + h / (2 * HALO);
            hx = h % (2 * HALO);
            if (hx >= HALO) hx += RX;
        }
        hl = hy * AW + hx;
        const int gx = x0 - 2 * HALO + hx, gy = y0 - 2 * HALO + hy;
        if (gx >= 0 && gx < a.nxp && gy >= 0 && gy < a.nyp) ho = (uint32_t)((gy + GH) * XS + gx + GH);
    }

    // the point source, relative to the region (first step) and the block (second)
    int srx = -1000, sry = -1000, srz = -1000;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    if constexpr ((FL & (F_SRC_POINT | F_SRC_REC | F_NORMAL | F_RUPD)) != 0) {
        sx = (float)a.src_pos[gs * 3 + 0];
        sz = (float)a.src_pos[gs * 3 + 1];
        sy = (float)a.src_pos[gs * 3 + 2];
        srx = a.src_pos[gs * 3 + 0] + a.nb - (x0 - HALO);
        sry = a.src_pos[gs * 3 + 2] + a.nb - (y0 - HALO);
        srz = a.src_pos[gs * 3 + 1] + a.nb;
    }
    float wavA = 0.f, wavB = 0.f;
    if constexpr ((FL & F_SRC_POINT) != 0) {
        wavA = a.wavelet[(int64_t)s * a.nt + tA];
        wavB = a.wavelet[(int64_t)s * a.nt + tB];
    }
    float alp = 0.f, bet = 0.f;
    if constexpr ((FL & F_CG_FUSE) != 0) {
        alp = (float)a.cg_alpha[s];
        bet = (float)a.cg_beta[s];
    }

    const int64_t nrec_s = (FL & (F_INJ | F_GATHER)) ? a.rec_ptr[gs + 1] - a.rec_ptr[gs] : 0;
    const int64_t doff = (FL & (F_INJ | F_GATHER)) ? (int64_t)a.nt * (a.rec_ptr[gs] - a.rec_ptr[a.shot0]) : 0;
    int ge = 0, gend = 0;
    if constexpr ((FL & F_GATHER) != 0) {
        const int32_t* gp = a.gat_ptr + (int64_t)gs * (a.tiles + 1);
        ge = gp[t];
        gend = gp[t + 1];
        // d^{tA-1} = R u^{tA}, straight from u^{tA}
        if (tA > 0) {
            float* dn = a.gat_data + doff + (int64_t)(tA - 1) * nrec_s;
            for (int e = ge + tid; e < gend; e += NTH) {
                const int cell = a.gat_cell[e];
                const int lz = cell / (BX * BY), r2 = cell - lz * BX * BY;
                const int cy = r2 / BX, cx = r2 - cy * BX;
                dn[a.gat_rid[e]] = cur[((zc0 + lz + GH) * YS + y0 + cy + GH) * XS + x0 + cx + GH];
            }
        }
    }
    int ie = 0, iend = 0, ie2 = 0, iend2 = 0;
    const float* djA = nullptr;
    const float* djB = nullptr;
    if constexpr ((FL & F_INJ) != 0) {
        const int32_t* ip = a.inj_ptr + (int64_t)gs * (a.tiles + 1);
        ie = ip[t];
        iend = ip[t + 1];
        const int32_t* ip2 = a.inj2_ptr + (int64_t)gs * (a.tiles + 1);
        ie2 = ip2[t];
        iend2 = ip2[t + 1];
        djA = a.inj_data + doff + (int64_t)tA * nrec_s;
        djB = a.inj_data + doff + (int64_t)tB * nrec_s;
    }

    // register windows: wn[r][k] = u^n at z1 - 4 + k; w1[r][k] = u^{n+1} at
    // z1 - 9 + k before iteration i's first step (z1 - 8 + k after it);
    // dq[r][k] = d^{n+1} at z1 - 5 + k (z1 - 4 + k after it)
    float wn[RPT][WIN], w1[RPT][WIN], dq[RPT][HALO + 1];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
#pragma unroll
        for (int k = 0; k < WIN; ++k) w1[r][k] = 0.f;
#pragma unroll
        for (int k = 0; k <= HALO; ++k) dq[r][k] = 0.f;
#pragma unroll
        for (int k = 0; k < 2 * HALO; ++k) {
            const int zz = zc0 - 2 * HALO + k;
            wn[r][k] = (cin[r] && zz >= 0 && zz < a.nzp) ? at(cur, (uint32_t)(zz + GH) * PS + col[r]) : 0.f;
        }
        wn[r][2 * HALO] = 0.f;
    }
    const int nit = min(BZ, a.nzp - zc0) + 2 * HALO;
    // state loads of the next PF iterations' planes z1: u^n at z1 + 4, c and
    // d^n at z1, the halo cell's u^n at z1 (set 0 is the next to be used)
    float nw[PF][RPT], nc[PF][RPT], nd[PF][RPT], nh[PF];
    auto load_plane = [&](int z1, float* w4, float* cc, float* dd, float& hh) {
        const bool zin = z1 >= 0 && z1 < a.nzp;
        const bool zin4 = z1 + HALO >= 0 && z1 + HALO < a.nzp;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            w4[r] = (cin[r] && zin4) ? at(cur, (uint32_t)(z1 + HALO + GH) * PS + col[r]) : 0.f;
            cc[r] = (cin[r] && zin) ? at(a.c2, (uint32_t)(z1 + GH) * PS + col[r]) : 0.f;
            dd[r] = (cin[r] && zin) ? at(din, (uint32_t)(z1 + GH) * PS + col[r]) : 0.f;
        }
        hh = (zin && ho != ~0u) ? at(cur, (uint32_t)(z1 + GH) * PS + ho) : 0.f;
    };
#pragma unroll
    for (int k = 0; k < PF; ++k) load_plane(zc0 - HALO + k, nw[k], nc[k], nd[k], nh[k]);
    // c on the block for the second step of iteration ii (plane z2 = zc0 - 8
    // + ii), issued one iteration ahead (the correlation's loads gain nothing
    // from that: they stay in their own iteration)
    float nc2[RPT];
    auto load_c2 = [&](int ii) {
        const int zz = zc0 - 2 * HALO + ii;
        const bool on = ii >= 2 * HALO && ii < nit;   // uniform
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            nc2[r] = (on && cout[r] && zz < a.nzp) ? at(a.c2, (uint32_t)(zz + GH) * PS + col[r]) : 0.f;
    };
    load_c2(0);

    double acc = 0.0;
    for (int i = 0; i < nit; ++i) {
        const int z1 = zc0 - HALO + i, z2 = z1 - HALO;
        const bool z1in = z1 >= 0 && z1 < a.nzp;
        const bool l2 = i >= 2 * HALO;                        // second step active (z2 < nzp by nit)
        const bool z1out = z1 >= zc0 && z1 < zc0 + BZ && z1in; // first step's plane is an output plane
        float* const Ab = A[i & 1];
        float* const Bb = B[i & 1];
        // ---- publish this iteration's planes
        float c1[RPT], d1v[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            wn[r][2 * HALO] = nw[0][r];
            Ab[(ry[r] + HALO) * AW + lane + HALO] = wn[r][HALO];
            Bb[ry[r] * RX + lane] = w1[r][HALO + 1];          // u^{n+1} at z2
            c1[r] = nc[0][r];
            d1v[r] = nd[0][r];
        }
        if (hl >= 0) Ab[hl] = nh[0];
        // ---- this iteration's dense loads and the next iteration's state loads
        const int iz1 = z1 - a.nb, iz2 = z2 - a.nb;
        const bool z1ph = iz1 >= 0 && iz1 < a.nz, z2ph = iz2 >= 0 && iz2 < a.nz;
        float qA[RPT], poA[RPT], xoA[RPT], pvA[RPT], rvA[RPT];
        float c2B[RPT], qB[RPT], poB[RPT], xoB[RPT], pvB[RPT], rvB[RPT], stA[RPT], stB[RPT], gB[RPT];
        uint32_t piA[RPT], piB[RPT];
        bool phA[RPT], phB[RPT], oA[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            phA[r] = xyph[r] && z1ph;
            oA[r] = phA[r] && cout[r] && z1out;
            phB[r] = xyph[r] && z2ph && cout[r] && l2;
            piA[r] = phA[r] ? (uint32_t)((iz1 * a.ny + iy[r]) * a.nx + ix) : 0u;
            piB[r] = phB[r] ? (uint32_t)((iz2 * a.ny + iy[r]) * a.nx + ix) : 0u;
            qA[r] = 0.f; poA[r] = 0.f; xoA[r] = 0.f; pvA[r] = 0.f; rvA[r] = 0.f;
            qB[r] = 0.f; poB[r] = 0.f; xoB[r] = 0.f; pvB[r] = 0.f; rvB[r] = 0.f; stA[r] = 0.f; stB[r] = 0.f;
            gB[r] = 0.f;
            c2B[r] = nc2[r];
            if constexpr ((FL & F_SRC_DENSE) != 0) {
                qA[r] = phA[r] ? at(a.dsrc + voff(a, s, tA), piA[r]) : 0.f;
                qB[r] = phB[r] ? at(a.dsrc + voff(a, s, tB), piB[r]) : 0.f;
            }
            if constexpr ((FL & F_CG_FUSE) != 0) {
                const int64_t vA = ((int64_t)s * a.nt + tA) * a.nphys, vB = ((int64_t)s * a.nt + tB) * a.nphys;
                if (phA[r]) {
                    poA[r] = at(a.cg_p + vA, piA[r]);
                    qA[r] = fmaf(bet, poA[r], at(a.cg_r + vA, piA[r]));
                    if (oA[r]) xoA[r] = at(a.cg_x + vA, piA[r]);
                }
                if (phB[r]) {
                    poB[r] = at(a.cg_p + vB, piB[r]);
                    qB[r] = fmaf(bet, poB[r], at(a.cg_r + vB, piB[r]));
                    xoB[r] = at(a.cg_x + vB, piB[r]);
                }
            }
            if constexpr ((FL & F_NORMAL) != 0) {
                const int64_t vA = ((int64_t)s * a.nt + tA) * a.nphys, vB = ((int64_t)s * a.nt + tB) * a.nphys;
                if (oA[r]) {
                    pvA[r] = at(a.dp + vA, piA[r]);
                    if constexpr ((FL & F_RUPD) != 0) rvA[r] = at(a.cg_rw + vA, piA[r]);
                }
                if (phB[r]) {
                    pvB[r] = at(a.dp + vB, piB[r]);
                    if constexpr ((FL & F_RUPD) != 0) rvB[r] = at(a.cg_rw + vB, piB[r]);
                }
            }
            if constexpr ((FL & F_CORR) != 0) {
                if (phB[r]) {
                    const float* st = a.store + s * a.store_stride;
                    stA[r] = at(st + (int64_t)a.store_slot * a.nphys, piB[r]);
                    stB[r] = at(st + (int64_t)a.store_slot2 * a.nphys, piB[r]);
                    // the accumulator with the other dense loads: its latency
                    // overlaps the first step
                    gB[r] = at(a.gacc + (int64_t)s * a.nphys, piB[r]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k + 1 < PF; ++k) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                nw[k][r] = nw[k + 1][r];
                nc[k][r] = nc[k + 1][r];
                nd[k][r] = nd[k + 1][r];
            }
            nh[k] = nh[k + 1];
        }
        if (i + PF < nit)   // uniform over the workgroup
            load_plane(z1 + PF, nw[PF - 1], nc[PF - 1], nd[PF - 1], nh[PF - 1]);
        load_c2(i + 1);
        // ---- injection planes of this iteration (entries sorted by cell, i.e. by plane)
        bool injA = false, injB = false;
        if constexpr ((FL & F_INJ) != 0) {
            injA = ie2 < iend2 && a.inj2_cell[ie2] / (RX * RY) == i;
            injB = l2 && ie < iend && a.inj_cell[ie] / (BX * BY) == i - 2 * HALO;
            if (injA || injB) {   // uniform
                __syncthreads();   // the last injection planes have been read
                if (injA)
                    for (int k = tid; k < RX * RY; k += NTH) IA[k] = 0.f;
                if (injB)
                    for (int k = tid; k < BX * BY; k += NTH) IB[k] = 0.f;
                __syncthreads();
                if (injA) {
                    for (int e = ie2 + tid; e < iend2 && a.inj2_cell[e] / (RX * RY) == i; e += NTH) {
                        float v = 0.f;
                        for (int k = a.inj2_rptr[e]; k < a.inj2_rptr[e + 1]; ++k) v += djA[a.inj2_rid[k]];
                        IA[a.inj2_cell[e] - i * RX * RY] = v;
                    }
                    while (ie2 < iend2 && a.inj2_cell[ie2] / (RX * RY) == i) ++ie2;
                }
                if (injB) {
                    const int lz = i - 2 * HALO;
                    for (int e = ie + tid; e < iend && a.inj_cell[e] / (BX * BY) == lz; e += NTH) {
                        float v = 0.f;
                        for (int k = a.inj_rptr[e]; k < a.inj_rptr[e + 1]; ++k) v += djB[a.inj_rid[k]];
                        IB[a.inj_cell[e] - lz * BX * BY] = v;
                    }
                    while (ie < iend && a.inj_cell[ie] / (BX * BY) == lz) ++ie;
                }
            }
        }
        __syncthreads();

        // ---- first step on plane z1 (the region)
        const float kz1 = at(a.kz, (uint32_t)min(max(z1, 0), a.nzp - 1));
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            float un = 0.f, dn = 0.f;
            if (cin[r] && z1in) {
                const float lap = lap3(a, Ab + (ry[r] + HALO) * AW + lane + HALO, AW, wn[r]);
                float q = qA[r];
                const float qd = q;   // the extended (dense) part of the source
                const bool at_src = lane == srx && ry[r] == sry && z1 == srz;
                if constexpr ((FL & F_SRC_POINT) != 0) {
                    if (at_src) q += wavA;
                }
                if constexpr ((FL & F_INJ) != 0) {
                    if (injA) q += IA[ry[r] * RX + lane];
                }
                const float lq = fmaf(a.dx2, q, lap);
                dn = incr3(c1[r], lq, d1v[r], kxy[r] + kz1);
                un = wn[r][HALO] + dn;
                if (oA[r]) {
                    const int64_t vA = ((int64_t)s * a.nt + tA) * a.nphys;
                    if constexpr ((FL & F_CG_FUSE) != 0) {
                        at(a.cg_pn + vA, piA[r]) = qd;
                        if (alp != 0.f) at(a.cg_x + vA, piA[r]) = fmaf(alp, poA[r], xoA[r]);
                    }
                    float wb = 0.f;
                    if constexpr ((FL & (F_NORMAL | F_RUPD)) != 0) wb = annih3(a, ix, iy[r], iz1, sx, sy, sz);
                    outputs3<FL>(a, s, tA, piA[r], un, qd, lq, c1[r], wb, pvA[r], rvA[r], at_src, acc);
                }
            }
#pragma unroll
            for (int k = 0; k < 2 * HALO; ++k) w1[r][k] = w1[r][k + 1];
            w1[r][2 * HALO] = un;
#pragma unroll
            for (int k = 0; k < HALO; ++k) dq[r][k] = dq[r][k + 1];
            dq[r][HALO] = dn;
        }

        // ---- second step on plane z2 (the block)
        if (l2) {   // uniform
            const float kz2 = at(a.kz, (uint32_t)min(max(z2, 0), a.nzp - 1));
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                if (!cout[r]) continue;
                const float lap = lap3(a, Bb + ry[r] * RX + lane, RX, w1[r]);
                float q = qB[r];
                const float qd = q;
                const bool at_src = lane == srx && ry[r] == sry && z2 == srz;
                if constexpr ((FL & F_SRC_POINT) != 0) {
                    if (at_src) q += wavB;
                }
                if constexpr ((FL & F_INJ) != 0) {
                    if (injB) q += IB[(ry[r] - HALO) * BX + lane - HALO];
                }
                const float lq = fmaf(a.dx2, q, lap);
                const float dn = incr3(c2B[r], lq, dq[r][0], kxy[r] + kz2);
                const float un = w1[r][HALO] + dn;
                const uint32_t so = (uint32_t)(z2 + GH) * PS + col[r];
                at(dnx, so) = dn;
                at(nxt, so) = un;
                if (!phB[r]) continue;
                const int64_t vB = ((int64_t)s * a.nt + tB) * a.nphys;
                if constexpr ((FL & F_CG_FUSE) != 0) {
                    at(a.cg_pn + vB, piB[r]) = qd;
                    if (alp != 0.f) at(a.cg_x + vB, piB[r]) = fmaf(alp, poB[r], xoB[r]);
                }
                float wb = 0.f;
                if constexpr ((FL & (F_NORMAL | F_RUPD)) != 0) wb = annih3(a, ix, iy[r], iz2, sx, sy, sz);
                outputs3<FL>(a, s, tB, piB[r], un, qd, lq, c2B[r], wb, pvB[r], rvB[r], at_src, acc);
                if constexpr ((FL & F_CORR) != 0) {
                    // both steps' products chained, as two one-step launches add them
                    float* g = a.gacc + (int64_t)s * a.nphys;
                    const float gA = fmaf(w1[r][HALO], stA[r], gB[r]);
                    at(g, piB[r]) = fmaf(un, stB[r], gA);
                }
            }
            if constexpr ((FL & F_GATHER) != 0) {
                // d^{tA} = R u^{tA+1} for the receivers on plane z2
                const int lz = i - 2 * HALO;
                float* dn = a.gat_data + doff + (int64_t)tA * nrec_s;
                for (int e = ge + tid; e < gend && a.gat_cell[e] / (BX * BY) == lz; e += NTH) {
                    const int r2 = a.gat_cell[e] - lz * BX * BY;
                    const int cy = r2 / BX, cx = r2 - cy * BX;
                    dn[a.gat_rid[e]] = Bb[(cy + HALO) * RX + cx + HALO];
                }
                while (ge < gend && a.gat_cell[ge] / (BX * BY) == lz) ++ge;
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r)
#pragma unroll
            for (int k = 0; k < 2 * HALO; ++k) wn[r][k] = wn[r][k + 1];
    }

    if constexpr ((FL & (F_NORMAL | F_RUPD)) != 0) {
        if (a.part) {   // uniform over the launch
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (lane == 0) sred[wv] = acc;
            __syncthreads();
            if (tid == 0) {
                double sum = 0.0;
                for (int k = 0; k < NW; ++k) sum += sred[k];
                a.part[(int64_t)s * a.part_stride + t] += sum;
            }
        }
    }
}

template <unsigned FL>
esi_status_t launch3d_t2(Plan* P, const StepArgs& a) {
    const int blocks = a.tiles * a.nshots;
    hipLaunchKernelGGL(k_step3d_t2<FL>, dim3(blocks), dim3(NTH), 0, P->stream, a);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

}  // namespace

bool step3d_t2_has(unsigned flags) {
    switch (flags) {
        case F_SRC_POINT: case F_SRC_POINT | F_GATHER: case F_SRC_POINT | F_STORE:
        case F_SRC_POINT | F_GATHER | F_STORE: case F_SRC_DENSE: case F_SRC_DENSE | F_GATHER:
        case F_SRC_DENSE | F_STORE: case F_SRC_DENSE | F_GATHER | F_STORE:
        case F_CG_FUSE | F_GATHER | F_RUPD: case F_SRC_DENSE | F_GATHER | F_RUPD:
        case F_INJ: case F_INJ | F_OUT: case F_INJ | F_NORMAL: case F_INJ | F_NORMAL | F_RUPD:
        case F_INJ | F_CORR: case F_INJ | F_CORR | F_OUT: case F_INJ | F_CORR | F_SRC_REC:
            return true;
        default:
            return false;
    }
}

esi_status_t launch_step3d_t2(Plan* P, unsigned flags, const StepArgs& a) {
    switch (flags) {
#define ESI_CASE(F) case (F): return launch3d_t2<(F)>(P, a);
        ESI_CASE(F_SRC_POINT)
        ESI_CASE(F_SRC_POINT | F_GATHER)
        ESI_CASE(F_SRC_POINT | F_STORE)
        ESI_CASE(F_SRC_POINT | F_GATHER | F_STORE)
        ESI_CASE(F_SRC_DENSE)
        ESI_CASE(F_SRC_DENSE | F_GATHER)
        ESI_CASE(F_SRC_DENSE | F_STORE)
        ESI_CASE(F_SRC_DENSE | F_GATHER | F_STORE)
        ESI_CASE(F_CG_FUSE | F_GATHER | F_RUPD)
        ESI_CASE(F_SRC_DENSE | F_GATHER | F_RUPD)
        ESI_CASE(F_INJ)
        ESI_CASE(F_INJ | F_OUT)
        ESI_CASE(F_INJ | F_NORMAL)
        ESI_CASE(F_INJ | F_NORMAL | F_RUPD)
        ESI_CASE(F_INJ | F_CORR)
        ESI_CASE(F_INJ | F_CORR | F_OUT)
        ESI_CASE(F_INJ | F_CORR | F_SRC_REC)
#undef ESI_CASE
        default: return fail(ESI_ERR_ARG, "internal: unsupported 3D two-step flags " + std::to_string(flags));
    }
}

void step3d_t2_tile_shape(int* tx, int* ty, int* tz) { *tx = BX; *ty = BY; *tz = BZ; }

}  // namespace esi
