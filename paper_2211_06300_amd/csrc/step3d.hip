// One time step of the 3D 8th-order acoustic scheme (Sec. 4.1) with the same
// fused work as the 2D kernels (injection, recording, CG direction update,
// N p with p.Np partials, gradient correlations).
//
// 2.5D sweep: a 512-thread workgroup owns a 64 (x) x 16 (y) block of columns
// and a chunk of 32 z-planes; a thread owns two columns, rows ly and ly + 8.
// Each thread keeps the 9-value z windows of its columns in registers; the
// current plane of the block plus a 4-cell x/y halo is staged in a
// double-buffered LDS plane, so one barrier per plane suffices.  Sixteen rows
// per block put the y halo at half the block's rows, where eight rows per
// block read a plane's cells twice over.
// Receiver injection is applied per plane through a small LDS plane; the
// recording reads u^n straight from memory.  Storage is the padded grid with
// a zero ghost frame of GH cells, planes YS x XS floats apart.
#include "esi_internal.h"

namespace esi {

namespace {

constexpr int TX = 64, WY = 8, RY = 2;     // threads: 64 x 8, two rows each
constexpr int TY = WY * RY, TZC = 32;      // block of columns, z-chunk
constexpr int NTH = TX * WY;               // 512 threads
constexpr int PW = TX + 2 * HALO, PH = TY + 2 * HALO;   // staged plane 72 x 24
constexpr int NHALO = PW * PH - TX * TY;   // 704 halo cells per plane
static_assert(NHALO <= 2 * NTH, "two halo cells per thread");

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

template <unsigned FL>
__global__ __launch_bounds__(NTH) void k_step3d(const StepArgs a) {
    __shared__ float P[2][PH * PW];
    __shared__ float sinj[(FL & F_INJ) ? TX * TY : 1];
    __shared__ double sred[NTH / 64];

    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int s = L / a.tiles;
    const int t = L - s * a.tiles;
    if (a.active && !a.active[s]) return;   // uniform over the workgroup
    const int gs = a.shot0 + s;
    const int tzi = t / (a.tiles_x * a.tiles_y);
    const int rem = t - tzi * a.tiles_x * a.tiles_y;
    const int tyi = rem / a.tiles_x, txi = rem - tyi * a.tiles_x;
    const int x0 = txi * TX, y0 = tyi * TY, zc0 = tzi * TZC;
    const int tid = threadIdx.x, lx = tid & 63;
    const int ly = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int XS = a.XS, YS = a.YS;
    const uint32_t PS = (uint32_t)(YS * XS);                 // plane stride
    const float* __restrict__ cur = a.cur + s * a.fstride;
    float* __restrict__ nxt = a.nxt + s * a.fstride;
    const float* __restrict__ din = a.din + s * a.fstride;
    float* __restrict__ dnx = a.dnx + s * a.fstride;

    // this thread's columns: rows yr = ly + r * WY of the block
    const int x = x0 + lx;
    const int ix = x - a.nb;
    uint32_t col[RY];
    float kxy[RY];
    bool xyphys[RY], cin[RY];   // cin: the column lies on the padded grid
    int iy[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = y0 + ly + r * WY;
        col[r] = (uint32_t)((y + GH) * XS + x + GH);
        kxy[r] = at(a.kx, (uint32_t)min(x, a.nxp - 1)) + at(a.ky, (uint32_t)min(y, a.nyp - 1));
        iy[r] = y - a.nb;
        xyphys[r] = ix >= 0 && ix < a.nx && iy[r] >= 0 && iy[r] < a.ny;
        cin[r] = x < a.nxp && y < a.nyp;
    }
    // halo cells this thread stages: LDS index and in-plane storage offset
    int hl[2];
    uint32_t ho[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        int h = tid + k * NTH;
        hl[k] = -1;
        ho[k] = 0;
        if (h < NHALO) {
            int ry, rx;
            if (h < 2 * HALO * PW) {                          // y-halo slabs, full width
                ry = h / PW;
                rx = h - ry * PW;
                if (ry >= HALO) ry += TY;
            } else {                                          // x-halo, body rows
                h -= 2 * HALO * PW;
                ry = HALO + h / (2 * HALO);
                rx = h % (2 * HALO);
                if (rx >= HALO) rx += TX;
            }
            const int hx = x0 - HALO + rx, hy = y0 - HALO + ry;
            // cells off the padded grid sit in the zero ghost frame: LDS takes 0, no load
            hl[k] = ry * PW + rx;
            ho[k] = (hx >= 0 && hx < a.nxp && hy >= 0 && hy < a.nyp) ? (uint32_t)((hy + GH) * XS + hx + GH) : ~0u;
        }
    }

    const int64_t vbase = ((int64_t)s * a.nt + a.step) * a.nphys;
    // dsrc / dout hold the whole time axis, or blk_T steps (step n in slot n % blk_T)
    const int64_t vblk = a.blk_T ? ((int64_t)s * a.blk_T + a.step % a.blk_T) * a.nphys : vbase;
    const float* dsrc = (FL & F_SRC_DENSE) ? a.dsrc + vblk : nullptr;
    float* dout = (FL & (F_OUT | F_NORMAL)) ? a.dout + vblk : nullptr;
    const float* csc = ((FL & F_SRC_DENSE) && (FL & F_SCALE)) ? a.cg_s + (int64_t)s * a.nphys : nullptr;
    const float* dp = (FL & F_NORMAL) ? a.dp + vbase : nullptr;
    float* rw = ((FL & F_NORMAL) && (FL & F_RUPD)) ? a.cg_rw + vbase : nullptr;
    const float ral = ((FL & F_NORMAL) && (FL & F_RUPD)) ? (float)a.cg_alpha[s] : 0.f;
    float* gacc = (FL & (F_PENALTY | F_CORR)) ? a.gacc + (int64_t)s * a.nphys : nullptr;
    float* store = (FL & (F_STORE | F_CORR)) ? a.store + s * a.store_stride + (int64_t)a.store_slot * a.nphys : nullptr;
    // paired correlation: this launch also adds the previous step's product,
    // its input field times store slot store_slot2, first (uniform)
    const bool pair = (FL & F_CORR) != 0 && a.corr_pair;
    const float* store_prev = pair ? a.store + s * a.store_stride + (int64_t)a.store_slot2 * a.nphys : nullptr;
    float alp = 0.f, bet = 0.f;
    const float* cgp = nullptr; const float* cgr = nullptr; float* cgpn = nullptr; float* cgx = nullptr;
    if constexpr ((FL & F_CG_FUSE) != 0) {
        alp = (float)a.cg_alpha[s];
        bet = (float)a.cg_beta[s];
        cgp = a.cg_p + vbase; cgr = a.cg_r + vbase; cgpn = a.cg_pn + vbase; cgx = a.cg_x + vbase;
    }

    const int64_t nrec_s = (FL & (F_INJ | F_GATHER)) ? a.rec_ptr[gs + 1] - a.rec_ptr[gs] : 0;
    const int64_t doff = (FL & (F_INJ | F_GATHER)) ? (int64_t)a.nt * (a.rec_ptr[gs] - a.rec_ptr[a.shot0]) : 0;
    if constexpr ((FL & F_GATHER) != 0) {
        // d^{n-1} = R u^n for the receivers of this block, straight from u^n
        if (a.step > 0) {
            const int32_t* gp = a.gat_ptr + (int64_t)gs * (a.tiles + 1);
            float* dn = a.gat_data + doff + (int64_t)(a.step - 1) * nrec_s;
            for (int e = gp[t] + tid; e < gp[t + 1]; e += NTH) {
                const int cell = a.gat_cell[e];
                const int lz = cell / (TX * TY), r2 = cell - lz * TX * TY;
                const int cy = r2 / TX, cx = r2 - cy * TX;
                dn[a.gat_rid[e]] = cur[((zc0 + lz + GH) * YS + y0 + cy + GH) * XS + x0 + cx + GH];
            }
        }
    }
    int ie = 0, iend = 0;
    const float* dj = nullptr;
    if constexpr ((FL & F_INJ) != 0) {
        const int32_t* ip = a.inj_ptr + (int64_t)gs * (a.tiles + 1);
        ie = ip[t];
        iend = ip[t + 1];
        dj = a.inj_data + doff + (int64_t)a.step * nrec_s;
    }
    int src_cell = -1;
    float src_val = 0.f;
    if constexpr ((FL & (F_SRC_POINT | F_SRC_REC)) != 0) {
        if (a.src_tile[gs] == t) {
            src_cell = a.src_cell[gs];
            if constexpr ((FL & F_SRC_POINT) != 0) src_val = a.wavelet[(int64_t)s * a.nt + a.step];
        }
    }
    float sx = 0.f, sy = 0.f, sz = 0.f;
    if constexpr ((FL & (F_NORMAL | F_PENALTY | F_RUPD)) != 0) {
        sx = (float)a.src_pos[gs * 3 + 0];
        sz = (float)a.src_pos[gs * 3 + 1];
        sy = (float)a.src_pos[gs * 3 + 2];
    }

    // z windows of this thread's columns: w[r][k] = u at z - 4 + k.  A plane's
    // own loads (the windows' new values, the halo cells, c, d) are issued one
    // plane ahead, before the barrier of the plane in between, so their
    // latency overlaps that plane's stencil work.
    float w[RY][2 * HALO + 1];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int k = 0; k < 2 * HALO; ++k) {
            const int zz = zc0 - HALO + k;
            w[r][k] = (cin[r] && zz >= 0 && zz < a.nzp) ? at(cur, (uint32_t)(zz + GH) * PS + col[r]) : 0.f;
        }
    const int zend = min(zc0 + TZC, a.nzp);
    float nw[RY], nc[RY], nd[RY], nh[2];   // the next plane's loads
    {
        const uint32_t pz = (uint32_t)(zc0 + GH) * PS;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            nw[r] = (cin[r] && zc0 + 4 < a.nzp) ? at(cur, pz + 4u * PS + col[r]) : 0.f;
            nc[r] = cin[r] ? at(a.c2, pz + col[r]) : 0.f;
            nd[r] = cin[r] ? at(din, pz + col[r]) : 0.f;
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) nh[k] = (hl[k] >= 0 && ho[k] != ~0u) ? at(cur, pz + ho[k]) : 0.f;
    }
    double acc = 0.0;
    for (int z = zc0; z < zend; ++z) {
        const int lz = z - zc0;
        const uint32_t pz = (uint32_t)(z + GH) * PS;
        float* Pb = P[lz & 1];
        float c2v[RY], dv[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            w[r][2 * HALO] = nw[r];
            Pb[(ly + r * WY + HALO) * PW + lx + HALO] = w[r][HALO];
            c2v[r] = nc[r];
            dv[r] = nd[r];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (hl[k] >= 0) Pb[hl[k]] = nh[k];
        // this plane's dense loads
        const float kz = at(a.kz, (uint32_t)min(z, a.nzp - 1));
        const int iz = z - a.nb;
        bool ph[RY];
        uint32_t pi[RY];
        float q[RY], po[RY], xo[RY], pv[RY], stv[RY], rv[RY], gv[RY], stp[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            ph[r] = xyphys[r] && iz >= 0 && iz < a.nz;
            pi[r] = ph[r] ? (uint32_t)((iz * a.ny + iy[r]) * a.nx + ix) : 0u;
            q[r] = 0.f; po[r] = 0.f; xo[r] = 0.f; pv[r] = 0.f; stv[r] = 0.f; rv[r] = 0.f; gv[r] = 0.f; stp[r] = 0.f;
            if constexpr ((FL & F_SRC_DENSE) != 0) {
                q[r] = ph[r] ? at(dsrc, pi[r]) : 0.f;
                if constexpr ((FL & F_SCALE) != 0) q[r] = q[r] * at(csc, pi[r]);   // cell-scaled dense source
            }
            if constexpr ((FL & F_CG_FUSE) != 0) {
                po[r] = at(cgp, pi[r]);
                xo[r] = at(cgx, pi[r]);
                q[r] = ph[r] ? fmaf(bet, po[r], at(cgr, pi[r])) : 0.f;
            }
            if constexpr ((FL & F_NORMAL) != 0) pv[r] = at(dp, pi[r]);
            if constexpr ((FL & F_NORMAL) != 0 && (FL & F_RUPD) != 0) rv[r] = at(rw, pi[r]);
            // the accumulator is read here, with the other dense loads, so that
            // its latency overlaps the plane's stencil work
            if constexpr ((FL & (F_PENALTY | F_CORR)) != 0) gv[r] = at(gacc, pi[r]);
            if constexpr ((FL & F_CORR) != 0) {
                stv[r] = at(store, pi[r]);
                if (pair) stp[r] = at(store_prev, pi[r]);
            }
        }
        bool inj_here = false;
        if constexpr ((FL & F_INJ) != 0) {
            // entries are sorted by cell, i.e. by plane first
            if (ie < iend && a.inj_cell[ie] / (TX * TY) == lz) {
                inj_here = true;
                __syncthreads();                  // the last injection plane has been read
                for (int i = tid; i < TX * TY; i += NTH) sinj[i] = 0.f;
                __syncthreads();
                int e = ie + tid;
                while (e < iend && a.inj_cell[e] / (TX * TY) == lz) {
                    float v = 0.f;
                    for (int k = a.inj_rptr[e]; k < a.inj_rptr[e + 1]; ++k) v += dj[a.inj_rid[k]];
                    sinj[a.inj_cell[e] - lz * TX * TY] = v;
                    e += NTH;
                }
                while (ie < iend && a.inj_cell[ie] / (TX * TY) == lz) ++ie;
            }
        }
        if (z + 1 < zend) {   // uniform over the workgroup
            const uint32_t pn = pz + PS;
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                nw[r] = (cin[r] && z + 5 < a.nzp) ? at(cur, pn + 4u * PS + col[r]) : 0.f;
                nc[r] = cin[r] ? at(a.c2, pn + col[r]) : 0.f;
                nd[r] = cin[r] ? at(din, pn + col[r]) : 0.f;
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) nh[k] = (hl[k] >= 0 && ho[k] != ~0u) ? at(cur, pn + ho[k]) : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int yl = ly + r * WY;                     // row within the block
            const float* cp = Pb + (yl + HALO) * PW + lx + HALO;
            const float cv = w[r][HALO];
            float lx_ = a.w1 * ((cp[-1] - cv) + (cp[1] - cv));
            lx_ = fmaf(a.w2, (cp[-2] - cv) + (cp[2] - cv), lx_);
            lx_ = fmaf(a.w3, (cp[-3] - cv) + (cp[3] - cv), lx_);
            lx_ = fmaf(a.w4, (cp[-4] - cv) + (cp[4] - cv), lx_);
            float ly_ = a.w1 * ((cp[-PW] - cv) + (cp[PW] - cv));
            ly_ = fmaf(a.w2, (cp[-2 * PW] - cv) + (cp[2 * PW] - cv), ly_);
            ly_ = fmaf(a.w3, (cp[-3 * PW] - cv) + (cp[3 * PW] - cv), ly_);
            ly_ = fmaf(a.w4, (cp[-4 * PW] - cv) + (cp[4 * PW] - cv), ly_);
            float lz_ = a.w1 * ((w[r][3] - cv) + (w[r][5] - cv));
            lz_ = fmaf(a.w2, (w[r][2] - cv) + (w[r][6] - cv), lz_);
            lz_ = fmaf(a.w3, (w[r][1] - cv) + (w[r][7] - cv), lz_);
            lz_ = fmaf(a.w4, (w[r][0] - cv) + (w[r][8] - cv), lz_);
            const float lap = (lx_ + ly_) + lz_;
            const int pcell = yl * TX + lx;                 // cell within the plane
            const int cell = lz * TX * TY + pcell;
            float qq = q[r];
            const float qd = qq;   // the extended (dense) part of the source
            if constexpr ((FL & F_SRC_POINT) != 0) {
                if (cell == src_cell) qq += src_val;
            }
            if constexpr ((FL & F_INJ) != 0) {
                if (inj_here) qq += sinj[pcell];
            }
            const float kap = kxy[r] + kz;
            const float lq = fmaf(a.dx2, qq, lap);
            const float dn = fmaf(c2v[r], lq, (1.f - kap) * dv[r]) * __builtin_amdgcn_rcpf(1.f + kap);
            const float un = cv + dn;
            // cells past the padded grid sit in the zero ghost frame (they would
            // compute 0): neither loaded nor stored
            const uint32_t so = pz + col[r];
            if (cin[r]) {
                at(dnx, so) = dn;
                at(nxt, so) = un;
            }
            if (ph[r]) {
                const uint32_t pr = pi[r];
                if constexpr ((FL & F_CG_FUSE) != 0) {
                    at(cgpn, pr) = qq;
                    if (alp != 0.f) at(cgx, pr) = fmaf(alp, po[r], xo[r]);
                }
                if constexpr ((FL & F_OUT) != 0) at(dout, pr) = un;
                if constexpr ((FL & F_SRC_REC) != 0) {
                    if (cell == src_cell) a.src_rec[(int64_t)s * a.nt + a.step] = un;
                }
                float wb = 0.f;
                if constexpr ((FL & (F_NORMAL | F_PENALTY | F_RUPD)) != 0) {
                    if (a.w_identity) {
                        wb = a.beta;
                    } else {
                        // the hardware square root (within 1 ulp; the argument
                        // is a sum of squared integers, never denormal)
                        const float ddx = (float)ix - sx, ddy = (float)iy[r] - sy, ddz = (float)iz - sz;
                        const float bb = __builtin_amdgcn_sqrtf(ddx * ddx + ddy * ddy + ddz * ddz) + a.b_eps;
                        wb = a.beta * (bb * bb);
                    }
                }
                if constexpr ((FL & (F_CG_FUSE | F_SRC_DENSE)) != 0 && (FL & F_RUPD) != 0)
                    acc += (double)(qd * (wb * qd));   // beta B^2 p.p of the direction (dense source)
                if constexpr ((FL & F_NORMAL) != 0) {
                    const float np = fmaf(wb, pv[r], un);
                    if constexpr ((FL & F_RUPD) != 0) {   // r -= alpha N p, as a separate pass would
                        const float rn = fmaf(-ral, np, rv[r]);
                        at(rw, pr) = rn;
                        acc += (double)(rn * rn);
                    } else {
                        at(dout, pr) = np;
                        acc += (double)pv[r] * (double)np;
                    }
                }
                if constexpr ((FL & F_PENALTY) != 0) {
                    at(gacc, pr) = fmaf(wb * qd, c2v[r] * a.inv_dt2 * lq, gv[r]);
                    acc += (double)(wb * qd) * (double)qd;   // penalty term (kept when a.part is set)
                }
                if constexpr ((FL & F_STORE) != 0) at(store, pr) = c2v[r] * a.inv_dt2 * lq;
                if constexpr ((FL & F_CORR) != 0) {
                    // the previous step's product first, as a two-step launch chains them
                    const float g = pair ? fmaf(cv, stp[r], gv[r]) : gv[r];
                    at(gacc, pr) = fmaf(un, stv[r], g);
                }
            }
#pragma unroll
            for (int k = 0; k < 2 * HALO; ++k) w[r][k] = w[r][k + 1];
        }
    }

    if constexpr ((FL & (F_NORMAL | F_PENALTY | F_RUPD)) != 0) {
        if (a.part) {   // uniform over the launch
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (lx == 0) sred[ly] = acc;
            __syncthreads();
            if (tid == 0) {
                double sum = 0.0;
                for (int k = 0; k < NTH / 64; ++k) sum += sred[k];
                a.part[(int64_t)s * a.part_stride + t] += sum;
            }
        }
    }
}

template <unsigned FL>
esi_status_t launch3d(Plan* P, const StepArgs& a) {
    const int blocks = a.tiles * a.nshots;
    hipLaunchKernelGGL(k_step3d<FL>, dim3(blocks), dim3(NTH), 0, P->stream, a);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

}  // namespace

esi_status_t launch_step3d(Plan* P, unsigned flags, const StepArgs& a) {
    switch (flags) {
#define ESI_CASE(F) case (F): return launch3d<(F)>(P, a);
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
        ESI_CASE(F_CG_FUSE | F_GATHER | F_RUPD)
        ESI_CASE(F_SRC_DENSE | F_GATHER | F_RUPD)
        ESI_CASE(F_SRC_DENSE | F_SCALE | F_GATHER)
        ESI_CASE(F_INJ)
        ESI_CASE(F_INJ | F_OUT)
        ESI_CASE(F_INJ | F_SRC_REC)
        ESI_CASE(F_INJ | F_NORMAL)
        ESI_CASE(F_INJ | F_NORMAL | F_RUPD)
        ESI_CASE(F_INJ | F_CORR)
        ESI_CASE(F_INJ | F_CORR | F_OUT)
        ESI_CASE(F_INJ | F_CORR | F_SRC_REC)
#undef ESI_CASE
        default: return fail(ESI_ERR_ARG, "internal: unsupported 3D step flags " + std::to_string(flags));
    }
}

void step3d_tile_shape(int* tx, int* ty, int* tz) { *tx = TX; *ty = TY; *tz = TZC; }

}  // namespace esi
