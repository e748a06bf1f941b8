// Learned preconditioner network: a four-level U-Net (channels 16/32/64/128)
// with bfloat16 weights and activations and float32 accumulation, trained and
// run entirely by the kernels below.  The paper leaves the preconditioner of
// its CG open (Sec. 4.2 and Sec. 6: fewer inner iterations need an efficient
// preconditioner); the network, its loss and its use are this library's.
//
// Activations are NHWC bfloat16 (channels contiguous, 16-byte aligned groups
// of eight).  A decoder level's concatenation [upsampled, skip] is one buffer
// of two planar halves, each a dense NHWC tensor of ch channels: the
// transposed convolution writes the first, the encoder's second convolution
// writes its output straight into the second, and the decoder's first
// convolution reads the pair as 2 ch channels.  The skip costs no copy, and
// no kernel writes part of another's cache lines.
//
// 3x3 convolutions (forward and data gradient) are implicit GEMMs on
// v_mfma_f32_16x16x32_bf16: D[cout][pixel] = sum_{tap, ci} W[tap][cout][ci]
// X[pixel + tap][ci], with each input tile staged in LDS once and read by all
// nine taps, and the weights packed in the instruction's operand order.  A
// lane stores four consecutive output channels of one pixel (8 bytes).  The
// data gradient is the same kernel with taps reversed and weights transposed.
// Transposed convolutions use the same instruction with operands loaded
// straight from memory (each input pixel is read once); their data gradient
// and the weight gradients use v_mfma_f32_16x16x16_bf16.  The weight gradient
// is a GEMM over pixels (split into fixed chunks, partials summed in a fixed
// order).
#include <cmath>
#include <cstring>
#include <vector>

#include "esi_internal.h"

namespace esi {
namespace {

typedef uint16_t bf16_t;
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
union bf8u {   // eight bf16 values as one 16-byte load or store
    uint4 u;
    uint16_t h[8];
};

constexpr int NT = 256;

__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }
// round to nearest even (finite inputs)
__device__ __forceinline__ bf16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
static uint16_t f2bf_host(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// 3x3 convolution, same size, zero padding, as an implicit GEMM on
// v_mfma_f32_16x16x32_bf16: D[m][pixel] = sum over (tap, k) of
// A[tap][m][k] X[pixel + tap][k].  X and Y are NHWC views with pixel strides
// sx, sy (elements); K input and M output channels, multiples of 16.  A view
// may hold its channels as two planar halves: channels from xsplit on
// (ysplit for Y) live xhs (yhs) elements further on, at channel c - xsplit.
//
// The contraction runs in blocks of 32: (tap, 32 channels) when K is a
// multiple of 32 (CK = 32, nine blocks per chunk of 32 channels), else (two
// taps, 16 channels) (CK = 16, five blocks, the tenth tap with zero weights).
// Lane l of a block holds the 8 consecutive contraction indices of k-group
// l / 16, for row (A) or pixel (B) l % 16; A is packed in that order by
// k_pack_frag, so a lane's weights are one coalesced 16-byte load.
//
// Workgroup: NWV waves, RPW output rows each, 64 pixels (4 groups of 16) x
// 16 CB output channels.  Per chunk of CK input channels the (NWV RPW + 2) x 66
// input tile and the chunk's weight operands are staged in LDS once; every
// tap then reads its shifted operands from there.  (Padding the pixel stride
// by 8 or 16 elements measured 1.5-4 % slower: the smaller tile keeps more
// workgroups resident.)
//
// The grid is persistent: workgroup b takes the (tile, chunk) steps of tiles
// b, b + gridDim.x, ...  The global loads of the next step are issued
// before the current step's MFMAs and land in registers, so memory latency
// overlaps the arithmetic; a tile's outputs are stored after its last chunk.
constexpr int frag_ck(int K) { return K % 32 == 0 ? 32 : 16; }
constexpr int frag_nkb(int ck) { return ck == 32 ? 9 : 5; }

template <int CB, int RPW, int CK, int NWV>
struct Conv3Tile {
    static constexpr int NTW = 64 * NWV;                  // threads of a workgroup
    static constexpr int ROWS = NWV * RPW;                // output rows of a tile
    static constexpr int NKB = frag_nkb(CK);
    static constexpr int TR = ROWS + 2, TC = 66, PS = CK, SUB = CK / 8;
    static constexpr int NQ = TR * TC * SUB, NL = (NQ + NTW - 1) / NTW;   // 16-byte pieces of a tile, per thread
    static constexpr int NWQ = NKB * CB * 64, NWL = (NWQ + NTW - 1) / NTW;  // and of a chunk's weights
};

template <int CB, int RPW, int CK, int NWV>
__global__ __launch_bounds__(64 * NWV) __attribute__((amdgpu_waves_per_eu(2))) void k_conv3(
    const bf16_t* __restrict__ X, int sx, int64_t xhs, int xsplit, int K, const bf16_t* __restrict__ Af, int ncb,
    const float* __restrict__ bias, bf16_t* __restrict__ Y, int sy, int64_t yhs, int ysplit, int M, int H, int W,
    int N, int relu) {
    using T = Conv3Tile<CB, RPW, CK, NWV>;
    __shared__ __align__(16) bf16_t xs[T::TR * T::TC * T::PS];
    __shared__ __align__(16) bf16_t ws[T::NWQ * 8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int jl = lane & 15, g = lane >> 4;
    const int ncog = M / (16 * CB), nchunk = K / CK;
    const int ntx = (W + 63) / 64, nty = (H + T::ROWS - 1) / T::ROWS;
    const int ntiles = ntx * nty * N * ncog;
    // tiles b, b + gridDim.x, ... of this workgroup b
    const int nmine = blockIdx.x < ntiles ? (ntiles - 1 - (int)blockIdx.x) / (int)gridDim.x + 1 : 0;
    const int nsteps = nmine * nchunk;

    // step -> tile origin, image, output-channel group, chunk
    auto decode = [&](int step, int& x0, int& y0, int& n, int& cbg, int& chunk) {
        const int t = (int)blockIdx.x + (step / nchunk) * (int)gridDim.x;
        chunk = step % nchunk;
        x0 = (t % ntx) * 64;
        y0 = ((t / ntx) % nty) * T::ROWS;
        const int z = t / (ntx * nty);
        n = z / ncog;
        cbg = z % ncog;
    };
    uint4 st[T::NL], sw[T::NWL];
    auto fetch = [&](int step) {
        int x0, y0, n, cbg, chunk;
        decode(step, x0, y0, n, cbg, chunk);
        const bf16_t* Xn = X + (int64_t)n * H * W * sx;
#pragma unroll
        for (int l = 0; l < T::NL; ++l) {
            const int q = threadIdx.x + l * T::NTW;
            const int sub = q % T::SUB, px = (q / T::SUB) % T::TC, row = q / (T::SUB * T::TC);
            const int yy = y0 - 1 + row, xx = x0 - 1 + px;
            const int ch = chunk * CK + sub * 8;             // channels at or past xsplit: second half
            const int64_t hoff = ch >= xsplit ? xhs - xsplit : 0;
            st[l] = uint4{0u, 0u, 0u, 0u};
            if (q < T::NQ && yy >= 0 && yy < H && xx >= 0 && xx < W)
                st[l] = *reinterpret_cast<const uint4*>(Xn + ((int64_t)yy * W + xx) * sx + hoff + ch);
        }
        // the workgroup's weight operands of the chunk: [kb][c][lane][8]
#pragma unroll
        for (int l = 0; l < T::NWL; ++l) {
            const int q = threadIdx.x + l * T::NTW;
            const int kbc = q / 64, kb = kbc / CB, c = kbc % CB;
            sw[l] = uint4{0u, 0u, 0u, 0u};
            if (q < T::NWQ)
                sw[l] = *reinterpret_cast<const uint4*>(
                    Af + (((int64_t)chunk * T::NKB + kb) * ncb + cbg * CB + c) * 512 + (q % 64) * 8);
        }
    };

    f4 acc[RPW][4][CB];
#pragma unroll
    for (int r = 0; r < RPW; ++r)
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int c = 0; c < CB; ++c) acc[r][p][c] = f4{0.f, 0.f, 0.f, 0.f};

    if (nsteps > 0) fetch(0);
    for (int step = 0; step < nsteps; ++step) {
        if (step) __syncthreads();   // every wave is done reading the previous step's LDS
#pragma unroll
        for (int l = 0; l < T::NL; ++l) {
            const int q = threadIdx.x + l * T::NTW;
            const int sub = q % T::SUB, px = (q / T::SUB) % T::TC, row = q / (T::SUB * T::TC);
            if (q < T::NQ) *reinterpret_cast<uint4*>(xs + (row * T::TC + px) * T::PS + sub * 8) = st[l];
        }
#pragma unroll
        for (int l = 0; l < T::NWL; ++l) {
            const int q = threadIdx.x + l * T::NTW;
            if (q < T::NWQ) *reinterpret_cast<uint4*>(ws + q * 8) = sw[l];
        }
        __syncthreads();
        if (step + 1 < nsteps) fetch(step + 1);   // lands while this step computes
#pragma unroll
        for (int kb = 0; kb < T::NKB; ++kb) {
            const int tap = CK == 32 ? kb : min(2 * kb + (g >> 1), 8);
            const int koff = CK == 32 ? 8 * g : 8 * (g & 1);
            const int dy = tap / 3, dx = tap % 3;
            bf16x8 a[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c)
                a[c] = *reinterpret_cast<const bf16x8*>(ws + ((kb * CB + c) * 64 + lane) * 8);
#pragma unroll
            for (int r = 0; r < RPW; ++r)
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const bf16x8 b = *reinterpret_cast<const bf16x8*>(
                        xs + ((wave * RPW + r + dy) * T::TC + p * 16 + jl + dx) * T::PS + koff);
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        acc[r][p][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[c], b, acc[r][p][c], 0, 0, 0);
                }
        }
        if (step % nchunk != nchunk - 1) continue;
        // the tile's last chunk: bias, ReLU, bf16, store; clear the sums
        int x0, y0, n, cbg, chunk;
        decode(step, x0, y0, n, cbg, chunk);
        bf16_t* Yn = Y + (int64_t)n * H * W * sy;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int yo = y0 + wave * RPW + r;
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const int xo = x0 + p * 16 + jl;
#pragma unroll
                for (int c = 0; c < CB; ++c) {
                    const int co = (cbg * CB + c) * 16 + 4 * g;
                    if (yo < H && xo < W) {
                        s4 o;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            float v = acc[r][p][c][e] + (bias ? bias[co + e] : 0.f);
                            if (relu) v = fmaxf(v, 0.f);
                            o[e] = (short)f2bf(v);
                        }
                        const int64_t hoff = co >= ysplit ? yhs - ysplit : 0;
                        *reinterpret_cast<s4*>(Yn + ((int64_t)yo * W + xo) * sy + hoff + co) = o;
                    }
                    acc[r][p][c] = f4{0.f, 0.f, 0.f, 0.f};
                }
            }
        }
    }
}

// Weight gradient of a 3x3 convolution: part[chunk][tap][co][ci] =
// sum over the chunk's rows of gy[p][co] x[p + tap][ci], and the bias partial
// bpart[chunk][co] = sum gy[p][co] (written by the ci-block 0 waves).
// One wave per (chunk, co block, ci block); rows of all images are chunked.
__global__ __launch_bounds__(64) void k_conv3_wgrad(const bf16_t* __restrict__ GY, int sg, int Cout,
                                                    const bf16_t* __restrict__ X, int sx, int64_t xhs, int xsplit,
                                                    int Cin,
                                                    int H, int W, int nrows, int rows_per_chunk,
                                                    float* __restrict__ part, float* __restrict__ bpart) {
    const int lane = threadIdx.x;
    const int nci = Cin / 16;
    const int blk = blockIdx.y;
    const int co0 = (blk / nci) * 16, ci0 = (blk % nci) * 16;
    const int chunk = blockIdx.x;
    const int r0 = chunk * rows_per_chunk, r1 = min(nrows, r0 + rows_per_chunk);
    const int jl = lane & 15, kq = (lane >> 4) * 4;
    f4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (int r = r0; r < r1; ++r) {
        const int n = r / H, y = r % H;
        const bf16_t* Gr = GY + (int64_t)r * W * sg;
        const bf16_t* Xn = X + (int64_t)n * H * W * sx + (ci0 >= xsplit ? xhs - xsplit : 0);
        for (int x0 = 0; x0 < W; x0 += 16) {
            s4 a;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int xp = x0 + kq + e;
                a[e] = xp < W ? (short)Gr[(int64_t)xp * sg + co0 + jl] : (short)0;
                bsum += bf2f((bf16_t)a[e]);
            }
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int yy = y + tap / 3 - 1, dx = tap % 3 - 1;
                s4 b;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int xp = x0 + kq + e, xx = xp + dx;
                    b[e] = (xp < W && yy >= 0 && yy < H && xx >= 0 && xx < W)
                               ? (short)Xn[((int64_t)yy * W + xx) * sx + ci0 + jl] : (short)0;
                }
                acc[tap] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[tap], 0, 0, 0);
            }
        }
    }
    // D[co][ci]: lane holds ci = ci0 + jl, co = co0 + kq + e
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            part[(((int64_t)chunk * 9 + tap) * Cout + co0 + kq + e) * Cin + ci0 + jl] = acc[tap][e];
    if (ci0 == 0) {
        // lanes jl, jl+16, jl+32, jl+48 hold partial sums of channel co0 + jl
        bsum += __shfl_xor(bsum, 16, 64);
        bsum += __shfl_xor(bsum, 32, 64);
        if (lane < 16) bpart[(int64_t)chunk * Cout + co0 + lane] = bsum;
    }
}

// Sum the chunk partials of a 3x3 layer into the flat gradient: weights in
// [co][ci][3][3] for ci < cin_real, then the bias.  Threads walk the partials
// in their own layout (ci fastest) so the reads over chunks are coalesced.
__global__ void k_conv3_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ bpart,
                                     int nchunks, int Cout, int Cin, int cin_real,
                                     float* __restrict__ gflat) {
    const int64_t per = (int64_t)9 * Cout * Cin;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < per + Cout;
         i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        if (i < per) {
            const int ci = (int)(i % Cin), co = (int)((i / Cin) % Cout), tap = (int)(i / ((int64_t)Cin * Cout));
            if (ci >= cin_real) continue;
            for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * per + i];
            gflat[((int64_t)co * cin_real + ci) * 9 + tap] = s;
        } else {
            const int co = (int)(i - per);
            for (int c = 0; c < nchunks; ++c) s += bpart[(int64_t)c * Cout + co];
            gflat[(int64_t)Cout * cin_real * 9 + co] = s;
        }
    }
}

// 2x2 average pool: out[n][i][j][c] = bf16(mean of the 2x2 block).
__global__ void k_pool(const bf16_t* __restrict__ X, int sx, bf16_t* __restrict__ Y, int sy, int C,
                       int N, int H2, int W2) {
    // one thread per 8 channels of an output pixel (16-byte loads and store)
    const int C8 = C / 8;
    const int64_t total = (int64_t)N * H2 * W2 * C8;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
        const int c = (int)(i % C8) * 8;
        const int64_t pix = i / C8;
        const int j = (int)(pix % W2), ii = (int)((pix / W2) % H2), n = (int)(pix / ((int64_t)W2 * H2));
        const int64_t base = ((int64_t)n * 2 * H2 + 2 * ii) * (2 * W2) + 2 * j;
        bf8u v[4];
        v[0].u = *reinterpret_cast<const uint4*>(X + base * sx + c);
        v[1].u = *reinterpret_cast<const uint4*>(X + (base + 1) * sx + c);
        v[2].u = *reinterpret_cast<const uint4*>(X + (base + 2 * W2) * sx + c);
        v[3].u = *reinterpret_cast<const uint4*>(X + (base + 2 * W2 + 1) * sx + c);
        bf8u o;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float s = bf2f(v[0].h[e]) + bf2f(v[1].h[e]) + bf2f(v[2].h[e]) + bf2f(v[3].h[e]);
            o.h[e] = f2bf(0.25f * s);
        }
        *reinterpret_cast<uint4*>(Y + pix * sy + c) = o.u;
    }
}

// Gradient into an encoder output: g[n][y][x][c] = bf16(gp[n][y/2][x/2][c] / 4
// + gskip[n][y][x][c]), then the ReLU mask of that output.
__global__ void k_pool_back(const bf16_t* __restrict__ GP, int sp, const bf16_t* __restrict__ GS, int ss,
                            const bf16_t* __restrict__ Yact, int sa, bf16_t* __restrict__ G, int sg,
                            int C, int N, int H, int W) {
    const int64_t total = (int64_t)N * H * W * C;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
        const int c = (int)(i % C);
        const int64_t pix = i / C;
        const int x = (int)(pix % W), y = (int)((pix / W) % H), n = (int)(pix / ((int64_t)W * H));
        const int64_t pp = ((int64_t)n * (H / 2) + y / 2) * (W / 2) + x / 2;
        const float v = 0.25f * bf2f(GP[pp * sp + c]) + bf2f(GS[pix * ss + c]);
        G[pix * sg + c] = bf2f(Yact[pix * sa + c]) > 0.f ? f2bf(v) : (bf16_t)0;
    }
}

// g *= (y > 0), in place.
__global__ void k_relu_mask(bf16_t* __restrict__ G, int sg, const bf16_t* __restrict__ Yact, int sa,
                            int C, int64_t npix) {
    const int64_t total = npix * C;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
        const int c = (int)(i % C);
        const int64_t pix = i / C;
        if (!(bf2f(Yact[pix * sa + c]) > 0.f)) G[pix * sg + c] = 0;
    }
}

// Transposed 2x2 convolution, stride 2, as a GEMM per input pixel on
// v_mfma_f32_16x16x32_bf16: D[(a d) Cout + co][pixel] = sum_ci W[ci][co][a][d]
// X[pixel][ci], stored with its bias at output pixel (2i + a, 2j + d).  A is
// packed by k_pack_frag_t in the instruction's operand order ([ci / 32][row
// block][lane][8]).  Workgroup: 4 waves, one input row each, 64 input pixels
// x 16 CB rows of D; every operand load of the launch (NKC = Cin / 32 blocks)
// is issued before the first MFMA.
template <int CB, int NKC>
__global__ __launch_bounds__(NT) void k_convT_mfma(const bf16_t* __restrict__ X, int sx,
                                                   const bf16_t* __restrict__ Af, const float* __restrict__ bias,
                                                   bf16_t* __restrict__ Y, int sy, int Cout, int Hi, int Wi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int jl = lane & 15, g = lane >> 4;
    const int M = 4 * Cout, nmb = M / 16;
    const int ncog = M / (16 * CB);
    const int n = blockIdx.z / ncog;
    const int mb0 = (blockIdx.z % ncog) * CB;
    const int y = blockIdx.y * 4 + wave;
    if (y >= Hi) return;
    const int x0 = blockIdx.x * 64;
    const bf16_t* Xr = X + ((int64_t)n * Hi + y) * Wi * sx;
    bf16x8 b[NKC][4], a[NKC][CB];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int xx = x0 + p * 16 + jl;
            b[kc][p] = bf16x8{};
            if (xx < Wi) b[kc][p] = *reinterpret_cast<const bf16x8*>(Xr + (int64_t)xx * sx + kc * 32 + 8 * g);
        }
#pragma unroll
        for (int c = 0; c < CB; ++c)
            a[kc][c] = *reinterpret_cast<const bf16x8*>(Af + (((int64_t)kc * nmb + mb0 + c) * 64 + lane) * 8);
    }
    f4 acc[4][CB];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            acc[p][c] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < NKC; ++kc)
                acc[p][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kc][c], b[kc][p], acc[p][c], 0, 0, 0);
        }
    const int Wo = 2 * Wi;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int xx = x0 + p * 16 + jl;
        if (xx >= Wi) continue;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int mrow = (mb0 + c) * 16 + 4 * g;     // four consecutive rows: same (a, d)
            const int ad = mrow / Cout, co = mrow - ad * Cout;
            const int yo = 2 * y + (ad >> 1), xo = 2 * xx + (ad & 1);
            s4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (short)f2bf(acc[p][c][e] + bias[co + e]);
            *reinterpret_cast<s4*>(Y + (((int64_t)n * 2 * Hi + yo) * Wo + xo) * sy + co) = o;
        }
    }
}

// Data gradient of the transposed convolution: D[ci][pixel] = sum over
// (a d, co) of WT[ci][(a d) Cout + co] GY[(2i + a, 2j + d)][co]; WT is
// [Cin][4 Cout] bf16.  Same workgroup shape as k_convT_mfma.
template <int CB>
__global__ __launch_bounds__(NT) void k_convT_dgrad_mfma(const bf16_t* __restrict__ GY, int sg, int Cout,
                                                         const bf16_t* __restrict__ WT, bf16_t* __restrict__ GX,
                                                         int sx, int Cin, int Hi, int Wi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ncog = Cin / (16 * CB);
    const int n = blockIdx.z / ncog;
    const int c0 = (blockIdx.z % ncog) * 16 * CB;
    const int y = blockIdx.y * 4 + wave;
    if (y >= Hi) return;
    const int x0 = blockIdx.x * 64;
    const int jl = lane & 15, kq = (lane >> 4) * 4;
    const int K = 4 * Cout, Wo = 2 * Wi;
    f4 acc[4][CB];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[p][c] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < K; k += 16) {
        const int ad = k / Cout, co = k - ad * Cout;
        const bf16_t* Gr = GY + (((int64_t)n * 2 * Hi + 2 * y + (ad >> 1)) * Wo + (ad & 1)) * sg + co + kq;
        s4 b[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int xx = x0 + p * 16 + jl;
            b[p] = xx < Wi ? *reinterpret_cast<const s4*>(Gr + (int64_t)2 * xx * sg) : s4{0, 0, 0, 0};
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const s4 av = *reinterpret_cast<const s4*>(WT + (int64_t)(c0 + c * 16 + jl) * K + k + kq);
#pragma unroll
            for (int p = 0; p < 4; ++p)
                acc[p][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, b[p], acc[p][c], 0, 0, 0);
        }
    }
    bf16_t* Gxr = GX + ((int64_t)n * Hi + y) * Wi * sx;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int xx = x0 + p * 16 + jl;
        if (xx >= Wi) continue;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            s4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (short)f2bf(acc[p][c][e]);
            *reinterpret_cast<s4*>(Gxr + (int64_t)xx * sx + c0 + c * 16 + kq) = o;
        }
    }
}

// Weight gradient of the transposed convolution: part[chunk][ad][co][ci] =
// sum over the chunk's input rows of GY[(2i + a, 2j + d)][co] X[(i, j)][ci]
// (a GEMM over pixels per sub-position ad), and bpart[chunk][co] = the sum of
// GY over the chunk's output pixels (ci-block 0 waves).  One wave per (chunk,
// co block, ci block).
__global__ __launch_bounds__(64) void k_convT_wgrad_mfma(const bf16_t* __restrict__ X, int sx, int Cin,
                                                         const bf16_t* __restrict__ GY, int sg, int Cout, int Hi,
                                                         int Wi, int nrows, int rows_per_chunk,
                                                         float* __restrict__ part, float* __restrict__ bpart) {
    const int lane = threadIdx.x;
    const int nci = Cin / 16;
    const int co0 = (blockIdx.y / nci) * 16, ci0 = (blockIdx.y % nci) * 16;
    const int chunk = blockIdx.x;
    const int r0 = chunk * rows_per_chunk, r1 = min(nrows, r0 + rows_per_chunk);
    const int jl = lane & 15, kq = (lane >> 4) * 4;
    const int Wo = 2 * Wi;
    f4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (int r = r0; r < r1; ++r) {                       // r = n Hi + i
        const int n = r / Hi, i = r - n * Hi;
        const bf16_t* Xr = X + (int64_t)r * Wi * sx;
        for (int x0 = 0; x0 < Wi; x0 += 16) {
            s4 b;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int xp = x0 + kq + e;
                b[e] = xp < Wi ? (short)Xr[(int64_t)xp * sx + ci0 + jl] : (short)0;
            }
#pragma unroll
            for (int ad = 0; ad < 4; ++ad) {
                const bf16_t* Gr = GY + (((int64_t)n * 2 * Hi + 2 * i + (ad >> 1)) * Wo + (ad & 1)) * sg + co0 + jl;
                s4 av;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int xp = x0 + kq + e;
                    av[e] = xp < Wi ? (short)Gr[(int64_t)2 * xp * sg] : (short)0;
                    bsum += bf2f((bf16_t)av[e]);
                }
                acc[ad] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, b, acc[ad], 0, 0, 0);
            }
        }
    }
    // D[co][ci]: lane holds ci = ci0 + jl, co = co0 + kq + e
#pragma unroll
    for (int ad = 0; ad < 4; ++ad)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            part[(((int64_t)chunk * 4 + ad) * Cout + co0 + kq + e) * Cin + ci0 + jl] = acc[ad][e];
    if (ci0 == 0) {
        bsum += __shfl_xor(bsum, 16, 64);
        bsum += __shfl_xor(bsum, 32, 64);
        if (lane < 16) bpart[(int64_t)chunk * Cout + co0 + lane] = bsum;
    }
}

// Transposed-convolution partials into the flat gradient [ci][co][a][d] + bias.
__global__ void k_convT_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ bpart, int nchunks,
                                     int Cout, int Cin, float* __restrict__ gflat) {
    const int64_t per = (int64_t)4 * Cout * Cin;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < per + Cout;
         i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        if (i < per) {
            const int ci = (int)(i % Cin), co = (int)((i / Cin) % Cout), ad = (int)(i / ((int64_t)Cin * Cout));
            for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * per + i];
            gflat[((int64_t)ci * Cout + co) * 4 + ad] = s;
        } else {
            const int co = (int)(i - per);
            for (int c = 0; c < nchunks; ++c) s += bpart[(int64_t)c * Cout + co];
            gflat[per + co] = s;
        }
    }
}

// Sum per-chunk partials laid out [chunk][n] into out[n].
__global__ void k_sum_chunks(const float* __restrict__ part, int nchunks, int64_t n, float* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        float s = 0.f;
        for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * n + i];
        out[i] = s;
    }
}

// Output layer (1x1, 16 -> 1): o[p] = b + sum_c w[c] x[p][c], float32.
__global__ void k_out(const bf16_t* __restrict__ X, int sx, const bf16_t* __restrict__ w, const float* bias,
                      float* __restrict__ o, int64_t npix) {
    for (int64_t p = blockIdx.x * (int64_t)NT + threadIdx.x; p < npix; p += (int64_t)gridDim.x * NT) {
        bf8u x[2];
        x[0].u = *reinterpret_cast<const uint4*>(X + p * sx);
        x[1].u = *reinterpret_cast<const uint4*>(X + p * sx + 8);
        float s = bias[0];
#pragma unroll
        for (int c = 0; c < 16; ++c) s += bf2f(w[c]) * bf2f(x[c >> 3].h[c & 7]);
        o[p] = s;
    }
}

// Back through the output layer: g[p][c] = bf16(w[c] go[p]) masked by the
// ReLU of its input x; weight and bias partials per chunk: part[chunk][17].
__global__ void k_out_back(const float* __restrict__ go, const bf16_t* __restrict__ X, int sx,
                           const bf16_t* __restrict__ w, bf16_t* __restrict__ G, int sg, int64_t npix,
                           int64_t pix_per_chunk, float* __restrict__ part) {
    __shared__ float red[17][NT / 64];
    const int chunk = blockIdx.x;
    const int64_t p0 = chunk * pix_per_chunk, p1 = min(npix, p0 + pix_per_chunk);
    float acc[17];
#pragma unroll
    for (int c = 0; c < 17; ++c) acc[c] = 0.f;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += NT) {
        const float g = go[p];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const float xv = bf2f(X[p * sx + c]);
            acc[c] += g * xv;
            G[p * sg + c] = xv > 0.f ? f2bf(bf2f(w[c]) * g) : (bf16_t)0;
        }
        acc[16] += g;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 17; ++c) {
        float v = acc[c];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) red[c][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 17) {
        float s = 0.f;
        for (int k = 0; k < NT / 64; ++k) s += red[threadIdx.x][k];
        part[(int64_t)chunk * 17 + threadIdx.x] = s;
    }
}

// Default per-sample loss weight sum_x a / (sum_x c)^2 (0 when sum_x c <= 0).
// One workgroup per sample.
__global__ __launch_bounds__(NT) void k_loss_weights(const float* __restrict__ a, const float* __restrict__ c,
                                                     int64_t npix, float* __restrict__ w) {
    __shared__ double red[2][NT / 64];
    const int s = blockIdx.x;
    double sa = 0.0, sc = 0.0;
    for (int64_t p = threadIdx.x; p < npix; p += NT) {
        sa += a[(int64_t)s * npix + p];
        sc += c[(int64_t)s * npix + p];
    }
    for (int k = 32; k > 0; k >>= 1) {
        sa += __shfl_xor(sa, k, 64);
        sc += __shfl_xor(sc, k, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sa;
        red[1][threadIdx.x >> 6] = sc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tc = 0.0;
        for (int k = 0; k < NT / 64; ++k) { ta += red[0][k]; tc += red[1][k]; }
        w[s] = (tc > 0.0 && ta > 0.0) ? (float)(ta / (tc * tc)) : 0.f;
    }
}

// Scaling loss per sample s: L_s = w_s sum_x (a e^{2o} - 2 c e^{o}) and
// go = w_s (2 a e^{2o} - 2 c e^{o}) / nbatch, with w from `weight` or the
// default sum_x a / (sum_x c)^2 of the image.  One workgroup per sample;
// loss[s] in float64.
__global__ __launch_bounds__(NT) void k_scaling_loss(const float* __restrict__ o, const float* __restrict__ a,
                                                     const float* __restrict__ c, const float* __restrict__ weight,
                                                     int64_t npix, int nbatch, float* __restrict__ go,
                                                     double* __restrict__ loss) {
    __shared__ double red[NT / 64];
    const int s = blockIdx.x;
    const float* os = o + (int64_t)s * npix;
    const float* as = a + (int64_t)s * npix;
    const float* cs = c + (int64_t)s * npix;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    auto block_sum = [&](double v) -> double {
        for (int k = 32; k > 0; k >>= 1) v += __shfl_xor(v, k, 64);
        __syncthreads();
        if (lane == 0) red[wv] = v;
        __syncthreads();
        double t = 0.0;
        for (int k = 0; k < NT / 64; ++k) t += red[k];
        return t;
    };
    double wt;
    if (weight) {
        wt = weight[s];
    } else {
        double suma = 0.0, sumc = 0.0;
        for (int64_t p = threadIdx.x; p < npix; p += NT) {
            suma += as[p];
            sumc += cs[p];
        }
        suma = block_sum(suma);
        sumc = block_sum(sumc);
        wt = (sumc > 0.0 && suma > 0.0) ? (double)(float)(suma / (sumc * sumc)) : 0.0;
    }
    const float inv = (float)wt;
    double sl = 0.0;
    for (int64_t p = threadIdx.x; p < npix; p += NT) {
        const float e = expf(os[p]);
        const float ae = as[p] * e, ce = cs[p];
        sl += (double)(ae * e - 2.f * ce * e);
        go[(int64_t)s * npix + p] = (2.f * ae * e - 2.f * ce * e) * inv / (float)nbatch;
    }
    sl = block_sum(sl);
    if (threadIdx.x == 0) loss[s] = sl * wt;
}

// Squared gradient norm: partials per block, summed by k_norm_finish.
__global__ __launch_bounds__(NT) void k_sqnorm(const float* __restrict__ g, int64_t n, double* __restrict__ part) {
    __shared__ double red[NT / 64];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        acc += (double)g[i] * (double)g[i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NT / 64; ++k) t += red[k];
        part[blockIdx.x] = t;
    }
}

// factor[0] = min(1, clip / ||g||) from the block partials (one thread).
__global__ void k_clip_factor(const double* __restrict__ part, int nb, float clip, float* __restrict__ factor) {
    if (threadIdx.x != 0) return;
    double t = 0.0;
    for (int k = 0; k < nb; ++k) t += part[k];
    const double nrm = sqrt(t);
    factor[0] = (clip > 0.f && nrm > clip) ? (float)(clip / nrm) : 1.f;
}

// Adam (Kingma & Ba 2015) on the float32 master parameters, the gradient
// scaled by factor[0] (gradient-norm clipping) when factor is given.
__global__ void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2, const float* __restrict__ factor) {
    const float f = factor ? factor[0] : 1.f;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const float gi = g[i] * f;
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// bf16 weights of a 3x3 layer in the operand order of k_conv3, from the
// master weights w[co][ci][3][3] (cin real input channels): forward (bwd = 0)
// A[tap][m = co][k = ci], the data gradient (bwd = 1) A[tap][m = ci][k = co]
// with the taps reversed.  Element (chunk, kb, cb, lane, e) is A at
// m = 16 cb + lane % 16 and the lane's tap and channel k of block kb
// (k_conv3's contraction order); zero beyond M, K, cin or the ninth tap.
__global__ void k_pack_frag(const float* __restrict__ w, int cout, int cin, int M, int K, int bwd,
                            bf16_t* __restrict__ af, int64_t n) {
    const int ck = frag_ck(K), nkb = frag_nkb(ck), ncb = (M + 15) / 16;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
        const int64_t rest = i >> 9;
        const int cb = (int)(rest % ncb), kb = (int)((rest / ncb) % nkb), chunk = (int)(rest / ((int64_t)ncb * nkb));
        const int g = lane >> 4, m = cb * 16 + (lane & 15);
        const int tap = ck == 32 ? kb : 2 * kb + (g >> 1);
        const int k = chunk * ck + (ck == 32 ? 8 * g : 8 * (g & 1)) + e;
        float v = 0.f;
        if (tap < 9 && m < M && k < K) {
            const int co = bwd ? k : m, ci = bwd ? m : k;
            if (ci < cin) v = w[((int64_t)co * cin + ci) * 9 + (bwd ? 8 - tap : tap)];
        }
        af[i] = f2bf(v);
    }
}

int64_t convT_frag_elems(int Cin, int Cout) { return (int64_t)((Cin + 31) / 32) * (4 * Cout / 16) * 512; }

int64_t frag_elems(int M, int K) {
    const int ck = frag_ck(K);
    return (int64_t)(K / ck) * frag_nkb(ck) * ((M + 15) / 16) * 512;
}

// bf16 data-gradient copy of transposed-convolution weights from
// [ci][co][a][d]: WT[ci][(a d) Cout + co].
__global__ void k_pack_convT(const float* __restrict__ w, int Cin, int Cout, bf16_t* __restrict__ wt) {
    const int64_t n = (int64_t)4 * Cin * Cout;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const int ad = (int)(i % 4), co = (int)((i / 4) % Cout), ci = (int)(i / (4 * Cout));
        wt[(int64_t)ci * 4 * Cout + ad * Cout + co] = f2bf(w[i]);
    }
}

// Transposed-convolution weights w[ci][co][a][d] in k_convT_mfma's operand
// order: element (kc, mb, lane, e) is W at row m = 16 mb + lane % 16 =
// (a d) Cout + co and ci = 32 kc + 8 (lane / 16) + e.
__global__ void k_pack_frag_t(const float* __restrict__ w, int Cin, int Cout, bf16_t* __restrict__ af, int64_t n) {
    const int nmb = 4 * Cout / 16;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
        const int64_t rest = i >> 9;
        const int mb = (int)(rest % nmb), kc = (int)(rest / nmb);
        const int m = mb * 16 + (lane & 15), ci = kc * 32 + 8 * (lane >> 4) + e;
        const int ad = m / Cout, co = m % Cout;
        af[i] = f2bf(ci < Cin ? w[((int64_t)ci * Cout + co) * 4 + ad] : 0.f);
    }
}

__global__ void k_to_bf16(const float* __restrict__ w, bf16_t* __restrict__ o, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) o[i] = f2bf(w[i]);
}

// Network input: NCHW float32 [n][3][H][W] to NHWC bf16 with 16 channels
// (channels 3..15 zero), one thread per pixel.
__global__ void k_input(const float* __restrict__ x, bf16_t* __restrict__ X, int N, int64_t HW) {
    const int64_t total = (int64_t)N * HW;
    for (int64_t pix = blockIdx.x * (int64_t)NT + threadIdx.x; pix < total; pix += (int64_t)gridDim.x * NT) {
        const int64_t n = pix / HW, p = pix % HW;
        bf8u lo;
        lo.u = uint4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int c = 0; c < 3; ++c) lo.h[c] = f2bf(x[(n * 3 + c) * HW + p]);
        *reinterpret_cast<uint4*>(X + pix * 16) = lo.u;
        *reinterpret_cast<uint4*>(X + pix * 16 + 8) = uint4{0u, 0u, 0u, 0u};
    }
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 8192)); }

}  // namespace

// ---------------------------------------------------------------------------
// Network state and the layer sequence.
struct Layer {
    int kind;            // 0 conv3x3, 1 convT 2x2, 2 conv1x1
    int cin, cout;       // real channel counts
    int64_t off;         // offset of the weights in the flat vector (bias follows)
    int64_t nw;          // weight count
    bf16_t *wf = nullptr, *wb = nullptr;   // packed bf16 weights
};

struct Unet {
    int H = 0, W = 0, maxb = 0;
    hipStream_t stream = nullptr;
    std::vector<Layer> L;
    int64_t P = 0;
    float *theta = nullptr, *m = nullptr, *v = nullptr;
    bf16_t* act = nullptr;       // all activation buffers
    bf16_t* grad = nullptr;      // all gradient buffers
    float* go = nullptr;         // dL/do [maxb][H][W]
    float* part = nullptr;       // reduction partials
    int64_t part_cap = 0;
    double* dloss = nullptr;     // per-sample loss
    // activation views (element offsets into act / grad, per-image strides)
    // C channels per pixel at pixel stride `stride`; a concatenation buffer
    // holds its two halves of C / 2 channels as planar tensors hs apart
    struct View { int64_t off; int stride; int C; int lvl; int64_t hs; };
    std::vector<View> av;        // named below
};

enum {
    A_X, A_A1, A_CAT1, A_D1A, A_D1B,
    A_P1, A_A2, A_CAT2, A_D2A, A_D2B,
    A_P2, A_A3, A_CAT3, A_D3A, A_D3B,
    A_P3, A_A4, A_B4, A_COUNT
};

// layer indices in flat order
enum { C1A, C1B, C2A, C2B, C3A, C3B, C4A, C4B, U3, D3A, D3B, U2, D2A, D2B, U1, D1A, D1B, OUT, NLAYERS };

}  // namespace esi

using namespace esi;

namespace {

const int kLayerDef[NLAYERS][3] = {
    {0, 3, 16}, {0, 16, 16}, {0, 16, 32}, {0, 32, 32}, {0, 32, 64}, {0, 64, 64},
    {0, 64, 128}, {0, 128, 128}, {1, 128, 64}, {0, 128, 64}, {0, 64, 64},
    {1, 64, 32}, {0, 64, 32}, {0, 32, 32}, {1, 32, 16}, {0, 32, 16}, {0, 16, 16}, {2, 16, 1}};

int64_t layer_weights(int kind, int ci, int co) { return kind == 0 ? (int64_t)9 * ci * co : kind == 1 ? (int64_t)4 * ci * co : ci * co; }

// A tensor view handed to the convolution launchers: pointer, pixel stride and,
// for a concatenation buffer, the distance to the second half and the first
// channel that lives there (no split: hs = 0, split beyond every channel).
struct Tv {
    bf16_t* p;
    int s;
    int64_t hs = 0;
    int split = 1 << 30;
};

struct Ctx {
    Unet* U;
    int N;
    int64_t pix(int lvl) const { return (int64_t)N * (U->H >> lvl) * (U->W >> lvl); }
    bf16_t* a(int id) const { return U->act + U->av[id].off; }
    bf16_t* g(int id) const { return U->grad + U->av[id].off; }
    // half h (0: upsampled decoder input, 1: encoder skip) of a concatenation buffer
    bf16_t* ah(int id, int h) const { return U->act + U->av[id].off + h * U->av[id].hs; }
    bf16_t* gh(int id, int h) const { return U->grad + U->av[id].off + h * U->av[id].hs; }
    Tv at(int id) const { return view(U->act, id); }
    Tv gt(int id) const { return view(U->grad, id); }
    Tv view(bf16_t* base, int id) const {
        const Unet::View& v = U->av[id];
        Tv t{base + v.off, v.stride};
        if (v.hs) { t.hs = v.hs; t.split = v.C / 2; }
        return t;
    }
    int h(int lvl) const { return U->H >> lvl; }
    int w(int lvl) const { return U->W >> lvl; }
};

// Eight waves of one output row each: a chunk's weight operands, staged once
// per workgroup, feed twice the MFMAs of a four-wave workgroup (0.68 against
// 0.70 ms for the network forward on 8 images of 408 x 808; two rows per wave
// or sixteen waves were slower, the latter spilling).
template <int CB, int RPW, int CK, int NWV = 8>
void launch_conv3(const Ctx& c, const Tv& X, int K, const bf16_t* Af, const float* bias, const Tv& Y, int M, int H,
                  int W, bool relu) {
    // persistent grid: as many workgroups as the device holds at once
    static int resident = 0;
    if (!resident) {
        int per_cu = 0, cus = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_conv3<CB, RPW, CK, NWV>, 64 * NWV, 0) != hipSuccess)
            per_cu = 1, cus = 256;
        resident = std::max(1, per_cu) * std::max(1, cus);
    }
    const int rows = NWV * RPW;
    const int64_t ntiles = (int64_t)((W + 63) / 64) * ((H + rows - 1) / rows) * c.N * (M / (16 * CB));
    const int grid = (int)std::min<int64_t>(ntiles, resident);
    hipLaunchKernelGGL((k_conv3<CB, RPW, CK, NWV>), dim3(grid), dim3(64 * NWV), 0, c.U->stream, X.p, X.s, X.hs, X.split, K, Af,
                       (M + 15) / 16, bias, Y.p, Y.s, Y.hs, Y.split, M, H, W, c.N, relu ? 1 : 0);
}

// K input channels (Cin, or Cout for the data gradient) to M outputs
esi_status_t conv3(const Ctx& c, const Tv& X, int K, int layer, bool bwd, const Tv& Y, int M, int lvl, bool relu) {
    Unet* U = c.U;
    const Layer& Ly = U->L[layer];
    const bf16_t* Af = bwd ? Ly.wb : Ly.wf;
    const float* bias = bwd ? nullptr : U->theta + Ly.off + Ly.nw;
    const int H = c.h(lvl), W = c.w(lvl);
    if (K % 16 || M % 16) return fail(ESI_ERR_SHAPE, "3x3 convolution channels must be multiples of 16");
    const int cb = M >= 64 ? 4 : M / 16;
    if (frag_ck(K) == 32) {
        if (cb == 4) launch_conv3<4, 1, 32>(c, X, K, Af, bias, Y, M, H, W, relu);
        else if (cb == 2) launch_conv3<2, 1, 32>(c, X, K, Af, bias, Y, M, H, W, relu);
        else launch_conv3<1, 1, 32>(c, X, K, Af, bias, Y, M, H, W, relu);
    } else {
        if (cb == 4) launch_conv3<4, 1, 16>(c, X, K, Af, bias, Y, M, H, W, relu);
        else if (cb == 2) launch_conv3<2, 1, 16>(c, X, K, Af, bias, Y, M, H, W, relu);
        else launch_conv3<1, 1, 16>(c, X, K, Af, bias, Y, M, H, W, relu);
    }
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t need_part(Unet* U, int64_t n) {
    return grow_t(&U->part, &U->part_cap, n, U->stream);
}

// weight + bias gradient of a 3x3 layer into gflat
esi_status_t conv3_wgrad(const Ctx& c, const Tv& GY, int Cout, const Tv& X, int Cin, int cin_real, int lvl,
                         float* gflat) {
    Unet* U = c.U;
    const int H = c.h(lvl), W = c.w(lvl);
    const int nrows = c.N * H;
    const int nblocks = (Cout / 16) * (Cin / 16);
    const int want = std::max(1, std::min(nrows, 2048 / nblocks));
    const int rpc = (nrows + want - 1) / want;
    const int nchunks = (nrows + rpc - 1) / rpc;
    const int64_t np = (int64_t)nchunks * 9 * Cout * Cin;
    ESI_TRY(need_part(U, np + (int64_t)nchunks * Cout));
    float* part = U->part;
    float* bpart = U->part + np;
    hipLaunchKernelGGL(k_conv3_wgrad, dim3(nchunks, nblocks), dim3(64), 0, U->stream, GY.p, GY.s, Cout, X.p, X.s,
                       X.hs, X.split, Cin, H, W, nrows, rpc, part, bpart);
    const int64_t nout = (int64_t)9 * Cout * Cin + Cout;
    hipLaunchKernelGGL(k_conv3_wgrad_reduce, dim3(grid_for(nout)), dim3(NT), 0, U->stream, part, bpart, nchunks,
                       Cout, Cin, cin_real, gflat);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

template <int CB, int NKC>
void launch_convT(const Ctx& c, const Layer& Ly, const bf16_t* X, int sx, const float* bias, bf16_t* Y, int sy,
                  int Hi, int Wi) {
    dim3 grid((Wi + 63) / 64, (Hi + 3) / 4, c.N * (4 * Ly.cout / (16 * CB)));
    hipLaunchKernelGGL((k_convT_mfma<CB, NKC>), grid, dim3(NT), 0, c.U->stream, X, sx, Ly.wf, bias, Y, sy, Ly.cout,
                       Hi, Wi);
}

esi_status_t convT_fwd(const Ctx& c, int layer, const bf16_t* X, int sx, bf16_t* Y, int sy, int lvl_in) {
    Unet* U = c.U;
    const Layer& Ly = U->L[layer];
    const int Hi = c.h(lvl_in), Wi = c.w(lvl_in);
    const float* bias = U->theta + Ly.off + Ly.nw;
    // 4 Cout rows of D in blocks of 64; Cin in blocks of 32 (32, 64 or 128)
    if (Ly.cout % 16 || (Ly.cin != 32 && Ly.cin != 64 && Ly.cin != 128))
        return fail(ESI_ERR_SHAPE, "transposed convolution channels outside the supported set");
    if (Ly.cin == 32) launch_convT<4, 1>(c, Ly, X, sx, bias, Y, sy, Hi, Wi);
    else if (Ly.cin == 64) launch_convT<4, 2>(c, Ly, X, sx, bias, Y, sy, Hi, Wi);
    else launch_convT<4, 4>(c, Ly, X, sx, bias, Y, sy, Hi, Wi);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t convT_back(const Ctx& c, int layer, const bf16_t* X, int sx, const bf16_t* GY, int sg,
                        bf16_t* GX, int sgx, int lvl_in, float* gflat) {
    Unet* U = c.U;
    const Layer& Ly = U->L[layer];
    const int Hi = c.h(lvl_in), Wi = c.w(lvl_in);
    {
        const int cb = Ly.cin >= 64 ? 4 : Ly.cin / 16;
        dim3 grid((Wi + 63) / 64, (Hi + 3) / 4, c.N * (Ly.cin / (16 * cb)));
        if (cb == 4)
            hipLaunchKernelGGL(k_convT_dgrad_mfma<4>, grid, dim3(NT), 0, U->stream, GY, sg, Ly.cout, Ly.wb, GX,
                               sgx, Ly.cin, Hi, Wi);
        else
            hipLaunchKernelGGL(k_convT_dgrad_mfma<2>, grid, dim3(NT), 0, U->stream, GY, sg, Ly.cout, Ly.wb, GX,
                               sgx, Ly.cin, Hi, Wi);
    }
    const int nrows = c.N * Hi;
    const int nblocks = (Ly.cout / 16) * (Ly.cin / 16);
    const int want = std::max(1, std::min(nrows, 2048 / nblocks));
    const int rpc = (nrows + want - 1) / want;
    const int nchunks = (nrows + rpc - 1) / rpc;
    const int64_t per = (int64_t)4 * Ly.cout * Ly.cin;
    ESI_TRY(need_part(U, nchunks * per + (int64_t)nchunks * Ly.cout));
    float* part = U->part;
    float* bpart = U->part + nchunks * per;
    hipLaunchKernelGGL(k_convT_wgrad_mfma, dim3(nchunks, nblocks), dim3(64), 0, U->stream, X, sx, Ly.cin, GY, sg,
                       Ly.cout, Hi, Wi, nrows, rpc, part, bpart);
    hipLaunchKernelGGL(k_convT_wgrad_reduce, dim3(grid_for(per + Ly.cout)), dim3(NT), 0, U->stream, part, bpart,
                       nchunks, Ly.cout, Ly.cin, gflat + Ly.off);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t pool(const Ctx& c, const bf16_t* X, int sx, bf16_t* Y, int sy, int C, int lvl_in) {
    const int64_t n = c.pix(lvl_in + 1) * (C / 8);
    hipLaunchKernelGGL(k_pool, dim3(grid_for(n)), dim3(NT), 0, c.U->stream, X, sx, Y, sy, C, c.N,
                       c.h(lvl_in + 1), c.w(lvl_in + 1));
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t mask(const Ctx& c, bf16_t* G, int sg, const bf16_t* Y, int sa, int C, int lvl) {
    const int64_t n = c.pix(lvl) * C;
    hipLaunchKernelGGL(k_relu_mask, dim3(grid_for(n)), dim3(NT), 0, c.U->stream, G, sg, Y, sa, C, c.pix(lvl));
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t forward(const Ctx& c, const float* x, float* o) {
    Unet* U = c.U;
    const int64_t HW = (int64_t)U->H * U->W;
    auto T = [](bf16_t* p, int s) { return Tv{p, s}; };
    hipLaunchKernelGGL(k_input, dim3(grid_for(c.N * HW)), dim3(NT), 0, U->stream, x, c.a(A_X), c.N, HW);
    // encoder: each level's second convolution writes the skip half of the
    // decoder's concatenation buffer, which the pooling reads
    ESI_TRY(conv3(c, c.at(A_X), 16, C1A, false, c.at(A_A1), 16, 0, true));
    ESI_TRY(conv3(c, c.at(A_A1), 16, C1B, false, T(c.ah(A_CAT1, 1), 16), 16, 0, true));
    ESI_TRY(pool(c, c.ah(A_CAT1, 1), 16, c.a(A_P1), 16, 16, 0));
    ESI_TRY(conv3(c, c.at(A_P1), 16, C2A, false, c.at(A_A2), 32, 1, true));
    ESI_TRY(conv3(c, c.at(A_A2), 32, C2B, false, T(c.ah(A_CAT2, 1), 32), 32, 1, true));
    ESI_TRY(pool(c, c.ah(A_CAT2, 1), 32, c.a(A_P2), 32, 32, 1));
    ESI_TRY(conv3(c, c.at(A_P2), 32, C3A, false, c.at(A_A3), 64, 2, true));
    ESI_TRY(conv3(c, c.at(A_A3), 64, C3B, false, T(c.ah(A_CAT3, 1), 64), 64, 2, true));
    ESI_TRY(pool(c, c.ah(A_CAT3, 1), 64, c.a(A_P3), 64, 64, 2));
    ESI_TRY(conv3(c, c.at(A_P3), 64, C4A, false, c.at(A_A4), 128, 3, true));
    ESI_TRY(conv3(c, c.at(A_A4), 128, C4B, false, c.at(A_B4), 128, 3, true));
    // decoder: the transposed convolution writes the first half
    ESI_TRY(convT_fwd(c, U3, c.a(A_B4), 128, c.ah(A_CAT3, 0), 64, 3));
    ESI_TRY(conv3(c, c.at(A_CAT3), 128, D3A, false, c.at(A_D3A), 64, 2, true));
    ESI_TRY(conv3(c, c.at(A_D3A), 64, D3B, false, c.at(A_D3B), 64, 2, true));
    ESI_TRY(convT_fwd(c, U2, c.a(A_D3B), 64, c.ah(A_CAT2, 0), 32, 2));
    ESI_TRY(conv3(c, c.at(A_CAT2), 64, D2A, false, c.at(A_D2A), 32, 1, true));
    ESI_TRY(conv3(c, c.at(A_D2A), 32, D2B, false, c.at(A_D2B), 32, 1, true));
    ESI_TRY(convT_fwd(c, U1, c.a(A_D2B), 32, c.ah(A_CAT1, 0), 16, 1));
    ESI_TRY(conv3(c, c.at(A_CAT1), 32, D1A, false, c.at(A_D1A), 16, 0, true));
    ESI_TRY(conv3(c, c.at(A_D1A), 16, D1B, false, c.at(A_D1B), 16, 0, true));
    const Layer& Lo = U->L[OUT];
    hipLaunchKernelGGL(k_out, dim3(grid_for(c.pix(0))), dim3(NT), 0, U->stream, c.a(A_D1B), 16, Lo.wf,
                       U->theta + Lo.off + Lo.nw, o, c.pix(0));
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

// Backward pass from U->go into the flat gradient gflat (after forward()).
esi_status_t backward(const Ctx& c, float* gflat) {
    Unet* U = c.U;
    auto T = [](bf16_t* p, int s) { return Tv{p, s}; };
    // output layer: g_d1b = bf16(w go) masked by d1b > 0; weight / bias sums
    {
        const int64_t npx = c.pix(0);
        const int nchunks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, npx / 4096));
        const int64_t ppc = (npx + nchunks - 1) / nchunks;
        ESI_TRY(need_part(U, (int64_t)nchunks * 17));
        const Layer& Lo = U->L[OUT];
        hipLaunchKernelGGL(k_out_back, dim3(nchunks), dim3(NT), 0, U->stream, U->go, c.a(A_D1B), 16, Lo.wf,
                           c.g(A_D1B), 16, npx, ppc, U->part);
        hipLaunchKernelGGL(k_sum_chunks, dim3(1), dim3(NT), 0, U->stream, U->part, nchunks, (int64_t)17,
                           gflat + Lo.off);
        ESI_HIP_TRY(hipGetLastError());
    }
    // weight gradient of a 3x3 layer from its output gradient GY and input X,
    // then (GX.p non-null) the gradient of its input
    auto conv_back = [&](int layer, const Tv& GY, int Cout, const Tv& X, int Cin, int lvl,
                         const Tv& GX) -> esi_status_t {
        const Layer& Ly = U->L[layer];
        ESI_TRY(conv3_wgrad(c, GY, Cout, X, Cin, Ly.cin, lvl, gflat + Ly.off));
        if (GX.p) ESI_TRY(conv3(c, GY, Cout, layer, true, GX, Cin, lvl, false));
        return ESI_OK;
    };
    // level 1 decoder: d1b, d1a (d1b's gradient is already masked)
    ESI_TRY(conv_back(D1B, c.gt(A_D1B), 16, c.at(A_D1A), 16, 0, c.gt(A_D1A)));
    ESI_TRY(mask(c, c.g(A_D1A), 16, c.a(A_D1A), 16, 16, 0));
    ESI_TRY(conv_back(D1A, c.gt(A_D1A), 16, c.at(A_CAT1), 32, 0, c.gt(A_CAT1)));
    ESI_TRY(convT_back(c, U1, c.a(A_D2B), 32, c.gh(A_CAT1, 0), 16, c.g(A_D2B), 32, 1, gflat));
    // level 2 decoder
    ESI_TRY(mask(c, c.g(A_D2B), 32, c.a(A_D2B), 32, 32, 1));
    ESI_TRY(conv_back(D2B, c.gt(A_D2B), 32, c.at(A_D2A), 32, 1, c.gt(A_D2A)));
    ESI_TRY(mask(c, c.g(A_D2A), 32, c.a(A_D2A), 32, 32, 1));
    ESI_TRY(conv_back(D2A, c.gt(A_D2A), 32, c.at(A_CAT2), 64, 1, c.gt(A_CAT2)));
    ESI_TRY(convT_back(c, U2, c.a(A_D3B), 64, c.gh(A_CAT2, 0), 32, c.g(A_D3B), 64, 2, gflat));
    // level 3 decoder
    ESI_TRY(mask(c, c.g(A_D3B), 64, c.a(A_D3B), 64, 64, 2));
    ESI_TRY(conv_back(D3B, c.gt(A_D3B), 64, c.at(A_D3A), 64, 2, c.gt(A_D3A)));
    ESI_TRY(mask(c, c.g(A_D3A), 64, c.a(A_D3A), 64, 64, 2));
    ESI_TRY(conv_back(D3A, c.gt(A_D3A), 64, c.at(A_CAT3), 128, 2, c.gt(A_CAT3)));
    ESI_TRY(convT_back(c, U3, c.a(A_B4), 128, c.gh(A_CAT3, 0), 64, c.g(A_B4), 128, 3, gflat));
    // bottleneck
    ESI_TRY(mask(c, c.g(A_B4), 128, c.a(A_B4), 128, 128, 3));
    ESI_TRY(conv_back(C4B, c.gt(A_B4), 128, c.at(A_A4), 128, 3, c.gt(A_A4)));
    ESI_TRY(mask(c, c.g(A_A4), 128, c.a(A_A4), 128, 128, 3));
    ESI_TRY(conv_back(C4A, c.gt(A_A4), 128, c.at(A_P3), 64, 3, c.gt(A_P3)));
    // encoder levels: gradient into e_l = pool path + skip, masked by e_l > 0;
    // the e_l gradient goes into the skip half of the concat gradient buffer
    struct Enc { int lvl, ch, cat, p, a, cb, ca, pin; };
    const Enc enc[3] = {{2, 64, A_CAT3, A_P3, A_A3, C3B, C3A, A_P2},
                        {1, 32, A_CAT2, A_P2, A_A2, C2B, C2A, A_P1},
                        {0, 16, A_CAT1, A_P1, A_A1, C1B, C1A, A_X}};
    for (const Enc& e : enc) {
        const int64_t n = c.pix(e.lvl) * e.ch;
        hipLaunchKernelGGL(k_pool_back, dim3(grid_for(n)), dim3(NT), 0, U->stream, c.g(e.p), e.ch,
                           c.gh(e.cat, 1), e.ch, c.ah(e.cat, 1), e.ch, c.gh(e.cat, 1), e.ch,
                           e.ch, c.N, c.h(e.lvl), c.w(e.lvl));
        ESI_HIP_TRY(hipGetLastError());
        const int cin_a = e.lvl == 0 ? 16 : e.ch / 2;
        ESI_TRY(conv_back(e.cb, T(c.gh(e.cat, 1), e.ch), e.ch, c.at(e.a), e.ch, e.lvl, c.gt(e.a)));
        ESI_TRY(mask(c, c.g(e.a), e.ch, c.a(e.a), e.ch, e.ch, e.lvl));
        ESI_TRY(conv_back(e.ca, c.gt(e.a), e.ch, c.at(e.pin), cin_a, e.lvl,
                          e.lvl == 0 ? Tv{nullptr, 0} : c.gt(e.pin)));
    }
    return ESI_OK;
}

esi_status_t pack(Unet* U) {
    for (Layer& Ly : U->L) {
        const float* w = U->theta + Ly.off;
        if (Ly.kind == 0) {
            const int cpad = Ly.cin < 16 ? 16 : Ly.cin;
            const int64_t nf = frag_elems(Ly.cout, cpad), nb = frag_elems(cpad, Ly.cout);
            hipLaunchKernelGGL(k_pack_frag, dim3(grid_for(nf)), dim3(NT), 0, U->stream, w, Ly.cout, Ly.cin, Ly.cout,
                               cpad, 0, Ly.wf, nf);
            hipLaunchKernelGGL(k_pack_frag, dim3(grid_for(nb)), dim3(NT), 0, U->stream, w, Ly.cout, Ly.cin, Ly.cin,
                               Ly.cout, 1, Ly.wb, nb);
        } else if (Ly.kind == 1) {
            const int64_t nf = convT_frag_elems(Ly.cin, Ly.cout);
            hipLaunchKernelGGL(k_pack_frag_t, dim3(grid_for(nf)), dim3(NT), 0, U->stream, w, Ly.cin, Ly.cout,
                               Ly.wf, nf);
            hipLaunchKernelGGL(k_pack_convT, dim3(grid_for(Ly.nw)), dim3(NT), 0, U->stream, w, Ly.cin, Ly.cout,
                               Ly.wb);
        } else {
            hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(Ly.nw)), dim3(NT), 0, U->stream, w, Ly.wf, Ly.nw);
        }
    }
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

void free_unet(Unet* U) {
    for (Layer& Ly : U->L) {
        if (Ly.wf) hipFree(Ly.wf);
        if (Ly.wb) hipFree(Ly.wb);
    }
    void* b[] = {U->theta, U->m, U->v, U->act, U->grad, U->go, U->part, U->dloss};
    for (void* p : b)
        if (p) hipFree(p);
    delete U;
}

Unet* as_unet(esi_unet_t u) { return reinterpret_cast<Unet*>(u); }

}  // namespace

extern "C" int64_t esi_unet_num_params(void) {
    int64_t P = 0;
    for (int l = 0; l < NLAYERS; ++l)
        P += layer_weights(kLayerDef[l][0], kLayerDef[l][1], kLayerDef[l][2]) + kLayerDef[l][2];
    return P;
}

extern "C" esi_status_t esi_unet_create(esi_unet_t* out, int32_t H, int32_t W, int32_t max_batch,
                                        void* stream) {
    set_error("");
    if (!out) return fail(ESI_ERR_ARG, "null output");
    *out = nullptr;
    if (H < 8 || W < 8 || H % 8 || W % 8) return fail(ESI_ERR_SHAPE, "H and W must be positive multiples of 8");
    if (max_batch < 1) return fail(ESI_ERR_ARG, "max_batch must be >= 1");
    if ((int64_t)H * W * max_batch > ((int64_t)1 << 31) / 128)
        return fail(ESI_ERR_SHAPE, "batch of images too large for one network buffer");
    Unet* U = new Unet;
    U->H = H; U->W = W; U->maxb = max_batch;
    U->stream = (hipStream_t)stream;
    int64_t off = 0;
    for (int l = 0; l < NLAYERS; ++l) {
        Layer Ly;
        Ly.kind = kLayerDef[l][0]; Ly.cin = kLayerDef[l][1]; Ly.cout = kLayerDef[l][2];
        Ly.off = off;
        Ly.nw = layer_weights(Ly.kind, Ly.cin, Ly.cout);
        off += Ly.nw + Ly.cout;
        U->L.push_back(Ly);
    }
    U->P = off;
    // activation views: offset, channels per pixel, level
    const int defs[A_COUNT][2] = {{16, 0}, {16, 0}, {32, 0}, {16, 0}, {16, 0},
                                  {16, 1}, {32, 1}, {64, 1}, {32, 1}, {32, 1},
                                  {32, 2}, {64, 2}, {128, 2}, {64, 2}, {64, 2},
                                  {64, 3}, {128, 3}, {128, 3}};
    int64_t aoff = 0;
    for (int i = 0; i < A_COUNT; ++i) {
        Unet::View vw;
        const bool cat = i == A_CAT1 || i == A_CAT2 || i == A_CAT3;
        vw.off = aoff; vw.C = defs[i][0]; vw.lvl = defs[i][1];
        vw.stride = cat ? vw.C / 2 : vw.C;
        vw.hs = cat ? (int64_t)max_batch * (H >> vw.lvl) * (W >> vw.lvl) * (vw.C / 2) : 0;
        aoff += (int64_t)max_batch * (H >> vw.lvl) * (W >> vw.lvl) * vw.C;
        aoff = (aoff + 63) / 64 * 64;
        U->av.push_back(vw);
    }
    auto fail_oom = [&]() { free_unet(U); return fail(ESI_ERR_OOM, "network allocation failed"); };
    if (hipMalloc(&U->theta, U->P * 4) != hipSuccess || hipMalloc(&U->m, U->P * 4) != hipSuccess ||
        hipMalloc(&U->v, U->P * 4) != hipSuccess || hipMalloc(&U->act, aoff * 2) != hipSuccess ||
        hipMalloc(&U->grad, aoff * 2) != hipSuccess ||
        hipMalloc(&U->go, (int64_t)max_batch * H * W * 4) != hipSuccess ||
        hipMalloc(&U->dloss, (int64_t)max_batch * 8) != hipSuccess)
        return fail_oom();
    for (Layer& Ly : U->L) {
        const int cpad = Ly.cin < 16 ? 16 : Ly.cin;
        const int64_t nf = Ly.kind == 0 ? frag_elems(Ly.cout, cpad) : Ly.kind == 1 ? convT_frag_elems(Ly.cin, Ly.cout)
                                                                            : Ly.nw;
        if (hipMalloc(&Ly.wf, nf * 2) != hipSuccess) return fail_oom();
        if (Ly.kind == 0 && hipMalloc(&Ly.wb, frag_elems(cpad, Ly.cout) * 2) != hipSuccess) return fail_oom();
        if (Ly.kind == 1 && hipMalloc(&Ly.wb, Ly.nw * 2) != hipSuccess) return fail_oom();
    }
    // zero everything so unused padding channels never hold garbage
    if (hipMemsetAsync(U->act, 0, aoff * 2, U->stream) != hipSuccess ||
        hipMemsetAsync(U->grad, 0, aoff * 2, U->stream) != hipSuccess ||
        hipMemsetAsync(U->theta, 0, U->P * 4, U->stream) != hipSuccess ||
        hipMemsetAsync(U->m, 0, U->P * 4, U->stream) != hipSuccess ||
        hipMemsetAsync(U->v, 0, U->P * 4, U->stream) != hipSuccess ||
        hipStreamSynchronize(U->stream) != hipSuccess) {
        free_unet(U);
        return fail(ESI_ERR_HIP, "network initialisation failed");
    }
    *out = reinterpret_cast<esi_unet_t>(U);
    return ESI_OK;
}

extern "C" esi_status_t esi_unet_destroy(esi_unet_t u) {
    set_error("");
    if (!u) return ESI_OK;
    Unet* U = as_unet(u);
    hipStreamSynchronize(U->stream);
    free_unet(U);
    return ESI_OK;
}

extern "C" esi_status_t esi_unet_set_params(esi_unet_t u, const float* theta) {
    set_error("");
    if (!u || !theta) return fail(ESI_ERR_ARG, "null argument");
    Unet* U = as_unet(u);
    ESI_HIP_TRY(hipMemcpyAsync(U->theta, theta, U->P * 4, hipMemcpyDefault, U->stream));
    ESI_HIP_TRY(hipMemsetAsync(U->m, 0, U->P * 4, U->stream));
    ESI_HIP_TRY(hipMemsetAsync(U->v, 0, U->P * 4, U->stream));
    ESI_TRY(pack(U));
    ESI_HIP_TRY(hipStreamSynchronize(U->stream));
    return ESI_OK;
}

extern "C" esi_status_t esi_unet_get_params(esi_unet_t u, float* theta) {
    set_error("");
    if (!u || !theta) return fail(ESI_ERR_ARG, "null argument");
    Unet* U = as_unet(u);
    ESI_HIP_TRY(hipMemcpyAsync(theta, U->theta, U->P * 4, hipMemcpyDefault, U->stream));
    ESI_HIP_TRY(hipStreamSynchronize(U->stream));
    return ESI_OK;
}

extern "C" esi_status_t esi_unet_forward(esi_unet_t u, const float* x, float* o, int32_t batch) {
    set_error("");
    if (!u || !x || !o) return fail(ESI_ERR_ARG, "null argument");
    Unet* U = as_unet(u);
    if (batch < 1 || batch > U->maxb) return fail(ESI_ERR_ARG, "batch outside [1, max_batch]");
    Ctx c{U, batch};
    return forward(c, x, o);
}

extern "C" esi_status_t esi_unet_loss_weights(const float* a, const float* c, int32_t batch, int64_t npix,
                                              float* w, void* stream) {
    set_error("");
    if (!a || !c || !w) return fail(ESI_ERR_ARG, "null argument");
    if (batch < 1 || npix < 1) return fail(ESI_ERR_ARG, "empty batch");
    hipLaunchKernelGGL(k_loss_weights, dim3(batch), dim3(NT), 0, (hipStream_t)stream, a, c, npix, w);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

extern "C" esi_status_t esi_unet_loss_grad(esi_unet_t u, const float* x, const float* a, const float* cc,
                                           const float* weight, int32_t batch, float* grad, double* loss) {
    set_error("");
    if (!u || !x || !a || !cc || !grad) return fail(ESI_ERR_ARG, "null argument");
    Unet* U = as_unet(u);
    if (batch < 1 || batch > U->maxb) return fail(ESI_ERR_ARG, "batch outside [1, max_batch]");
    Ctx c{U, batch};
    const int64_t npix = (int64_t)U->H * U->W;
    ESI_TRY(grow_t(&U->part, &U->part_cap, (int64_t)batch * npix, U->stream));   // o scratch
    float* o = U->part;
    ESI_TRY(forward(c, x, o));
    hipLaunchKernelGGL(k_scaling_loss, dim3(batch), dim3(NT), 0, U->stream, o, a, cc, weight, npix, batch, U->go,
                       U->dloss);
    ESI_HIP_TRY(hipGetLastError());
    ESI_TRY(backward(c, grad));
    if (loss) {
        std::vector<double> h(batch);
        ESI_HIP_TRY(hipMemcpyAsync(h.data(), U->dloss, batch * 8, hipMemcpyDeviceToHost, U->stream));
        ESI_HIP_TRY(hipStreamSynchronize(U->stream));
        double s = 0.0;
        for (double v : h) s += v;
        *loss = s / batch;
    }
    return ESI_OK;
}

extern "C" esi_status_t esi_unet_adam(esi_unet_t u, const float* grad, float lr, float beta1, float beta2,
                                      float eps, int32_t step, float clip_norm) {
    set_error("");
    if (!u || !grad) return fail(ESI_ERR_ARG, "null argument");
    if (step < 1) return fail(ESI_ERR_ARG, "Adam step counts from 1");
    Unet* U = as_unet(u);
    const float bc1 = (float)(1.0 - std::pow((double)beta1, step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, step));
    float* factor = nullptr;
    if (clip_norm > 0.f) {
        const int nb = 256;
        ESI_TRY(grow_t(&U->part, &U->part_cap, (int64_t)2 * nb + 2, U->stream));
        double* part = reinterpret_cast<double*>(U->part);
        factor = U->part + 2 * nb;
        hipLaunchKernelGGL(k_sqnorm, dim3(nb), dim3(NT), 0, U->stream, grad, U->P, part);
        hipLaunchKernelGGL(k_clip_factor, dim3(1), dim3(64), 0, U->stream, part, nb, clip_norm, factor);
    }
    hipLaunchKernelGGL(k_adam, dim3(grid_for(U->P)), dim3(NT), 0, U->stream, U->theta, U->m, U->v, grad, U->P,
                       lr, beta1, beta2, eps, bc1, bc2, factor);
    ESI_HIP_TRY(hipGetLastError());
    return pack(U);
}

namespace esi {

esi_status_t unet_dims(esi_unet_t u, int* H, int* W, int* maxb) {
    if (!u) return fail(ESI_ERR_ARG, "null network");
    Unet* U = as_unet(u);
    *H = U->H; *W = U->W; *maxb = U->maxb;
    return ESI_OK;
}

// Forward pass queued on `stream` (the caller's) instead of the network's own.
esi_status_t unet_forward_on(esi_unet_t u, hipStream_t stream, const float* x, float* o, int batch) {
    Unet* U = as_unet(u);
    if (batch < 1 || batch > U->maxb) return fail(ESI_ERR_ARG, "batch outside [1, max_batch]");
    hipStream_t own = U->stream;
    U->stream = stream;
    Ctx c{U, batch};
    esi_status_t st = forward(c, x, o);
    U->stream = own;
    return st;
}

}  // namespace esi
