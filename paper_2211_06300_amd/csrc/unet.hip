// Learned preconditioner network: a four-level U-Net (channels 16/32/64/128)
// with bfloat16 weights and activations and float32 accumulation, trained and
// run entirely by the kernels below.  The paper leaves the preconditioner of
// its CG open (Sec. 4.2 and Sec. 6: fewer inner iterations need an efficient
// preconditioner); the network, its loss and its use are this library's.
//
// Activations are NHWC bfloat16 (channels contiguous, 8-byte aligned groups of
// four).  A decoder level's concatenation [upsampled, skip] is one buffer: the
// transposed convolution writes channels [0, ch) and the encoder's second
// convolution writes its output straight into [ch, 2ch), so the skip costs
// no copy.
//
// 3x3 convolutions (forward and data gradient) are implicit GEMMs on
// v_mfma_f32_16x16x16_bf16: D[cout][pixel] = sum_{tap, ci} W[tap][cout][ci]
// X[pixel + tap][ci].  With the operand layout of that instruction a lane
// holds four consecutive input channels of one pixel (one 8-byte load) and
// four consecutive output channels of one pixel (one 8-byte store).  The data
// gradient is the same kernel with taps reversed and weights transposed.  The
// weight gradient is a GEMM over pixels (split into fixed chunks, partials
// summed in a fixed order).
#include <cmath>
#include <cstring>
#include <vector>

#include "esi_internal.h"

namespace esi {
namespace {

typedef uint16_t bf16_t;
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;
#ifndef ESI_CONV_TAPG
#define ESI_CONV_TAPG 3
#endif
constexpr int TG = ESI_CONV_TAPG;   // 3x3 taps whose operands are loaded together (1, 3 or 9)
static_assert(9 % TG == 0, "tap groups must split the 9 taps");

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
// 3x3 convolution, same size, zero padding; X and Y are NHWC views with pixel
// strides sx, sy (elements) and Cin, Cout channels (multiples of 16).
// Workgroup: 4 waves, one output row each, 64 pixels (4 groups of 16) x
// 16*CB output channels.  Wp is [9][Cout][Cin] bf16.
template <int CB>
__global__ __launch_bounds__(NT) void k_conv3(const bf16_t* __restrict__ X, int sx, int Cin,
                                              const bf16_t* __restrict__ Wp,
                                              const float* __restrict__ bias, bf16_t* __restrict__ Y,
                                              int sy, int Cout, int H, int W, int relu) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ncog = Cout / (16 * CB);
    const int n = blockIdx.z / ncog;
    const int co0 = (blockIdx.z % ncog) * 16 * CB;
    const int y = blockIdx.y * 4 + wave;
    if (y >= H) return;
    const int x0 = blockIdx.x * 64;
    const int jl = lane & 15, kq = (lane >> 4) * 4;
    f4 acc[4][CB];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[p][c] = f4{0.f, 0.f, 0.f, 0.f};
    const bf16_t* Xn = X + (int64_t)n * H * W * sx;
    for (int ci = 0; ci < Cin; ci += 16) {
        // the operands of TG taps first (TG x 4 pixel groups, TG x CB weight
        // blocks), so their loads overlap; then the MFMAs
#pragma unroll
        for (int t0 = 0; t0 < 9; t0 += TG) {
            s4 b[TG][4], a[TG][CB];
#pragma unroll
            for (int g = 0; g < TG; ++g) {
                const int tap = t0 + g;
                const int yy = y + tap / 3 - 1;
                const bool rowok = yy >= 0 && yy < H;
                const int dx = tap % 3 - 1;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int xx = x0 + p * 16 + jl + dx;
                    b[g][p] = (rowok && xx >= 0 && xx < W)
                                  ? *reinterpret_cast<const s4*>(Xn + ((int64_t)yy * W + xx) * sx + ci + kq)
                                  : s4{0, 0, 0, 0};
                }
#pragma unroll
                for (int c = 0; c < CB; ++c)
                    a[g][c] = *reinterpret_cast<const s4*>(Wp + ((int64_t)tap * Cout + co0 + c * 16 + jl) * Cin + ci + kq);
            }
#pragma unroll
            for (int g = 0; g < TG; ++g)
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int c = 0; c < CB; ++c)
                        acc[p][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[g][c], b[g][p], acc[p][c], 0, 0, 0);
        }
    }
    bf16_t* Yn = Y + (int64_t)n * H * W * sy;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int xo = x0 + p * 16 + jl;
        if (xo >= W) continue;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int co = co0 + c * 16 + kq;
            s4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float v = acc[p][c][e] + (bias ? bias[co + e] : 0.f);
                if (relu) v = fmaxf(v, 0.f);
                o[e] = (short)f2bf(v);
            }
            *reinterpret_cast<s4*>(Yn + ((int64_t)y * W + xo) * sy + co) = o;
        }
    }
}

// Weight gradient of a 3x3 convolution: part[chunk][tap][co][ci] =
// sum over the chunk's rows of gy[p][co] x[p + tap][ci], and the bias partial
// bpart[chunk][co] = sum gy[p][co] (written by the ci-block 0 waves).
// One wave per (chunk, co block, ci block); rows of all images are chunked.
__global__ __launch_bounds__(64) void k_conv3_wgrad(const bf16_t* __restrict__ GY, int sg, int Cout,
                                                    const bf16_t* __restrict__ X, int sx, int Cin,
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
        const bf16_t* Xn = X + (int64_t)n * H * W * sx;
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
    const int64_t total = (int64_t)N * H2 * W2 * C;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
        const int c = (int)(i % C);
        const int64_t pix = i / C;
        const int j = (int)(pix % W2), ii = (int)((pix / W2) % H2), n = (int)(pix / ((int64_t)W2 * H2));
        const int64_t base = ((int64_t)n * 2 * H2 + 2 * ii) * (2 * W2) + 2 * j;
        const float s = bf2f(X[base * sx + c]) + bf2f(X[(base + 1) * sx + c]) +
                        bf2f(X[(base + 2 * W2) * sx + c]) + bf2f(X[(base + 2 * W2 + 1) * sx + c]);
        Y[pix * sy + c] = f2bf(0.25f * s);
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
// v_mfma_f32_16x16x16_bf16: D[(a d) Cout + co][pixel] = sum_ci W4[(a d) Cout +
// co][ci] X[pixel][ci], stored with its bias at output pixel (2i + a, 2j + d).
// W4 is [4 Cout][Cin] bf16.  Workgroup: 4 waves, one input row each, 64 input
// pixels x 16 CB rows of D.
template <int CB>
__global__ __launch_bounds__(NT) void k_convT_mfma(const bf16_t* __restrict__ X, int sx, int Cin,
                                                   const bf16_t* __restrict__ W4, const float* __restrict__ bias,
                                                   bf16_t* __restrict__ Y, int sy, int Cout, int Hi, int Wi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int M = 4 * Cout;
    const int ncog = M / (16 * CB);
    const int n = blockIdx.z / ncog;
    const int m0 = (blockIdx.z % ncog) * 16 * CB;
    const int y = blockIdx.y * 4 + wave;
    if (y >= Hi) return;
    const int x0 = blockIdx.x * 64;
    const int jl = lane & 15, kq = (lane >> 4) * 4;
    f4 acc[4][CB];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[p][c] = f4{0.f, 0.f, 0.f, 0.f};
    const bf16_t* Xr = X + ((int64_t)n * Hi + y) * Wi * sx;
    for (int ci = 0; ci < Cin; ci += 16) {
        s4 b[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int xx = x0 + p * 16 + jl;
            b[p] = xx < Wi ? *reinterpret_cast<const s4*>(Xr + (int64_t)xx * sx + ci + kq) : s4{0, 0, 0, 0};
        }
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const s4 av = *reinterpret_cast<const s4*>(W4 + (int64_t)(m0 + c * 16 + jl) * Cin + ci + kq);
#pragma unroll
            for (int p = 0; p < 4; ++p)
                acc[p][c] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, b[p], acc[p][c], 0, 0, 0);
        }
    }
    const int Wo = 2 * Wi;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int xx = x0 + p * 16 + jl;
        if (xx >= Wi) continue;
#pragma unroll
        for (int c = 0; c < CB; ++c) {
            const int mrow = m0 + c * 16 + kq;            // four consecutive rows: same (a, d)
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
        float s = bias[0];
#pragma unroll
        for (int c = 0; c < 16; ++c) s += bf2f(w[c]) * bf2f(X[p * sx + c]);
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

// bf16 copies of the master weights: conv3x3 forward [9][Cout][cin_pad] and
// data-gradient [9][Cin][Cout] (taps reversed) from [co][ci][3][3].
__global__ void k_pack_conv3(const float* __restrict__ w, int Cout, int cin_real, int cin_pad,
                             bf16_t* __restrict__ wf, bf16_t* __restrict__ wb) {
    const int64_t n = (int64_t)9 * Cout * cin_pad;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const int ci = (int)(i % cin_pad), co = (int)((i / cin_pad) % Cout), tap = (int)(i / ((int64_t)cin_pad * Cout));
        const float v = ci < cin_real ? w[((int64_t)co * cin_real + ci) * 9 + tap] : 0.f;
        const bf16_t h = f2bf(v);
        wf[i] = h;
        if (wb && ci < cin_real) wb[((int64_t)(8 - tap) * cin_real + ci) * Cout + co] = h;
    }
}

// bf16 copies of transposed-convolution weights from [ci][co][a][d]: forward
// W4[(a d) Cout + co][ci] and data-gradient WT[ci][(a d) Cout + co].
__global__ void k_pack_convT(const float* __restrict__ w, int Cin, int Cout, bf16_t* __restrict__ w4,
                             bf16_t* __restrict__ wt) {
    const int64_t n = (int64_t)4 * Cin * Cout;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        const int ad = (int)(i % 4), co = (int)((i / 4) % Cout), ci = (int)(i / (4 * Cout));
        const bf16_t h = f2bf(w[i]);
        w4[((int64_t)ad * Cout + co) * Cin + ci] = h;
        wt[(int64_t)ci * 4 * Cout + ad * Cout + co] = h;
    }
}

__global__ void k_to_bf16(const float* __restrict__ w, bf16_t* __restrict__ o, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) o[i] = f2bf(w[i]);
}

// Network input: NCHW float32 [n][3][H][W] to NHWC bf16 with 16 channels
// (channels 3..15 zero).
__global__ void k_input(const float* __restrict__ x, bf16_t* __restrict__ X, int N, int64_t HW) {
    const int64_t total = (int64_t)N * HW * 16;
    for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < total; i += (int64_t)gridDim.x * NT) {
        const int c = (int)(i % 16);
        const int64_t pix = i / 16;
        const int64_t n = pix / HW, p = pix % HW;
        X[i] = c < 3 ? f2bf(x[(n * 3 + c) * HW + p]) : (bf16_t)0;
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
    struct View { int64_t off; int stride; int C; int lvl; };
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

struct Ctx {
    Unet* U;
    int N;
    int64_t pix(int lvl) const { return (int64_t)N * (U->H >> lvl) * (U->W >> lvl); }
    bf16_t* a(int id, int choff = 0) const { return U->act + U->av[id].off * 1 + choff; }
    bf16_t* g(int id, int choff = 0) const { return U->grad + U->av[id].off + choff; }
    int s(int id) const { return U->av[id].stride; }
    int h(int lvl) const { return U->H >> lvl; }
    int w(int lvl) const { return U->W >> lvl; }
};

esi_status_t conv3(const Ctx& c, const bf16_t* X, int sx, int Cin, int layer, bool bwd, bf16_t* Y, int sy,
                   int Cout, int lvl, bool relu) {
    Unet* U = c.U;
    const Layer& Ly = U->L[layer];
    const bf16_t* Wp = bwd ? Ly.wb : Ly.wf;
    const float* bias = bwd ? nullptr : U->theta + Ly.off + Ly.nw;
    const int H = c.h(lvl), W = c.w(lvl);
    const int cb = Cout >= 64 ? 4 : Cout / 16;
    dim3 grid((W + 63) / 64, (H + 3) / 4, c.N * (Cout / (16 * cb)));
    if (cb == 4)
        hipLaunchKernelGGL(k_conv3<4>, grid, dim3(NT), 0, U->stream, X, sx, Cin, Wp, bias, Y, sy, Cout, H, W, relu ? 1 : 0);
    else if (cb == 2)
        hipLaunchKernelGGL(k_conv3<2>, grid, dim3(NT), 0, U->stream, X, sx, Cin, Wp, bias, Y, sy, Cout, H, W, relu ? 1 : 0);
    else
        hipLaunchKernelGGL(k_conv3<1>, grid, dim3(NT), 0, U->stream, X, sx, Cin, Wp, bias, Y, sy, Cout, H, W, relu ? 1 : 0);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t need_part(Unet* U, int64_t n) {
    return grow_t(&U->part, &U->part_cap, n, U->stream);
}

// weight + bias gradient of a 3x3 layer into gflat
esi_status_t conv3_wgrad(const Ctx& c, const bf16_t* GY, int sg, int Cout, const bf16_t* X, int sx, int Cin,
                         int cin_real, int lvl, float* gflat) {
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
    hipLaunchKernelGGL(k_conv3_wgrad, dim3(nchunks, nblocks), dim3(64), 0, U->stream, GY, sg, Cout, X, sx,
                       Cin, H, W, nrows, rpc, part, bpart);
    const int64_t nout = (int64_t)9 * Cout * Cin + Cout;
    hipLaunchKernelGGL(k_conv3_wgrad_reduce, dim3(grid_for(nout)), dim3(NT), 0, U->stream, part, bpart, nchunks,
                       Cout, Cin, cin_real, gflat);
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

esi_status_t convT_fwd(const Ctx& c, int layer, const bf16_t* X, int sx, bf16_t* Y, int sy, int lvl_in) {
    Unet* U = c.U;
    const Layer& Ly = U->L[layer];
    const int Hi = c.h(lvl_in), Wi = c.w(lvl_in);
    const int M = 4 * Ly.cout;
    const int cb = M >= 64 ? 4 : M / 16;
    dim3 grid((Wi + 63) / 64, (Hi + 3) / 4, c.N * (M / (16 * cb)));
    const float* bias = U->theta + Ly.off + Ly.nw;
    if (cb == 4)
        hipLaunchKernelGGL(k_convT_mfma<4>, grid, dim3(NT), 0, U->stream, X, sx, Ly.cin, Ly.wf, bias, Y, sy,
                           Ly.cout, Hi, Wi);
    else
        hipLaunchKernelGGL(k_convT_mfma<1>, grid, dim3(NT), 0, U->stream, X, sx, Ly.cin, Ly.wf, bias, Y, sy,
                           Ly.cout, Hi, Wi);
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
    const int64_t n = c.pix(lvl_in + 1) * C;
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
    hipLaunchKernelGGL(k_input, dim3(grid_for(c.N * HW * 16)), dim3(NT), 0, U->stream, x, c.a(A_X), c.N, HW);
    // encoder
    ESI_TRY(conv3(c, c.a(A_X), 16, 16, C1A, false, c.a(A_A1), 16, 16, 0, true));
    ESI_TRY(conv3(c, c.a(A_A1), 16, 16, C1B, false, c.a(A_CAT1, 16), 32, 16, 0, true));
    ESI_TRY(pool(c, c.a(A_CAT1, 16), 32, c.a(A_P1), 16, 16, 0));
    ESI_TRY(conv3(c, c.a(A_P1), 16, 16, C2A, false, c.a(A_A2), 32, 32, 1, true));
    ESI_TRY(conv3(c, c.a(A_A2), 32, 32, C2B, false, c.a(A_CAT2, 32), 64, 32, 1, true));
    ESI_TRY(pool(c, c.a(A_CAT2, 32), 64, c.a(A_P2), 32, 32, 1));
    ESI_TRY(conv3(c, c.a(A_P2), 32, 32, C3A, false, c.a(A_A3), 64, 64, 2, true));
    ESI_TRY(conv3(c, c.a(A_A3), 64, 64, C3B, false, c.a(A_CAT3, 64), 128, 64, 2, true));
    ESI_TRY(pool(c, c.a(A_CAT3, 64), 128, c.a(A_P3), 64, 64, 2));
    ESI_TRY(conv3(c, c.a(A_P3), 64, 64, C4A, false, c.a(A_A4), 128, 128, 3, true));
    ESI_TRY(conv3(c, c.a(A_A4), 128, 128, C4B, false, c.a(A_B4), 128, 128, 3, true));
    // decoder
    ESI_TRY(convT_fwd(c, U3, c.a(A_B4), 128, c.a(A_CAT3), 128, 3));
    ESI_TRY(conv3(c, c.a(A_CAT3), 128, 128, D3A, false, c.a(A_D3A), 64, 64, 2, true));
    ESI_TRY(conv3(c, c.a(A_D3A), 64, 64, D3B, false, c.a(A_D3B), 64, 64, 2, true));
    ESI_TRY(convT_fwd(c, U2, c.a(A_D3B), 64, c.a(A_CAT2), 64, 2));
    ESI_TRY(conv3(c, c.a(A_CAT2), 64, 64, D2A, false, c.a(A_D2A), 32, 32, 1, true));
    ESI_TRY(conv3(c, c.a(A_D2A), 32, 32, D2B, false, c.a(A_D2B), 32, 32, 1, true));
    ESI_TRY(convT_fwd(c, U1, c.a(A_D2B), 32, c.a(A_CAT1), 32, 1));
    ESI_TRY(conv3(c, c.a(A_CAT1), 32, 32, D1A, false, c.a(A_D1A), 16, 16, 0, true));
    ESI_TRY(conv3(c, c.a(A_D1A), 16, 16, D1B, false, c.a(A_D1B), 16, 16, 0, true));
    const Layer& Lo = U->L[OUT];
    hipLaunchKernelGGL(k_out, dim3(grid_for(c.pix(0))), dim3(NT), 0, U->stream, c.a(A_D1B), 16, Lo.wf,
                       U->theta + Lo.off + Lo.nw, o, c.pix(0));
    ESI_HIP_TRY(hipGetLastError());
    return ESI_OK;
}

// Backward pass from U->go into the flat gradient gflat (after forward()).
esi_status_t backward(const Ctx& c, float* gflat) {
    Unet* U = c.U;
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
    auto conv_back = [&](int layer, int gid, int gchoff, int gstride, int Cout, const bf16_t* X, int sx,
                         int Cin, int lvl, bf16_t* GX, int sgx) -> esi_status_t {
        const Layer& Ly = U->L[layer];
        ESI_TRY(conv3_wgrad(c, c.g(gid, gchoff), gstride, Cout, X, sx, Cin, Ly.cin, lvl, gflat + Ly.off));
        if (GX) ESI_TRY(conv3(c, c.g(gid, gchoff), gstride, Cout, layer, true, GX, sgx, Cin, lvl, false));
        return ESI_OK;
    };
    // level 1 decoder: d1b, d1a (d1b's gradient is already masked)
    ESI_TRY(conv_back(D1B, A_D1B, 0, 16, 16, c.a(A_D1A), 16, 16, 0, c.g(A_D1A), 16));
    ESI_TRY(mask(c, c.g(A_D1A), 16, c.a(A_D1A), 16, 16, 0));
    ESI_TRY(conv_back(D1A, A_D1A, 0, 16, 16, c.a(A_CAT1), 32, 32, 0, c.g(A_CAT1), 32));
    ESI_TRY(convT_back(c, U1, c.a(A_D2B), 32, c.g(A_CAT1), 32, c.g(A_D2B), 32, 1, gflat));
    // level 2 decoder
    ESI_TRY(mask(c, c.g(A_D2B), 32, c.a(A_D2B), 32, 32, 1));
    ESI_TRY(conv_back(D2B, A_D2B, 0, 32, 32, c.a(A_D2A), 32, 32, 1, c.g(A_D2A), 32));
    ESI_TRY(mask(c, c.g(A_D2A), 32, c.a(A_D2A), 32, 32, 1));
    ESI_TRY(conv_back(D2A, A_D2A, 0, 32, 32, c.a(A_CAT2), 64, 64, 1, c.g(A_CAT2), 64));
    ESI_TRY(convT_back(c, U2, c.a(A_D3B), 64, c.g(A_CAT2), 64, c.g(A_D3B), 64, 2, gflat));
    // level 3 decoder
    ESI_TRY(mask(c, c.g(A_D3B), 64, c.a(A_D3B), 64, 64, 2));
    ESI_TRY(conv_back(D3B, A_D3B, 0, 64, 64, c.a(A_D3A), 64, 64, 2, c.g(A_D3A), 64));
    ESI_TRY(mask(c, c.g(A_D3A), 64, c.a(A_D3A), 64, 64, 2));
    ESI_TRY(conv_back(D3A, A_D3A, 0, 64, 64, c.a(A_CAT3), 128, 128, 2, c.g(A_CAT3), 128));
    ESI_TRY(convT_back(c, U3, c.a(A_B4), 128, c.g(A_CAT3), 128, c.g(A_B4), 128, 3, gflat));
    // bottleneck
    ESI_TRY(mask(c, c.g(A_B4), 128, c.a(A_B4), 128, 128, 3));
    ESI_TRY(conv_back(C4B, A_B4, 0, 128, 128, c.a(A_A4), 128, 128, 3, c.g(A_A4), 128));
    ESI_TRY(mask(c, c.g(A_A4), 128, c.a(A_A4), 128, 128, 3));
    ESI_TRY(conv_back(C4A, A_A4, 0, 128, 128, c.a(A_P3), 64, 64, 3, c.g(A_P3), 64));
    // encoder levels: gradient into e_l = pool path + skip, masked by e_l > 0;
    // the e_l gradient goes into the skip half of the concat gradient buffer
    struct Enc { int lvl, ch, cat, p, a, cb, ca, pin; };
    const Enc enc[3] = {{2, 64, A_CAT3, A_P3, A_A3, C3B, C3A, A_P2},
                        {1, 32, A_CAT2, A_P2, A_A2, C2B, C2A, A_P1},
                        {0, 16, A_CAT1, A_P1, A_A1, C1B, C1A, A_X}};
    for (const Enc& e : enc) {
        const int64_t n = c.pix(e.lvl) * e.ch;
        hipLaunchKernelGGL(k_pool_back, dim3(grid_for(n)), dim3(NT), 0, U->stream, c.g(e.p), e.ch,
                           c.g(e.cat, e.ch), 2 * e.ch, c.a(e.cat, e.ch), 2 * e.ch, c.g(e.cat, e.ch), 2 * e.ch,
                           e.ch, c.N, c.h(e.lvl), c.w(e.lvl));
        ESI_HIP_TRY(hipGetLastError());
        const int cin_a = e.lvl == 0 ? 16 : e.ch / 2;
        ESI_TRY(conv_back(e.cb, e.cat, e.ch, 2 * e.ch, e.ch, c.a(e.a), e.ch, e.ch, e.lvl, c.g(e.a), e.ch));
        ESI_TRY(mask(c, c.g(e.a), e.ch, c.a(e.a), e.ch, e.ch, e.lvl));
        ESI_TRY(conv_back(e.ca, e.a, 0, e.ch, e.ch, c.a(e.pin), cin_a, cin_a, e.lvl,
                          e.lvl == 0 ? nullptr : c.g(e.pin), cin_a));
    }
    return ESI_OK;
}

esi_status_t pack(Unet* U) {
    for (Layer& Ly : U->L) {
        const float* w = U->theta + Ly.off;
        if (Ly.kind == 0) {
            const int cpad = Ly.cin < 16 ? 16 : Ly.cin;
            const int64_t n = (int64_t)9 * Ly.cout * cpad;
            hipLaunchKernelGGL(k_pack_conv3, dim3(grid_for(n)), dim3(NT), 0, U->stream, w, Ly.cout, Ly.cin, cpad,
                               Ly.wf, Ly.wb);
        } else if (Ly.kind == 1) {
            hipLaunchKernelGGL(k_pack_convT, dim3(grid_for(Ly.nw)), dim3(NT), 0, U->stream, w, Ly.cin, Ly.cout,
                               Ly.wf, Ly.wb);
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
        vw.off = aoff; vw.stride = defs[i][0]; vw.C = defs[i][0]; vw.lvl = defs[i][1];
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
        const int64_t nf = Ly.kind == 0 ? (int64_t)9 * Ly.cout * cpad : Ly.nw;
        if (hipMalloc(&Ly.wf, nf * 2) != hipSuccess) return fail_oom();
        if (Ly.kind == 0 && hipMalloc(&Ly.wb, (int64_t)9 * Ly.cin * Ly.cout * 2) != hipSuccess) return fail_oom();
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
