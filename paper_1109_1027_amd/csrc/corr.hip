// Learned coarse-grid corrector: a 3-layer 3x3 convolutional network on 2D fields,
// BF16 operands on the MFMA units (v_mfma_f32_32x32x16_bf16) with FP32 accumulation.
//
//   A0 = bf16(features(Psi))                        [P, 8]   (P = pixels = batch x H x W, NHWC)
//   Z1 = conv(A0, W1) + b1,  A1 = bf16(silu(Z1))      [P, 32]
//   Z2 = conv(A1, W2) + b2,  A2 = bf16(silu(Z2))      [P, 32]
//   Y  = conv(A2, W3) + b3                          [P, 2]   FP32
//   Psi <- Psi + scale (Y0 + i Y1) on interior nodes
//
// Every convolution is an implicit GEMM.  Forward and input-gradient passes share
// one kernel: a wave owns 32 consecutive pixels of a row (the MFMA M dimension)
// and all 32 output channels (N); the reduction K = 9 taps x C_in runs in chunks
// of 16, each lane loading one 16-byte NHWC vector (8 channels of one tap).  The
// input-gradient pass is the same convolution with mirrored taps and transposed,
// repacked weights.  The weight gradient reduces over pixels: a block stages 64
// pixels of the input patches and of the output gradient in LDS, transposed so
// that each MFMA operand is one 16-byte LDS read, and accumulates a (9 C_in + 1)
// x 32 tile (the extra row, a constant 1, gives the bias gradient); per-block
// partial sums are added in a fixed order by a second pass.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"

using namespace nlse;

namespace nlse {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int CORR_CIN = 8, CORR_HID = 32, CORR_OUT = 2;
constexpr float LAP_SCALE = 16.0f, V_SCALE = 0.25f;
// flat FP32 parameter vector: W1[32][9][8] b1[32] W2[32][9][32] b2[32] W3[2][9][32] b3[2]
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + 32 * 9 * 8, OFF_W2 = OFF_B1 + 32, OFF_B2 = OFF_W2 + 32 * 9 * 32,
              OFF_W3 = OFF_B2 + 32, OFF_B3 = OFF_W3 + 2 * 9 * 32, NPARAM = OFF_B3 + 2;

__host__ __device__ inline int tap_dy(int t) { return t / 3 - 1; }
__host__ __device__ inline int tap_dx(int t) { return t % 3 - 1; }

// float -> bfloat16 bits, round to nearest even
__device__ __forceinline__ unsigned short f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

// SiLU and its derivative through the hardware exponential and reciprocal (about 1 ulp
// each, far below the bf16 rounding of every activation); training and inference use the
// same functions, so their forward passes agree bit for bit.
__device__ __forceinline__ float sigmoid_f(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float silu_f(float z) { return z * sigmoid_f(z); }
__device__ __forceinline__ float dsilu_f(float z)
{
    const float s = sigmoid_f(z);
    return s * (1.0f + z * (1.0f - s));
}

// ------------------------------------------------------------- features --
// Training-time input augmentation: a Gaussian of standard deviation sigma added to each
// real and imaginary part of the input field, drawn from a counter-based generator:
// splitmix64 (Steele, Lea & Flood 2014) of (seed, node, part) gives two uniforms, the
// Box-Muller transform one normal deviate.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ float gauss(uint64_t seed, uint64_t node, int part)
{
    const uint64_t a = splitmix64(seed * 0x100000001B3ull + node * 4 + part);
    const uint64_t b = splitmix64(a);
    const float u1 = ((float)(a >> 40) + 1.0f) * (1.0f / 16777216.0f);   // (0, 1]
    const float u2 = (float)(b >> 40) * (1.0f / 16777216.0f);            // [0, 1)
    return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

// The 8 input channels of node (y, x), packed as bf16: Re, Im, 16 h^2 Lap (Re, Im) with the
// 5-point Laplacian, |Psi|^2, V/4, 0, 0.  at(yy, xx) returns the field (zero outside it).
template <typename At>
__device__ __forceinline__ uint4 feat8(const At &at, int y, int x, float v)
{
    const float2 u = at(y, x);
    const float2 n = at(y - 1, x), s = at(y + 1, x), w = at(y, x - 1), e = at(y, x + 1);
    const float lr = (((n.x + s.x) + w.x) + e.x) - 4.0f * u.x;
    const float li = (((n.y + s.y) + w.y) + e.y) - 4.0f * u.y;
    uint4 pk;
    pk.x = f2bf(u.x) | ((unsigned)f2bf(u.y) << 16);
    pk.y = f2bf(LAP_SCALE * lr) | ((unsigned)f2bf(LAP_SCALE * li) << 16);
    pk.z = f2bf(u.x * u.x + u.y * u.y) | ((unsigned)f2bf(V_SCALE * v) << 16);
    pk.w = 0;
    return pk;
}

// X0[p][0..7] for every node of B dense complex fields [B][H][W] (complex64) or of a
// context's padded master field (templated on the master type).  aug_sigma > 0 adds
// the augmentation noise to the field before the features are formed.
template <typename M>
__global__ void features_kernel(const C<M> *psi, int64_t pitch_row, int64_t pitch_field, int64_t off,
                                const float *V, int B, int H, int W, unsigned short *X0, float aug_sigma,
                                uint64_t aug_seed)
{
    const int64_t P = (int64_t)B * H * W;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((int64_t)W * H));
        const C<M> *f = psi + b * pitch_field + off;
        auto at = [&](int yy, int xx) -> float2 {
            if (yy < 0 || yy >= H || xx < 0 || xx >= W) return make_float2(0.f, 0.f);
            const C<M> v = f[(int64_t)yy * pitch_row + xx];
            float2 r = make_float2((float)v.x, (float)v.y);
            if (aug_sigma > 0.f && yy > 0 && yy < H - 1 && xx > 0 && xx < W - 1) {
                const uint64_t node = ((uint64_t)b * H + yy) * W + xx;
                r.x += aug_sigma * gauss(aug_seed, node, 0);
                r.y += aug_sigma * gauss(aug_seed, node, 1);
            }
            return r;
        };
        reinterpret_cast<uint4 *>(X0)[p] = feat8(at, y, x, V[(int64_t)y * W + x]);
    }
}

// --------------------------------------------------- convolution (MFMA) --
// MODE 0: hidden forward  -> Z (FP32) and A = bf16(silu(Z + b))
// MODE 1: output forward  -> Y (FP32, channels 0..1) = acc + b
// MODE 2: input gradient  -> dZprev = bf16(acc * silu'(Zprev))   (taps mirrored by dir = -1)
template <int CI, int MODE>
__global__ __launch_bounds__(256) void conv_kernel(const unsigned short *X, const bf16x8 *Bpk, const float *bias,
                                                   int B, int H, int W, float *Zout, unsigned short *Aout,
                                                   const float *Zprev, float *Yout, int dir)
{
    constexpr int K = 9 * CI, NCH = (K + 15) / 16;
    const int lane = threadIdx.x & 63;
    const int64_t tiles_row = (W + 31) / 32;
    const int64_t tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t ntiles = (int64_t)B * H * tiles_row;
    if (tile >= ntiles) return;   // no barriers in this kernel
    const int x0 = (int)(tile % tiles_row) * 32;
    const int64_t row = tile / tiles_row;   // b * H + y
    const int y = (int)(row % H);
    const int64_t rowbase = row - y;        // b * H
    const int m = lane & 31, half = lane >> 5;
    const int x = x0 + m;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int k0 = 16 * c + 8 * half;
        const int t = k0 / CI, cb = k0 % CI;
        uint4 a = make_uint4(0, 0, 0, 0);
        if (t < 9) {
            const int yy = y + dir * tap_dy(t), xx = x + dir * tap_dx(t);
            if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                a = *reinterpret_cast<const uint4 *>(X + ((rowbase + yy) * W + xx) * CI + cb);
        }
        const bf16x8 av = __builtin_bit_cast(bf16x8, a);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, Bpk[c * 64 + lane], acc, 0, 0, 0);
    }
    // accumulator i of lane l holds row 8(i/4) + 4(l/32) + i%4, column l%32
    const int n = lane & 31;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int mm = 8 * (i / 4) + 4 * half + (i % 4);
        const int xo = x0 + mm;
        if (xo >= W) continue;
        const int64_t p = (rowbase + y) * W + xo;
        if (MODE == 0) {
            const float z = acc[i] + bias[n];
            Zout[p * 32 + n] = z;
            Aout[p * 32 + n] = f2bf(silu_f(z));
        } else if (MODE == 1) {
            if (n < CORR_OUT) Yout[p * CORR_OUT + n] = acc[i] + bias[n];
        } else {
            Aout[p * 32 + n] = f2bf(acc[i] * dsilu_f(Zprev[p * 32 + n]));
        }
    }
}

// ---------------------------------------------------- inference (tiled) --
// The forward pass without the training outputs, three launches per application:
//   layer 1: features of Psi (computed into LDS) -> A1,   layer 2: A1 -> A2,
//   layer 3: A2 -> Y, written out (inference) or added to the interior of Psi (apply).
// A block of 4 waves owns an output tile of 8 rows x 32 pixels; its 10 x 34-pixel input
// tile (zero outside the field) is staged in LDS once and every wave reads its 9 taps
// from there; the packed weights sit in registers.  Each wave computes 2 rows, the
// reduction over K in the same chunk order with the same operands as conv_kernel, so the
// results are bit-identical to the training forward pass.
constexpr int IT_R = 8, IT_W = 32, IT_IR = IT_R + 2, IT_IW = IT_W + 2, IT_PIX = IT_IR * IT_IW;

struct InfArgs {
    const void *psi;          // layer 1: the field (master of a context, or dense complex64 batch)
    int64_t pitch_row, pitch_field, off;
    const float *V;           // dense [H][W]
    int B, H, W;
    const unsigned short *X;  // layers 2, 3: input activations [P][32] bf16
    const bf16x8 *Bpk;        // packed weights of the layer
    const float *bias;
    unsigned short *Aout;     // layers 1, 2
    float *Yout;              // layer 3 (inference) or nullptr
    void *psi_out;            // layer 3 (apply): the context's master, or nullptr
    float scale;
};

template <int L, typename M>
__global__ __launch_bounds__(256) void infer_kernel(InfArgs A)
{
    constexpr int CI = L == 1 ? CORR_CIN : 32;
    constexpr int SP = CI + 8;                  // LDS pixel stride in bf16 (16-byte pad against bank conflicts)
    constexpr int NCH = (9 * CI + 15) / 16;
    __shared__ __attribute__((aligned(16))) unsigned short tile[IT_PIX * SP];
    __shared__ float ybuf[IT_R][IT_W][2];
    // per-wave staging of its two output rows as bf16 [row][pixel][channel] (+8 pad), so
    // that every lane stores 16 contiguous bytes
    __shared__ __attribute__((aligned(16))) unsigned short obuf[L < 3 ? 4 : 1][2][IT_W][40];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tiles_x = (A.W + IT_W - 1) / IT_W, tiles_y = (A.H + IT_R - 1) / IT_R;
    const int bx = blockIdx.x % tiles_x, by = (blockIdx.x / tiles_x) % tiles_y, b = blockIdx.x / (tiles_x * tiles_y);
    const int x0 = bx * IT_W, y0 = by * IT_R;
    const int64_t fbase = (int64_t)b * A.H * A.W;   // pixel index of this field's (0, 0)

    bf16x8 breg[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) breg[c] = A.Bpk[c * 64 + lane];

    // stage the input tile: pixel (ty, tx) is field node (y0 - 1 + ty, x0 - 1 + tx)
    if (L == 1) {
        const C<M> *f = (const C<M> *)A.psi + b * A.pitch_field + A.off;
        auto at = [&](int yy, int xx) -> float2 {
            if (yy < 0 || yy >= A.H || xx < 0 || xx >= A.W) return make_float2(0.f, 0.f);
            const C<M> v = f[(int64_t)yy * A.pitch_row + xx];
            return make_float2((float)v.x, (float)v.y);
        };
        for (int e = threadIdx.x; e < IT_PIX; e += blockDim.x) {
            const int yy = y0 - 1 + e / IT_IW, xx = x0 - 1 + e % IT_IW;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (yy >= 0 && yy < A.H && xx >= 0 && xx < A.W) v = feat8(at, yy, xx, A.V[(int64_t)yy * A.W + xx]);
            *reinterpret_cast<uint4 *>(tile + e * SP) = v;
        }
    } else {
        for (int e = threadIdx.x; e < IT_PIX * 4; e += blockDim.x) {
            const int px = e >> 2, part = e & 3;
            const int yy = y0 - 1 + px / IT_IW, xx = x0 - 1 + px % IT_IW;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (yy >= 0 && yy < A.H && xx >= 0 && xx < A.W)
                v = *reinterpret_cast<const uint4 *>(A.X + (fbase + (int64_t)yy * A.W + xx) * 32 + part * 8);
            *reinterpret_cast<uint4 *>(tile + px * SP + part * 8) = v;
        }
    }
    __syncthreads();

    const int m = lane & 31, half = lane >> 5;
    f32x16 acc[2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[r][i] = 0.f;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const int k0 = 16 * c + 8 * half;
        const int t = k0 / CI, cb = k0 % CI;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int ty = 2 * wv + r;              // output row within the tile
            uint4 a = make_uint4(0, 0, 0, 0);
            if (t < 9) a = *reinterpret_cast<const uint4 *>(tile + ((ty + 1 + tap_dy(t)) * IT_IW + (m + 1 + tap_dx(t))) * SP + cb);
            acc[r] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), breg[c], acc[r], 0, 0, 0);
        }
    }

    // accumulator i of lane l holds pixel 8(i/4) + 4(l/32) + i%4, channel l%32
    const int n = lane & 31;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int ty = 2 * wv + r, y = y0 + ty;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int mm = 8 * (i / 4) + 4 * half + (i % 4);
            const int xo = x0 + mm;
            if (L < 3) {
                obuf[L < 3 ? wv : 0][r][mm][n] = f2bf(silu_f(acc[r][i] + A.bias[n]));
            } else if (n < CORR_OUT) {
                ybuf[ty][mm][n] = acc[r][i] + A.bias[n];
            }
        }
    }
    if (L < 3) {
        __builtin_amdgcn_wave_barrier();   // the wave reads back only what it wrote
        // 2 rows x 32 pixels x 64 B = 256 16-byte pieces, 4 per lane
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = q * 64 + lane, r = e >> 7, px = (e >> 2) & 31, part = e & 3;
            const int y = y0 + 2 * wv + r, xo = x0 + px;
            if (y < A.H && xo < A.W)
                *reinterpret_cast<uint4 *>(A.Aout + (fbase + (int64_t)y * A.W + xo) * 32 + part * 8) =
                    *reinterpret_cast<const uint4 *>(&obuf[L < 3 ? wv : 0][r][px][part * 8]);
        }
    }
    if (L == 3) {
        __syncthreads();
        const int ty = threadIdx.x / IT_W, tx = threadIdx.x % IT_W;   // 256 threads = 8 x 32 pixels
        const int y = y0 + ty, x = x0 + tx;
        if (y < A.H && x < A.W) {
            const float y0v = ybuf[ty][tx][0], y1v = ybuf[ty][tx][1];
            if (A.Yout) {
                float *o = A.Yout + (fbase + (int64_t)y * A.W + x) * 2;
                o[0] = y0v;
                o[1] = y1v;
            } else if (x > 0 && x < A.W - 1 && y > 0 && y < A.H - 1) {
                C<M> *q = (C<M> *)A.psi_out + A.off + (int64_t)y * A.pitch_row + x;
                C<M> v = *q;
                v.x += (M)(A.scale * y0v);
                v.y += (M)(A.scale * y1v);
                *q = v;
            }
        }
    }
}

// ------------------------------------------------------- weight gradient --
// dW[k][n] for k = t*CI + c (t = tap) and the bias row k = 9*CI, summed over pixels:
//   dW[k][n] = sum_p G[p][n] X[p + off_t][c],   dB[n] = sum_p G[p][n].
// G has GC channels (32, or 8 for the 2-channel output gradient padded to 8).
constexpr int WG_PIX = 64;

template <int CI, int GC>
__global__ __launch_bounds__(256) void wgrad_kernel(const unsigned short *X, const unsigned short *G, int B, int H,
                                                    int W, float *partials)
{
    constexpr int K = 9 * CI + 1, MT = (K + 31) / 32;
    __shared__ unsigned short Xs[MT * 32][WG_PIX];
    __shared__ unsigned short Gs[32][WG_PIX];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t segs_row = (W + WG_PIX - 1) / WG_PIX;
    const int64_t nseg = (int64_t)B * H * segs_row;
    f32x16 acc[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[j][i] = 0.f;
    for (int64_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        const int x0 = (int)(seg % segs_row) * WG_PIX;
        const int64_t row = seg / segs_row;
        const int y = (int)(row % H);
        const int64_t rowbase = row - y;
        __syncthreads();
        // stage X patches transposed: Xs[t*CI + c][i] = X[(y+dy, x0+i+dx)][c]; row K = 1 (bias)
        for (int e = threadIdx.x; e < MT * 32 * WG_PIX; e += blockDim.x) {
            const int k = e / WG_PIX, i = e % WG_PIX;
            unsigned short v = 0;
            if (k < 9 * CI) {
                const int t = k / CI, c = k % CI;
                const int yy = y + tap_dy(t), xx = x0 + i + tap_dx(t);
                if (x0 + i < W && yy >= 0 && yy < H && xx >= 0 && xx < W) v = X[((rowbase + yy) * W + xx) * CI + c];
            } else if (k == 9 * CI) {
                v = (x0 + i < W) ? (unsigned short)0x3F80 : (unsigned short)0;   // 1.0 in bf16
            }
            Xs[k][i] = v;
        }
        for (int e = threadIdx.x; e < 32 * WG_PIX; e += blockDim.x) {
            const int n = e / WG_PIX, i = e % WG_PIX;
            unsigned short v = 0;
            if (n < GC && x0 + i < W) v = G[((rowbase + y) * W + x0 + i) * GC + n];
            Gs[n][i] = v;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int mt = wv + 4 * j;
            if (mt >= MT) break;
#pragma unroll
            for (int ch = 0; ch < WG_PIX / 16; ++ch) {
                const int pofs = 16 * ch + 8 * (lane >> 5);
                const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&Xs[mt * 32 + (lane & 31)][pofs]);
                const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&Gs[lane & 31][pofs]);
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[j], 0, 0, 0);
            }
        }
    }
    // partials[block][k][n]
    float *out = partials + (int64_t)blockIdx.x * MT * 32 * 32;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int mt = wv + 4 * j;
        if (mt >= MT) break;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int k = mt * 32 + 8 * (i / 4) + 4 * (lane >> 5) + (i % 4);
            out[k * 32 + (lane & 31)] = acc[j][i];
        }
    }
}

// sum the per-block partials in block order; scatter into the flat gradient vector
__global__ void wgrad_finish_kernel(const float *partials, int nblocks, int rows, int CI, int cout, float *gW,
                                    float *gB)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // e = k * 32 + n
    if (e >= rows * 32) return;
    const int k = e / 32, n = e % 32;
    if (n >= cout) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += partials[(int64_t)b * rows * 32 + e];
    if (k < 9 * CI) gW[(n * 9 + k / CI) * CI + k % CI] = s;   // W[n][t][c]
    else if (k == 9 * CI) gB[n] = s;
}

// ------------------------------------------------------- loss and dY --
// d = (Y - (ref - pred)/scale) on interior nodes; dY = bf16(2 d / count) into [P][8];
// per-block partial sums of d^2 (FP64) for the loss.
// With smooth = R > 0 the target is the residual filtered by the binomial kernel of
// width 2R + 1 along each axis (weights C(2R, k) / 4^R: [1 2 1]/4 for R = 1,
// [1 4 6 4 1]/16 for R = 2, ...), nodes outside the field taken as zero: only
// resolved scales are learned.
constexpr int MAX_SMOOTH = 4;
__global__ void loss_kernel(const float *Y, const float2 *pred, const float2 *ref, int B, int H, int W,
                            float inv_scale, float gscale, int smooth, unsigned short *dY, double *partials)
{
    __shared__ double sh[256];
    const int64_t P = (int64_t)B * H * W;
    double acc = 0.0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(p % W), y = (int)((p / W) % H);
        float d0 = 0.f, d1 = 0.f;
        if (x > 0 && x < W - 1 && y > 0 && y < H - 1) {
            float t0, t1;
            if (!smooth) {
                const float2 r = ref[p], q = pred[p];
                t0 = r.x - q.x;
                t1 = r.y - q.y;
            } else {
                float w[2 * MAX_SMOOTH + 1];
                float c = 1.f;
                for (int k = 0; k <= 2 * smooth; ++k) {      // C(2R, k) by the multiplicative formula
                    w[k] = c;
                    c = c * (float)(2 * smooth - k) / (float)(k + 1);
                }
                const float norm = 1.f / (float)(1u << (2 * smooth));
                t0 = 0.f;
                t1 = 0.f;
                for (int dy = -smooth; dy <= smooth; ++dy)
                    for (int dx = -smooth; dx <= smooth; ++dx) {
                        const int yy = y + dy, xx = x + dx;
                        if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                        const int64_t q2 = p + (int64_t)dy * W + dx;
                        const float wt = w[dy + smooth] * norm * w[dx + smooth] * norm;
                        const float2 r = ref[q2], q = pred[q2];
                        t0 += wt * (r.x - q.x);
                        t1 += wt * (r.y - q.y);
                    }
            }
            d0 = Y[p * 2] - t0 * inv_scale;
            d1 = Y[p * 2 + 1] - t1 * inv_scale;
        }
        acc += (double)d0 * d0 + (double)d1 * d1;
        uint4 pk = make_uint4(f2bf(gscale * d0) | ((unsigned)f2bf(gscale * d1) << 16), 0, 0, 0);
        reinterpret_cast<uint4 *>(dY)[p] = pk;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void sum_partials_kernel(const double *partials, int n, double *out)
{
    __shared__ double sh[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += partials[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// ------------------------------------------------------- weights, Adam --
// Forward B operand of layer (CI -> CO): chunk c, lane l: column n = l%32, rows
// k = 16c + 8(l/32) + j (j < 8), value W[n][k/CI][k%CI] (0 past K or n >= CO).
// Input-gradient B operand of the same layer: its input is the output gradient with
// GC channels (CO padded), its output the CI input channels: column c' = l%32, rows
// k = t*GC + n, value W[n][t][c'] (0 for n >= CO or c' >= CI).
__global__ void pack_kernel(const float *Wt, int CI, int CO, int GC, int transposed, unsigned short *out, int nch)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // e = (c * 64 + lane) * 8 + j
    if (e >= nch * 64 * 8) return;
    const int j = e % 8, lane = (e / 8) % 64, c = e / 512;
    const int col = lane % 32, k = 16 * c + 8 * (lane / 32) + j;
    float v = 0.f;
    if (!transposed) {
        if (k < 9 * CI && col < CO) v = Wt[(col * 9 + k / CI) * CI + k % CI];
    } else {
        const int t = k / GC, n = k % GC;
        if (k < 9 * GC && n < CO && col < CI) v = Wt[(n * 9 + t) * CI + col];
    }
    out[e] = f2bf(v);
}

__global__ void adam_kernel(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    m[i] = b1 * m[i] + (1.f - b1) * gi;
    v[i] = b2 * v[i] + (1.f - b2) * gi * gi;
    const float mh = m[i] / c1, vh = v[i] / c2;
    w[i] -= lr * mh / (sqrtf(vh) + eps);
}

// Psi <- Psi + scale (Y0 + i Y1) on the interior of a context's padded master field
// injection restriction: dst[y][x] = src[f y][f x] (dense complex fields)
template <typename S, typename D>
__global__ void inject_kernel(const C<S> *src, int64_t src_w, C<D> *dst, int64_t dst_h, int64_t dst_w, int factor)
{
    const int64_t P = dst_h * dst_w;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = p % dst_w, y = p / dst_w;
        dst[p] = cvt<D, S>(src[(y * factor) * src_w + x * factor]);
    }
}

}  // namespace nlse

// ------------------------------------------------------------------ host --

struct nlse_corr {
    int H, W, maxB;
    hipStream_t stream;
    float *params = nullptr, *grads = nullptr, *mom = nullptr, *vel = nullptr;
    unsigned short *pk1 = nullptr, *pk2 = nullptr, *pk3 = nullptr, *pk2t = nullptr, *pk3t = nullptr;
    float *V = nullptr;
    unsigned short *X0 = nullptr, *A1 = nullptr, *A2 = nullptr, *dY = nullptr, *dZ2 = nullptr, *dZ1 = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *Y = nullptr, *wpart = nullptr;
    double *lpart = nullptr, *lout = nullptr;
    double scale = 1.0;
    int smooth = 0;             // filter the training targets (see loss_kernel)
    double aug_sigma = 0.0;     // training-input augmentation noise (features_kernel)
    uint64_t aug_seed = 0;
    int adam_t = 0;
    bool packed = false;
};

namespace {
constexpr int NCH1 = (9 * CORR_CIN + 15) / 16, NCH2 = (9 * 32 + 15) / 16;
constexpr int NCH3T = (9 * 8 + 15) / 16;     // output gradient (2 channels padded to 8) -> 32
constexpr int WG_BLOCKS = 512, LOSS_BLOCKS = 512;

int pack_all(nlse_corr *m)
{
    auto pack = [&](const float *Wt, int CI, int CO, int GC, int tr, unsigned short *out, int nch) {
        const int n = nch * 64 * 8;
        hipLaunchKernelGGL(pack_kernel, dim3((n + 255) / 256), dim3(256), 0, m->stream, Wt, CI, CO, GC, tr, out, nch);
        return hipGetLastError();
    };
    HIPTRY(pack(m->params + OFF_W1, CORR_CIN, 32, 0, 0, m->pk1, NCH1));
    HIPTRY(pack(m->params + OFF_W2, 32, 32, 0, 0, m->pk2, NCH2));
    HIPTRY(pack(m->params + OFF_W3, 32, CORR_OUT, 0, 0, m->pk3, NCH2));
    HIPTRY(pack(m->params + OFF_W2, 32, 32, 32, 1, m->pk2t, NCH2));
    HIPTRY(pack(m->params + OFF_W3, 32, CORR_OUT, 8, 1, m->pk3t, NCH3T));
    m->packed = true;
    return NLSE_OK;
}

int64_t conv_blocks(int B, int H, int W) { return ((int64_t)B * H * ((W + 31) / 32) + 3) / 4; }

// forward of B fields whose features are already in X0
int forward(nlse_corr *m, int B)
{
    if (!m->packed) {
        int rc = pack_all(m);
        if (rc) return rc;
    }
    const unsigned g = (unsigned)conv_blocks(B, m->H, m->W);
    hipLaunchKernelGGL((conv_kernel<CORR_CIN, 0>), dim3(g), dim3(256), 0, m->stream, m->X0,
                       (const bf16x8 *)m->pk1, m->params + OFF_B1, B, m->H, m->W, m->Z1, m->A1, nullptr, nullptr, 1);
    HIPTRY(hipGetLastError());
    hipLaunchKernelGGL((conv_kernel<32, 0>), dim3(g), dim3(256), 0, m->stream, m->A1, (const bf16x8 *)m->pk2,
                       m->params + OFF_B2, B, m->H, m->W, m->Z2, m->A2, nullptr, nullptr, 1);
    HIPTRY(hipGetLastError());
    hipLaunchKernelGGL((conv_kernel<32, 1>), dim3(g), dim3(256), 0, m->stream, m->A2, (const bf16x8 *)m->pk3,
                       m->params + OFF_B3, B, m->H, m->W, nullptr, nullptr, nullptr, m->Y, 1);
    HIPTRY(hipGetLastError());
    return NLSE_OK;
}

template <int L, typename M>
hipError_t launch_infer(const InfArgs &a, hipStream_t st)
{
    const int tiles = a.B * ((a.H + IT_R - 1) / IT_R) * ((a.W + IT_W - 1) / IT_W);
    hipLaunchKernelGGL((infer_kernel<L, M>), dim3(tiles), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Inference of B fields straight from Psi (master type M at psi + off, rows pitch_row apart,
// fields pitch_field apart): Y to Yout, or (Yout = nullptr) Psi += scale Y on the interior.
template <typename M>
int infer_tiled(nlse_corr *m, const void *psi, int64_t pitch_row, int64_t pitch_field, int64_t off, int B,
                float *Yout, void *psi_out)
{
    if (!m->packed) {
        int rc = pack_all(m);
        if (rc) return rc;
    }
    InfArgs a;
    std::memset(&a, 0, sizeof a);
    a.psi = psi;
    a.pitch_row = pitch_row;
    a.pitch_field = pitch_field;
    a.off = off;
    a.V = m->V;
    a.B = B;
    a.H = m->H;
    a.W = m->W;
    a.Bpk = (const bf16x8 *)m->pk1;
    a.bias = m->params + OFF_B1;
    a.Aout = m->A1;
    HIPTRY((launch_infer<1, M>(a, m->stream)));
    a.X = m->A1;
    a.Bpk = (const bf16x8 *)m->pk2;
    a.bias = m->params + OFF_B2;
    a.Aout = m->A2;
    HIPTRY((launch_infer<2, M>(a, m->stream)));
    a.X = m->A2;
    a.Bpk = (const bf16x8 *)m->pk3;
    a.bias = m->params + OFF_B3;
    a.Aout = nullptr;
    a.Yout = Yout;
    a.psi_out = psi_out;
    a.scale = (float)m->scale;
    HIPTRY((launch_infer<3, M>(a, m->stream)));
    return NLSE_OK;
}

int features_dense(nlse_corr *m, const void *psi, int B, float aug_sigma = 0.f, uint64_t aug_seed = 0)
{
    const int64_t P = (int64_t)B * m->H * m->W;
    const unsigned g = (unsigned)std::min<int64_t>((P + 255) / 256, 65535);
    hipLaunchKernelGGL((features_kernel<float>), dim3(g), dim3(256), 0, m->stream, (const C<float> *)psi,
                       (int64_t)m->W, (int64_t)m->H * m->W, (int64_t)0, m->V, B, m->H, m->W, m->X0, aug_sigma,
                       aug_seed);
    HIPTRY(hipGetLastError());
    return NLSE_OK;
}

template <int CI, int GC>
int wgrad(nlse_corr *m, const unsigned short *X, const unsigned short *G, int B, float *gW, float *gB, int cout)
{
    constexpr int rows = ((9 * CI + 1 + 31) / 32) * 32;
    hipLaunchKernelGGL((wgrad_kernel<CI, GC>), dim3(WG_BLOCKS), dim3(256), 0, m->stream, X, G, B, m->H, m->W,
                       m->wpart);
    HIPTRY(hipGetLastError());
    hipLaunchKernelGGL(wgrad_finish_kernel, dim3((rows * 32 + 255) / 256), dim3(256), 0, m->stream, m->wpart,
                       WG_BLOCKS, rows, CI, cout, gW, gB);
    HIPTRY(hipGetLastError());
    return NLSE_OK;
}

// loss and gradients of B (pred, ref) pairs; grads land in m->grads
int loss_grads(nlse_corr *m, const void *pred, const void *ref, int B, double *loss)
{
    int rc = features_dense(m, pred, B, (float)m->aug_sigma, m->aug_seed + (uint64_t)m->adam_t);
    if (!rc) rc = forward(m, B);
    if (rc) return rc;
    const int H = m->H, W = m->W;
    const double count = 2.0 * B * (double)(H - 2) * (W - 2);
    hipLaunchKernelGGL(loss_kernel, dim3(LOSS_BLOCKS), dim3(256), 0, m->stream, m->Y, (const float2 *)pred,
                       (const float2 *)ref, B, H, W, (float)(1.0 / m->scale), (float)(2.0 / count), m->smooth, m->dY, m->lpart);
    HIPTRY(hipGetLastError());
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, m->stream, m->lpart, LOSS_BLOCKS, m->lout);
    HIPTRY(hipGetLastError());
    const unsigned g = (unsigned)conv_blocks(B, H, W);
    // layer 3: weight gradient, then input gradient through silu'(Z2)
    if ((rc = wgrad<32, 8>(m, m->A2, m->dY, B, m->grads + OFF_W3, m->grads + OFF_B3, CORR_OUT))) return rc;
    hipLaunchKernelGGL((conv_kernel<8, 2>), dim3(g), dim3(256), 0, m->stream, m->dY, (const bf16x8 *)m->pk3t,
                       nullptr, B, H, W, nullptr, m->dZ2, m->Z2, nullptr, -1);
    HIPTRY(hipGetLastError());
    // layer 2
    if ((rc = wgrad<32, 32>(m, m->A1, m->dZ2, B, m->grads + OFF_W2, m->grads + OFF_B2, 32))) return rc;
    hipLaunchKernelGGL((conv_kernel<32, 2>), dim3(g), dim3(256), 0, m->stream, m->dZ2, (const bf16x8 *)m->pk2t,
                       nullptr, B, H, W, nullptr, m->dZ1, m->Z1, nullptr, -1);
    HIPTRY(hipGetLastError());
    // layer 1
    if ((rc = wgrad<CORR_CIN, 32>(m, m->X0, m->dZ1, B, m->grads + OFF_W1, m->grads + OFF_B1, 32))) return rc;
    if (loss) {
        double l;
        HIPTRY(hipMemcpyAsync(&l, m->lout, sizeof l, hipMemcpyDeviceToHost, m->stream));
        HIPTRY(hipStreamSynchronize(m->stream));
        *loss = l / count;
    }
    return NLSE_OK;
}
}  // namespace

extern "C" {

int32_t nlse_corr_param_count(void) { return NPARAM; }

void nlse_corr_destroy(nlse_corr *m)
{
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    void *bufs[] = {m->params, m->grads, m->mom, m->vel, m->pk1, m->pk2, m->pk3, m->pk2t, m->pk3t, m->V, m->X0,
                    m->A1, m->A2, m->dY, m->dZ2, m->dZ1, m->Z1, m->Z2, m->Y, m->wpart, m->lpart, m->lout};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete m;
}

int nlse_corr_create(nlse_corr **out, int32_t H, int32_t W, int32_t max_batch, const double *V, void *stream)
{
    if (!out || H < 3 || W < 3 || max_batch < 1) return fail(NLSE_E_INVAL, "nlse_corr_create: bad arguments");
    *out = nullptr;
    nlse_corr *m = new nlse_corr();
    m->H = H;
    m->W = W;
    m->maxB = max_batch;
    m->stream = (hipStream_t)stream;
    const int64_t P = (int64_t)max_batch * H * W;
    struct A { void **p; size_t bytes; };
    const size_t wrows = ((9 * 32 + 1 + 31) / 32) * 32;
    A allocs[] = {{(void **)&m->params, NPARAM * 4}, {(void **)&m->grads, NPARAM * 4},
                  {(void **)&m->mom, NPARAM * 4}, {(void **)&m->vel, NPARAM * 4},
                  {(void **)&m->pk1, NCH1 * 64 * 16}, {(void **)&m->pk2, NCH2 * 64 * 16},
                  {(void **)&m->pk3, NCH2 * 64 * 16}, {(void **)&m->pk2t, NCH2 * 64 * 16},
                  {(void **)&m->pk3t, NCH3T * 64 * 16}, {(void **)&m->V, (size_t)H * W * 4},
                  {(void **)&m->X0, (size_t)P * 16}, {(void **)&m->A1, (size_t)P * 64}, {(void **)&m->A2, (size_t)P * 64},
                  {(void **)&m->dY, (size_t)P * 16}, {(void **)&m->dZ2, (size_t)P * 64}, {(void **)&m->dZ1, (size_t)P * 64},
                  {(void **)&m->Z1, (size_t)P * 128}, {(void **)&m->Z2, (size_t)P * 128}, {(void **)&m->Y, (size_t)P * 8},
                  {(void **)&m->wpart, (size_t)WG_BLOCKS * wrows * 32 * 4}, {(void **)&m->lpart, LOSS_BLOCKS * 8},
                  {(void **)&m->lout, 16}};
    for (auto &a : allocs) {
        hipError_t e = hipMalloc(a.p, a.bytes);
        if (e == hipSuccess) e = hipMemset(*a.p, 0, a.bytes);
        if (e != hipSuccess) {
            nlse_corr_destroy(m);
            return fail(NLSE_E_NOMEM, std::string("nlse_corr_create: ") + hipGetErrorString(e));
        }
    }
    if (V) {
        std::vector<float> vf((size_t)H * W);
        for (size_t i = 0; i < vf.size(); ++i) vf[i] = (float)V[i];
        hipError_t e = hipMemcpy(m->V, vf.data(), vf.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            nlse_corr_destroy(m);
            return hipfail(e, "nlse_corr_create: V");
        }
    }
    *out = m;
    return NLSE_OK;
}

int nlse_corr_set_params(nlse_corr *m, const float *params, double scale)
{
    if (!m || !params || !(scale > 0.0)) return fail(NLSE_E_INVAL, "nlse_corr_set_params: bad arguments");
    HIPTRY(hipMemcpyAsync(m->params, params, NPARAM * 4, hipMemcpyHostToDevice, m->stream));
    HIPTRY(hipMemsetAsync(m->mom, 0, NPARAM * 4, m->stream));
    HIPTRY(hipMemsetAsync(m->vel, 0, NPARAM * 4, m->stream));
    HIPTRY(hipStreamSynchronize(m->stream));
    m->scale = scale;
    m->adam_t = 0;
    m->packed = false;
    return NLSE_OK;
}

int nlse_corr_set_target_filter(nlse_corr *m, int32_t smooth)
{
    if (!m) return fail(NLSE_E_INVAL, "NULL corrector");
    if (smooth < 0 || smooth > MAX_SMOOTH) return fail(NLSE_E_INVAL, "target filter width out of range (0..4)");
    m->smooth = smooth;
    return NLSE_OK;
}

int nlse_corr_set_augment(nlse_corr *m, double sigma, uint64_t seed)
{
    if (!m || !(sigma >= 0.0)) return fail(NLSE_E_INVAL, "nlse_corr_set_augment: bad arguments");
    m->aug_sigma = sigma;
    m->aug_seed = seed;
    return NLSE_OK;
}

int nlse_corr_get_params(nlse_corr *m, float *params)
{
    if (!m || !params) return fail(NLSE_E_INVAL, "nlse_corr_get_params: bad arguments");
    HIPTRY(hipMemcpyAsync(params, m->params, NPARAM * 4, hipMemcpyDeviceToHost, m->stream));
    HIPTRY(hipStreamSynchronize(m->stream));
    return NLSE_OK;
}

int nlse_corr_infer(nlse_corr *m, const void *psi, int32_t batch, float *y_out)
{
    if (!m || !psi || !y_out || batch < 1 || batch > m->maxB) return fail(NLSE_E_INVAL, "nlse_corr_infer: bad arguments");
    return infer_tiled<float>(m, psi, m->W, (int64_t)m->H * m->W, 0, batch, y_out, nullptr);
}

int nlse_corr_grads(nlse_corr *m, const void *pred, const void *ref, int32_t batch, float *grads, double *loss)
{
    if (!m || !pred || !ref || batch < 1 || batch > m->maxB) return fail(NLSE_E_INVAL, "nlse_corr_grads: bad arguments");
    int rc = loss_grads(m, pred, ref, batch, loss);
    if (rc) return rc;
    if (grads) {
        HIPTRY(hipMemcpyAsync(grads, m->grads, NPARAM * 4, hipMemcpyDeviceToHost, m->stream));
        HIPTRY(hipStreamSynchronize(m->stream));
    }
    return NLSE_OK;
}

int nlse_corr_train_step(nlse_corr *m, const void *pred, const void *ref, int32_t batch, double lr, double *loss)
{
    if (!m || !pred || !ref || batch < 1 || batch > m->maxB || !(lr > 0.0))
        return fail(NLSE_E_INVAL, "nlse_corr_train_step: bad arguments");
    int rc = loss_grads(m, pred, ref, batch, loss);
    if (rc) return rc;
    m->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
    hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->params, m->grads, m->mom,
                       m->vel, NPARAM, (float)lr, b1, b2, 1e-8f, c1, c2);
    HIPTRY(hipGetLastError());
    return pack_all(m);
}

// Internal tensors of the training passes, for validation (see nlse.h).
int nlse_corr_tensor(nlse_corr *m, int32_t which, int32_t to_device, void *host, int64_t bytes)
{
    if (!m || !host || bytes < 0) return fail(NLSE_E_INVAL, "nlse_corr_tensor: bad arguments");
    const int64_t P = (int64_t)m->maxB * m->H * m->W;
    void *buf = nullptr;
    int64_t cap = 0;
    switch (which) {
    case NLSE_CORR_X0: buf = m->X0; cap = P * 16; break;
    case NLSE_CORR_A1: buf = m->A1; cap = P * 64; break;
    case NLSE_CORR_A2: buf = m->A2; cap = P * 64; break;
    case NLSE_CORR_Z1: buf = m->Z1; cap = P * 128; break;
    case NLSE_CORR_Z2: buf = m->Z2; cap = P * 128; break;
    case NLSE_CORR_Y: buf = m->Y; cap = P * 8; break;
    case NLSE_CORR_DY: buf = m->dY; cap = P * 16; break;
    case NLSE_CORR_DZ2: buf = m->dZ2; cap = P * 64; break;
    case NLSE_CORR_DZ1: buf = m->dZ1; cap = P * 64; break;
    case NLSE_CORR_GRADS: buf = m->grads; cap = NPARAM * 4; break;
    default: return fail(NLSE_E_INVAL, "nlse_corr_tensor: unknown tensor");
    }
    if (bytes > cap) return fail(NLSE_E_INVAL, "nlse_corr_tensor: more bytes than the tensor holds");
    HIPTRY(hipMemcpyAsync(to_device ? buf : host, to_device ? host : buf, (size_t)bytes,
                          to_device ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost, m->stream));
    HIPTRY(hipStreamSynchronize(m->stream));
    return NLSE_OK;
}

// One stage of the training passes on the internal tensors (see nlse.h).
int nlse_corr_stage(nlse_corr *m, int32_t op, int32_t batch)
{
    if (!m || batch < 1 || batch > m->maxB) return fail(NLSE_E_INVAL, "nlse_corr_stage: bad arguments");
    if (!m->packed) {
        const int rc = pack_all(m);
        if (rc) return rc;
    }
    const int B = batch, H = m->H, W = m->W;
    const unsigned g = (unsigned)conv_blocks(B, H, W);
    switch (op) {
    case NLSE_CORR_FWD1:
        hipLaunchKernelGGL((conv_kernel<CORR_CIN, 0>), dim3(g), dim3(256), 0, m->stream, m->X0, (const bf16x8 *)m->pk1,
                           m->params + OFF_B1, B, H, W, m->Z1, m->A1, nullptr, nullptr, 1);
        break;
    case NLSE_CORR_FWD2:
        hipLaunchKernelGGL((conv_kernel<32, 0>), dim3(g), dim3(256), 0, m->stream, m->A1, (const bf16x8 *)m->pk2,
                           m->params + OFF_B2, B, H, W, m->Z2, m->A2, nullptr, nullptr, 1);
        break;
    case NLSE_CORR_FWD3:
        hipLaunchKernelGGL((conv_kernel<32, 1>), dim3(g), dim3(256), 0, m->stream, m->A2, (const bf16x8 *)m->pk3,
                           m->params + OFF_B3, B, H, W, nullptr, nullptr, nullptr, m->Y, 1);
        break;
    case NLSE_CORR_WGRAD3: return wgrad<32, 8>(m, m->A2, m->dY, B, m->grads + OFF_W3, m->grads + OFF_B3, CORR_OUT);
    case NLSE_CORR_BWD3:
        hipLaunchKernelGGL((conv_kernel<8, 2>), dim3(g), dim3(256), 0, m->stream, m->dY, (const bf16x8 *)m->pk3t,
                           nullptr, B, H, W, nullptr, m->dZ2, m->Z2, nullptr, -1);
        break;
    case NLSE_CORR_WGRAD2: return wgrad<32, 32>(m, m->A1, m->dZ2, B, m->grads + OFF_W2, m->grads + OFF_B2, 32);
    case NLSE_CORR_BWD2:
        hipLaunchKernelGGL((conv_kernel<32, 2>), dim3(g), dim3(256), 0, m->stream, m->dZ2, (const bf16x8 *)m->pk2t,
                           nullptr, B, H, W, nullptr, m->dZ1, m->Z1, nullptr, -1);
        break;
    case NLSE_CORR_WGRAD1: return wgrad<CORR_CIN, 32>(m, m->X0, m->dZ1, B, m->grads + OFF_W1, m->grads + OFF_B1, 32);
    default: return fail(NLSE_E_INVAL, "nlse_corr_stage: unknown stage");
    }
    HIPTRY(hipGetLastError());
    return NLSE_OK;
}

int nlse_corr_apply(nlse_corr *m, nlse_ctx *c)
{
    if (!m || !c) return fail(NLSE_E_INVAL, "nlse_corr_apply: NULL argument");
    if (c->p.ndim != 2 || c->L.nx + 1 != m->W || c->L.ny + 1 != m->H)
        return fail(NLSE_E_INVAL, "nlse_corr_apply: context grid does not match the corrector");
    if (c->stream != m->stream) return fail(NLSE_E_INVAL, "nlse_corr_apply: corrector and context streams differ");
    const int64_t pitch = c->L.px, off = c->L.ox;
    const int rc = c->esM == 16 ? infer_tiled<double>(m, c->psi, pitch, 0, off, 1, nullptr, c->psi)
                                : infer_tiled<float>(m, c->psi, pitch, 0, off, 1, nullptr, c->psi);
    if (rc) return rc;
    // stage fields hold the master's boundary values only; their interiors are rewritten by the next step
    return NLSE_OK;
}

int nlse_step_corrected(nlse_ctx *c, nlse_corr *m, int64_t nsteps, double dt, int32_t every)
{
    if (!c || !m || every < 1 || nsteps < 0) return fail(NLSE_E_INVAL, "nlse_step_corrected: bad arguments");
    for (int64_t done = 0; done < nsteps;) {
        const int64_t n = std::min<int64_t>(every, nsteps - done);
        int rc = nlse_step(c, n, dt);
        if (rc) return rc;
        done += n;
        if (n == every) {
            rc = nlse_corr_apply(m, c);
            if (rc) return rc;
        }
    }
    return NLSE_OK;
}

int nlse_inject(const void *src, int32_t src_prec, int64_t src_n, void *dst, int64_t dst_n, int32_t factor,
                void *stream)
{
    if (!src || !dst || factor < 1 || dst_n * factor != src_n) return fail(NLSE_E_INVAL, "nlse_inject: bad sizes");
    const int64_t P = (dst_n + 1) * (dst_n + 1);
    const unsigned g = (unsigned)std::min<int64_t>((P + 255) / 256, 65535);
    hipStream_t st = (hipStream_t)stream;
    if (src_prec == NLSE_F32)
        hipLaunchKernelGGL((inject_kernel<float, float>), dim3(g), dim3(256), 0, st, (const C<float> *)src, src_n + 1,
                           (C<float> *)dst, dst_n + 1, dst_n + 1, factor);
    else
        hipLaunchKernelGGL((inject_kernel<double, float>), dim3(g), dim3(256), 0, st, (const C<double> *)src,
                           src_n + 1, (C<float> *)dst, dst_n + 1, dst_n + 1, factor);
    HIPTRY(hipGetLastError());
    return NLSE_OK;
}

}  // extern "C"
