// Learned preconditioner for the single-layer system: a convolutional network
// that acts patch by patch on the tensor-product coefficient grid of the spline
// space (a patch of S is a (2^m+p) x (2^m+p) grid of coefficients, Sec. 2.2) as
// an approximate inverse of the Jacobi-scaled Galerkin matrix.  Its purpose is
// the observation of Sec. 5 that diagonally preconditioned Krylov iterations
// grow costly for fine meshes and higher degrees.
//
// Network: five 3x3 convolutions, 1 -> C -> C -> C -> C -> 1 channels (C = 32),
// ReLU (or the identity: a linear network) after the first four, no biases,
// zero padding at the patch edges.  The
// preconditioner is the residual map y -> y + f(y) with y = D^-1 r (D the
// diagonal of the Galerkin matrix), so a network whose last layer is zero is
// the Jacobi preconditioner.  Without biases f is positively homogeneous,
// f(a y) = a f(y) for a > 0, so it needs no input normalisation.
//
// Precision: FP32 master weights for the optimiser (Adam), rounded to BF16
// (nearest even) for every forward and backward pass; activations, gradients
// and all sums in FP32.  Loss: L = sum (y + f(y) - x)^2 / (2 N) over the N
// coefficients of a batch of (y, x) pairs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/igabem.h"
#include "cnn.h"

namespace {

constexpr int kC = 32;               // hidden channels
constexpr int kLayers = 5;
constexpr int kTile = 16;            // convolution output tile: 16 RT x 16 pixels, RT per thread
constexpr int kCiChunk = 8;          // input channels staged in LDS at a time
constexpr int kGTH = 8, kGTW = 16;   // pixel tile of the weight-gradient kernel
constexpr int kGBlocks = 1024;       // weight-gradient blocks (partials summed in a fixed order)
constexpr int kLossBlocks = 1024;

constexpr int kCin[kLayers] = {1, kC, kC, kC, kC};
constexpr int kCout[kLayers] = {kC, kC, kC, kC, 1};

struct Dims {
    int64_t off[kLayers + 1];
    int cin[kLayers], cout[kLayers];
};

Dims make_dims()
{
    Dims d{};
    d.off[0] = 0;
    for (int l = 0; l < kLayers; ++l) {
        d.cin[l] = kCin[l];
        d.cout[l] = kCout[l];
        d.off[l + 1] = d.off[l] + (int64_t)9 * kCin[l] * kCout[l];
    }
    return d;
}

__device__ inline float bf16_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline uint16_t float_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even (finite inputs)
    return (uint16_t)(u >> 16);
}

// out[n][co][y][x] = sum_ci sum_{dy,dx} w[co][ci][dy][dx] a[n][ci][y+dy-1][x+dx-1]
// with a = relu(in) when RELU_IN, else in; zero outside the grid.  When
// MASK_OUT, out is multiplied by (mask > 0) (the ReLU derivative of the layer
// below, for the data gradient).  Grid: (tiles of 16 RT rows x 16 columns,
// images); each thread computes the pixels (py + 16 r, px), r < RT, so every
// weight read from LDS feeds RT multiply-adds (RT = 2 for several output
// channels, 1 for one, where more waves matter more).
template <int CIN, int COUT, bool RELU_IN, bool MASK_OUT>
constexpr int conv_rows() { return COUT > 1 ? 2 : 1; }

template <int CIN, int COUT, bool RELU_IN, bool MASK_OUT>
__global__ void __launch_bounds__(256) k_conv3(const float *__restrict__ in, const uint16_t *__restrict__ wgt,
                                               float *__restrict__ out, const float *__restrict__ mask, int H, int W,
                                               int tiles_x)
{
    constexpr int CC = CIN < kCiChunk ? CIN : kCiChunk;
    static_assert(CIN % CC == 0, "input channels in whole chunks");
    constexpr int RT = conv_rows<CIN, COUT, RELU_IN, MASK_OUT>();
    constexpr int SH = RT * kTile + 2, SW = kTile + 2;
    __shared__ float xs[CC][SH][SW + 1];
    __shared__ float ws[CC * 9][COUT];
    const int n = blockIdx.y;
    const int ty0 = (blockIdx.x / tiles_x) * (RT * kTile), tx0 = (blockIdx.x % tiles_x) * kTile;
    const int tid = threadIdx.x, py = tid / kTile, px = tid % kTile;
    const size_t plane = (size_t)H * W;
    float acc[RT][COUT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int co = 0; co < COUT; ++co) acc[r][co] = 0.f;
    for (int c0 = 0; c0 < CIN; c0 += CC) {
        __syncthreads();
        for (int i = tid; i < CC * SH * SW; i += 256) {
            const int cc = i / (SH * SW), r = i % (SH * SW), yy = r / SW, xx = r % SW;
            const int y = ty0 + yy - 1, x = tx0 + xx - 1;
            float v = 0.f;
            if (y >= 0 && y < H && x >= 0 && x < W) {
                v = in[((size_t)n * CIN + c0 + cc) * plane + (size_t)y * W + x];
                if (RELU_IN) v = fmaxf(v, 0.f);
            }
            xs[cc][yy][xx] = v;
        }
        for (int i = tid; i < CC * 9 * COUT; i += 256) {
            const int co = i / (CC * 9), r = i % (CC * 9);
            ws[r][co] = bf16_to_float(wgt[((size_t)co * CIN + c0) * 9 + r]);
        }
        __syncthreads();
        for (int cc = 0; cc < CC; ++cc) {
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                float xv[RT];
#pragma unroll
                for (int r = 0; r < RT; ++r) xv[r] = xs[cc][py + r * kTile + t / 3][px + t % 3];
#pragma unroll
                for (int co = 0; co < COUT; ++co) {
                    const float wv = ws[cc * 9 + t][co];
#pragma unroll
                    for (int r = 0; r < RT; ++r) acc[r][co] = fmaf(wv, xv[r], acc[r][co]);
                }
            }
        }
    }
    const int x = tx0 + px;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
        const int y = ty0 + py + r * kTile;
        if (y < H && x < W) {
            const size_t o = (size_t)n * COUT * plane + (size_t)y * W + x;
#pragma unroll
            for (int co = 0; co < COUT; ++co) {
                float v = acc[r][co];
                if (MASK_OUT && !(mask[o + co * plane] > 0.f)) v = 0.f;
                out[o + co * plane] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The 32 -> 32 channel layers on the matrix cores (v_mfma_f32_16x16x32_bf16: D = A B + C with A 16 x 32,
// B 32 x 16, FP32 C and D; lane l holds A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16], j < 8,
// and D[4 (l / 16) + i][l % 16], i < 4).  The weights are BF16 already; an FP32 value v enters as
// three BF16 terms, hi = bf16(v), mid = bf16(v - hi), lo = bf16(v - hi - mid), with hi + mid + lo = v
// exactly (each rounding to nearest removes at least eight of the 24 significant bits).  Their products
// with a BF16 weight are exact in FP32, so a convolution differs from FP32 arithmetic only in the order
// of the FP32 additions.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ inline f4_t mfma_bf16(const uint4 &a, const uint4 &b, const f4_t &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                   c, 0, 0, 0);
}

// the three BF16 terms of v
__device__ inline void split_bf16(float v, uint16_t &hi, uint16_t &mid, uint16_t &lo)
{
    hi = float_to_bf16(v);
    const float r = v - bf16_to_float(hi);
    mid = float_to_bf16(r);
    lo = float_to_bf16(r - bf16_to_float(mid));
}

// eight values split into three terms, each term's eight BF16 values packed in a uint4 (value j in the
// low half of word j / 2 for even j)
__device__ inline void split8_bf16(const float (&v)[8], uint4 &hi, uint4 &mid, uint4 &lo)
{
    uint32_t h[4], m[4], l[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint16_t h0, m0, l0, h1, m1, l1;
        split_bf16(v[2 * k], h0, m0, l0);
        split_bf16(v[2 * k + 1], h1, m1, l1);
        h[k] = (uint32_t)h0 | ((uint32_t)h1 << 16);
        m[k] = (uint32_t)m0 | ((uint32_t)m1 << 16);
        l[k] = (uint32_t)l0 | ((uint32_t)l1 << 16);
    }
    hi = uint4{h[0], h[1], h[2], h[3]};
    mid = uint4{m[0], m[1], m[2], m[3]};
    lo = uint4{l[0], l[1], l[2], l[3]};
}

constexpr int kMT = 16;               // convolution output tile: 16 x 16 pixels per workgroup
constexpr int kMS = kMT + 2;          // staged input side (one pixel of halo)
constexpr int kMPS = 40;              // LDS stride of a staged pixel in BF16: 32 channels + 8 padding, so
                                      // 16 lanes reading 16 bytes at consecutive pixels hit distinct banks

// MFMA operand order of a 32 -> 32 layer: wm[((t * 2 + mt) * 64 + lane) * 8 + j] =
// w[co = 16 mt + lane % 16][ci = 8 (lane / 16) + j][t] (w in the [co][ci][t] layout of wb or wt).
__global__ void k_pack_mfma(const uint16_t *__restrict__ w, uint16_t *__restrict__ wm)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9 * kC * kC) return;
    const int j = i % 8, lane = (i / 8) % 64, mt = (i / 512) % 2, t = i / 1024;
    const int co = 16 * mt + lane % 16, ci = 8 * (lane / 16) + j;
    wm[i] = w[(co * kC + ci) * 9 + t];
}

// out[n][co][y][x] = sum_ci sum_t w[co][ci][t] a[n][ci][y + dy - 1][x + dx - 1] for 32 channels in and
// out, as k_conv3<32, 32, RELU_IN, MASK_OUT>.  Workgroup: one 16 x 16 output tile of one image; the
// input tile with its halo is staged in LDS as hi, mid and lo planes, pixel-major with the 32 channels
// innermost.  Wave w takes output rows w, w + 4, w + 8, w + 12: per tap and row, six MFMAs (two halves
// of the output channels times the three terms) on A = the tap's weights (from wm, in operand order) and
// B = 16 pixels x 32 channels read straight from the staged tile.  The three planes take 77,760 bytes of
// LDS (gfx950 grants up to 160 KB to a workgroup; two workgroups fit a CU).
template <bool RELU_IN, bool MASK_OUT>
__global__ void __launch_bounds__(256) k_conv3_mfma(const float *__restrict__ in, const uint4 *__restrict__ wm,
                                                    float *__restrict__ out, const float *__restrict__ mask, int H,
                                                    int W, int tiles_x)
{
    __shared__ __attribute__((aligned(16))) uint16_t xs[3][kMS * kMS * kMPS];
    const int n = blockIdx.y;
    const int ty0 = (blockIdx.x / tiles_x) * kMT, tx0 = (blockIdx.x % tiles_x) * kMT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const size_t plane = (size_t)H * W;
    // one item = one staged pixel and eight channels (consecutive pixels over the lanes): all of a
    // thread's loads are issued before the first use, then three 16-byte LDS writes per item
    constexpr int NIT = (4 * kMS * kMS + 255) / 256;
    float v[NIT][8];
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
        const int it = tid + 256 * k;
        const int g = it / (kMS * kMS), r = it % (kMS * kMS);
        const int y = ty0 + r / kMS - 1, x = tx0 + r % kMS - 1;
        const bool inside = it < 4 * kMS * kMS && y >= 0 && y < H && x >= 0 && x < W;
        const float *src = in + ((size_t)n * kC + 8 * (inside ? g : 0)) * plane + (inside ? (size_t)y * W + x : 0);
#pragma unroll
        for (int j = 0; j < 8; ++j) v[k][j] = inside ? src[(size_t)j * plane] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
        const int it = tid + 256 * k;
        if (it >= 4 * kMS * kMS) break;
        const int g = it / (kMS * kMS), r = it % (kMS * kMS);
        if (RELU_IN)
#pragma unroll
            for (int j = 0; j < 8; ++j) v[k][j] = fmaxf(v[k][j], 0.f);
        uint4 h, md, l;
        split8_bf16(v[k], h, md, l);
        *(uint4 *)&xs[0][r * kMPS + 8 * g] = h;
        *(uint4 *)&xs[1][r * kMPS + 8 * g] = md;
        *(uint4 *)&xs[2][r * kMPS + 8 * g] = l;
    }
    __syncthreads();
    const int pn = lane & 15, kq = lane >> 4;
    f4_t acc[4][2];
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc[rr][0] = acc[rr][1] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int t = 0; t < 9; ++t) {
        const int dy = t / 3, dx = t % 3;
        const uint4 a0 = wm[(t * 2) * 64 + lane], a1 = wm[(t * 2 + 1) * 64 + lane];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int off = ((wave + 4 * rr + dy) * kMS + pn + dx) * kMPS + 8 * kq;
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
                const uint4 b = *(const uint4 *)&xs[pl][off];
                acc[rr][0] = mfma_bf16(a0, b, acc[rr][0]);
                acc[rr][1] = mfma_bf16(a1, b, acc[rr][1]);
            }
        }
    }
    const int x = tx0 + pn;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int y = ty0 + wave + 4 * rr;
        if (y >= H || x >= W) continue;
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const size_t o = ((size_t)n * kC + 16 * mt + 4 * kq + i) * plane + (size_t)y * W + x;
                float v = acc[rr][mt][i];
                if (MASK_OUT && !(mask[o] > 0.f)) v = 0.f;
                out[o] = v;
            }
    }
}

// Weight gradient of one layer: g[co][ci][t] = sum_{n,p} dz[n][co][p] a[n][ci][p + o_t]
// (a = relu(in) when RELU_IN), as per-block partial sums part[block][co][ci][t];
// block b takes the 8 x 16 pixel tiles b, b + gridDim.x, ...
template <int CIN, int COUT, bool RELU_IN>
__global__ void __launch_bounds__(256) k_wgrad3(const float *__restrict__ in, const float *__restrict__ dz,
                                                float *__restrict__ part, int H, int W, int tiles_x,
                                                int64_t tiles_per_img, int64_t ntiles)
{
    constexpr int NP = CIN * COUT;
    constexpr int PPT = (NP + 255) / 256;
    static_assert(256 % CIN == 0, "a thread keeps one input channel");
    constexpr int AW = kGTW + 2, AS = (kGTH + 2) * AW + 1;
    __shared__ float as[CIN * AS];
    __shared__ float ds[COUT][kGTH * kGTW];
    const int tid = threadIdx.x, ci = tid % CIN;
    const size_t plane = (size_t)H * W;
    float acc[PPT][9];
#pragma unroll
    for (int j = 0; j < PPT; ++j)
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[j][t] = 0.f;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int n = (int)(tile / tiles_per_img);
        const int r = (int)(tile % tiles_per_img);
        const int ty0 = (r / tiles_x) * kGTH, tx0 = (r % tiles_x) * kGTW;
        __syncthreads();
        for (int i = tid; i < CIN * (kGTH + 2) * AW; i += 256) {
            const int c = i / ((kGTH + 2) * AW), rr = i % ((kGTH + 2) * AW);
            const int y = ty0 + rr / AW - 1, x = tx0 + rr % AW - 1;
            float v = 0.f;
            if (y >= 0 && y < H && x >= 0 && x < W) {
                v = in[((size_t)n * CIN + c) * plane + (size_t)y * W + x];
                if (RELU_IN) v = fmaxf(v, 0.f);
            }
            as[c * AS + rr] = v;
        }
        for (int i = tid; i < COUT * kGTH * kGTW; i += 256) {
            const int co = i / (kGTH * kGTW), pp = i % (kGTH * kGTW);
            const int y = ty0 + pp / kGTW, x = tx0 + pp % kGTW;
            ds[co][pp] = (y < H && x < W) ? dz[((size_t)n * COUT + co) * plane + (size_t)y * W + x] : 0.f;
        }
        __syncthreads();
        if (tid < NP) {
            for (int pp = 0; pp < kGTH * kGTW; ++pp) {
                const int py = pp / kGTW, px = pp % kGTW;
                float a9[9];
#pragma unroll
                for (int t = 0; t < 9; ++t) a9[t] = as[ci * AS + (py + t / 3) * AW + px + t % 3];
#pragma unroll
                for (int j = 0; j < PPT; ++j) {
                    const int k = tid + 256 * j;
                    if (k < NP) {
                        const float d = ds[k / CIN][pp];
#pragma unroll
                        for (int t = 0; t < 9; ++t) acc[j][t] = fmaf(d, a9[t], acc[j][t]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const int k = tid + 256 * j;
        if (k < NP)
#pragma unroll
            for (int t = 0; t < 9; ++t) part[(size_t)blockIdx.x * NP * 9 + (size_t)k * 9 + t] = acc[j][t];
    }
}

constexpr int kWR = 4, kWC = 32;                     // weight-gradient tile: 4 rows x 32 columns
constexpr int kDZS = kWR * kWC + 8;                  // LDS stride of one channel of dz (BF16, padded)
constexpr int kASW = kWC + 8;                        // staged activation columns: x0 - 1 .. x0 + 38
constexpr int kAS = (kWR + 2) * kASW + 8;            // LDS stride of one channel of the activation

// (d0..d3, d4..d7) as 16 BF16 values; the 8 starting at element s (0..2)
__device__ inline uint4 shift_bf16(const uint4 &a, const uint4 &b, int s)
{
    auto fun = [](uint32_t lo, uint32_t hi) { return (uint32_t)((((uint64_t)hi << 32) | lo) >> 16); };
    if (s == 0) return a;
    if (s == 2) return uint4{a.y, a.z, a.w, b.x};
    return uint4{fun(a.x, a.y), fun(a.y, a.z), fun(a.z, a.w), fun(a.w, b.x)};
}

// Weight gradient of a 32 -> 32 layer on the matrix cores, as k_wgrad3<32, 32, RELU_IN>:
// g[co][ci][t] = sum over images and pixels p of dz[co][p] a[ci][p + o_t], one 32 x 32 product per tap
// with the pixels as the reduction.  Workgroup b takes the 4 x 32 pixel tiles b, b + gridDim.x, ...;
// dz (rows of the tile) and a (with a one-pixel halo) are staged in LDS as hi, mid and lo planes,
// channel by channel with the columns innermost.  Wave w owns the 16 x 16 block (co half w / 2, ci half
// w % 2) of all nine taps.  Per staged activation row s it reads the 16 channels' 32 columns once (two
// aligned 16-byte pieces per lane and term, shifted by dx in registers) and, for each dy with output row
// s - dy in the tile, adds the six products of terms of combined order at most two (hi hi, hi mid,
// mid hi, hi lo, lo hi, mid mid) for dx = 0, 1, 2; the three left out are below 2^-23 of the product.
// Partial sums per workgroup as k_wgrad3's, reduced by k_wreduce.  73,728 bytes of LDS per workgroup.
template <bool RELU_IN>
__global__ void __launch_bounds__(256) k_wgrad3_mfma(const float *__restrict__ in, const float *__restrict__ dz,
                                                     float *__restrict__ part, int H, int W, int tiles_x,
                                                     int64_t tiles_per_img, int64_t ntiles)
{
    __shared__ __attribute__((aligned(16))) uint16_t ds[3][kC * kDZS];
    __shared__ __attribute__((aligned(16))) uint16_t as[3][kC * kAS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mt = wave >> 1, nt = wave & 1, li = lane & 15, h = lane >> 4;
    const size_t plane = (size_t)H * W;
    f4_t acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f4_t{0.f, 0.f, 0.f, 0.f};
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int n = (int)(tile / tiles_per_img);
        const int r = (int)(tile % tiles_per_img);
        const int y0 = (r / tiles_x) * kWR, x0 = (r % tiles_x) * kWC;
        __syncthreads();
        // one item = eight consecutive pixels of one row and channel; all of a thread's loads (two dz
        // items, four activation items) are issued before the first use, then three 16-byte LDS writes
        // per item
        constexpr int ND = kC * kWR * (kWC / 8), NA = kC * (kWR + 2) * (kASW / 8);
        constexpr int KD = (ND + 255) / 256, KA = (NA + 255) / 256;
        float vd[KD][8], va[KA][8];
#pragma unroll
        for (int k = 0; k < KD; ++k) {
            const int it = tid + 256 * k;
            const int c = it / (kWR * kWC / 8), q = it % (kWR * kWC / 8);
            const int y = y0 + q / (kWC / 8), xb = x0 + 8 * (q % (kWC / 8));
            const bool ok = it < ND && y < H;
            const float *src = dz + ((size_t)n * kC + (ok ? c : 0)) * plane + (size_t)(ok ? y : 0) * W;
#pragma unroll
            for (int j = 0; j < 8; ++j) vd[k][j] = (ok && xb + j < W) ? src[xb + j] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < KA; ++k) {
            const int it = tid + 256 * k;
            const int c = it / ((kWR + 2) * (kASW / 8)), q = it % ((kWR + 2) * (kASW / 8));
            const int y = y0 + q / (kASW / 8) - 1, xb = x0 + 8 * (q % (kASW / 8)) - 1;
            const bool ok = it < NA && y >= 0 && y < H;
            const float *src = in + ((size_t)n * kC + (ok ? c : 0)) * plane + (size_t)(ok ? y : 0) * W;
#pragma unroll
            for (int j = 0; j < 8; ++j) va[k][j] = (ok && xb + j >= 0 && xb + j < W) ? src[xb + j] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < KD; ++k) {
            const int it = tid + 256 * k;
            if (it >= ND) break;
            const int c = it / (kWR * kWC / 8), q = it % (kWR * kWC / 8);
            uint4 hi, md, lo;
            split8_bf16(vd[k], hi, md, lo);
            const int o = c * kDZS + 8 * q;
            *(uint4 *)&ds[0][o] = hi;
            *(uint4 *)&ds[1][o] = md;
            *(uint4 *)&ds[2][o] = lo;
        }
#pragma unroll
        for (int k = 0; k < KA; ++k) {
            const int it = tid + 256 * k;
            if (it >= NA) break;
            const int c = it / ((kWR + 2) * (kASW / 8)), q = it % ((kWR + 2) * (kASW / 8));
            if (RELU_IN)
#pragma unroll
                for (int j = 0; j < 8; ++j) va[k][j] = fmaxf(va[k][j], 0.f);
            uint4 hi, md, lo;
            split8_bf16(va[k], hi, md, lo);
            const int o = c * kAS + 8 * q;
            *(uint4 *)&as[0][o] = hi;
            *(uint4 *)&as[1][o] = md;
            *(uint4 *)&as[2][o] = lo;
        }
        __syncthreads();
        const int co = 16 * mt + li, ci = 16 * nt + li;
#pragma unroll 1
        for (int sr = 0; sr < kWR + 2; ++sr) {
            uint4 b[3][3];  // [term][dx]
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
                const uint16_t *src = &as[pl][ci * kAS + sr * kASW + 8 * h];
                const uint4 c0 = *(const uint4 *)src, c1 = *(const uint4 *)(src + 8);
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) b[pl][dx] = shift_bf16(c0, c1, dx);
            }
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const int orow = sr - dy;
                if (orow < 0 || orow >= kWR) continue;
                uint4 a[3];
#pragma unroll
                for (int pl = 0; pl < 3; ++pl) a[pl] = *(const uint4 *)&ds[pl][co * kDZS + orow * kWC + 8 * h];
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    f4_t c = acc[dy * 3 + dx];
                    c = mfma_bf16(a[0], b[0][dx], c);
                    c = mfma_bf16(a[0], b[1][dx], c);
                    c = mfma_bf16(a[1], b[0][dx], c);
                    c = mfma_bf16(a[0], b[2][dx], c);
                    c = mfma_bf16(a[2], b[0][dx], c);
                    c = mfma_bf16(a[1], b[1][dx], c);
                    acc[dy * 3 + dx] = c;
                }
            }
        }
    }
    // D[m][n]: m = co within the half (4 (lane / 16) + i), n = ci within the half (lane % 16)
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = 16 * mt + 4 * h + i, ci = 16 * nt + li;
            part[(size_t)blockIdx.x * kC * kC * 9 + ((size_t)co * kC + ci) * 9 + t] = acc[t][i];
        }
}

// g[i] = sum over blocks b of part[b][i] in a fixed order: 32 weights per workgroup, 8 groups of
// threads summing the partials b = grp, grp + 8, ..., then the 8 group sums added in order.
__global__ void __launch_bounds__(256) k_wreduce(int nblk, int cnt, const float *__restrict__ part,
                                                 float *__restrict__ g)
{
    __shared__ float red[8][32];
    const int lane = threadIdx.x % 32, grp = threadIdx.x / 32;
    const int i = blockIdx.x * 32 + lane;
    float s = 0.f;
    if (i < cnt)
        for (int b = grp; b < nblk; b += 8) s += part[(size_t)b * cnt + i];
    red[grp][lane] = s;
    __syncthreads();
    if (grp == 0 && i < cnt) {
        float t = red[0][lane];
        for (int k = 1; k < 8; ++k) t += red[k][lane];
        g[i] = t;
    }
}

// d = y + f - x; dout = d * scale; per-block partial sums of d^2 (FP64).
__global__ void __launch_bounds__(256) k_loss(int64_t n, const float *__restrict__ y, const float *__restrict__ f,
                                              const float *__restrict__ x, float scale, float *__restrict__ dout,
                                              double *__restrict__ lpart)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float d = y[i] + f[i] - x[i];
        dout[i] = d * scale;
        s += (double)d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

__global__ void k_add_in(int64_t n, const float *__restrict__ y, float *__restrict__ f)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] += y[i];
}

__global__ void k_adam(int64_t n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi, vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 copies of the weights: wb in the forward layout [co][ci][t], wt for the
// data gradient, [ci][co][8 - t] (channels swapped, taps flipped).
__global__ void k_pack(Dims D, int64_t nw, const float *__restrict__ w, uint16_t *__restrict__ wb,
                       uint16_t *__restrict__ wt)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    int l = 0;
    while (l + 1 < kLayers && i >= D.off[l + 1]) ++l;
    const int64_t r = i - D.off[l];
    const int cin = D.cin[l], cout = D.cout[l];
    const int co = (int)(r / (9 * cin)), ci = (int)((r / 9) % cin), t = (int)(r % 9);
    const uint16_t h = float_to_bf16(w[i]);
    wb[i] = h;
    wt[D.off[l] + ((int64_t)ci * cout + co) * 9 + (8 - t)] = h;
}

__global__ void k_pc_in(int64_t n, const double *__restrict__ v, const double *__restrict__ D, float *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)(v[i] / D[i]);
}

__global__ void k_pc_out(int64_t n, const double *__restrict__ v, const double *__restrict__ D,
                         const float *__restrict__ f, double *__restrict__ z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = v[i] / D[i] + (double)f[i];
}

unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

struct igb_cnn {
    hipStream_t st = nullptr;
    bool relu = true;                  // IGB_CNN_RELU; false: identity activation (a linear network)
    Dims dims{};
    int64_t nw = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *part = nullptr;
    uint16_t *wb = nullptr, *wt = nullptr;
    uint16_t *wm = nullptr, *wtm = nullptr;  // the 32 -> 32 layers 1..3 in MFMA operand order (forward, backward)
    double *lpart = nullptr;
    int64_t step = 0;
    int64_t cap = 0;                   // pixels per activation buffer
    float *z[4] = {}, *da = nullptr, *db = nullptr, *f = nullptr, *d1 = nullptr, *yin = nullptr;
};

namespace {

igb_status err(igb_status s, const std::string &m)
{
    igb_set_error(m);
    return s;
}

#define CNNCHK(x)                                                                                         \
    do {                                                                                                  \
        hipError_t e_ = (x);                                                                              \
        if (e_ != hipSuccess)                                                                             \
            return err(e_ == hipErrorOutOfMemory ? IGB_ENOMEM : IGB_EHIP, std::string("HIP: ") + hipGetErrorString(e_)); \
    } while (0)
#define CNNLAUNCH() CNNCHK(hipGetLastError())

void free_acts(igb_cnn *net)
{
    for (float **p : {&net->z[0], &net->z[1], &net->z[2], &net->z[3], &net->da, &net->db, &net->f, &net->d1, &net->yin}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    net->cap = 0;
}

igb_status ensure(igb_cnn *net, int64_t npix)
{
    if (npix <= net->cap) return IGB_OK;
    CNNCHK(hipStreamSynchronize(net->st));
    free_acts(net);
    for (int l = 0; l < 4; ++l) CNNCHK(hipMalloc(&net->z[l], (size_t)npix * kC * sizeof(float)));
    CNNCHK(hipMalloc(&net->da, (size_t)npix * kC * sizeof(float)));
    CNNCHK(hipMalloc(&net->db, (size_t)npix * kC * sizeof(float)));
    CNNCHK(hipMalloc(&net->f, (size_t)npix * sizeof(float)));
    CNNCHK(hipMalloc(&net->d1, (size_t)npix * sizeof(float)));
    CNNCHK(hipMalloc(&net->yin, (size_t)npix * sizeof(float)));
    net->cap = npix;
    return IGB_OK;
}

// 32 -> 32 layers: wm holds the layer's weights in MFMA operand order
template <bool RELU_IN, bool MASK_OUT>
igb_status conv_mfma(const igb_cnn *net, const float *in, const uint16_t *wm, float *out, const float *mask, int nimg,
                     int H, int W)
{
    const int tx = (W + kMT - 1) / kMT, ty = (H + kMT - 1) / kMT;
    hipLaunchKernelGGL((k_conv3_mfma<RELU_IN, MASK_OUT>), dim3((unsigned)(tx * ty), (unsigned)nimg), dim3(256), 0,
                       net->st, in, (const uint4 *)wm, out, mask, H, W, tx);
    CNNLAUNCH();
    return IGB_OK;
}

template <int CIN, int COUT, bool RELU_IN, bool MASK_OUT>
igb_status conv(const igb_cnn *net, const float *in, const uint16_t *w, float *out, const float *mask, int nimg, int H,
                int W)
{
    constexpr int RT = conv_rows<CIN, COUT, RELU_IN, MASK_OUT>();
    const int tx = (W + kTile - 1) / kTile, ty = (H + RT * kTile - 1) / (RT * kTile);
    hipLaunchKernelGGL((k_conv3<CIN, COUT, RELU_IN, MASK_OUT>), dim3((unsigned)(tx * ty), (unsigned)nimg), dim3(256), 0,
                       net->st, in, w, out, mask, H, W, tx);
    CNNLAUNCH();
    return IGB_OK;
}

template <int CIN, int COUT, bool RELU_IN>
igb_status wgrad(igb_cnn *net, int layer, const float *in, const float *dz, int nimg, int H, int W)
{
    const bool mfma = CIN == kC && COUT == kC;
    const int tx = mfma ? (W + kWC - 1) / kWC : (W + kGTW - 1) / kGTW;
    const int ty = mfma ? (H + kWR - 1) / kWR : (H + kGTH - 1) / kGTH;
    const int64_t tpi = (int64_t)tx * ty, nt = tpi * nimg;
    const int nb = (int)std::min<int64_t>(kGBlocks, nt);
    if constexpr (CIN == kC && COUT == kC)
        hipLaunchKernelGGL((k_wgrad3_mfma<RELU_IN>), dim3((unsigned)nb), dim3(256), 0, net->st, in, dz, net->part, H, W,
                           tx, tpi, nt);
    else
        hipLaunchKernelGGL((k_wgrad3<CIN, COUT, RELU_IN>), dim3((unsigned)nb), dim3(256), 0, net->st, in, dz, net->part,
                           H, W, tx, tpi, nt);
    CNNLAUNCH();
    const int cnt = 9 * CIN * COUT;
    hipLaunchKernelGGL(k_wreduce, dim3(nblk(cnt, 32)), dim3(256), 0, net->st, nb, cnt, (const float *)net->part,
                       net->g + net->dims.off[layer]);
    CNNLAUNCH();
    return IGB_OK;
}

// f = network(in) (correction only) into net->f; pre-activations into z[0..3].
template <bool ACT>
igb_status forward_t(const igb_cnn *net, const float *in, int nimg, int H, int W)
{
    igb_status rc;
    const int64_t *o = net->dims.off;
    if ((rc = conv<1, kC, false, false>(net, in, net->wb + o[0], net->z[0], nullptr, nimg, H, W))) return rc;
    constexpr int64_t L = 9 * kC * kC;  // weights of one 32 -> 32 layer
    (void)o;
    if ((rc = conv_mfma<ACT, false>(net, net->z[0], net->wm, net->z[1], nullptr, nimg, H, W))) return rc;
    if ((rc = conv_mfma<ACT, false>(net, net->z[1], net->wm + L, net->z[2], nullptr, nimg, H, W))) return rc;
    if ((rc = conv_mfma<ACT, false>(net, net->z[2], net->wm + 2 * L, net->z[3], nullptr, nimg, H, W))) return rc;
    return conv<kC, 1, ACT, false>(net, net->z[3], net->wb + o[4], net->f, nullptr, nimg, H, W);
}

igb_status forward(const igb_cnn *net, const float *in, int nimg, int H, int W)
{
    return net->relu ? forward_t<true>(net, in, nimg, H, W) : forward_t<false>(net, in, nimg, H, W);
}

// Weight gradient into net->g from dL/df in net->d1 (activations of the last forward pass).
template <bool ACT>
igb_status backward_t(igb_cnn *net, const float *in, int nimg, int H, int W)
{
    igb_status rc;
    const int64_t *o = net->dims.off;
    const uint16_t *wt = net->wt;
    float **z = net->z;
    if ((rc = wgrad<kC, 1, ACT>(net, 4, z[3], net->d1, nimg, H, W))) return rc;
    if ((rc = conv<1, kC, false, ACT>(net, net->d1, wt + o[4], net->da, z[3], nimg, H, W))) return rc;
    if ((rc = wgrad<kC, kC, ACT>(net, 3, z[2], net->da, nimg, H, W))) return rc;
    constexpr int64_t L = 9 * kC * kC;
    if ((rc = conv_mfma<false, ACT>(net, net->da, net->wtm + 2 * L, net->db, z[2], nimg, H, W))) return rc;
    if ((rc = wgrad<kC, kC, ACT>(net, 2, z[1], net->db, nimg, H, W))) return rc;
    if ((rc = conv_mfma<false, ACT>(net, net->db, net->wtm + L, net->da, z[1], nimg, H, W))) return rc;
    if ((rc = wgrad<kC, kC, ACT>(net, 1, z[0], net->da, nimg, H, W))) return rc;
    if ((rc = conv_mfma<false, ACT>(net, net->da, net->wtm, net->db, z[0], nimg, H, W))) return rc;
    return wgrad<1, kC, false>(net, 0, in, net->db, nimg, H, W);
}

igb_status backward(igb_cnn *net, const float *in, int nimg, int H, int W)
{
    return net->relu ? backward_t<true>(net, in, nimg, H, W) : backward_t<false>(net, in, nimg, H, W);
}

// Loss of (in + f, target) and the weight gradient into net->g; returns sum d^2.
igb_status loss_grad(igb_cnn *net, const float *in, const float *tgt, int nimg, int H, int W, double *sumsq)
{
    igb_status rc;
    const int64_t npix = (int64_t)nimg * H * W;
    if ((rc = forward(net, in, nimg, H, W))) return rc;
    hipLaunchKernelGGL(k_loss, dim3(kLossBlocks), dim3(256), 0, net->st, npix, in, (const float *)net->f, tgt,
                       (float)(1.0 / (double)npix), net->d1, net->lpart);
    CNNLAUNCH();
    if ((rc = backward(net, in, nimg, H, W))) return rc;
    std::vector<double> lp(kLossBlocks);
    CNNCHK(hipMemcpyAsync(lp.data(), net->lpart, kLossBlocks * sizeof(double), hipMemcpyDeviceToHost, net->st));
    CNNCHK(hipStreamSynchronize(net->st));
    double s = 0.0;
    for (double x : lp) s += x;
    *sumsq = s;
    return IGB_OK;
}

igb_status adam_step(igb_cnn *net, float lr);

igb_status pack(igb_cnn *net)
{
    hipLaunchKernelGGL(k_pack, dim3(nblk(net->nw, 256)), dim3(256), 0, net->st, net->dims, net->nw, (const float *)net->w,
                       net->wb, net->wt);
    CNNLAUNCH();
    for (int l = 1; l <= 3; ++l) {
        const int64_t L = 9 * kC * kC;
        hipLaunchKernelGGL(k_pack_mfma, dim3(nblk(L, 256)), dim3(256), 0, net->st, (const uint16_t *)net->wb + net->dims.off[l],
                           net->wm + (l - 1) * L);
        hipLaunchKernelGGL(k_pack_mfma, dim3(nblk(L, 256)), dim3(256), 0, net->st, (const uint16_t *)net->wt + net->dims.off[l],
                           net->wtm + (l - 1) * L);
    }
    CNNLAUNCH();
    return IGB_OK;
}

igb_status adam_step(igb_cnn *net, float lr)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    ++net->step;
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)net->step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)net->step));
    hipLaunchKernelGGL(k_adam, dim3(nblk(net->nw, 256)), dim3(256), 0, net->st, net->nw, net->w, (const float *)net->g,
                       net->m, net->v, lr, b1, b2, eps, c1, c2);
    CNNLAUNCH();
    return pack(net);
}

struct StreamSwap {
    igb_cnn *net;
    hipStream_t keep;
    StreamSwap(igb_cnn *n, hipStream_t st) : net(n), keep(n->st) { n->st = st; }
    ~StreamSwap() { net->st = keep; }
};

igb_status check_grid(int64_t nimg, int64_t h, int64_t w)
{
    if (nimg < 1 || h < 1 || w < 1) return err(IGB_EINVAL, "image count and sizes must be >= 1");
    if (nimg > 65535) return err(IGB_EINVAL, "at most 65535 images per call");
    if (h > 4096 || w > 4096) return err(IGB_EINVAL, "image sides above 4096");
    return IGB_OK;
}

}  // namespace

int32_t cnn_precondition(const igb_cnn *cnet, int32_t n_img, int32_t h, int32_t w, const double *v, const double *D,
                         double *z, hipStream_t st)
{
    igb_cnn *net = const_cast<igb_cnn *>(cnet);
    igb_status rc;
    if ((rc = check_grid(n_img, h, w))) return rc;
    const int64_t n = (int64_t)n_img * h * w;
    if ((rc = ensure(net, n))) return rc;
    hipStream_t keep = net->st;
    net->st = st;
    hipLaunchKernelGGL(k_pc_in, dim3(nblk(n, 256)), dim3(256), 0, st, n, v, D, net->yin);
    rc = hipGetLastError() == hipSuccess ? IGB_OK : err(IGB_EHIP, "kernel launch failed");
    if (!rc) rc = forward(net, net->yin, n_img, h, w);
    if (!rc) {
        hipLaunchKernelGGL(k_pc_out, dim3(nblk(n, 256)), dim3(256), 0, st, n, v, D, (const float *)net->f, z);
        if (hipGetLastError() != hipSuccess) rc = err(IGB_EHIP, "kernel launch failed");
    }
    net->st = keep;
    return rc;
}

int32_t cnn_batch_forward(igb_cnn *net, const float *in, int32_t n_img, int32_t h, int32_t w, hipStream_t st,
                          float **f_out, float **dout)
{
    igb_status rc;
    if ((rc = check_grid(n_img, h, w))) return rc;
    if ((rc = ensure(net, (int64_t)n_img * h * w))) return rc;
    StreamSwap sw(net, st);
    if ((rc = forward(net, in, n_img, h, w))) return rc;
    *f_out = net->f;
    *dout = net->d1;
    return IGB_OK;
}

int32_t cnn_batch_backward_adam(igb_cnn *net, const float *in, int32_t n_img, int32_t h, int32_t w, float lr,
                                hipStream_t st)
{
    StreamSwap sw(net, st);
    igb_status rc;
    if ((rc = backward(net, in, n_img, h, w))) return rc;
    return adam_step(net, lr);
}

extern "C" {

igb_status igb_cnn_create(const float *weights_host, int32_t activation, void *hip_stream, igb_cnn **out)
{
    if (!out) return err(IGB_EINVAL, "null argument");
    *out = nullptr;
    if (!weights_host) return err(IGB_EINVAL, "null weights");
    if (activation != IGB_CNN_RELU && activation != IGB_CNN_LINEAR) return err(IGB_EINVAL, "unknown activation");
    igb_cnn *net = new igb_cnn();
    net->relu = activation == IGB_CNN_RELU;
    net->st = (hipStream_t)hip_stream;
    net->dims = make_dims();
    net->nw = net->dims.off[kLayers];
    if (net->nw != IGB_CNN_NUM_WEIGHTS) {
        delete net;
        return err(IGB_EINVAL, "weight count mismatch");
    }
    for (int64_t i = 0; i < net->nw; ++i)
        if (!std::isfinite(weights_host[i])) {
            delete net;
            return err(IGB_EINVAL, "weights must be finite");
        }
    auto fail_free = [&](igb_status s) {
        igb_cnn_destroy(net);
        return s;
    };
    const size_t fb = (size_t)net->nw * sizeof(float);
    hipError_t e = hipSuccess;
    for (auto a : {std::make_pair((void **)&net->w, fb), std::make_pair((void **)&net->g, fb),
                   std::make_pair((void **)&net->m, fb), std::make_pair((void **)&net->v, fb),
                   std::make_pair((void **)&net->wb, net->nw * sizeof(uint16_t)),
                   std::make_pair((void **)&net->wt, net->nw * sizeof(uint16_t)),
                   std::make_pair((void **)&net->wm, (size_t)3 * 9 * kC * kC * sizeof(uint16_t)),
                   std::make_pair((void **)&net->wtm, (size_t)3 * 9 * kC * kC * sizeof(uint16_t)),
                   std::make_pair((void **)&net->part, (size_t)kGBlocks * 9 * kC * kC * sizeof(float)),
                   std::make_pair((void **)&net->lpart, kLossBlocks * sizeof(double))})
        if (e == hipSuccess) e = hipMalloc(a.first, a.second);
    if (e != hipSuccess)
        return fail_free(err(e == hipErrorOutOfMemory ? IGB_ENOMEM : IGB_EHIP,
                             std::string("device allocation: ") + hipGetErrorString(e)));
    if (hipMemcpyAsync(net->w, weights_host, fb, hipMemcpyHostToDevice, net->st) != hipSuccess ||
        hipMemsetAsync(net->m, 0, fb, net->st) != hipSuccess || hipMemsetAsync(net->v, 0, fb, net->st) != hipSuccess)
        return fail_free(err(IGB_EHIP, "weight upload failed"));
    igb_status rc = pack(net);
    if (!rc && hipStreamSynchronize(net->st) != hipSuccess) rc = err(IGB_EHIP, "weight upload failed");
    if (rc) return fail_free(rc);
    *out = net;
    return IGB_OK;
}

void igb_cnn_destroy(igb_cnn *net)
{
    if (!net) return;
    (void)hipStreamSynchronize(net->st);
    free_acts(net);
    for (void *p : {(void *)net->w, (void *)net->g, (void *)net->m, (void *)net->v, (void *)net->wb, (void *)net->wt,
                    (void *)net->wm, (void *)net->wtm, (void *)net->part, (void *)net->lpart})
        if (p) (void)hipFree(p);
    delete net;
}

igb_status igb_cnn_get_weights(const igb_cnn *net, float *weights_host)
{
    if (!net || !weights_host) return err(IGB_EINVAL, "null argument");
    CNNCHK(hipMemcpyAsync(weights_host, net->w, net->nw * sizeof(float), hipMemcpyDeviceToHost, net->st));
    CNNCHK(hipStreamSynchronize(net->st));
    return IGB_OK;
}

igb_status igb_cnn_forward(const igb_cnn *cnet, const float *in_dev, int32_t n_img, int32_t h, int32_t w, float *out_dev)
{
    if (!cnet || !in_dev || !out_dev) return err(IGB_EINVAL, "null argument");
    igb_cnn *net = const_cast<igb_cnn *>(cnet);
    igb_status rc;
    if ((rc = check_grid(n_img, h, w))) return rc;
    const int64_t n = (int64_t)n_img * h * w;
    if ((rc = ensure(net, n))) return rc;
    if ((rc = forward(net, in_dev, n_img, h, w))) return rc;
    hipLaunchKernelGGL(k_add_in, dim3(nblk(n, 256)), dim3(256), 0, net->st, n, in_dev, net->f);
    CNNLAUNCH();
    CNNCHK(hipMemcpyAsync(out_dev, net->f, n * sizeof(float), hipMemcpyDeviceToDevice, net->st));
    return IGB_OK;
}

igb_status igb_cnn_gradient(igb_cnn *net, const float *in_dev, const float *target_dev, int32_t n_img, int32_t h,
                            int32_t w, double *loss_host, float *grad_host)
{
    if (!net || !in_dev || !target_dev || !loss_host || !grad_host) return err(IGB_EINVAL, "null argument");
    igb_status rc;
    if ((rc = check_grid(n_img, h, w))) return rc;
    const int64_t n = (int64_t)n_img * h * w;
    if ((rc = ensure(net, n))) return rc;
    double s;
    if ((rc = loss_grad(net, in_dev, target_dev, n_img, h, w, &s))) return rc;
    *loss_host = s / (2.0 * (double)n);
    CNNCHK(hipMemcpyAsync(grad_host, net->g, net->nw * sizeof(float), hipMemcpyDeviceToHost, net->st));
    CNNCHK(hipStreamSynchronize(net->st));
    return IGB_OK;
}

igb_status igb_cnn_train(igb_cnn *net, const float *y_dev, const float *x_dev, int64_t n_pairs, int32_t imgs_per_pair,
                         int32_t h, int32_t w, int32_t epochs, int32_t batch, float lr, double *loss_host)
{
    if (!net || !y_dev || !x_dev) return err(IGB_EINVAL, "null argument");
    if (n_pairs < 1 || epochs < 0 || batch < 1) return err(IGB_EINVAL, "n_pairs and batch must be >= 1, epochs >= 0");
    if (!(lr > 0.f) || !std::isfinite(lr)) return err(IGB_EINVAL, "learning rate must be > 0");
    igb_status rc;
    const int64_t b = std::min<int64_t>(batch, n_pairs);
    if ((rc = check_grid(b * imgs_per_pair, h, w))) return rc;
    const int64_t per = (int64_t)imgs_per_pair * h * w;
    if ((rc = ensure(net, b * per))) return rc;
    for (int e = 0; e < epochs; ++e) {
        double tot = 0.0;
        for (int64_t s0 = 0; s0 < n_pairs; s0 += b) {
            const int64_t nb = std::min(b, n_pairs - s0);
            double s;
            if ((rc = loss_grad(net, y_dev + s0 * per, x_dev + s0 * per, (int)(nb * imgs_per_pair), h, w, &s))) return rc;
            tot += s;
            if ((rc = adam_step(net, lr))) return rc;
        }
        if (loss_host) loss_host[e] = tot / (2.0 * (double)(n_pairs * per));
    }
    CNNCHK(hipStreamSynchronize(net->st));
    return IGB_OK;
}

}  // extern "C"
