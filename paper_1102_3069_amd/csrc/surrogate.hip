// Learned surrogate: a six-layer 3x3 convolutional network that proposes
// the magnetisation ten fixed steps ahead, trained and evaluated with BF16
// MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
//   input  x: m as a BF16 pair (hi, 256 (m - hi): 6 channels) and the
//          applied field B / 50 mT (3 channels)
//   net    conv3x3(9->32) SiLU, 4 x [conv3x3(32->32) SiLU], conv3x3(32->3)
//   output o; proposal m' = normalize(base + s o) for a base state (m or a
//          coarse step of it) and an output scale s; loss mean
//          (o - (m_t - base) / s)^2
//
// Every convolution is an implicit GEMM over (pixels) x (output channels)
// with K = 9 taps x 32 input channels.  Activations are BF16, channels
// last ([n][y][x][32], channel counts padded to 32 with zeros), weights
// BF16 [tap][cout][cin]; the data gradient is the same kernel with the
// weights flipped in space and transposed in channels, with the SiLU
// derivative of the layer below applied in its epilogue; the weight
// gradient is an MFMA reduction over pixel chunks into per-block partial
// sums that two more kernels add in a fixed order (deterministic).  Master
// weights and the Adam moments stay FP32.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "host_common.hpp"
#include "internal.hpp"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int CH = 32;          // padded channel count of every activation
constexpr int KC = 4;           // channels of the compact network output (3 used)
constexpr int NL = 6;           // layers
constexpr int CIN[NL] = {9, 32, 32, 32, 32, 32};
constexpr int COUT[NL] = {32, 32, 32, 32, 32, 3};
constexpr float B_SCALE = 0.05f;
constexpr float LO_SCALE = 256.0f;   // the low part of m is scaled by 2^8 before its own BF16 rounding
constexpr int kVerifyPart = 4;       // start states per verification batch

// round-to-nearest-even FP32 -> BF16 bits (NaN kept quiet)
__host__ __device__ inline u16 f2bf(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
// the same rounding by the hardware conversion (v_cvt_pk_bf16_f32)
__device__ inline u16 f2bf_hw(float f) { return __builtin_bit_cast(u16, (__bf16)f); }
__host__ __device__ inline float bf2f(u16 h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

__device__ inline bf16x8 load8(const u16* p) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    bf16x8 r;
    memcpy(&r, &v, 16);
    return r;
}
__device__ inline bf16x8 zero8() {
    bf16x8 r;
    const uint4 z = make_uint4(0, 0, 0, 0);
    memcpy(&r, &z, 16);
    return r;
}

// SiLU and its derivative on the hardware exp2 and reciprocal (about 1 ulp
// each; every result is rounded to BF16 afterwards, 2^-9)
__device__ inline float sigmoid_hw(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigmoid_hw(z); }
__device__ inline float silu_grad(float z) {
    const float s = sigmoid_hw(z);
    return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// MFMA lane layout of v_mfma_f32_16x16x32_bf16 (C = A B, A 16x32, B 32x16):
//   A: lane l holds row (l % 16), k = 8 (l / 16) + 0..7
//   B: lane l holds column (l % 16), k = 8 (l / 16) + 0..7
//   C: lane l holds column (l % 16), rows 4 (l / 16) + 0..3
// The self-test below multiplies known matrices to confirm it.
// ---------------------------------------------------------------------------
__global__ void mfma_selftest_kernel(const u16* A, const u16* B, float* C) {
    const int l = threadIdx.x;
    bf16x8 a = load8(A + (l % 16) * 32 + 8 * (l / 16));
    u16 bt[8];
    for (int i = 0; i < 8; ++i) bt[i] = B[(8 * (l / 16) + i) * 16 + (l % 16)];
    bf16x8 b;
    memcpy(&b, bt, 16);
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    for (int r = 0; r < 4; ++r) C[(4 * (l / 16) + r) * 16 + (l % 16)] = c[r];
}

// ---------------------------------------------------------------------------
// forward convolution (also the data gradient with transposed weights)
//   in   [N][H][W][32] bf16, wt [9][32 cout][32 cin] bf16, bias [32] (may be null)
//   z    [N][H][W][32] float (pre-activation, may be null)
//   zc   [N][H][W][4] float (its first four channels: the network output, may be null)
//   zb   [N][H][W][32] bf16 (pre-activation kept for the backward pass, may be null)
//   a    [N][H][W][32] bf16 (SiLU(z) if act, else z; may be null)
//   zg   [N][H][W][32] bf16 (may be null): data-gradient mode, a is then
//        z times SiLU'(zg), the gradient at the previous layer's pre-activation
// block: 4 waves, 64 pixels of `rows` consecutive rows; a wave: 16 pixels x
// 32 channels per row, with the weight fragments of all nine taps held in
// registers across the rows.  The bf16 tiles (a, zb, zg) pass through LDS so
// that every lane reads or writes 16 contiguous bytes (8 channels of one
// pixel).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void conv_fwd_kernel(const u16* __restrict__ in, const u16* __restrict__ wt,
                                                       const float* __restrict__ bias, float* __restrict__ z,
                                                       float* __restrict__ zc, u16* __restrict__ zb, u16* __restrict__ a,
                                                       const u16* __restrict__ zg, int H, int W, int act, int rows) {
    __shared__ u16 ws[9 * CH * CH];
    __shared__ u16 tile[4][2][16 * CH];   // per wave: [0] a, [1] zb or zg; [pixel][channel]
    const int tid = threadIdx.x;
    for (int i = tid; i < 9 * CH * CH / 8; i += 256)
        reinterpret_cast<uint4*>(ws)[i] = reinterpret_cast<const uint4*>(wt)[i];
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int n = blockIdx.z;
    const int x0 = blockIdx.x * 64 + wave * 16;
    const int col = lane % 16, kg = lane / 16;
    const size_t img = (size_t)n * H * W;
    u16* ta = tile[wave][0];
    u16* tz = tile[wave][1];
    // the lane's 16-byte chunk of a tile row: pixel lane / 4, channels 8 (lane % 4)
    const int cpx = lane >> 2, cch = 8 * (lane & 3);
    bf16x8 B0[9], B1[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        B0[t] = load8(ws + t * CH * CH + col * CH + 8 * kg);
        B1[t] = load8(ws + t * CH * CH + (16 + col) * CH + 8 * kg);
    }
    const float bias0 = bias ? bias[col] : 0.f, bias1 = bias ? bias[16 + col] : 0.f;
    const int ya = blockIdx.y * rows, yb = min(ya + rows, H);
    // the A fragments of input rows y-1, y, y+1 (taps v = 0, 1, 2) roll down
    // the rows; the next input row is read while this row's epilogue runs.
    // Every lane reads (outside the image: the nearest pixel inside), so that
    // no load is conditional and the waits stay exact; a row's fragments
    // outside the image are zeroed in place once they have arrived.
    auto load_row = [&](int yy, bf16x8 (&dst)[3]) {
        const int yc = min(max(yy, 0), H - 1);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const int xc = min(max(x0 + col + v - 1, 0), W - 1);
            dst[v] = load8(in + ((img + (size_t)yc * W + xc) * CH + 8 * kg));
        }
    };
    auto mask_row = [&](int yy, bf16x8 (&r)[3]) {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const int xx = x0 + col + v - 1;
            if (!(yy >= 0 && yy < H && xx >= 0 && xx < W)) r[v] = zero8();
        }
    };
    bf16x8 Ar[3][3];
    load_row(ya - 1, Ar[0]);
    load_row(ya, Ar[1]);
    load_row(ya + 1, Ar[2]);
    mask_row(ya - 1, Ar[0]);
    mask_row(ya, Ar[1]);
    for (int y = ya; y < yb; ++y) {
        mask_row(y + 1, Ar[2]);
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
#pragma unroll
        for (int u = 0; u < 3; ++u) {
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ar[u][v], B0[u * 3 + v], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ar[u][v], B1[u * 3 + v], acc1, 0, 0, 0);
            }
        }
        const size_t crow = (img + (size_t)y * W + x0 + cpx) * CH + cch;   // the lane's chunk in global memory
        const bool cin = x0 + cpx < W;
        uint4 gch = make_uint4(0, 0, 0, 0);
        if (zg) gch = *reinterpret_cast<const uint4*>(zg + (img + (size_t)y * W + min(x0 + cpx, W - 1)) * CH + cch);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            Ar[0][v] = Ar[1][v];
            Ar[1][v] = Ar[2][v];
        }
        load_row(y + 1 < yb ? y + 2 : H, Ar[2]);   // (row H: zeros, nothing read)
        if (zg) *reinterpret_cast<uint4*>(tz + cpx * CH + cch) = gch;
        __builtin_amdgcn_wave_barrier();
        // C layout: lane holds channels col and 16 + col of pixel 4 kg + r
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int px = 4 * kg + r;
            const float v0 = acc0[r] + bias0, v1 = acc1[r] + bias1;
            if (z && x0 + px < W) {
                const size_t p = (img + (size_t)y * W + x0 + px) * CH;
                z[p + col] = v0;
                z[p + 16 + col] = v1;
            }
            if (zc && col < KC && x0 + px < W) zc[(img + (size_t)y * W + x0 + px) * KC + col] = v0;
            float o0 = v0, o1 = v1;
            if (zg) {
                o0 *= silu_grad(bf2f(tz[px * CH + col]));
                o1 *= silu_grad(bf2f(tz[px * CH + 16 + col]));
            } else if (act) {
                o0 = silu(v0);
                o1 = silu(v1);
            }
            ta[px * CH + col] = f2bf_hw(o0);
            ta[px * CH + 16 + col] = f2bf_hw(o1);
            if (zb) {
                tz[px * CH + col] = f2bf_hw(v0);
                tz[px * CH + 16 + col] = f2bf_hw(v1);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (cin) {
            if (a) *reinterpret_cast<uint4*>(a + crow) = *reinterpret_cast<const uint4*>(ta + cpx * CH + cch);
            if (zb) *reinterpret_cast<uint4*>(zb + crow) = *reinterpret_cast<const uint4*>(tz + cpx * CH + cch);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[u][v][co][ci] = sum over pixels p of gz[p][co] times
// a_in[p + (u - 1, v - 1)][ci], db[co] = sum_p gz[p][co].  Summed over the
// input pixel q = p + (u - 1, v - 1) instead, the input is staged unshifted
// and the gradient row in three horizontally shifted copies, so every MFMA
// fragment is one aligned 16-byte LDS read.  A block owns 64 input columns
// of `rows` consecutive gradient rows; the three input rows a gradient row
// pairs with rotate through a ring in LDS, so each input row is staged
// once.  Staging transposes channels-last data to [channel][pixel] in
// registers (4 pixels x 8 channels per thread).  Wave w accumulates the
// input-channel half 16 (w & 1) and the pixel half 32 (w >> 1) of every
// tap; the two pixel halves are added in LDS at the end in a fixed order
// and the block writes one partial sum, reduced by the two reduce kernels.
// ---------------------------------------------------------------------------
constexpr int WG_LD = 72;          // LDS row stride (u16): 64 pixels + 8, rows 16-byte aligned
constexpr int WG_TARGET = 1024;    // blocks a weight-gradient launch aims for
constexpr int WG_SEG = 64;         // segments of the first reduction stage
constexpr int NWG = 9 * CH * CH;   // weight-gradient entries of one layer

// pixels xs + 4 q .. xs + 4 q + 3 of row y, channels 8 cg .. 8 cg + 7, into
// dst[channel][4 q + i] (zero outside the image), in two halves: the reads
// into registers, then the transposed LDS stores
__device__ inline void load_quad(uint4 (&v)[4], const u16* __restrict__ src, size_t img, int H, int W, int y, int xs,
                                 int q, int cg) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int x = xs + 4 * q + i;
        v[i] = make_uint4(0, 0, 0, 0);
        if (y >= 0 && y < H && x >= 0 && x < W)
            v[i] = *reinterpret_cast<const uint4*>(src + (img + (size_t)y * W + x) * CH + 8 * cg);
    }
}
__device__ inline void store_quad(u16* dst, const uint4 (&v)[4], int q, int cg) {
    unsigned w[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        w[i][0] = v[i].x;
        w[i][1] = v[i].y;
        w[i][2] = v[i].z;
        w[i][3] = v[i].w;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // word k of a pixel holds channels 2k (low half) and 2k + 1 (high half)
        uint2 lo, hi;
        lo.x = (w[0][k] & 0xffffu) | (w[1][k] << 16);
        lo.y = (w[2][k] & 0xffffu) | (w[3][k] << 16);
        hi.x = (w[0][k] >> 16) | (w[1][k] & 0xffff0000u);
        hi.y = (w[2][k] >> 16) | (w[3][k] & 0xffff0000u);
        *reinterpret_cast<uint2*>(dst + (8 * cg + 2 * k) * WG_LD + 4 * q) = lo;
        *reinterpret_cast<uint2*>(dst + (8 * cg + 2 * k + 1) * WG_LD + 4 * q) = hi;
    }
}
__device__ inline void stage_quad(u16* dst, const u16* __restrict__ src, size_t img, int H, int W, int y, int xs,
                                  int q, int cg) {
    uint4 v[4];
    load_quad(v, src, img, H, W, y, xs, q, cg);
    store_quad(dst, v, q, cg);
}

__global__ __launch_bounds__(256) void conv_wgrad_kernel(const u16* __restrict__ gz, const u16* __restrict__ ain,
                                                         float* __restrict__ part_w, float* __restrict__ part_b,
                                                         int H, int W, int rows) {
    // staging: gradient gT[3 shifts][32][72] and input aT[3 ring slots][32][72]
    // (27 KB); at the end the same memory holds the pixel-half exchange (36 KB)
    __shared__ __align__(16) unsigned char smem[2 * 72 * 64 * 4];
    u16* gT = reinterpret_cast<u16*>(smem);
    u16* aT = gT + 3 * CH * WG_LD;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane % 16, kg = lane / 16;
    const int cih = wave & 1, kh = wave >> 1;
    const int n = blockIdx.z, x0 = blockIdx.x * 64;
    const int ya = blockIdx.y * rows, yb = min(ya + rows, H);
    const size_t img = (size_t)n * H * W;
    f32x4 acc[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) acc[i] = (f32x4){0.f, 0.f, 0.f, 0.f};
    float bpart = 0.f;   // channel tid / 8, pixels 8 (tid % 8) ..
    // input rows ya - 1 and ya into their ring slots ((row + 3) mod 3)
    if (tid < 128) {
        const int r = ya - 1 + tid / 64;
        stage_quad(aT + ((r + 3) % 3) * CH * WG_LD, ain, img, H, W, r, x0, (tid / 4) % 16, tid % 4);
    }
    // per row y: gT[v][co][px] = gz[y][x0 + px + 1 - v] (threads < 192) and
    // input row y + 1 into its ring slot (the others); the reads of the next
    // row's share go out before this row's MFMAs
    auto load_share = [&](int y, uint4 (&v)[4]) {
        if (tid < 192) load_quad(v, gz, img, H, W, y, x0 + 1 - tid / 64, (tid / 4) % 16, tid % 4);
        else load_quad(v, ain, img, H, W, y + 1, x0, (tid - 192) / 4, (tid - 192) % 4);
    };
    uint4 share[4];
    load_share(ya, share);
    for (int y = ya; y < yb; ++y) {
        __syncthreads();
        if (tid < 192) store_quad(gT + (tid / 64) * CH * WG_LD, share, (tid / 4) % 16, tid % 4);
        else store_quad(aT + ((y + 1) % 3) * CH * WG_LD, share, (tid - 192) / 4, (tid - 192) % 4);
        __syncthreads();
        if (y + 1 < yb) load_share(y + 1, share);
        {
            const u16* g1 = gT + CH * WG_LD + (tid >> 3) * WG_LD + 8 * (tid & 7);
#pragma unroll
            for (int i = 0; i < 8; ++i) bpart += bf2f(g1[i]);
        }
        const int kc = 32 * kh + 8 * kg;
        bf16x8 Bu[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) Bu[u] = load8(aT + ((y + u + 2) % 3) * CH * WG_LD + (16 * cih + col) * WG_LD + kc);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
#pragma unroll
            for (int coh = 0; coh < 2; ++coh) {
                const bf16x8 A = load8(gT + v * CH * WG_LD + (16 * coh + col) * WG_LD + kc);
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    f32x4& c = acc[(u * 3 + v) * 2 + coh];
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bu[u], c, 0, 0, 0);
                }
            }
        }
    }
    // add the pixel halves: waves 2, 3 hand their sums to waves 0, 1
    __syncthreads();
    float* red = reinterpret_cast<float*>(smem);
    if (kh == 1) {
#pragma unroll
        for (int i = 0; i < 18; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[(cih * 72 + 4 * i + r) * 64 + lane] = acc[i][r];
    }
    __syncthreads();
    const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    if (kh == 0) {
        float* pw = part_w + (size_t)blk * NWG;
#pragma unroll
        for (int i = 0; i < 18; ++i) {
            const int tap = i / 2, coh = i % 2;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = 16 * coh + 4 * kg + r, ci = 16 * cih + col;
                pw[(tap * CH + co) * CH + ci] = acc[i][r] + red[(cih * 72 + 4 * i + r) * 64 + lane];
            }
        }
    }
    bpart += __shfl_xor(bpart, 4);
    bpart += __shfl_xor(bpart, 2);
    bpart += __shfl_xor(bpart, 1);
    if ((tid & 7) == 0) part_b[(size_t)blk * CH + (tid >> 3)] = bpart;
}

// first stage of the deterministic reduction: entry i (weights, then the 32
// bias entries) summed over segment blockIdx.y of the block partials, in
// block order
__global__ void wgrad_reduce1_kernel(const float* part_w, const float* part_b, int nblk, float* part2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NWG + CH) return;
    const int per = (nblk + gridDim.y - 1) / gridDim.y;
    const int b0 = blockIdx.y * per, b1 = min(nblk, b0 + per);
    float s = 0.f;
    if (i < NWG) {
#pragma unroll 8
        for (int b = b0; b < b1; ++b) s += part_w[(size_t)b * NWG + i];
    } else {
#pragma unroll 8
        for (int b = b0; b < b1; ++b) s += part_b[(size_t)b * CH + i - NWG];
    }
    part2[(size_t)blockIdx.y * (NWG + CH) + i] = s;
}

// second stage: the segments in order
__global__ void wgrad_reduce2_kernel(const float* part2, int nseg, float* gw, float* gb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NWG + CH) return;
    float s = 0.f;
#pragma unroll 8
    for (int k = 0; k < nseg; ++k) s += part2[(size_t)k * (NWG + CH) + i];
    if (i < NWG)
        gw[i] = s;
    else
        gb[i - NWG] = s;
}

// gz = g * silu'(z) (hidden layers) or g (last layer), as bf16
__global__ void act_bwd_kernel(const float* g, const float* z, u16* gz, size_t n, int act) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = act ? g[i] * silu_grad(z[i]) : g[i];
    gz[i] = f2bf(v);
}

// x = (m, B / 50 mT, 0...) bf16 channels-last; m is [n][3][H][W] float
__global__ void make_input_kernel(const float* m, const float* B, u16* x, int N, int H, int W) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t npx = (size_t)N * H * W;
    if (i >= npx) return;
    const int n = (int)(i / ((size_t)H * W));
    const size_t p = i - (size_t)n * H * W;
    // m as a BF16 pair: hi = bf16(m), lo = bf16(256 (m - hi)) (m - hi is
    // exact in FP32), so the first layer sees m to about 16 bits
    uint32_t ch[9];
    for (int c = 0; c < 3; ++c) {
        const float v = m[((size_t)n * 3 + c) * H * W + p];
        const u16 hi = f2bf(v);
        ch[c] = hi;
        ch[3 + c] = f2bf((v - bf2f(hi)) * LO_SCALE);
    }
    for (int c = 0; c < 3; ++c) ch[6 + c] = f2bf(B[n * 3 + c] / B_SCALE);
    // the pixel's 32 channels as four 16-byte stores (channels 9.. zero)
    uint4* xo = reinterpret_cast<uint4*>(x + i * CH);
    xo[0] = make_uint4(ch[0] | ch[1] << 16, ch[2] | ch[3] << 16, ch[4] | ch[5] << 16, ch[6] | ch[7] << 16);
    xo[1] = make_uint4(ch[8], 0u, 0u, 0u);
    xo[2] = make_uint4(0u, 0u, 0u, 0u);
    xo[3] = make_uint4(0u, 0u, 0u, 0u);
}

// loss gradient (bf16: the gradient at the last layer's pre-activation) of
// the mean squared error of the network output against
// (m_target - base) / scale, and per-block loss partials
__global__ void loss_kernel(const float* zout, const float* base, const float* mt, u16* gz, float* part, int N,
                            int H, int W, float inv_scale) {
    __shared__ float red[256];
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t npx = (size_t)N * H * W;
    const float inv = 1.0f / (3.0f * (float)npx);
    float l = 0.f;
    if (i < npx) {
        const int n = (int)(i / ((size_t)H * W));
        const size_t p = i - (size_t)n * H * W;
        uint32_t gb[3];
        for (int c = 0; c < 3; ++c) {
            const size_t q = ((size_t)n * 3 + c) * H * W + p;
            const float d = zout[i * KC + c] - (mt[q] - base[q]) * inv_scale;
            l += d * d;
            gb[c] = f2bf(2.0f * d * inv);
        }
        // the pixel's 32 gradient channels (3.. zero) as four 16-byte stores
        uint4* go = reinterpret_cast<uint4*>(gz + i * CH);
        go[0] = make_uint4(gb[0] | gb[1] << 16, gb[2], 0u, 0u);
        go[1] = make_uint4(0u, 0u, 0u, 0u);
        go[2] = make_uint4(0u, 0u, 0u, 0u);
        go[3] = make_uint4(0u, 0u, 0u, 0u);
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] * inv;
}

// one block of 256 threads: strided partial sums, then a fixed tree
__global__ void sum_kernel(const float* part, int n, float* out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// proposals m' = normalize(base + scale * out)
__global__ void propose_kernel(const float* base, const float* zout, float* mo, int N, int H, int W, float scale) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t npx = (size_t)N * H * W;
    if (i >= npx) return;
    const int n = (int)(i / ((size_t)H * W));
    const size_t p = i - (size_t)n * H * W;
    float v[3];
    for (int c = 0; c < 3; ++c) v[c] = base[((size_t)n * 3 + c) * H * W + p] + scale * zout[i * KC + c];
    const float inv = rsqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int c = 0; c < 3; ++c) mo[((size_t)n * 3 + c) * H * W + p] = v[c] * inv;
}

// FP32 master weights of one layer [cout][cin][3][3] + bias -> bf16 forward
// [tap][co][ci] and data-gradient [tap'][ci][co] (tap' = 8 - tap) layouts
__global__ void pack_kernel(const float* w, int cin, int cout, u16* wf, u16* wtr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9 * CH * CH) return;
    const int tap = i / (CH * CH), co = (i / CH) % CH, ci = i % CH;
    float v = 0.f;
    if (co < cout && ci < cin) v = w[((co * cin + ci) * 3 + tap / 3) * 3 + tap % 3];
    wf[i] = f2bf(v);
    wtr[((8 - tap) * CH + ci) * CH + co] = f2bf(v);
}

// the [tap][co][ci] weight gradient back to the [cout][cin][3][3] layout
__global__ void unpack_grad_kernel(const float* gwp, int cin, int cout, float* gw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cout * cin * 9) return;
    const int tap = i % 9, ci = (i / 9) % cin, co = i / (9 * cin);
    gw[i] = gwp[(tap * CH + co) * CH + ci];
}

__global__ void adam_kernel(float* p, const float* g, float* m1, float* m2, int n, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    m1[i] = 0.9f * m1[i] + 0.1f * gi;
    m2[i] = 0.999f * m2[i] + 0.001f * gi * gi;
    p[i] -= lr * (m1[i] / c1) / (sqrtf(m2[i] / c2) + 1e-8f);
}

// x (float, channels-last) -> bf16
__global__ void to_bf16_kernel(const float* x, u16* y, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// out[j] = max over cells of |a_j - b_j| (Euclidean norm per cell), as the
// bits of a non-negative float (ordered like unsigned integers)
__global__ void maxdiff_kernel(const float* a, const float* b, int ncells, unsigned* out) {
    __shared__ float red[256];
    float m = 0.f;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncells; i += gridDim.x * blockDim.x) {
        const float dx = a[i] - b[i];
        const float dy = a[ncells + i] - b[ncells + i];
        const float dz = a[2 * ncells + i] - b[2 * ncells + i];
        float d = sqrtf(dx * dx + dy * dy + dz * dz);
        if (!(d <= 3.0e38f)) d = INFINITY;   // NaN or Inf: infinitely far
        m = fmaxf(m, d);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

// ============================================================================
// host side
// ============================================================================
struct llg_sur {
    int device = 0;
    hipStream_t stream = nullptr;
    int H = 0, W = 0, maxb = 0;
    std::string err;
    long long nparam = 0;
    std::vector<long long> woff, boff;        // offsets of each layer's weights / bias in params
    float* params = nullptr;                   // FP32 master, oracle layout
    float* grads = nullptr;
    float* mom1 = nullptr;
    float* mom2 = nullptr;
    u16* wf[NL] = {};                          // bf16 forward weights
    u16* wtr[NL] = {};                         // bf16 transposed/flipped weights
    u16* act[NL] = {};                         // layer inputs (bf16, 32 ch)
    float* z[NL] = {};                         // pre-activations: bf16 32 ch kept for the backward pass
                                               // (hidden layers), float 4 ch (network output) or float
                                               // 32 ch (parity checks)
    float* g = nullptr;                        // gradient w.r.t. a layer's output (float, 32 ch)
    u16* gz = nullptr;                         // gradient w.r.t. pre-activation (bf16)
    u16* gz2 = nullptr;                        // the same for the layer below (ping-pong)
    float* gwp = nullptr;                      // reduced [tap][co][ci] weight gradient
    float* part_w = nullptr;
    float* part_b = nullptr;
    float* part2 = nullptr;                    // first-stage sums of the weight-gradient reduction
    float* part_l = nullptr;
    float* dloss = nullptr;
    float* dm_in = nullptr;                    // staging for host inputs
    float* dm_t = nullptr;
    float* dB = nullptr;
    float* dm_out = nullptr;
    long long adam_t = 0;
    bool packed = false;
    float out_scale = 1.f;                     // dm = out_scale * network output
    // speculative verification
    std::vector<llg_batch*> vb;                // the plain segments of a round, in parts of kVerifyPart
    llg_batch* eb = nullptr;                   // one film: the coarse step of the proposals' base
    llg_film_desc vdesc = {};                  // the film the batch was built for
    int vwin = 0;
    float* props = nullptr;                    // proposals: window + 1 states
    unsigned* dmax = nullptr;                  // per-proposal max-cell distance (float bits)
};

namespace {

llg_status sfail(llg_sur* s, llg_status c, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    return c;
}

#define SCHK(s, x)                                                                                \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess)                                                                     \
            return sfail(s, e_ == hipErrorOutOfMemory ? LLG_E_NOMEM : LLG_E_DEVICE, "%s: %s (%s:%d)", #x, \
                         hipGetErrorString(e_), __FILE__, __LINE__);                              \
    } while (0)

// gradient rows per weight-gradient block: about WG_TARGET blocks, at
// least 4 rows each
int wg_rows(const llg_sur* s, int N) {
    const long long rb = (long long)((s->W + 63) / 64) * s->H * N;
    return (int)std::min<long long>(s->H, std::max<long long>(4, (rb + WG_TARGET - 1) / WG_TARGET));
}
dim3 wg_grid(const llg_sur* s, int N) {
    const int r = wg_rows(s, N);
    return dim3((s->W + 63) / 64, (s->H + r - 1) / r, N);
}
int wg_blocks(const llg_sur* s, int N) {
    const dim3 g = wg_grid(s, N);
    return (int)(g.x * g.y * g.z);
}

// convolution rows per forward block: blocks of 64 pixels by `rows` rows,
// about 2048 of them, at most 16 rows
void launch_conv(llg_sur* s, const u16* in, const u16* wt, const float* bias, float* z, float* zc, u16* zb, u16* a,
                 const u16* zg, int N, int act) {
    const long long rb = (long long)((s->W + 63) / 64) * s->H * N;
    const int rows = (int)std::min<long long>(16, std::max<long long>(1, rb / 2048));
    hipLaunchKernelGGL(conv_fwd_kernel, dim3((s->W + 63) / 64, (s->H + rows - 1) / rows, N), dim3(256), 0,
                       s->stream, in, wt, bias, z, zc, zb, a, zg, s->H, s->W, act, rows);
}

// weight and bias gradient of one layer from the pre-activation gradient
// gz and the layer input ain: per-block partials, then two fixed-order
// reduction stages into gwp ([tap][co][ci]) and gb (32 entries)
void launch_wgrad(llg_sur* s, const u16* gz, const u16* ain, int N, float* gb) {
    const dim3 grid = wg_grid(s, N);
    const int nblk = (int)(grid.x * grid.y * grid.z);
    hipLaunchKernelGGL(conv_wgrad_kernel, grid, dim3(256), 0, s->stream, gz, ain, s->part_w, s->part_b, s->H, s->W,
                       wg_rows(s, N));
    const int nseg = std::min(WG_SEG, nblk);
    hipLaunchKernelGGL(wgrad_reduce1_kernel, dim3((NWG + CH + 255) / 256, nseg), dim3(256), 0, s->stream, s->part_w,
                       s->part_b, nblk, s->part2);
    hipLaunchKernelGGL(wgrad_reduce2_kernel, dim3((NWG + CH + 255) / 256), dim3(256), 0, s->stream, s->part2, nseg,
                       s->gwp, gb);
}

llg_status pack(llg_sur* s) {
    for (int l = 0; l < NL; ++l) {
        hipLaunchKernelGGL(pack_kernel, dim3((9 * CH * CH + 255) / 256), dim3(256), 0, s->stream,
                           s->params + s->woff[l], CIN[l], COUT[l], s->wf[l], s->wtr[l]);
        SCHK(s, hipGetLastError());
    }
    s->packed = true;
    return LLG_OK;
}

// keep_z: keep every hidden layer's pre-activation as bf16 for the backward
// pass (in the first half of its float buffer).  The last layer's (the
// network output) is written compact, four float channels per pixel, unless
// f32_layer asks for it; layer f32_layer's is written as float, 32 channels
llg_status forward(llg_sur* s, const float* m, const float* B, int N, bool keep_z, int f32_layer = -1) {
    const size_t npx = (size_t)N * s->H * s->W;
    hipLaunchKernelGGL(make_input_kernel, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, s->stream, m, B,
                       s->act[0], N, s->H, s->W);
    SCHK(s, hipGetLastError());
    for (int l = 0; l < NL; ++l) {
        // the bias of a layer with fewer than 32 outputs is read through a
        // zero-padded 32-entry copy kept in the gradient buffer's tail
        const bool f32 = l == f32_layer, out = l == NL - 1 && !f32;
        launch_conv(s, s->act[l], s->wf[l], s->params + s->boff[l], f32 ? s->z[l] : nullptr, out ? s->z[l] : nullptr,
                    keep_z && l < NL - 1 && !f32 ? reinterpret_cast<u16*>(s->z[l]) : nullptr,
                    l < NL - 1 ? s->act[l + 1] : nullptr, nullptr, N, l < NL - 1 ? 1 : 0);
        SCHK(s, hipGetLastError());
    }
    return LLG_OK;
}

}  // namespace

extern "C" {

llg_status llg_mfma_selftest(int device, const float* A, const float* B, float* C) {
    if (!A || !B || !C) return LLG_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return LLG_E_DEVICE;
    std::vector<u16> ha(16 * 32), hb(32 * 16);
    for (int i = 0; i < 16 * 32; ++i) ha[i] = f2bf(A[i]);
    for (int i = 0; i < 32 * 16; ++i) hb[i] = f2bf(B[i]);
    u16 *da = nullptr, *db = nullptr;
    float* dc = nullptr;
    if (hipMalloc(&da, 1024) != hipSuccess || hipMalloc(&db, 1024) != hipSuccess ||
        hipMalloc(&dc, 16 * 16 * 4) != hipSuccess)
        return LLG_E_DEVICE;
    (void)hipMemcpy(da, ha.data(), 1024, hipMemcpyHostToDevice);
    (void)hipMemcpy(db, hb.data(), 1024, hipMemcpyHostToDevice);
    hipLaunchKernelGGL(mfma_selftest_kernel, dim3(1), dim3(64), 0, 0, da, db, dc);
    hipError_t e = hipMemcpy(C, dc, 16 * 16 * 4, hipMemcpyDeviceToHost);
    (void)hipFree(da);
    (void)hipFree(db);
    (void)hipFree(dc);
    return e == hipSuccess ? LLG_OK : LLG_E_DEVICE;
}

llg_status llg_sur_create(int device, int H, int W, int max_batch, llg_sur** out) {
    if (!out || H < 1 || W < 1 || max_batch < 1) return LLG_E_ARG;
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return LLG_E_DEVICE;
    llg_sur* s = new llg_sur();
    *out = s;
    s->device = device;
    s->H = H;
    s->W = W;
    s->maxb = max_batch;
    SCHK(s, hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    long long off = 0;
    for (int l = 0; l < NL; ++l) {
        s->woff.push_back(off);
        off += (long long)COUT[l] * CIN[l] * 9;
        s->boff.push_back(off);
        off += COUT[l];
    }
    s->nparam = off;
    // bias reads cover 32 entries: pad the parameter arrays at the end
    const size_t pbytes = sizeof(float) * (size_t)(off + CH);
    SCHK(s, hipMalloc(&s->params, pbytes));
    SCHK(s, hipMalloc(&s->grads, pbytes));
    SCHK(s, hipMalloc(&s->mom1, pbytes));
    SCHK(s, hipMalloc(&s->mom2, pbytes));
    SCHK(s, hipMemset(s->params, 0, pbytes));
    SCHK(s, hipMemset(s->grads, 0, pbytes));
    SCHK(s, hipMemset(s->mom1, 0, pbytes));
    SCHK(s, hipMemset(s->mom2, 0, pbytes));
    const size_t npx = (size_t)max_batch * H * W;
    for (int l = 0; l < NL; ++l) {
        SCHK(s, hipMalloc(&s->wf[l], 9 * CH * CH * 2));
        SCHK(s, hipMalloc(&s->wtr[l], 9 * CH * CH * 2));
        SCHK(s, hipMalloc(&s->z[l], npx * CH * 4));
    }
    for (int l = 0; l < NL; ++l) SCHK(s, hipMalloc(&s->act[l], npx * CH * 2));
    SCHK(s, hipMalloc(&s->g, npx * CH * 4));
    SCHK(s, hipMalloc(&s->gz, npx * CH * 2));
    SCHK(s, hipMalloc(&s->gz2, npx * CH * 2));
    SCHK(s, hipMalloc(&s->gwp, 9 * CH * CH * 4));
    int maxblk = 0;
    for (int n = 1; n <= max_batch; ++n) maxblk = std::max(maxblk, wg_blocks(s, n));
    SCHK(s, hipMalloc(&s->part_w, (size_t)maxblk * NWG * 4));
    SCHK(s, hipMalloc(&s->part_b, (size_t)maxblk * CH * 4));
    SCHK(s, hipMalloc(&s->part2, (size_t)WG_SEG * (NWG + CH) * 4));
    SCHK(s, hipMalloc(&s->part_l, ((npx + 255) / 256) * 4));
    SCHK(s, hipMalloc(&s->dloss, 4));
    SCHK(s, hipMalloc(&s->dm_in, npx * 3 * 4));
    SCHK(s, hipMalloc(&s->dm_t, npx * 3 * 4));
    SCHK(s, hipMalloc(&s->dm_out, npx * 3 * 4));
    SCHK(s, hipMalloc(&s->dB, (size_t)max_batch * 3 * 4));
    return LLG_OK;
}

void llg_sur_destroy(llg_sur* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    void* ptrs[] = {s->params, s->grads, s->mom1, s->mom2, s->g, s->gz, s->gz2, s->gwp, s->part_w, s->part_b,
                    s->part2, s->part_l, s->dloss, s->dm_in, s->dm_t, s->dm_out, s->dB};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (int l = 0; l < NL; ++l) {
        if (s->wf[l]) (void)hipFree(s->wf[l]);
        if (s->wtr[l]) (void)hipFree(s->wtr[l]);
        if (s->z[l]) (void)hipFree(s->z[l]);
    }
    for (int l = 0; l < NL; ++l)
        if (s->act[l]) (void)hipFree(s->act[l]);
    if (s->props) (void)hipFree(s->props);
    if (s->dmax) (void)hipFree(s->dmax);
    for (llg_batch* v : s->vb)
        if (v) llg_batch_destroy(v);
    s->vb.clear();
    if (s->eb) llg_batch_destroy(s->eb);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

const char* llg_sur_last_error(const llg_sur* s) { return s ? s->err.c_str() : "null surrogate"; }

int64_t llg_sur_num_params(void) {
    long long n = 0;
    for (int l = 0; l < NL; ++l) n += (long long)COUT[l] * CIN[l] * 9 + COUT[l];
    return n;
}

llg_status llg_sur_set_params(llg_sur* s, const float* params, int64_t n) {
    if (!s || !params) return LLG_E_ARG;
    if (n != s->nparam) return sfail(s, LLG_E_ARG, "expected %lld parameters", s->nparam);
    SCHK(s, hipSetDevice(s->device));
    SCHK(s, hipMemcpyAsync(s->params, params, sizeof(float) * n, hipMemcpyHostToDevice, s->stream));
    SCHK(s, hipMemsetAsync(s->mom1, 0, sizeof(float) * (n + CH), s->stream));
    SCHK(s, hipMemsetAsync(s->mom2, 0, sizeof(float) * (n + CH), s->stream));
    s->adam_t = 0;
    llg_status rc = pack(s);
    if (rc != LLG_OK) return rc;
    SCHK(s, hipStreamSynchronize(s->stream));
    return LLG_OK;
}

llg_status llg_sur_set_output_scale(llg_sur* s, double scale) {
    if (!s || !(scale > 0) || !isfinite(scale) || scale > 1e30) return LLG_E_ARG;
    s->out_scale = (float)scale;
    return LLG_OK;
}

llg_status llg_sur_get_params(llg_sur* s, float* params, int64_t n) {
    if (!s || !params) return LLG_E_ARG;
    if (n != s->nparam) return sfail(s, LLG_E_ARG, "expected %lld parameters", s->nparam);
    SCHK(s, hipSetDevice(s->device));
    SCHK(s, hipMemcpyAsync(params, s->params, sizeof(float) * n, hipMemcpyDeviceToHost, s->stream));
    SCHK(s, hipStreamSynchronize(s->stream));
    return LLG_OK;
}

llg_status llg_sur_get_grads(llg_sur* s, float* grads, int64_t n) {
    if (!s || !grads) return LLG_E_ARG;
    if (n != s->nparam) return sfail(s, LLG_E_ARG, "expected %lld parameters", s->nparam);
    SCHK(s, hipSetDevice(s->device));
    SCHK(s, hipMemcpyAsync(grads, s->grads, sizeof(float) * n, hipMemcpyDeviceToHost, s->stream));
    SCHK(s, hipStreamSynchronize(s->stream));
    return LLG_OK;
}

// gradient of the loss (and optionally one Adam step) for a batch
llg_status llg_sur_train_step(llg_sur* s, const float* m_in, const float* m_target, const float* m_base,
                              const float* B, int batch, llg_mem where, float lr, float* loss) {
    llg::host::TraceRange trace_("llg_sur_train_step");
    if (!s || !m_in || !m_target || !B || batch < 1 || batch > s->maxb) return LLG_E_ARG;
    SCHK(s, hipSetDevice(s->device));
    if (!s->packed) return sfail(s, LLG_E_STATE, "parameters not set");
    const size_t npx = (size_t)batch * s->H * s->W;
    const float* mi = m_in;
    const float* mt = m_target;
    const float* mb = m_base;
    if (where != LLG_DEVICE) {
        SCHK(s, hipMemcpyAsync(s->dm_in, m_in, npx * 3 * 4, hipMemcpyHostToDevice, s->stream));
        SCHK(s, hipMemcpyAsync(s->dm_t, m_target, npx * 3 * 4, hipMemcpyHostToDevice, s->stream));
        mi = s->dm_in;
        mt = s->dm_t;
        if (m_base) {
            SCHK(s, hipMemcpyAsync(s->dm_out, m_base, npx * 3 * 4, hipMemcpyHostToDevice, s->stream));
            mb = s->dm_out;
        }
    }
    if (!mb) mb = mi;
    SCHK(s, hipMemcpyAsync(s->dB, B, (size_t)batch * 3 * 4, hipMemcpyHostToDevice, s->stream));
    llg_status rc = forward(s, mi, s->dB, batch, true);
    if (rc != LLG_OK) return rc;
    const int lb = (int)((npx + 255) / 256);
    hipLaunchKernelGGL(loss_kernel, dim3(lb), dim3(256), 0, s->stream, s->z[NL - 1], mb, mt, s->gz, s->part_l, batch,
                       s->H, s->W, 1.0f / s->out_scale);
    SCHK(s, hipGetLastError());
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s->stream, s->part_l, lb, s->dloss);
    SCHK(s, hipGetLastError());
    u16* gcur = s->gz;    // gradient at layer l's pre-activation
    u16* gnext = s->gz2;
    for (int l = NL - 1; l >= 0; --l) {
        launch_wgrad(s, gcur, s->act[l], batch, s->grads + s->boff[l]);
        SCHK(s, hipGetLastError());
        hipLaunchKernelGGL(unpack_grad_kernel, dim3((COUT[l] * CIN[l] * 9 + 255) / 256), dim3(256), 0, s->stream,
                           s->gwp, CIN[l], COUT[l], s->grads + s->woff[l]);
        SCHK(s, hipGetLastError());
        if (l > 0) {
            // data gradient: the same convolution with flipped, transposed
            // weights, times SiLU'(z) of layer l - 1 (every hidden layer has
            // the activation)
            launch_conv(s, gcur, s->wtr[l], nullptr, nullptr, nullptr, nullptr, gnext,
                        reinterpret_cast<const u16*>(s->z[l - 1]), batch, 0);
            SCHK(s, hipGetLastError());
            std::swap(gcur, gnext);
        }
    }
    // note: the reduce kernel wrote 32 bias entries; the parameter arrays
    // carry 32 floats of padding so this never runs past the end
    if (lr > 0.f) {
        s->adam_t += 1;
        const float c1 = 1.0f - powf(0.9f, (float)s->adam_t), c2 = 1.0f - powf(0.999f, (float)s->adam_t);
        const int n = (int)s->nparam;
        hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s->stream, s->params, s->grads, s->mom1,
                           s->mom2, n, lr, c1, c2);
        SCHK(s, hipGetLastError());
        rc = pack(s);
        if (rc != LLG_OK) return rc;
    }
    if (loss) {
        SCHK(s, hipMemcpyAsync(loss, s->dloss, 4, hipMemcpyDeviceToHost, s->stream));
    }
    SCHK(s, hipStreamSynchronize(s->stream));
    return LLG_OK;
}

llg_status llg_sur_predict(llg_sur* s, const float* m_in, const float* m_base, const float* B, int batch,
                           llg_mem where, float* m_out) {
    if (!s || !m_in || !B || !m_out || batch < 1 || batch > s->maxb) return LLG_E_ARG;
    SCHK(s, hipSetDevice(s->device));
    if (!s->packed) return sfail(s, LLG_E_STATE, "parameters not set");
    const size_t npx = (size_t)batch * s->H * s->W;
    const float* mi = m_in;
    const float* mb = m_base;
    float* mo = m_out;
    if (where != LLG_DEVICE) {
        SCHK(s, hipMemcpyAsync(s->dm_in, m_in, npx * 3 * 4, hipMemcpyHostToDevice, s->stream));
        mi = s->dm_in;
        mo = s->dm_out;
        if (m_base) {
            SCHK(s, hipMemcpyAsync(s->dm_t, m_base, npx * 3 * 4, hipMemcpyHostToDevice, s->stream));
            mb = s->dm_t;
        }
    }
    if (!mb) mb = mi;
    SCHK(s, hipMemcpyAsync(s->dB, B, (size_t)batch * 3 * 4, hipMemcpyHostToDevice, s->stream));
    llg_status rc = forward(s, mi, s->dB, batch, false);
    if (rc != LLG_OK) return rc;
    hipLaunchKernelGGL(propose_kernel, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, s->stream, mb,
                       s->z[NL - 1], mo, batch, s->H, s->W, s->out_scale);
    SCHK(s, hipGetLastError());
    if (where != LLG_DEVICE) SCHK(s, hipMemcpyAsync(m_out, s->dm_out, npx * 3 * 4, hipMemcpyDeviceToHost, s->stream));
    SCHK(s, hipStreamSynchronize(s->stream));
    return LLG_OK;
}

// the pre-activation of layer `layer` (the last one: the net's dm before
// padding) for a batch, [batch][H][W][32] float into host memory; for parity
// checks
llg_status llg_sur_forward_raw(llg_sur* s, const float* m_in, const float* B, int batch, int layer, float* z_out) {
    if (!s || !m_in || !B || !z_out || batch < 1 || batch > s->maxb || layer < 0 || layer >= NL) return LLG_E_ARG;
    SCHK(s, hipSetDevice(s->device));
    if (!s->packed) return sfail(s, LLG_E_STATE, "parameters not set");
    const size_t npx = (size_t)batch * s->H * s->W;
    SCHK(s, hipMemcpyAsync(s->dm_in, m_in, npx * 3 * 4, hipMemcpyHostToDevice, s->stream));
    SCHK(s, hipMemcpyAsync(s->dB, B, (size_t)batch * 3 * 4, hipMemcpyHostToDevice, s->stream));
    llg_status rc = forward(s, s->dm_in, s->dB, batch, false, layer);
    if (rc != LLG_OK) return rc;
    SCHK(s, hipMemcpyAsync(z_out, s->z[layer], npx * CH * 4, hipMemcpyDeviceToHost, s->stream));
    SCHK(s, hipStreamSynchronize(s->stream));
    return LLG_OK;
}

// one convolution layer through the training kernels, for parity checks:
// x and gy are [batch][H][W][32] float (host) and are rounded to bf16 as the
// training path rounds activations and gradients; y = conv(x) + bias, and if
// gy is given gw [cout][cin][3][3], gb [cout] and gx [batch][H][W][32]
llg_status llg_sur_conv_check(llg_sur* s, int layer, const float* x, const float* gy, int batch, float* y,
                              float* gx, float* gw, float* gb) {
    if (!s || !x || !y || batch < 1 || batch > s->maxb || layer < 0 || layer >= NL) return LLG_E_ARG;
    if (gy && (!gx || !gw || !gb)) return LLG_E_ARG;
    SCHK(s, hipSetDevice(s->device));
    if (!s->packed) return sfail(s, LLG_E_STATE, "parameters not set");
    const size_t n = (size_t)batch * s->H * s->W * CH;
    const unsigned nb = (unsigned)((n + 255) / 256);
    SCHK(s, hipMemcpyAsync(s->g, x, n * 4, hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL(to_bf16_kernel, dim3(nb), dim3(256), 0, s->stream, s->g, s->act[0], n);
    SCHK(s, hipGetLastError());
    launch_conv(s, s->act[0], s->wf[layer], s->params + s->boff[layer], s->z[0], nullptr, nullptr, nullptr, nullptr,
                batch, 0);
    SCHK(s, hipGetLastError());
    SCHK(s, hipMemcpyAsync(y, s->z[0], n * 4, hipMemcpyDeviceToHost, s->stream));
    if (gy) {
        float *dgw = nullptr, *dgb = nullptr;
        SCHK(s, hipMalloc(&dgw, sizeof(float) * COUT[layer] * CIN[layer] * 9));
        SCHK(s, hipMalloc(&dgb, sizeof(float) * CH));
        SCHK(s, hipMemcpyAsync(s->g, gy, n * 4, hipMemcpyHostToDevice, s->stream));
        hipLaunchKernelGGL(act_bwd_kernel, dim3(nb), dim3(256), 0, s->stream, s->g, (const float*)nullptr, s->gz, n, 0);
        SCHK(s, hipGetLastError());
        launch_wgrad(s, s->gz, s->act[0], batch, dgb);
        SCHK(s, hipGetLastError());
        hipLaunchKernelGGL(unpack_grad_kernel, dim3((COUT[layer] * CIN[layer] * 9 + 255) / 256), dim3(256), 0,
                           s->stream, s->gwp, CIN[layer], COUT[layer], dgw);
        SCHK(s, hipGetLastError());
        launch_conv(s, s->gz, s->wtr[layer], nullptr, s->z[1], nullptr, nullptr, nullptr, nullptr, batch, 0);
        SCHK(s, hipGetLastError());
        SCHK(s, hipMemcpyAsync(gx, s->z[1], n * 4, hipMemcpyDeviceToHost, s->stream));
        SCHK(s, hipMemcpyAsync(gw, dgw, sizeof(float) * COUT[layer] * CIN[layer] * 9, hipMemcpyDeviceToHost,
                               s->stream));
        SCHK(s, hipMemcpyAsync(gb, dgb, sizeof(float) * COUT[layer], hipMemcpyDeviceToHost, s->stream));
        SCHK(s, hipStreamSynchronize(s->stream));
        (void)hipFree(dgw);
        (void)hipFree(dgb);
    }
    SCHK(s, hipStreamSynchronize(s->stream));
    return LLG_OK;
}

// ---------------------------------------------------------------------------
// speculative verification: the surrogate chains up to `window` proposals,
// one plain batched launch advances every start state by seg_steps RK4
// steps, the prefix of proposals within max_dm of their plain counterparts
// is accepted and the plain state at the end of the accepted prefix (or at
// the first rejected proposal) is committed
// ---------------------------------------------------------------------------
namespace {

bool same_film(const llg_film_desc& a, const llg_film_desc& b) {
    if (a.nx != b.nx || a.ny != b.ny || a.dx != b.dx || a.dy != b.dy || a.dz != b.dz || a.Ms != b.Ms ||
        a.Aex != b.Aex || a.alpha != b.alpha || a.Ku != b.Ku)
        return false;
    for (int i = 0; i < 3; ++i)
        if (a.u[i] != b.u[i] || a.B[i] != b.B[i]) return false;
    return true;
}

llg_status max_distance(llg_sur* s, const float* a, const float* b, int ncells, unsigned* out) {
    const int blocks = std::min(1024, (ncells + 255) / 256);
    hipLaunchKernelGGL(maxdiff_kernel, dim3(blocks), dim3(256), 0, s->stream, a, b, ncells, out);
    SCHK(s, hipGetLastError());
    return LLG_OK;
}

float bits_to_float(unsigned u) {
    float f;
    memcpy(&f, &u, 4);
    return f;
}

}  // namespace

llg_status llg_sur_advance(llg_sur* s, const llg_film_desc* film, int window, int64_t n_segments, int seg_steps,
                           double dt, int predictor, double max_dm, float* m, llg_mem where, llg_sur_stats* out) {
    llg::host::TraceRange trace_("llg_sur_advance");
    if (!s || !film || !m || window < 1 || window > 256 || n_segments < 0 || seg_steps < 1 || !(dt > 0) ||
        !(max_dm >= 0) ||
        (predictor != LLG_SUR_BASE_STATE && predictor != LLG_SUR_BASE_EULER && predictor != LLG_SUR_BASE_RK4))
        return LLG_E_ARG;
    s->err.clear();
    SCHK(s, hipSetDevice(s->device));
    if (!s->packed) return sfail(s, LLG_E_STATE, "parameters not set");
    if (film->nx != s->W || film->ny != s->H)
        return sfail(s, LLG_E_ARG, "film %d x %d does not match the surrogate's %d x %d", film->nx, film->ny, s->W,
                     s->H);
    const int ncells = s->H * s->W;
    const size_t vec = sizeof(float) * 3 * (size_t)ncells;
    llg_sur_stats st = {};
    // the verification batches (start states kVerifyPart p ... of a round)
    // and the coarse-step batch: copies of the film
    const int nparts = (window + kVerifyPart - 1) / kVerifyPart;
    if (s->vb.empty() || s->vwin != window || !same_film(s->vdesc, *film)) {
        for (llg_batch* v : s->vb)
            if (v) llg_batch_destroy(v);
        s->vb.assign(nparts, nullptr);
        if (s->eb) llg_batch_destroy(s->eb);
        s->eb = nullptr;
        if (s->props) (void)hipFree(s->props);
        if (s->dmax) (void)hipFree(s->dmax);
        s->props = nullptr;
        s->dmax = nullptr;
        std::vector<float> h0(3 * (size_t)ncells);
        SCHK(s, hipMemcpy(h0.data(), m, vec, where == LLG_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
        std::vector<llg_film_desc> fd(window, *film);
        for (auto& f : fd) f.m0 = h0.data();
        for (int i = 0; i <= nparts; ++i) {
            const int count = i < nparts ? std::min(kVerifyPart, window - i * kVerifyPart) : 1;
            llg_batch** dst = i < nparts ? &s->vb[i] : &s->eb;
            const llg_status rc = llg_batch_create(s->device, fd.data(), count, dst);
            if (rc != LLG_OK) {
                const std::string why = *dst ? llg_batch_last_error(*dst) : "batch creation failed";
                if (*dst) llg_batch_destroy(*dst);
                *dst = nullptr;
                for (llg_batch* v : s->vb)   // the others are rebuilt by the next call
                    if (v) llg_batch_destroy(v);
                s->vb.clear();
                return sfail(s, rc, "%s batch: %s", i < nparts ? "verification" : "predictor", why.c_str());
            }
        }
        s->vdesc = *film;
        s->vdesc.m0 = nullptr;
        s->vwin = window;
        SCHK(s, hipMalloc(&s->props, vec * (window + 1)));
        SCHK(s, hipMalloc(&s->dmax, sizeof(unsigned) * 2 * window));
    }
    const float Bf[3] = {(float)film->B[0], (float)film->B[1], (float)film->B[2]};
    SCHK(s, hipMemcpyAsync(s->dB, Bf, sizeof Bf, hipMemcpyHostToDevice, s->stream));
    SCHK(s, hipMemcpyAsync(s->props, m, vec, where == LLG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           s->stream));
    // the start state is checked and renormalised as llg_set_m does
    {
        hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s->stream, s->dmax, 1);
        SCHK(s, hipGetLastError());
        SCHK(s, llg::launch_normalize_check(s->props, ncells, reinterpret_cast<int*>(s->dmax), s->stream));
        unsigned bad = 0;
        SCHK(s, hipMemcpyAsync(&bad, s->dmax, sizeof bad, hipMemcpyDeviceToHost, s->stream));
        SCHK(s, hipStreamSynchronize(s->stream));
        if (bad) return sfail(s, LLG_E_ARG, "m is not a field of unit vectors");
    }
    std::vector<float*> ptr(window);
    std::vector<unsigned> hd(2 * window);
    const llg_method coarse = predictor == LLG_SUR_BASE_EULER ? LLG_EULER : LLG_RK4;
    int64_t done = 0;
    while (done < n_segments) {
        const int w = (int)std::min<int64_t>(window, n_segments - done);
        const int parts = (w + kVerifyPart - 1) / kVerifyPart;   // parts this round
        float* P = s->props;
        const size_t stride = 3 * (size_t)ncells;
        // plain segments from the start states of part p, on the part's
        // batch stream, overlapping the proposals still to come
        auto verify = [&](int p) -> llg_status {
            const int first = p * kVerifyPart, count = std::min(kVerifyPart, w - first);
            const llg_status rc = llg_batch_fixed_async_(s->vb[p], LLG_RK4, dt, seg_steps, P + first * stride,
                                                         stride, count, s->stream, ptr.data() + first);
            if (rc != LLG_OK) return sfail(s, rc, "verification batch: %s", llg_batch_last_error(s->vb[p]));
            return LLG_OK;
        };
        // proposals 1..w, each from the previous one: normalize(base + dm)
        // with base the previous state or its one coarse step (Euler or
        // RK4) over the whole segment by the plain solver; a part starts as
        // soon as its last start state exists
        int launched = 0;
        for (int j = 1; j <= w; ++j) {
            llg_status rc = LLG_OK;
            while (launched < parts && std::min((launched + 1) * kVerifyPart, w) <= j)
                if ((rc = verify(launched++)) != LLG_OK) return rc;
            const float* prev = P + (size_t)(j - 1) * stride;
            const float* base = prev;
            if (predictor != LLG_SUR_BASE_STATE) {
                float* em = nullptr;
                rc = llg_batch_fixed_async_(s->eb, coarse, dt * seg_steps, 1, prev, 0, 1, s->stream, &em);
                if (rc == LLG_OK) rc = llg_batch_then_(s->eb, s->stream);
                if (rc != LLG_OK) return sfail(s, rc, "predictor batch: %s", llg_batch_last_error(s->eb));
                base = em;
            }
            rc = forward(s, prev, s->dB, 1, false);
            if (rc != LLG_OK) return rc;
            hipLaunchKernelGGL(propose_kernel, dim3((ncells + 255) / 256), dim3(256), 0, s->stream, base,
                               s->z[NL - 1], P + (size_t)j * stride, 1, s->H, s->W, s->out_scale);
            SCHK(s, hipGetLastError());
        }
        for (int p = 0; p < parts; ++p) {
            const llg_status rc = llg_batch_then_(s->vb[p], s->stream);
            if (rc != LLG_OK) return sfail(s, rc, "verification batch: %s", llg_batch_last_error(s->vb[p]));
        }
        // d_j = distance of proposal j to the plain result from its
        // predecessor (non-finite: infinite), and whether each plain result
        // is finite (0) or not
        hipLaunchKernelGGL(zero_u32_kernel, dim3((2 * window + 255) / 256), dim3(256), 0, s->stream, s->dmax,
                           2 * window);
        SCHK(s, hipGetLastError());
        for (int j = 1; j <= w; ++j) {
            llg_status rc = max_distance(s, P + (size_t)j * stride, ptr[j - 1], ncells, s->dmax + j - 1);
            if (rc == LLG_OK) rc = max_distance(s, ptr[j - 1], ptr[j - 1], ncells, s->dmax + window + j - 1);
            if (rc != LLG_OK) return rc;
        }
        SCHK(s, hipMemcpyAsync(hd.data(), s->dmax, sizeof(unsigned) * 2 * window, hipMemcpyDeviceToHost, s->stream));
        SCHK(s, hipStreamSynchronize(s->stream));
        int k = w;       // segments this round commits
        int acc = w;     // proposals accepted
        for (int j = 1; j <= w; ++j) {
            const float d = bits_to_float(hd[j - 1]);
            st.max_dm_seen = std::max(st.max_dm_seen, (double)d);
            if (!((double)d <= max_dm)) { k = j; acc = j - 1; break; }
            st.max_dm_accepted = std::max(st.max_dm_accepted, (double)d);
        }
        if (hd[window + k - 1] != 0u)
            return sfail(s, LLG_E_DIVERGED, "plain segment %lld: non-finite field or torque", (long long)(done + k - 1));
        st.proposals += w;
        st.accepted += acc;
        st.rounds += 1;
        st.segments += k;
        SCHK(s, hipMemcpyAsync(P, ptr[k - 1], vec, hipMemcpyDeviceToDevice, s->stream));
        done += k;
    }
    SCHK(s, hipMemcpyAsync(m, s->props, vec, where == LLG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           s->stream));
    SCHK(s, hipStreamSynchronize(s->stream));
    if (out) *out = st;
    return LLG_OK;
}

}  // extern "C"
