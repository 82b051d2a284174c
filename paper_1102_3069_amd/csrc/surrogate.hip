// Learned surrogate: a six-layer 3x3 convolutional network that proposes
// the magnetisation ten fixed steps ahead, trained and evaluated with BF16
// MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
//   input  x: m (3 channels) and the applied field B / 50 mT (3 channels)
//   net    conv3x3(6->32) SiLU, 4 x [conv3x3(32->32) SiLU], conv3x3(32->3)
//   output dm; proposal m' = normalize(m + dm); loss mean (dm - (m_t - m))^2
//
// Every convolution is an implicit GEMM over (pixels) x (output channels)
// with K = 9 taps x 32 input channels.  Activations are BF16, channels
// last ([n][y][x][32], channel counts padded to 32 with zeros), weights
// BF16 [tap][cout][cin]; the data gradient is the same kernel with the
// weights flipped in space and transposed in channels; the weight gradient
// is an MFMA reduction over pixel chunks into per-block partial sums that a
// second kernel adds in a fixed order (deterministic).  Master weights and
// the Adam moments stay FP32.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int CH = 32;          // padded channel count of every activation
constexpr int NL = 6;           // layers
constexpr int CIN[NL] = {9, 32, 32, 32, 32, 32};
constexpr int COUT[NL] = {32, 32, 32, 32, 32, 3};
constexpr float B_SCALE = 0.05f;
constexpr float LO_SCALE = 256.0f;   // the low part of m is scaled by 2^8 before its own BF16 rounding

// round-to-nearest-even FP32 -> BF16 bits (NaN kept quiet)
__host__ __device__ inline u16 f2bf(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
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

__device__ inline float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float silu_grad(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
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
//   a    [N][H][W][32] bf16 (SiLU(z) if act, else z; may be null)
// block: 4 waves, 64 pixels of one row; a wave: 16 pixels x 32 channels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void conv_fwd_kernel(const u16* __restrict__ in, const u16* __restrict__ wt,
                                                       const float* __restrict__ bias, float* __restrict__ z,
                                                       u16* __restrict__ a, int H, int W, int act) {
    __shared__ u16 ws[9 * CH * CH];
    const int tid = threadIdx.x;
    for (int i = tid; i < 9 * CH * CH / 8; i += 256)
        reinterpret_cast<uint4*>(ws)[i] = reinterpret_cast<const uint4*>(wt)[i];
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int n = blockIdx.z, y = blockIdx.y;
    const int x0 = blockIdx.x * 64 + wave * 16;
    const int col = lane % 16, kg = lane / 16;
    const size_t img = (size_t)n * H * W;
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
    for (int u = 0; u < 3; ++u) {
        const int yy = y + u - 1;
        for (int v = 0; v < 3; ++v) {
            const int xx = x0 + col + v - 1;
            bf16x8 A = zero8();
            if (yy >= 0 && yy < H && xx >= 0 && xx < W) A = load8(in + ((img + (size_t)yy * W + xx) * CH + 8 * kg));
            const u16* wb = ws + (u * 3 + v) * CH * CH;
            const bf16x8 B0 = load8(wb + col * CH + 8 * kg);
            const bf16x8 B1 = load8(wb + (16 + col) * CH + 8 * kg);
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B1, acc1, 0, 0, 0);
        }
    }
    // C layout: lane holds channel (col) of pixels 4 kg + r
    for (int r = 0; r < 4; ++r) {
        const int x = x0 + 4 * kg + r;
        if (x >= W) continue;
        const size_t p = (img + (size_t)y * W + x) * CH;
        float v0 = acc0[r], v1 = acc1[r];
        if (bias) { v0 += bias[col]; v1 += bias[16 + col]; }
        if (z) { z[p + col] = v0; z[p + 16 + col] = v1; }
        if (a) {
            a[p + col] = f2bf(act ? silu(v0) : v0);
            a[p + 16 + col] = f2bf(act ? silu(v1) : v1);
        }
    }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[tap][co][ci] = sum_p gz[p][co] a_in[p + tap][ci],
// db[co] = sum_p gz[p][co], over the pixel chunk of a block (64 pixels of
// ROWS rows); partial sums per block, reduced by wgrad_reduce_kernel.
// LDS holds gz^T [co][64 px] and the three input rows [ci][66 px] of a
// chunk, so the MFMA fragments read contiguous k (pixel) runs.
// ---------------------------------------------------------------------------
constexpr int WG_ROWS = 16;

__global__ __launch_bounds__(256) void conv_wgrad_kernel(const u16* __restrict__ gz, const u16* __restrict__ ain,
                                                         float* __restrict__ part_w, float* __restrict__ part_b,
                                                         int H, int W) {
    __shared__ u16 gT[CH][64];
    __shared__ u16 aT[3][CH][72];
    __shared__ float bsum[4][CH];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int col = lane % 16, kg = lane / 16;
    const int n = blockIdx.z;
    const int x0 = blockIdx.x * 64;
    const int yb = blockIdx.y * WG_ROWS;
    const size_t img = (size_t)n * H * W;
    // a wave owns taps wave, wave+4 (and 8 for wave 0); each tap: 4 tiles
    // (co half, ci half) of 16 x 16
    f32x4 acc[3][4];
    for (int t = 0; t < 3; ++t)
        for (int q = 0; q < 4; ++q) acc[t][q] = (f32x4){0.f, 0.f, 0.f, 0.f};
    float bpart = 0.f;   // lanes 0..31 of wave 0..3 keep a channel's bias sum
    for (int yy = yb; yy < yb + WG_ROWS && yy < H; ++yy) {
        __syncthreads();
        // stage gz^T for pixels x0..x0+63 of row yy
        for (int e = tid; e < 64 * CH; e += 256) {
            const int px = e / CH, c = e % CH;
            const int x = x0 + px;
            gT[c][px] = x < W ? gz[(img + (size_t)yy * W + x) * CH + c] : (u16)0;
        }
        // stage input rows yy-1..yy+1, pixels x0-1..x0+64 (66, padded to 72)
        for (int e = tid; e < 3 * 66 * CH; e += 256) {
            const int r = e / (66 * CH), t = e % (66 * CH);
            const int px = t / CH, c = t % CH;
            const int y = yy + r - 1, x = x0 + px - 1;
            aT[r][c][px] = (y >= 0 && y < H && x >= 0 && x < W) ? ain[(img + (size_t)y * W + x) * CH + c] : (u16)0;
        }
        __syncthreads();
        if (tid < CH) {
            float s = 0.f;
            for (int px = 0; px < 64; ++px) s += bf2f(gT[tid][px]);
            bpart += s;
        }
        for (int ti = 0; ti < 3; ++ti) {
            const int tap = wave + 4 * ti;
            if (tap >= 9) break;
            const int u = tap / 3, v = tap % 3;
            for (int kc = 0; kc < 64; kc += 32) {
                for (int coh = 0; coh < 2; ++coh) {
                    // A[co][p]: row co = 16 coh + col, k = pixels kc + 8 kg ..
                    const bf16x8 A = load8(&gT[16 * coh + col][kc + 8 * kg]);
                    for (int cih = 0; cih < 2; ++cih) {
                        // B[p][ci]: column ci = 16 cih + col; pixel p reads input x + v - 1
                        u16 bt[8];
                        for (int i = 0; i < 8; ++i) bt[i] = aT[u][16 * cih + col][kc + 8 * kg + i + v];
                        bf16x8 B;
                        memcpy(&B, bt, 16);
                        acc[ti][coh * 2 + cih] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[ti][coh * 2 + cih], 0, 0, 0);
                    }
                }
            }
        }
    }
    const int blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    float* pw = part_w + (size_t)blk * 9 * CH * CH;
    for (int ti = 0; ti < 3; ++ti) {
        const int tap = wave + 4 * ti;
        if (tap >= 9) break;
        for (int q = 0; q < 4; ++q) {
            const int coh = q / 2, cih = q % 2;
            for (int r = 0; r < 4; ++r) {
                const int co = 16 * coh + 4 * kg + r, ci = 16 * cih + col;
                pw[(tap * CH + co) * CH + ci] = acc[ti][q][r];
            }
        }
    }
    if (tid < CH) part_b[(size_t)blk * CH + tid] = bpart;
    (void)bsum;
}

// sums the per-block partials in block order (deterministic)
__global__ void wgrad_reduce_kernel(const float* part_w, const float* part_b, int nblk, float* gw, float* gb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 9 * CH * CH) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += part_w[(size_t)b * 9 * CH * CH + i];
        gw[i] = s;
    }
    if (i < CH) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += part_b[(size_t)b * CH + i];
        gb[i] = s;
    }
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
    u16* xo = x + i * CH;
    // m as a BF16 pair: hi = bf16(m), lo = bf16(256 (m - hi)) (m - hi is
    // exact in FP32), so the first layer sees m to about 16 bits
    for (int c = 0; c < 3; ++c) {
        const float v = m[((size_t)n * 3 + c) * H * W + p];
        const u16 hi = f2bf(v);
        xo[c] = hi;
        xo[3 + c] = f2bf((v - bf2f(hi)) * LO_SCALE);
    }
    for (int c = 0; c < 3; ++c) xo[6 + c] = f2bf(B[n * 3 + c] / B_SCALE);
    for (int c = 9; c < CH; ++c) xo[c] = 0;
}

// loss gradient of the mean squared error of the network output against
// (m_target - base) / scale, and per-block loss partials
__global__ void loss_kernel(const float* zout, const float* base, const float* mt, float* g, float* part, int N,
                            int H, int W, float inv_scale) {
    __shared__ float red[256];
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t npx = (size_t)N * H * W;
    const float inv = 1.0f / (3.0f * (float)npx);
    float l = 0.f;
    if (i < npx) {
        const int n = (int)(i / ((size_t)H * W));
        const size_t p = i - (size_t)n * H * W;
        for (int c = 0; c < CH; ++c) {
            float gv = 0.f;
            if (c < 3) {
                const size_t q = ((size_t)n * 3 + c) * H * W + p;
                const float d = zout[i * CH + c] - (mt[q] - base[q]) * inv_scale;
                l += d * d;
                gv = 2.0f * d * inv;
            }
            g[i * CH + c] = gv;
        }
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] * inv;
}

__global__ void sum_kernel(const float* part, int n, float* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s;
}

// proposals m' = normalize(base + scale * out)
__global__ void propose_kernel(const float* base, const float* zout, float* mo, int N, int H, int W, float scale) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t npx = (size_t)N * H * W;
    if (i >= npx) return;
    const int n = (int)(i / ((size_t)H * W));
    const size_t p = i - (size_t)n * H * W;
    float v[3];
    for (int c = 0; c < 3; ++c) v[c] = base[((size_t)n * 3 + c) * H * W + p] + scale * zout[i * CH + c];
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
    u16* act[NL + 1] = {};                     // activations (bf16, 32 ch)
    float* z[NL] = {};                         // pre-activations (float, 32 ch)
    float* g = nullptr;                        // gradient w.r.t. a layer's output (float, 32 ch)
    u16* gz = nullptr;                         // gradient w.r.t. pre-activation (bf16)
    float* gwp = nullptr;                      // reduced [tap][co][ci] weight gradient
    float* part_w = nullptr;
    float* part_b = nullptr;
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
    llg_batch* vb = nullptr;                   // window films advanced by the plain solver
    llg_batch* eb = nullptr;                   // one film: the Euler predictor
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

int wg_blocks(const llg_sur* s, int N) {
    return ((s->W + 63) / 64) * ((s->H + WG_ROWS - 1) / WG_ROWS) * N;
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

llg_status forward(llg_sur* s, const float* m, const float* B, int N) {
    const size_t npx = (size_t)N * s->H * s->W;
    hipLaunchKernelGGL(make_input_kernel, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, s->stream, m, B,
                       s->act[0], N, s->H, s->W);
    SCHK(s, hipGetLastError());
    const dim3 grid((s->W + 63) / 64, s->H, N);
    for (int l = 0; l < NL; ++l) {
        // the bias of a layer with fewer than 32 outputs is read through a
        // zero-padded 32-entry copy kept in the gradient buffer's tail
        hipLaunchKernelGGL(conv_fwd_kernel, grid, dim3(256), 0, s->stream, s->act[l], s->wf[l],
                           s->params + s->boff[l], s->z[l], s->act[l + 1], s->H, s->W, l < NL - 1 ? 1 : 0);
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
    for (int l = 0; l <= NL; ++l) SCHK(s, hipMalloc(&s->act[l], npx * CH * 2));
    SCHK(s, hipMalloc(&s->g, npx * CH * 4));
    SCHK(s, hipMalloc(&s->gz, npx * CH * 2));
    SCHK(s, hipMalloc(&s->gwp, 9 * CH * CH * 4));
    SCHK(s, hipMalloc(&s->part_w, (size_t)wg_blocks(s, max_batch) * 9 * CH * CH * 4));
    SCHK(s, hipMalloc(&s->part_b, (size_t)wg_blocks(s, max_batch) * CH * 4));
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
    void* ptrs[] = {s->params, s->grads, s->mom1, s->mom2, s->g, s->gz, s->gwp, s->part_w, s->part_b,
                    s->part_l, s->dloss, s->dm_in, s->dm_t, s->dm_out, s->dB};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (int l = 0; l < NL; ++l) {
        if (s->wf[l]) (void)hipFree(s->wf[l]);
        if (s->wtr[l]) (void)hipFree(s->wtr[l]);
        if (s->z[l]) (void)hipFree(s->z[l]);
    }
    for (int l = 0; l <= NL; ++l)
        if (s->act[l]) (void)hipFree(s->act[l]);
    if (s->props) (void)hipFree(s->props);
    if (s->dmax) (void)hipFree(s->dmax);
    if (s->vb) llg_batch_destroy(s->vb);
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
    llg_status rc = forward(s, mi, s->dB, batch);
    if (rc != LLG_OK) return rc;
    const int lb = (int)((npx + 255) / 256);
    hipLaunchKernelGGL(loss_kernel, dim3(lb), dim3(256), 0, s->stream, s->z[NL - 1], mb, mt, s->g, s->part_l, batch,
                       s->H, s->W, 1.0f / s->out_scale);
    SCHK(s, hipGetLastError());
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(64), 0, s->stream, s->part_l, lb, s->dloss);
    SCHK(s, hipGetLastError());
    const dim3 fgrid((s->W + 63) / 64, s->H, batch);
    const dim3 wgrid((s->W + 63) / 64, (s->H + WG_ROWS - 1) / WG_ROWS, batch);
    const int nwb = wg_blocks(s, batch);
    for (int l = NL - 1; l >= 0; --l) {
        hipLaunchKernelGGL(act_bwd_kernel, dim3((unsigned)((npx * CH + 255) / 256)), dim3(256), 0, s->stream, s->g,
                           s->z[l], s->gz, npx * CH, l < NL - 1 ? 1 : 0);
        SCHK(s, hipGetLastError());
        hipLaunchKernelGGL(conv_wgrad_kernel, wgrid, dim3(256), 0, s->stream, s->gz, s->act[l], s->part_w,
                           s->part_b, s->H, s->W);
        SCHK(s, hipGetLastError());
        hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((9 * CH * CH + 255) / 256), dim3(256), 0, s->stream, s->part_w,
                           s->part_b, nwb, s->gwp, s->grads + s->boff[l]);
        SCHK(s, hipGetLastError());
        hipLaunchKernelGGL(unpack_grad_kernel, dim3((COUT[l] * CIN[l] * 9 + 255) / 256), dim3(256), 0, s->stream,
                           s->gwp, CIN[l], COUT[l], s->grads + s->woff[l]);
        SCHK(s, hipGetLastError());
        if (l > 0) {
            // data gradient: the same convolution with flipped, transposed weights
            hipLaunchKernelGGL(conv_fwd_kernel, fgrid, dim3(256), 0, s->stream, s->gz, s->wtr[l], (const float*)nullptr,
                               s->g, (u16*)nullptr, s->H, s->W, 0);
            SCHK(s, hipGetLastError());
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
    llg_status rc = forward(s, mi, s->dB, batch);
    if (rc != LLG_OK) return rc;
    hipLaunchKernelGGL(propose_kernel, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, s->stream, mb,
                       s->z[NL - 1], mo, batch, s->H, s->W, s->out_scale);
    SCHK(s, hipGetLastError());
    if (where != LLG_DEVICE) SCHK(s, hipMemcpyAsync(m_out, s->dm_out, npx * 3 * 4, hipMemcpyDeviceToHost, s->stream));
    SCHK(s, hipStreamSynchronize(s->stream));
    return LLG_OK;
}

// the pre-activation of the last layer (the net's dm before padding) for a
// batch, [batch][H][W][32] float into host memory; for parity checks
llg_status llg_sur_forward_raw(llg_sur* s, const float* m_in, const float* B, int batch, int layer, float* z_out) {
    if (!s || !m_in || !B || !z_out || batch < 1 || batch > s->maxb || layer < 0 || layer >= NL) return LLG_E_ARG;
    SCHK(s, hipSetDevice(s->device));
    if (!s->packed) return sfail(s, LLG_E_STATE, "parameters not set");
    const size_t npx = (size_t)batch * s->H * s->W;
    SCHK(s, hipMemcpyAsync(s->dm_in, m_in, npx * 3 * 4, hipMemcpyHostToDevice, s->stream));
    SCHK(s, hipMemcpyAsync(s->dB, B, (size_t)batch * 3 * 4, hipMemcpyHostToDevice, s->stream));
    llg_status rc = forward(s, s->dm_in, s->dB, batch);
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
    const dim3 fgrid((s->W + 63) / 64, s->H, batch);
    hipLaunchKernelGGL(conv_fwd_kernel, fgrid, dim3(256), 0, s->stream, s->act[0], s->wf[layer],
                       s->params + s->boff[layer], s->z[0], (u16*)nullptr, s->H, s->W, 0);
    SCHK(s, hipGetLastError());
    SCHK(s, hipMemcpyAsync(y, s->z[0], n * 4, hipMemcpyDeviceToHost, s->stream));
    if (gy) {
        float *dgw = nullptr, *dgb = nullptr;
        SCHK(s, hipMalloc(&dgw, sizeof(float) * COUT[layer] * CIN[layer] * 9));
        SCHK(s, hipMalloc(&dgb, sizeof(float) * CH));
        SCHK(s, hipMemcpyAsync(s->g, gy, n * 4, hipMemcpyHostToDevice, s->stream));
        hipLaunchKernelGGL(act_bwd_kernel, dim3(nb), dim3(256), 0, s->stream, s->g, (const float*)nullptr, s->gz, n, 0);
        SCHK(s, hipGetLastError());
        const dim3 wgrid((s->W + 63) / 64, (s->H + WG_ROWS - 1) / WG_ROWS, batch);
        hipLaunchKernelGGL(conv_wgrad_kernel, wgrid, dim3(256), 0, s->stream, s->gz, s->act[0], s->part_w,
                           s->part_b, s->H, s->W);
        SCHK(s, hipGetLastError());
        hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((9 * CH * CH + 255) / 256), dim3(256), 0, s->stream, s->part_w,
                           s->part_b, wg_blocks(s, batch), s->gwp, dgb);
        SCHK(s, hipGetLastError());
        hipLaunchKernelGGL(unpack_grad_kernel, dim3((COUT[layer] * CIN[layer] * 9 + 255) / 256), dim3(256), 0,
                           s->stream, s->gwp, CIN[layer], COUT[layer], dgw);
        SCHK(s, hipGetLastError());
        hipLaunchKernelGGL(conv_fwd_kernel, fgrid, dim3(256), 0, s->stream, s->gz, s->wtr[layer],
                           (const float*)nullptr, s->z[1], (u16*)nullptr, s->H, s->W, 0);
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
    // the verification batch: `window` copies of the film
    if (!s->vb || s->vwin != window || !same_film(s->vdesc, *film)) {
        if (s->vb) llg_batch_destroy(s->vb);
        if (s->eb) llg_batch_destroy(s->eb);
        s->vb = nullptr;
        s->eb = nullptr;
        if (s->props) (void)hipFree(s->props);
        if (s->dmax) (void)hipFree(s->dmax);
        s->props = nullptr;
        s->dmax = nullptr;
        std::vector<float> h0(3 * (size_t)ncells);
        SCHK(s, hipMemcpy(h0.data(), m, vec, where == LLG_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
        std::vector<llg_film_desc> fd(window, *film);
        for (auto& f : fd) f.m0 = h0.data();
        llg_status rc = llg_batch_create(s->device, fd.data(), window, &s->vb);
        if (rc != LLG_OK) {
            const std::string why = s->vb ? llg_batch_last_error(s->vb) : "batch creation failed";
            if (s->vb) llg_batch_destroy(s->vb);
            s->vb = nullptr;
            return sfail(s, rc, "verification batch: %s", why.c_str());
        }
        rc = llg_batch_create(s->device, fd.data(), 1, &s->eb);
        if (rc != LLG_OK) {
            const std::string why = s->eb ? llg_batch_last_error(s->eb) : "batch creation failed";
            if (s->eb) llg_batch_destroy(s->eb);
            s->eb = nullptr;
            return sfail(s, rc, "predictor batch: %s", why.c_str());
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
    int64_t done = 0;
    while (done < n_segments) {
        const int w = (int)std::min<int64_t>(window, n_segments - done);
        float* P = s->props;
        // proposals 1..w, each from the previous one: normalize(base + dm)
        // with base the previous state or its one coarse step (Euler or
        // RK4) over the whole segment by the plain solver
        for (int j = 1; j <= w; ++j) {
            const float* prev = P + (size_t)(j - 1) * 3 * ncells;
            const float* base = prev;
            if (predictor != LLG_SUR_BASE_STATE) {
                float* em = nullptr;
                llg_status rc = llg_batch_state_ptr_(s->eb, 0, &em);
                if (rc != LLG_OK) return sfail(s, rc, "predictor batch: %s", llg_batch_last_error(s->eb));
                SCHK(s, hipMemcpyAsync(em, prev, vec, hipMemcpyDeviceToDevice, s->stream));
                SCHK(s, hipStreamSynchronize(s->stream));
                llg_batch_states_replaced_(s->eb);
                rc = llg_batch_step(s->eb, predictor == LLG_SUR_BASE_EULER ? LLG_EULER : LLG_RK4, dt * seg_steps, 1);
                if (rc != LLG_OK) return sfail(s, rc, "predictor batch: %s", llg_batch_last_error(s->eb));
                rc = llg_batch_state_ptr_(s->eb, 0, &em);
                if (rc != LLG_OK) return sfail(s, rc, "predictor batch: %s", llg_batch_last_error(s->eb));
                base = em;
            }
            llg_status rc = forward(s, prev, s->dB, 1);
            if (rc != LLG_OK) return rc;
            hipLaunchKernelGGL(propose_kernel, dim3((ncells + 255) / 256), dim3(256), 0, s->stream, base,
                               s->z[NL - 1], P + (size_t)j * 3 * ncells, 1, s->H, s->W, s->out_scale);
            SCHK(s, hipGetLastError());
        }
        // finiteness of the proposals (0 for finite, inf otherwise) and the
        // number of start states that may go to the plain solver
        hipLaunchKernelGGL(zero_u32_kernel, dim3((2 * window + 255) / 256), dim3(256), 0, s->stream, s->dmax,
                           2 * window);
        SCHK(s, hipGetLastError());
        for (int j = 1; j <= w; ++j) {
            const float* pj = P + (size_t)j * 3 * ncells;
            llg_status rc = max_distance(s, pj, pj, ncells, s->dmax + window + j - 1);
            if (rc != LLG_OK) return rc;
        }
        SCHK(s, hipMemcpyAsync(hd.data() + window, s->dmax + window, sizeof(unsigned) * window,
                               hipMemcpyDeviceToHost, s->stream));
        SCHK(s, hipStreamSynchronize(s->stream));
        int nstart = w;   // films 0..nstart-1 start from proposals 0..nstart-1
        for (int j = 1; j < w; ++j)
            if (hd[window + j - 1] != 0u) { nstart = j; break; }
        // plain segments from every start state, one batched launch per step
        for (int j = 0; j < nstart; ++j) {
            llg_status rc = llg_batch_state_ptr_(s->vb, j, &ptr[j]);
            if (rc != LLG_OK) return sfail(s, rc, "verification batch: %s", llg_batch_last_error(s->vb));
            SCHK(s, hipMemcpyAsync(ptr[j], P + (size_t)j * 3 * ncells, vec, hipMemcpyDeviceToDevice, s->stream));
        }
        SCHK(s, hipStreamSynchronize(s->stream));
        llg_batch_states_replaced_(s->vb);
        llg_status rc = llg_batch_step(s->vb, LLG_RK4, dt, seg_steps);
        if (rc != LLG_OK) return sfail(s, rc, "verification batch: %s", llg_batch_last_error(s->vb));
        for (int j = 0; j < nstart; ++j) {
            rc = llg_batch_state_ptr_(s->vb, j, &ptr[j]);
            if (rc != LLG_OK) return sfail(s, rc, "verification batch: %s", llg_batch_last_error(s->vb));
        }
        // distance of every proposal to the plain result from its predecessor
        for (int j = 1; j <= nstart; ++j) {
            rc = max_distance(s, P + (size_t)j * 3 * ncells, ptr[j - 1], ncells, s->dmax + j - 1);
            if (rc != LLG_OK) return rc;
        }
        SCHK(s, hipMemcpyAsync(hd.data(), s->dmax, sizeof(unsigned) * window, hipMemcpyDeviceToHost, s->stream));
        SCHK(s, hipStreamSynchronize(s->stream));
        int k = nstart;       // segments this round commits
        int acc = nstart;     // proposals accepted
        for (int j = 1; j <= nstart; ++j) {
            const float d = bits_to_float(hd[j - 1]);
            st.max_dm_seen = std::max(st.max_dm_seen, (double)d);
            if (!((double)d <= max_dm)) { k = j; acc = j - 1; break; }
            st.max_dm_accepted = std::max(st.max_dm_accepted, (double)d);
        }
        st.proposals += nstart;
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
