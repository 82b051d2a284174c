// Column passes of the 3D path (y forward, z with the kernel product, y
// inverse) for axes of compiled length.
//
// Layout: the passes run along an axis of a [c][outer][axis][kx] array
// (kx fastest, strides in ColArgs).  A block owns a tile of TW consecutive
// kx at one outer index, so its global reads and writes are rows of TW
// contiguous complex values; the tile is transposed through LDS so that
// every transform reads its line contiguously.  The pass with the kernel
// product needs the three components of a tile in one block (NC = 3); the
// plain forward and inverse passes take one component per block (NC = 1),
// which leaves room in LDS for wider tiles and more blocks per CU.  An open axis (zero padded
// to 2L) is split into its even and odd frequencies, X[2k] = FFT_L(x),
// X[2k+1] = FFT_L(x W^n) (W = exp(-2 pi i / 2L)), stored in that order (k
// of the even half, then of the odd half); one lane group per (component,
// column, half); the inverse keeps h[n] = IFFT_L(Y_even)[n] +
// W^-n IFFT_L(Y_odd)[n].  A periodic axis is one transform of length L.
// The z pass multiplies by the real symmetric 6-component kernel spectrum
// between the transforms (Sec. 3.2: the transformed kernel of a symmetric
// tensor is real).

#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "lane_fft.hpp"

namespace llg {

namespace {

// H = 2 halves (open axis) or 1 (periodic); E elements per lane; NC
// components per block (3, or 1 with the component from the block index)
template <int L, int E, int TW, int H, int NC>
struct Tile3 {
    static_assert(NC == 1 || NC == 3, "one or three components per block");
    static constexpr int P = L / E;             // lanes per transform
    static constexpr int NG = NC * TW * H;      // lane groups: component, column, half
    static constexpr int NT = NG * P;           // threads per block
    static_assert(64 % P == 0 && NT <= 1024 && NT % 64 == 0, "groups fill whole wavefronts");
    // one LDS line per group, long enough to be that group's FFT scratch;
    // an odd stride spreads the rows of the tile over the banks
    static constexpr int LS = LfScratch<L>::size + 1;
    using F = LaneFFT<L, E, H, float2>;
    static constexpr int O_TWS = H * L;         // after the twiddles exp(-2 pi i m / (H L))
    static constexpr int O_X = O_TWS + F::TWS_ALLOC;   // after the stage twiddle tables
    static constexpr int bytes() { return (O_X + NG * LS) * 8; }
    static __device__ __forceinline__ int line(int c, int w, int h) { return ((c * TW + w) * H + h) * LS; }
};

// kernel spectrum entries at (kx, ka along the pass, ko along y): mirror
// compressed along both; odd components change sign under a mirror
__device__ __forceinline__ void kernel6(const ColArgs& a, int kx, int ka, int ko, float* Kv) {
    bool fa = false, fo = false;
    int ia = ka, io = ko;
    if (ka > a.Pa - ka) { ia = a.Pa - ka; fa = true; }
    if (ko > a.Po - ko) { io = a.Po - ko; fo = true; }
    const long long cstride = (long long)a.no_c * a.nkx * a.na_c;
    const long long off = ((long long)io * a.nkx + kx) * a.na_c + ia;
#pragma unroll
    for (int c = 0; c < 6; ++c) Kv[c] = a.K[c * cstride + off];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        if (fa && a.sign_a[c] < 0) Kv[c] = -Kv[c];
        if (fo && a.sign_o[c] < 0) Kv[c] = -Kv[c];
    }
}

// frequency at position j of the order 0, 1, P-1, 2, P-2, ..., so that the
// two frequencies ko and P - ko that share mirror-compressed kernel rows are
// adjacent
__device__ __forceinline__ int mirror_pair_order(int j, int P) {
    if (j == 0) return 0;
    const int p = (j + 1) >> 1;
    if (2 * p == P) return p;
    return (j & 1) ? p : P - p;
}

template <int L, int E, int TW, int H, int NC, int MODE>
__global__ __launch_bounds__((Tile3<L, E, TW, H, NC>::NT)) void col3_tiled(ColArgs a, DevState* __restrict__ st) {
    using T = Tile3<L, E, TW, H, NC>;
    using F = typename T::F;
    constexpr int P = T::P, NT = T::NT;
    static_assert(MODE != COL_FULL || NC == 3, "the kernel product needs every component");
    extern __shared__ float2 lds[];
    float2* tw = lds;
    float2* tws = lds + T::O_TWS;
    float2* X = lds + T::O_X;
    if (st->done) return;
    const int tid = threadIdx.x;
    int lb = xcd_remap_blocks(blockIdx.x, gridDim.x);
    const int per_c = a.nouter * a.ntiles;      // blocks of one component (NC = 1)
    const int c0 = NC == 3 ? 0 : lb / per_c;    // first component of the block
    lb -= c0 * per_c;
    int o = lb / a.ntiles;
    const int tile = lb - o * a.ntiles;
    if (MODE == COL_FULL && a.nouter == a.Po) {
        // the product pass over every y frequency: mirror pairs (ko, Po - ko)
        // one after the other, so the second reads the kernel rows from L2
        const int ko = mirror_pair_order(o, a.Po);
        o = a.o_split ? (ko & 1) * (a.Po / 2) + (ko >> 1) : ko;
    }
    const int kx0 = tile * TW;
    const int Wt = min(TW, a.nkx - kx0);
    const float2* in = a.in + c0 * a.cs_in + o * a.os_in + kx0;
    float2* out = a.out + c0 * a.cs_out + o * a.os_out + kx0;

    // ---- the tile into the lines: n_in rows (zero beyond) into the h = 0
    // lines, or the H L stored frequencies into their half lines
    // (the loads of up to eight iterations issued before their LDS stores)
    StagedCopy<H * L, NT, float2> twc;
    twc.load(a.tw, tid);
    typename F::template TwFill<NT> twf;
    twf.load(a.tw, tid);
    constexpr int NIN = MODE != COL_INV ? NC * L * TW : NC * H * L * TW;
    constexpr int ITI = (NIN + NT - 1) / NT, CH = ITI < 8 ? ITI : 8;
#pragma unroll
    for (int i0 = 0; i0 < ITI; i0 += CH) {
        float2 v[CH];
        int dst[CH];
#pragma unroll
        for (int ii = 0; ii < CH; ++ii) {
            const int e = tid + (i0 + ii) * NT;
            dst[ii] = -1;
            if (i0 + ii >= ITI || e >= NIN) continue;
            const int w = e % TW, t = e / TW;
            v[ii] = make_float2(0.f, 0.f);
            if (MODE != COL_INV) {
                const int n = t % L, c = t / L;
                if (w < Wt && n < a.n_in) v[ii] = in[c * a.cs_in + n * a.as_in + w];
                dst[ii] = T::line(c, w, 0) + n;
            } else {
                const int k = t % (H * L), c = t / (H * L);
                if (w < Wt) v[ii] = in[c * a.cs_in + k * a.as_in + w];
                dst[ii] = T::line(c, w, k / L) + k % L;
            }
        }
        if (i0 == 0) {
            twc.store(tw, tid);
            twf.store(tws, tid);
        }
#pragma unroll
        for (int ii = 0; ii < CH; ++ii)
            if (dst[ii] >= 0) X[dst[ii]] = v[ii];
    }
    __syncthreads();

    const int gi = tid / P, lg = tid % P;
    const int h = gi % H, w = (gi / H) % TW, c = gi / (H * TW);
    float2* ln = X + T::line(c, w, h);
    float2 x[E];
    if (MODE != COL_INV) {
        // ---- forward transforms (the odd half of x W^n)
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int n = lg + P * i;
            const float2 v = X[T::line(c, w, 0) + n];
            x[i] = h ? cmul(v, tw[n]) : v;
        }
        __syncthreads();   // every half has read its input line
        F::template run<false>(x, ln, tws, lg);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < E; ++i) ln[lg + P * i] = x[i];
        __syncthreads();
        if constexpr (MODE == COL_FWD) {
            for (int e = tid; e < NC * H * L * TW; e += NT) {
                const int ww = e % TW, t = e / TW;
                const int k = t % (H * L), cc = t / (H * L);
                if (ww < Wt) out[cc * a.cs_out + k * a.as_out + ww] = X[T::line(cc, ww, k / L) + k % L];
            }
            return;
        } else {
            // ---- H = K M at every (kx, k) of the tile
            int ko = o;
            if (a.o_split) {
                const int hp = a.Po / 2;
                ko = 2 * (o % hp) + o / hp;
            }
            // consecutive threads take consecutive frequencies ka = H pos + hh,
            // so the kernel spectrum (stored along ka) is read in whole lines
            // (the kernel values of up to three iterations read before their
            // first use)
            constexpr int ITP = (TW * H * L + NT - 1) / NT, CK = ITP < 3 ? ITP : 3;
#pragma unroll
            for (int i0 = 0; i0 < ITP; i0 += CK) {
            float Kc[CK][6];
#pragma unroll
            for (int ii = 0; ii < CK; ++ii) {
                const int e = tid + (i0 + ii) * NT;
                if (i0 + ii >= ITP || e >= TW * H * L) continue;
                const int ka = e % (H * L), ww = e / (H * L);
                const int pos = ka / H, hh = ka % H;
                if (ww < Wt) kernel6(a, kx0 + ww, H * pos + hh, ko, Kc[ii]);
            }
#pragma unroll
            for (int ii = 0; ii < CK; ++ii) {
                const int e = tid + (i0 + ii) * NT;
                if (i0 + ii >= ITP || e >= TW * H * L) continue;
                const int ka = e % (H * L), ww = e / (H * L);
                const int pos = ka / H, hh = ka % H;
                if (ww >= Wt) continue;
                const float* Kv = Kc[ii];
                float2* px = X + T::line(0, ww, hh) + pos;
                float2* py = X + T::line(1, ww, hh) + pos;
                float2* pz = X + T::line(2, ww, hh) + pos;
                const float2 Mx = *px, My = *py, Mz = *pz;
                // K = [xx, yy, zz, xy, xz, yz]
                *px = make_float2(Kv[0] * Mx.x + Kv[3] * My.x + Kv[4] * Mz.x,
                                  Kv[0] * Mx.y + Kv[3] * My.y + Kv[4] * Mz.y);
                *py = make_float2(Kv[3] * Mx.x + Kv[1] * My.x + Kv[5] * Mz.x,
                                  Kv[3] * Mx.y + Kv[1] * My.y + Kv[5] * Mz.y);
                *pz = make_float2(Kv[4] * Mx.x + Kv[5] * My.x + Kv[2] * Mz.x,
                                  Kv[4] * Mx.y + Kv[5] * My.y + Kv[2] * Mz.y);
            }
            }
            __syncthreads();
        }
    }
    // ---- inverse transforms; the odd half leaves W^-n times its result
#pragma unroll
    for (int i = 0; i < E; ++i) x[i] = ln[lg + P * i];
    __builtin_amdgcn_wave_barrier();
    F::template run<true>(x, ln, tws, lg);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int n = lg + P * i;
        ln[n] = h ? cmul(x[i], cconj(tw[n])) : x[i];
    }
    __syncthreads();
    // ---- rows n < n_out of the tile (even + odd half on an open axis)
    for (int e = tid; e < NC * L * TW; e += NT) {
        const int ww = e % TW, t = e / TW;
        const int n = t % L, cc = t / L;
        if (ww >= Wt || n >= a.n_out) continue;
        float2 v = X[T::line(cc, ww, 0) + n];
        if (H == 2) {
            const float2 u = X[T::line(cc, ww, H - 1) + n];
            v = make_float2(v.x + u.x, v.y + u.y);
        }
        out[cc * a.cs_out + n * a.as_out + ww] = v;
    }
}

// compiled (length L of one transform, elements per lane, tile width,
// halves): open axes of 2 L = 32 ... 512, periodic axes of L = 32 ... 256.
// T3_FULL: the pass with the kernel product (three components per block);
// T3_ONE: the plain forward and inverse passes (one component per block,
// tiles twice as wide where that fits)
#define T3_FULL(X)                                                                                  \
    X(16, 4, 16, 2) X(32, 4, 8, 2) X(64, 8, 4, 2) X(128, 8, 4, 2) X(256, 16, 4, 2) X(32, 4, 16, 1) \
    X(64, 8, 16, 1) X(128, 8, 8, 1) X(256, 16, 8, 1)
#define T3_ONE(X)                                                                                     \
    X(16, 4, 32, 2) X(32, 4, 16, 2) X(64, 8, 16, 2) X(128, 8, 8, 2) X(256, 16, 8, 2) X(32, 4, 32, 1) \
    X(64, 8, 32, 1) X(128, 8, 16, 1) X(256, 16, 16, 1)

hipError_t allow_lds3(const void* fn, int bytes) { return raise_lds_limit(fn, bytes); }

template <int L, int E, int TW, int H, int NC>
hipError_t launch_t3(const ColArgs& a, int mode, DevState* st, hipStream_t s) {
    using T = Tile3<L, E, TW, H, NC>;
    if (a.ntiles != (a.nkx + TW - 1) / TW) return hipErrorInvalidValue;
    if ((mode == COL_FULL) != (NC == 3)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(a.nouter * a.ntiles * (3 / NC))), block(T::NT);
    if constexpr (NC == 3) {
        const void* fn = reinterpret_cast<const void*>(&col3_tiled<L, E, TW, H, 3, COL_FULL>);
        hipError_t e = allow_lds3(fn, T::bytes());
        if (e != hipSuccess) return e;
        hot_launch(col3_tiled<L, E, TW, H, 3, COL_FULL>, grid, block, T::bytes(), s, a, st);
    } else {
        const void* fn = mode == COL_FWD ? reinterpret_cast<const void*>(&col3_tiled<L, E, TW, H, 1, COL_FWD>)
                                         : reinterpret_cast<const void*>(&col3_tiled<L, E, TW, H, 1, COL_INV>);
        hipError_t e = allow_lds3(fn, T::bytes());
        if (e != hipSuccess) return e;
        if (mode == COL_FWD)
            hot_launch(col3_tiled<L, E, TW, H, 1, COL_FWD>, grid, block, T::bytes(), s, a, st);
        else
            hot_launch(col3_tiled<L, E, TW, H, 1, COL_INV>, grid, block, T::bytes(), s, a, st);
    }
    return hipGetLastError();
}

}  // namespace

// the transform length and halves of an axis of FFT length P: open axes
// (split) use two transforms of P/2; full: the pass with the kernel product
bool fast3d_col_ok(int P, int split, bool full) {
    const int H = split ? 2 : 1, L = P / H;
    if (full) {
#define CASE(LL, E, TW, HH) if (L == LL && H == HH) return Tile3<LL, E, TW, HH, 3>::bytes() <= 160 * 1024;
        T3_FULL(CASE)
#undef CASE
    } else {
#define CASE(LL, E, TW, HH) if (L == LL && H == HH) return Tile3<LL, E, TW, HH, 1>::bytes() <= 160 * 1024;
        T3_ONE(CASE)
#undef CASE
    }
    return false;
}

int fast3d_col_width(int P, int split, bool full) {
    const int H = split ? 2 : 1, L = P / H;
    if (full) {
#define CASE(LL, E, TW, HH) if (L == LL && H == HH) return TW;
        T3_FULL(CASE)
#undef CASE
    } else {
#define CASE(LL, E, TW, HH) if (L == LL && H == HH) return TW;
        T3_ONE(CASE)
#undef CASE
    }
    return 0;
}

// a.P the axis FFT length, a.split for an open axis; COL_FWD: n_in <= L
// rows in, P frequencies out; COL_INV: P in, n_out <= L rows out;
// COL_FULL: n_in = n_out <= L with the 6-component product; a.ntiles
// tiles of fast3d_col_width(P, split, mode == COL_FULL) columns per outer
// index
hipError_t launch_col3_tiled(const ColArgs& a, int mode, DevState* st, hipStream_t s) {
    const int H = a.split ? 2 : 1, L = a.P / H;
    if (a.P != H * L || a.nkx < 1 || a.nouter < 1 || a.n_in < 1 || a.n_out < 1) return hipErrorInvalidValue;
    if (mode == COL_FWD && !(a.n_in <= L && a.n_out == a.P)) return hipErrorInvalidValue;
    if (mode == COL_INV && !(a.n_in == a.P && a.n_out <= L)) return hipErrorInvalidValue;
    if (mode == COL_FULL && !(a.n_in == a.n_out && a.n_in <= L && a.ncomp == 6)) return hipErrorInvalidValue;
    if (mode != COL_FWD && mode != COL_FULL && mode != COL_INV) return hipErrorInvalidValue;
    if (mode == COL_FULL) {
#define CASE(LL, E, TW, HH) \
        if (L == LL && H == HH) return launch_t3<LL, E, TW, HH, 3>(a, mode, st, s);
        T3_FULL(CASE)
#undef CASE
    } else {
#define CASE(LL, E, TW, HH) \
        if (L == LL && H == HH) return launch_t3<LL, E, TW, HH, 1>(a, mode, st, s);
        T3_ONE(CASE)
#undef CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace llg
