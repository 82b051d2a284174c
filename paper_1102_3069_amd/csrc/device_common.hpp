// Device-side building blocks shared by the library's HIP kernels:
// complex helpers, a workgroup-wide Stockham FFT staged in LDS, the small
// DFT butterflies it uses, and the Philox4x32-10 generator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace llg {

constexpr int kMaxStages = 16;

// Factorisation of one FFT length into radices 2, 3, 4, 5, 7, 8 (stage
// order), built on the host.
struct FftPlan {
    int L;
    int ns;
    int rad[kMaxStages];
};

// ---------------------------------------------------------------------------
// complex arithmetic (float2 / double2)
// ---------------------------------------------------------------------------
template <typename C> struct real_of;
template <> struct real_of<float2> { using type = float; };
template <> struct real_of<double2> { using type = double; };

template <typename C>
__device__ __forceinline__ C cmk(typename real_of<C>::type x, typename real_of<C>::type y) {
    C c; c.x = x; c.y = y; return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmk<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, typename real_of<C>::type s) {
    return cmk<C>(a.x * s, a.y * s);
}
// multiply by -i (forward) or +i (inverse)
template <typename C> __device__ __forceinline__ C mul_mi(C a) { return cmk<C>(a.y, -a.x); }
template <typename C> __device__ __forceinline__ C mul_pi(C a) { return cmk<C>(-a.y, a.x); }
template <typename C> __device__ __forceinline__ C czero() { return cmk<C>(0, 0); }

// ---------------------------------------------------------------------------
// small DFTs: y_k = sum_n v_n w^(n k), w = exp(-2 pi i / R) forward,
// exp(+2 pi i / R) inverse
// ---------------------------------------------------------------------------
template <int R> struct RootTable;
// cos(2 pi j / R), sin(2 pi j / R) for j = 1 .. (R-1)/2
template <> struct RootTable<3> {
    static constexpr double c[2] = {1.0, -0.5};
    static constexpr double s[2] = {0.0, 0.86602540378443864676};
};
template <> struct RootTable<5> {
    static constexpr double c[3] = {1.0, 0.30901699437494742410, -0.80901699437494742410};
    static constexpr double s[3] = {0.0, 0.95105651629515357212, 0.58778525229247312917};
};
template <> struct RootTable<7> {
    static constexpr double c[4] = {1.0, 0.62348980185873353053, -0.22252093395631440429,
                                    -0.90096886790241912624};
    static constexpr double s[4] = {0.0, 0.78183148246802980871, 0.97492791218182360702,
                                    0.43388373911755812048};
};

// odd prime radix: pair the inputs n and R-n (cosine and sine parts)
template <int R, typename C>
__device__ __forceinline__ void dft_odd(C* v, bool inv) {
    using T = typename real_of<C>::type;
    constexpr int H = (R - 1) / 2;
    C a[H + 1], b[H + 1];
#pragma unroll
    for (int n = 1; n <= H; ++n) {
        a[n] = cadd(v[n], v[R - n]);
        b[n] = csub(v[n], v[R - n]);
    }
    C y0 = v[0];
#pragma unroll
    for (int n = 1; n <= H; ++n) y0 = cadd(y0, a[n]);
    C out[R];
    out[0] = y0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        C re = v[0];
        C im = czero<C>();
#pragma unroll
        for (int n = 1; n <= H; ++n) {
            int j = (n * k) % R;
            T cj, sj;
            if (j <= H) { cj = (T)RootTable<R>::c[j]; sj = (T)RootTable<R>::s[j]; }
            else { cj = (T)RootTable<R>::c[R - j]; sj = -(T)RootTable<R>::s[R - j]; }
            re = cadd(re, cscale(a[n], cj));
            im = cadd(im, cscale(b[n], sj));
        }
        // forward: y_k = re - i im, y_{R-k} = re + i im
        C t = inv ? mul_pi(im) : mul_mi(im);
        out[k] = cadd(re, t);
        out[R - k] = csub(re, t);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = out[k];
}

template <typename C>
__device__ __forceinline__ void dft4(C& v0, C& v1, C& v2, C& v3, bool inv) {
    C t0 = cadd(v0, v2), t1 = csub(v0, v2);
    C t2 = cadd(v1, v3), t3 = csub(v1, v3);
    t3 = inv ? mul_pi(t3) : mul_mi(t3);
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, t3);
    v3 = csub(t1, t3);
}

template <int R, typename C> struct Dft;
template <typename C> struct Dft<2, C> {
    static __device__ __forceinline__ void run(C* v, bool) {
        C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};
template <typename C> struct Dft<4, C> {
    static __device__ __forceinline__ void run(C* v, bool inv) { dft4(v[0], v[1], v[2], v[3], inv); }
};
template <typename C> struct Dft<8, C> {
    static __device__ __forceinline__ void run(C* v, bool inv) {
        using T = typename real_of<C>::type;
        const T r = (T)0.70710678118654752440;
        C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4(e0, e1, e2, e3, inv);
        dft4(o0, o1, o2, o3, inv);
        // w8^k, w8 = exp(-+ 2 pi i / 8)
        const T sg = inv ? (T)1 : (T)-1;
        C w1 = cmk<C>(r, sg * r), w3 = cmk<C>(-r, sg * r);
        o1 = cmul(o1, w1);
        o2 = inv ? mul_pi(o2) : mul_mi(o2);
        o3 = cmul(o3, w3);
        v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
        v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
        v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
        v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
    }
};
template <typename C> struct Dft<3, C> {
    static __device__ __forceinline__ void run(C* v, bool inv) { dft_odd<3, C>(v, inv); }
};
template <typename C> struct Dft<5, C> {
    static __device__ __forceinline__ void run(C* v, bool inv) { dft_odd<5, C>(v, inv); }
};
template <typename C> struct Dft<7, C> {
    static __device__ __forceinline__ void run(C* v, bool inv) { dft_odd<7, C>(v, inv); }
};

// ---------------------------------------------------------------------------
// Stockham autosort FFT in LDS (Stockham formulation as in Govindaraju et
// al., "High performance discrete Fourier transforms on graphics
// processors", SC'08): stage with radix R on sub-length Ns reads element
// j + r L/R, twiddles it by W_{Ns R}^{(j mod Ns) r}, and writes output r of
// butterfly j to ((j div Ns) Ns R + j mod Ns) + r Ns.  The stage is done in
// place: every thread first reads and transforms its butterflies into
// registers, the workgroup synchronises, then all write.
//
// `buf` holds `nbatch` transforms of length L back to back.  The twiddle
// table tw has tw[m] = exp(-2 pi i m / Lt) with Lt = L * tmul.
// MAXE bounds the elements one thread touches per stage: nbatch*L <= MAXE*nthr.
// ---------------------------------------------------------------------------
template <int R, int MAXE, typename C>
__device__ __forceinline__ void stockham_stage(C* buf, int L, int Ns, int nbatch,
                                               const C* __restrict__ tw, int tmul, bool inv,
                                               int tid, int nthr) {
    constexpr int MAXB = (MAXE + R - 1) / R;
    const int nb = L / R;
    const int total = nbatch * nb;
    const int step = (L / (Ns * R)) * tmul;
    C v[MAXB][R];
    int dst[MAXB];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int t = tid + q * nthr;
        dst[q] = -1;
        if (t < total) {
            const int b = t / nb;
            const int j = t - b * nb;
            const int k = j % Ns;
            const C* src = buf + b * L;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = src[j + r * nb];
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = tw[k * r * step];
                    if (inv) w.y = -w.y;
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            Dft<R, C>::run(v[q], inv);
            dst[q] = b * L + (j - k) * R + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        if (dst[q] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[q] + r * Ns] = v[q][r];
        }
    }
    __syncthreads();
}

// Whole transform; the caller synchronises before (data in buf) and the
// result is in buf, in natural order, when this returns (it ends with a
// barrier).  Unnormalised in both directions.
template <int MAXE, typename C>
__device__ __forceinline__ void lds_fft(C* buf, const FftPlan& p, int nbatch,
                                        const C* __restrict__ tw, int tmul, bool inv,
                                        int tid, int nthr) {
    int Ns = 1;
    for (int s = 0; s < p.ns; ++s) {
        const int R = p.rad[s];
        switch (R) {
            case 2: stockham_stage<2, MAXE>(buf, p.L, Ns, nbatch, tw, tmul, inv, tid, nthr); break;
            case 3: stockham_stage<3, MAXE>(buf, p.L, Ns, nbatch, tw, tmul, inv, tid, nthr); break;
            case 4: stockham_stage<4, MAXE>(buf, p.L, Ns, nbatch, tw, tmul, inv, tid, nthr); break;
            case 5: stockham_stage<5, MAXE>(buf, p.L, Ns, nbatch, tw, tmul, inv, tid, nthr); break;
            case 7: stockham_stage<7, MAXE>(buf, p.L, Ns, nbatch, tw, tmul, inv, tid, nthr); break;
            default: stockham_stage<8, MAXE>(buf, p.L, Ns, nbatch, tw, tmul, inv, tid, nthr); break;
        }
        Ns *= R;
    }
}

// dst[m] = src[m] for m < n (n <= N) by threads tid = 0 .. NT-1 of a
// workgroup, in two halves: load() issues every read into registers,
// store() writes them out.  Issuing the loads of several copies before the
// first store makes them cost one memory round trip together.
template <int N, int NT, typename T>
struct StagedCopy {
    static constexpr int IT = (N + NT - 1) / NT;
    T v[IT];
    __device__ __forceinline__ void load(const T* __restrict__ src, int tid, int n = N) {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int m = tid + it * NT;
            if (m < n) v[it] = src[m];
        }
    }
    __device__ __forceinline__ void store(T* __restrict__ dst, int tid, int n = N) const {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int m = tid + it * NT;
            if (m < n) dst[m] = v[it];
        }
    }
};

// Workgroups are dispatched round-robin over the 8 XCDs of the MI355X; give
// each XCD a contiguous range of logical tiles so that tiles sharing cache
// lines share one L2 (a bijection of [0, n)).
__device__ __forceinline__ int xcd_remap_blocks(int b, int n) {
    const int X = 8;
    const int x = b % X, i = b / X;
    const int q = n / X, rmd = n % X;
    return x * q + min(x, rmd) + i;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of
// (hi0,lo0) = M0*x0, (hi1,lo1) = M1*x2, x <- (hi1^x1^k0, lo1, hi0^x3^k1, lo0)
// with the key bumped by (W0, W1) between rounds.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        const uint32_t lo0 = M0 * c.x, hi0 = __umulhi(M0, c.x);
        const uint32_t lo1 = M1 * c.z, hi1 = __umulhi(M1, c.z);
        U4 n;
        n.x = hi1 ^ c.y ^ k0;
        n.y = lo1;
        n.z = hi0 ^ c.w ^ k1;
        n.w = lo0;
        c = n;
    }
    return c;
}

// 24-bit uniform in (0,1), exact in float
__device__ __forceinline__ float u24(uint32_t b) {
    return ((float)(b >> 8) + 0.5f) * 5.9604644775390625e-8f;
}

// unit Gaussian vector of cell `cell` at time step `step` (Box-Muller on
// the hardware transcendentals: v_log_f32 is log2, v_sin_f32 / v_cos_f32
// take their argument in turns, so sin(2 pi u) is one instruction for the
// uniforms u in (0, 1))
__device__ __forceinline__ void thermal_eta(uint32_t cell, uint64_t step, uint32_t k0, uint32_t k1,
                                            float& ex, float& ey, float& ez) {
    U4 c;
    c.x = cell;
    c.y = (uint32_t)(step & 0xffffffffu);
    c.z = (uint32_t)(step >> 32);
    c.w = 0u;
    U4 r = philox4x32_10(c, k0, k1);
    const float u0 = u24(r.x), u1 = u24(r.y), u2 = u24(r.z), u3 = u24(r.w);
    constexpr float kTwoLn2 = 1.38629436111989061883f;   // -2 ln u = -2 ln 2 log2 u
    const float a = sqrtf(-kTwoLn2 * __builtin_amdgcn_logf(u0));
    const float b = sqrtf(-kTwoLn2 * __builtin_amdgcn_logf(u2));
    ex = a * __builtin_amdgcn_cosf(u1);
    ey = a * __builtin_amdgcn_sinf(u1);
    ez = b * __builtin_amdgcn_cosf(u3);
}

}  // namespace llg
