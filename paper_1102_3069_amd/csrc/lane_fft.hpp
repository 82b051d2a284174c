// Compile-time-length FFTs computed by a group of P lanes of one wavefront.
//
// Lane lg (0 <= lg < P) of the group holds E = L/P elements in registers,
// element i being index lg + P*i of the sequence ("natural" layout).  The
// transform is a Stockham autosort sequence of radix-R stages (every R
// divides E): the first stage reads its butterfly inputs straight from the
// registers, the last one writes its outputs straight back to registers in
// the same natural layout, and the stages in between exchange through a
// per-group LDS scratch of L elements.  A group never spans two wavefronts,
// so no workgroup barrier is needed inside a transform: the lanes of one
// wavefront issue their LDS operations in program order.
//
// LDS banks: the scratch index is XOR-swizzled within aligned runs of 32
// elements (lf_swz), which spreads both the unit-stride reads and the
// R-strided Stockham stores of a stage over distinct banks; each stage's
// twiddles sit in a table of their own, ordered (r - 1) * Ns + k, so that
// the lanes of a wavefront read consecutive (or equal) entries.  The caller
// fills that table once per workgroup (TwFill) from the table
// exp(-2 pi i m / (L * TM)) it already holds (TM = 1 or 2 so that one table
// serves both the half-length transforms of a zero-padded axis and its
// pre/post twiddles).
#pragma once

#include "device_common.hpp"

namespace llg {

// one more DFT size used by the lane FFTs: 16 = 4 x 4
template <typename C> struct Dft<16, C> {
    static __device__ __forceinline__ void run(C* v, bool inv) {
        using T = typename real_of<C>::type;
        C a[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            a[n2][0] = v[n2]; a[n2][1] = v[4 + n2]; a[n2][2] = v[8 + n2]; a[n2][3] = v[12 + n2];
            dft4(a[n2][0], a[n2][1], a[n2][2], a[n2][3], inv);
        }
        // twiddles W16^(n2 k1)
        const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
        const T r2 = (T)0.70710678118654752440;
        const T sg = inv ? (T)1 : (T)-1;
        const C w1 = cmk<C>(c1, sg * s1), w2 = cmk<C>(r2, sg * r2), w3 = cmk<C>(s1, sg * c1);
        const C w6 = cmk<C>(-r2, sg * r2), w9 = cmk<C>(-c1, -sg * s1);
        a[1][1] = cmul(a[1][1], w1); a[1][2] = cmul(a[1][2], w2); a[1][3] = cmul(a[1][3], w3);
        a[2][1] = cmul(a[2][1], w2); a[2][2] = inv ? mul_pi(a[2][2]) : mul_mi(a[2][2]);
        a[2][3] = cmul(a[2][3], w6);
        a[3][1] = cmul(a[3][1], w3); a[3][2] = cmul(a[3][2], w6); a[3][3] = cmul(a[3][3], w9);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            C b0 = a[0][k1], b1 = a[1][k1], b2 = a[2][k1], b3 = a[3][k1];
            dft4(b0, b1, b2, b3, inv);
            v[k1] = b0; v[k1 + 4] = b1; v[k1 + 8] = b2; v[k1 + 12] = b3;
        }
    }
};

// ---------------------------------------------------------------------------
// stage plan: greedy radices from {16, 8, 4, 2, 3, 5, 7}, each dividing both
// the remaining length and E
// ---------------------------------------------------------------------------
constexpr int lf_pick(int rem, int E) {
    return (rem % 16 == 0 && E % 16 == 0) ? 16
         : (rem % 8 == 0 && E % 8 == 0) ? 8
         : (rem % 4 == 0 && E % 4 == 0) ? 4
         : (rem % 2 == 0 && E % 2 == 0) ? 2
         : (rem % 3 == 0 && E % 3 == 0) ? 3
         : (rem % 5 == 0 && E % 5 == 0) ? 5
         : (rem % 7 == 0 && E % 7 == 0) ? 7 : 0;
}
constexpr int lf_radix(int L, int E, int s) {
    int rem = L;
    for (int i = 0; i < s; ++i) {
        const int r = lf_pick(rem, E);
        if (r == 0) return 0;
        rem /= r;
    }
    return rem == 1 ? 1 : lf_pick(rem, E);
}
constexpr int lf_nstages(int L, int E) {
    int rem = L, n = 0;
    while (rem > 1) {
        const int r = lf_pick(rem, E);
        if (r == 0) return -1;
        rem /= r;
        ++n;
    }
    return n;
}
constexpr int lf_ns(int L, int E, int s) {
    int p = 1;
    for (int i = 0; i < s; ++i) p *= lf_radix(L, E, i);
    return p;
}

// shift/mask friendly modulo for the compile-time Ns
template <int N> __device__ __forceinline__ int cmod(int a) { return a % N; }

// LDS scratch index of element i of a length-L transform: a permutation of
// 0 .. L-1 that flips the low bits of i (within its aligned run of M + 1
// elements, M + 1 the largest power of two dividing L, at most 32) by bits
// A.. and B.. of i (each flipped bit taken from higher bits, so the map is
// invertible; it is linear over XOR).  Unit-stride runs and the R-strided
// runs of the Stockham stores then fall into distinct 8-byte bank pairs.
template <int L> struct LfSwz {
    static constexpr int low = L & -L;
    static constexpr int M = (low < 32 ? low : 32) - 1;
};
template <int L, int A = 3, int B = 7> __device__ __forceinline__ int lf_swz(int i) {
    return i ^ (((i >> A) ^ (i >> B)) & LfSwz<L>::M);
}

template <int L> struct LfScratch { static constexpr int size = L; };

template <int L, int E, int TM, typename C>
struct LaneFFT {
    static constexpr int P = L / E;
    static constexpr int NS = lf_nstages(L, E);
    static constexpr int SCRATCH = LfScratch<L>::size;   // elements per group
    // swizzle shifts: plans of radix 4 and below (E not a multiple of 8) take
    // bits 2 and 3, which spread their stride-2 and stride-4 stage stores
    // over the banks (bank conflicts of the 1024-point rows 104448 -> 6144
    // cycles per launch); radix-8 and radix-16 plans take 3 and 7
    static constexpr int SA = E % 8 == 0 ? 3 : 2, SB = E % 8 == 0 ? 7 : 3;
    static __device__ __forceinline__ int swz(int i) { return lf_swz<L, SA, SB>(i); }
    static_assert(L % E == 0 && NS >= 0, "length must factor into radices dividing E");
    static_assert(64 % P == 0, "a lane group must fit one wavefront");

    // twiddle table of stage s >= 1: entry (r - 1) Ns + k = w^(k r TS) of the
    // caller's table, r = 1 .. R-1, k < Ns
    static constexpr int tws_count(int s) { return s == 0 ? 0 : (lf_radix(L, E, s) - 1) * lf_ns(L, E, s); }
    static constexpr int tws_off(int s) {
        int o = 0;
        for (int i = 1; i < s; ++i) o += tws_count(i);
        return o;
    }
    static constexpr int TWS = tws_off(NS);                // entries of all stage tables
    static constexpr int TWS_ALLOC = TWS > 0 ? TWS : 1;    // LDS entries to reserve

    template <int S>
    static __device__ __forceinline__ void tw_index(int e, int& idx) {
        if constexpr (S < NS) {
            constexpr int R = lf_radix(L, E, S), Ns = lf_ns(L, E, S);
            constexpr int TS = (L / (Ns * R)) * TM, B = tws_off(S), CNT = (R - 1) * Ns;
            if (e >= B && e < B + CNT) {
                const int t = e - B;
                idx = (t % Ns) * (t / Ns + 1) * TS;
            }
            tw_index<S + 1>(e, idx);
        }
    }
    // the stage tables from the table full[m] = exp(-2 pi i m / (L TM)),
    // by threads tid = 0 .. NT-1 of the workgroup (a barrier must follow),
    // in two halves like StagedCopy: load() issues the reads, store()
    // writes the tables
    template <int NT>
    struct TwFill {
        static constexpr int IT = (TWS + NT - 1) / NT;
        C v[IT > 0 ? IT : 1];
        template <typename Src>
        __device__ __forceinline__ void load(const Src* __restrict__ full, int tid) {
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int e = tid + it * NT;
                if (e < TWS) {
                    int idx = 0;
                    tw_index<1>(e, idx);
                    v[it] = full[idx];
                }
            }
        }
        __device__ __forceinline__ void store(C* __restrict__ tws, int tid) const {
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int e = tid + it * NT;
                if (e < TWS) tws[e] = v[it];
            }
        }
    };
    template <int S, bool INV>
    static __device__ __forceinline__ void stage(C (&x)[E], C* sc, const C* tws, int lg) {
        constexpr int R = lf_radix(L, E, S);
        constexpr int Ns = lf_ns(L, E, S);
        constexpr int U = E / R;          // butterflies per lane
        constexpr int LR = L / R;
        constexpr int B = tws_off(S);
        constexpr bool FIRST = S == 0, LAST = S == NS - 1;
        // power-of-two lengths: every radix, Ns and P are powers of two, so a
        // scratch index splits into the lane's part and a part fixed by
        // (u, r) with disjoint bits, and the swizzle (linear over XOR) of the
        // index is the XOR of the parts' swizzles: one lane value per stage
        // and a constant per access
        constexpr bool P2 = (L & (L - 1)) == 0;
        const int rl = swz(lg);
        C v[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = lg + P * u;
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[u][r] = FIRST ? x[u + r * U]
                        : sc[P2 ? (rl ^ swz(P * u + r * LR)) : swz(j + r * LR)];
            if (Ns > 1) {
                const int k = cmod<Ns>(j);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = tws[B + (r - 1) * Ns + k];
                    if (INV) w.y = -w.y;
                    v[u][r] = cmul(v[u][r], w);
                }
            }
            Dft<R, C>::run(v[u], INV);
        }
        if (LAST) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int r = 0; r < R; ++r) x[u + r * U] = v[u][r];
        } else {
            __builtin_amdgcn_wave_barrier();
            // the lane's part of the store index: d(lg) with d(j) = (j - j mod Ns) R + j mod Ns
            const int wl = swz((lg - cmod<Ns>(lg)) * R + cmod<Ns>(lg));
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = lg + P * u;
                const int k = cmod<Ns>(j);
                const int d = (j - k) * R + k;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int c = (P * u - cmod<Ns>(P * u)) * R + cmod<Ns>(P * u) + r * Ns;
                    sc[P2 ? (wl ^ swz(c)) : swz(d + r * Ns)] = v[u][r];
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }

    template <int S, bool INV>
    static __device__ __forceinline__ void stages(C (&x)[E], C* sc, const C* tws, int lg) {
        if constexpr (S < NS) {
            stage<S, INV>(x, sc, tws, lg);
            stages<S + 1, INV>(x, sc, tws, lg);
        }
    }

    // unnormalised transform, forward (exp(-i...)) or inverse (exp(+i...));
    // tws: the stage tables (TwFill)
    template <bool INV>
    static __device__ __forceinline__ void run(C (&x)[E], C* sc, const C* tws, int lg) {
        stages<0, INV>(x, sc, tws, lg);
    }
};

// value held by lane `src` (absolute lane id in the wavefront) of register v
__device__ __forceinline__ float2 lane_shfl(float2 v, int src) {
    float2 r;
    r.x = __shfl(v.x, src);
    r.y = __shfl(v.y, src);
    return r;
}

}  // namespace llg
