// Fast path of the 2D (one cell thick) effective-field evaluation, for FFT
// lengths known at compile time.
//
// Spectrum layout ("packed"): S[c][y][kx], kx < Px/2.  For a real row the
// k = 0 and k = Px/2 coefficients are both real, so column 0 carries
// (X[0], X[Px/2]) as one complex number; the column pass separates the two
// with the Hermitian symmetry of their y transforms, multiplies each by its
// own kernel column and packs them again.
//
// Row kernels: a block owns RP row pairs and three lane groups per pair
// (two packed rows (mx + i my) and the pair (mz_r0 + i mz_r1)); every
// transform is a LaneFFT of one lane group.  Column kernel: a block owns W
// columns; each (column, frequency half, component group) is one lane
// group, the two halves of a zero-padded axis meet in LDS at the end.
#include <hip/hip_runtime.h>

#include "cell_physics.hpp"
#include "internal.hpp"
#include "lane_fft.hpp"

namespace llg {

namespace {

constexpr int FRT = 192;   // threads of a fast row block (three wavefronts)

__device__ __forceinline__ float2 mk2(float x, float y) { float2 r; r.x = x; r.y = y; return r; }

// Hermitian partner Z[(L - k) mod L] of element i of lane lg (k = lg + P i),
// element layout of LaneFFT; every lane of the group must call this.
template <int E, int P>
__device__ __forceinline__ float2 partner_mirror(const float2 (&z)[E], int i, int lg, int gbase) {
    const float2 t = lane_shfl(z[(E - 1 - i) % E], gbase + (P - lg) % P);
    if (lg != 0) return t;
    return z[(E - i) % E];
}
// partner Z[L - 1 - k] (odd half of a split axis)
template <int E, int P>
__device__ __forceinline__ float2 partner_odd(const float2 (&z)[E], int i, int lg, int gbase) {
    return lane_shfl(z[E - 1 - i], gbase + (P - 1 - lg));
}

// ---------------------------------------------------------------------------
// rows: forward transform of the new magnetisation and packed store
// ---------------------------------------------------------------------------
constexpr int lds_align(int b) { return (b + 15) / 16 * 16; }

template <int PX, int E>
struct RowFast {
    static constexpr int P = PX / E;
    static constexpr int RP = 64 / P;
    static constexpr int HE = E / 2;
    static constexpr int SC = LfScratch<PX>::size;
    static constexpr int NR = 2 * RP + 2;               // staged m rows
    using F = LaneFFT<PX, E, 1, float2>;
    // dynamic LDS carve-up (bytes): twiddles, FFT scratch, exchange rows,
    // staged m rows, staged m0 rows, reduction slots
    static constexpr int O_TW = 0;
    static constexpr int O_SCR = lds_align(O_TW + PX * 8);
    static constexpr int O_XCH = lds_align(O_SCR + 3 * RP * SC * 8);
    static constexpr int O_M = lds_align(O_XCH + RP * 2 * PX * 4);
    static constexpr int fwd_bytes() { return O_M; }
    template <bool XPER> static constexpr int nxm() { return XPER ? PX : PX / 2; }
    template <bool XPER> static constexpr int o_m0() { return lds_align(O_M + NR * 3 * nxm<XPER>() * 4); }
    template <bool XPER> static constexpr int o_wmax() { return lds_align(o_m0<XPER>() + 2 * RP * 3 * nxm<XPER>() * 4); }
    template <bool XPER> static constexpr int inv_bytes() { return lds_align(o_wmax<XPER>() + 16); }

    // kind 0/1 lanes hold the new (mx, my, mz) of their row in nx/ny/nz
    // (cells x = lg + P i); kind 2 lanes collect mz of both rows from xch.
    static __device__ __forceinline__ void forward_store(const Grid& g, float2* __restrict__ S,
                                                         float2* scr, const float2* tw, float* xch,
                                                         const float (&nmx)[E], const float (&nmy)[E],
                                                         const float (&nmz)[E], int kind, int lg,
                                                         int gbase, int r0, bool v0, bool v1) {
        const int nx = g.nx;
        float* xr = xch + (kind & 1) * PX;
        if (kind < 2) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int x = lg + P * i;
                if (x < nx) xr[x] = nmz[i];
            }
        }
        __syncthreads();
        float2 z[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int x = lg + P * i;
            z[i] = mk2(0.f, 0.f);
            if (x < nx) {
                if (kind < 2) {
                    z[i] = mk2(nmx[i], nmy[i]);
                } else {
                    z[i] = mk2(v0 ? xch[x] : 0.f, v1 ? xch[PX + x] : 0.f);
                }
            }
        }
        F::template run<false>(z, scr, tw, lg);
        const long long cs = (long long)g.nrows * g.nkxp;
        const float2 zN = z[HE];   // k = Px/2 on lane 0
#pragma unroll
        for (int i = 0; i < HE; ++i) {
            const int k = lg + P * i;
            const float2 zk = z[i];
            const float2 zm = partner_mirror<E, P>(z, i, lg, gbase);
            float2 A = mk2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            float2 B = mk2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
            if (k == 0) {   // pack the real DC and Nyquist coefficients
                A = mk2(zk.x, zN.x);
                B = mk2(zk.y, zN.y);
            }
            if (kind == 0 && v0) {
                S[(long long)r0 * g.nkxp + k] = A;
                S[cs + (long long)r0 * g.nkxp + k] = B;
            } else if (kind == 1 && v1) {
                S[(long long)(r0 + 1) * g.nkxp + k] = A;
                S[cs + (long long)(r0 + 1) * g.nkxp + k] = B;
            } else if (kind == 2) {
                if (v0) S[2 * cs + (long long)r0 * g.nkxp + k] = A;
                if (v1) S[2 * cs + (long long)(r0 + 1) * g.nkxp + k] = B;
            }
        }
    }
};

template <int PX, int E>
__device__ __forceinline__ void row_fwd_body(const Grid& g, const float2* __restrict__ twx,
                                             float2* __restrict__ S, const FwdArgs& fa,
                                             DevState* __restrict__ st, int blk, char* lds) {
    using R = RowFast<PX, E>;
    constexpr int P = R::P, RP = R::RP;
    float2* tw = (float2*)(lds + R::O_TW);
    float2* scr = (float2*)(lds + R::O_SCR);
    float* xch = (float*)(lds + R::O_XCH);
    if (st->done) return;
    const int tid = threadIdx.x;
    const int gi = tid / P, lg = tid % P;
    const int pair = gi / 3, kind = gi % 3;
    const int gbase = (tid & 63) - lg;
    const int r0 = 2 * (blk * RP + pair);
    const bool v0 = r0 < g.nrows, v1 = r0 + 1 < g.nrows;
    for (int m = tid; m < PX; m += FRT) tw[m] = twx[m];
    const int cur = st->cur;
    const float c1 = st->dtau * fa.a1;
    const long long cs = g.ncells;
    const float* mi = resolve(fa.m_in, cur);
    const float* m0 = resolve(fa.m0, cur);
    const float* k1 = resolve(fa.k1, cur);
    float* mo = resolve(fa.m_out, cur);
    float nmx[E], nmy[E], nmz[E];
    const int r = r0 + (kind & 1);
    const bool vr = kind < 2 && ((kind == 0) ? v0 : v1);
#pragma unroll
    for (int i = 0; i < E; ++i) {
        nmx[i] = nmy[i] = nmz[i] = 0.f;
        const int x = lg + P * i;
        if (vr && x < g.nx) {
            const long long q = (long long)r * g.nx + x;
            if (fa.combine) {
                float ax = m0[q] + c1 * k1[q];
                float ay = m0[cs + q] + c1 * k1[cs + q];
                float az = m0[2 * cs + q] + c1 * k1[2 * cs + q];
                const float inv = rsqrtf(ax * ax + ay * ay + az * az);
                ax *= inv; ay *= inv; az *= inv;
                mo[q] = ax; mo[cs + q] = ay; mo[2 * cs + q] = az;
                nmx[i] = ax; nmy[i] = ay; nmz[i] = az;
            } else {
                nmx[i] = mi[q]; nmy[i] = mi[cs + q]; nmz[i] = mi[2 * cs + q];
            }
        }
    }
    __syncthreads();   // twiddle table
    R::forward_store(g, S, scr + gi * R::SC, tw, xch + pair * 2 * PX, nmx, nmy, nmz, kind, lg, gbase, r0, v0, v1);
}

template <int PX, int E>
__global__ __launch_bounds__(FRT) void row_fwd_fast(Grid g, const float2* __restrict__ twx,
                                                    float2* __restrict__ S, FwdArgs fa,
                                                    DevState* __restrict__ st) {
    extern __shared__ char dyn_lds[];
    row_fwd_body<PX, E>(g, twx, S, fa, st, blockIdx.x, dyn_lds);
}

// exchange + anisotropy + applied + thermal field of cell x of a row whose
// magnetisation and that of its y neighbours sit in LDS (rm, rc, rp: rows
// y-1, y, y+1, component stride nx; null where the neighbour is missing)
__device__ __forceinline__ void local_field_lds(const Grid& g, const Phys& p, const float* rm,
                                                const float* rc, const float* rp, int r, int x,
                                                uint64_t step, float& hx, float& hy, float& hz) {
    const int nx = g.nx;
    const float mx = rc[x], my = rc[nx + x], mz = rc[2 * nx + x];
    float sx = 0.f, sy = 0.f, sz = 0.f;
    auto nb = [&](const float* row, int xx, float c) {
        sx += c * (row[xx] - mx);
        sy += c * (row[nx + xx] - my);
        sz += c * (row[2 * nx + xx] - mz);
    };
    if (p.cex[0] != 0.f && nx > 1) {
        const float c = p.cex[0];
        if (x > 0) nb(rc, x - 1, c); else if (g.pbc[0]) nb(rc, nx - 1, c);
        if (x < nx - 1) nb(rc, x + 1, c); else if (g.pbc[0]) nb(rc, 0, c);
    }
    if (p.cex[1] != 0.f) {
        if (rm) nb(rm, x, p.cex[1]);
        if (rp) nb(rp, x, p.cex[1]);
    }
    hx += sx; hy += sy; hz += sz;
    if (p.ku != 0.f) {
        const float mu = p.ku * (mx * p.u[0] + my * p.u[1] + mz * p.u[2]);
        hx += mu * p.u[0]; hy += mu * p.u[1]; hz += mu * p.u[2];
    }
    hx += p.hz[0]; hy += p.hz[1]; hz += p.hz[2];
    if (p.sig_th != 0.f) {
        float ex, ey, ez;
        thermal_eta((uint32_t)((long long)r * nx + x), step, p.seed_lo, p.seed_hi, ex, ey, ez);
        hx += p.sig_th * ex; hy += p.sig_th * ey; hz += p.sig_th * ez;
    }
}

// XPER: the x axis is periodic (nx == PX), else nx <= PX/2
template <int PX, int E, bool XPER>
__device__ __forceinline__ void row_inv_body(const Grid& g, const Phys& p, const float2* __restrict__ twx,
                                             float2* __restrict__ S, const StageArgs& sa,
                                             DevState* __restrict__ st, int blk, char* lds) {
    using R = RowFast<PX, E>;
    using F = typename R::F;
    constexpr int P = R::P, RP = R::RP;
    constexpr int NXM = R::template nxm<XPER>();     // largest nx
    constexpr int IC = XPER ? E : E / 2;             // cell slots per lane
    constexpr int NR = R::NR;                        // staged m rows (with the y neighbours)
    float2* tw = (float2*)(lds + R::O_TW);
    float2* scr = (float2*)(lds + R::O_SCR);
    float* xch = (float*)(lds + R::O_XCH);
    float* mrow = (float*)(lds + R::O_M);
    float* m0row = (float*)(lds + R::template o_m0<XPER>());
    float* wmax = (float*)(lds + R::template o_wmax<XPER>());
    if (st->done) return;
    const int tid = threadIdx.x;
    const int gi = tid / P, lg = tid % P;
    const int pair = gi / 3, kind = gi % 3;
    const int gbase = (tid & 63) - lg;
    const int rb = 2 * blk * RP;                    // first row of the block
    const int r0 = rb + 2 * pair;
    const bool v0 = r0 < g.nrows, v1 = r0 + 1 < g.nrows;
    const int cur = st->cur;
    const float dtau = st->dtau;
    const uint64_t step = (uint64_t)st->step;
    const int nx = g.nx, ny = g.ny;
    const long long cs = g.ncells;
    const float* mi = resolve(sa.m_in, cur);
    const float* m0 = resolve(sa.m0, cur);
    float* mo = resolve(sa.m_out, cur);
    float* ko = resolve(sa.k_out, cur);
    const bool stage = sa.mode == ROW_STAGE;

    // ---- issue every global read of the block up front (coalesced rows)
    for (int m = tid; m < PX; m += FRT) tw[m] = twx[m];
    // rows rb-1 .. rb+2RP (y neighbours wrap on a periodic y axis)
    for (int e = tid; e < NR * 3 * nx; e += FRT) {
        const int q = e / (3 * nx), t = e - q * 3 * nx;
        const int c = t / nx, x = t - c * nx;
        int row = rb - 1 + q;
        bool ok = row >= 0 && row < g.nrows;
        if (g.pbc[1]) { row = (row + ny) % ny; ok = true; }
        mrow[q * 3 * NXM + t] = ok ? mi[c * cs + (long long)row * nx + x] : 0.f;
    }
    if (stage) {
        for (int e = tid; e < 2 * RP * 3 * nx; e += FRT) {
            const int q = e / (3 * nx), t = e - q * 3 * nx;
            const int c = t / nx, x = t - c * nx;
            const int row = rb + q;
            m0row[q * 3 * NXM + t] = row < g.nrows ? m0[c * cs + (long long)row * nx + x] : 0.f;
        }
    }
    float2 z[E];
#pragma unroll
    for (int i = 0; i < E; ++i) z[i] = mk2(0.f, 0.f);
    if (p.demag_on) {
        const long long scs = (long long)g.nrows * g.nkxp;
        const float2* sa_ = nullptr;
        const float2* sb_ = nullptr;
        if (kind == 0) { if (v0) { sa_ = S + (long long)r0 * g.nkxp; sb_ = sa_ + scs; } }
        else if (kind == 1) { if (v1) { sa_ = S + (long long)(r0 + 1) * g.nkxp; sb_ = sa_ + scs; } }
        else {
            if (v0) sa_ = S + 2 * scs + (long long)r0 * g.nkxp;
            if (v1) sb_ = S + 2 * scs + (long long)(r0 + 1) * g.nkxp;
        }
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int k = lg + P * i;
            const bool up = k > PX / 2;
            const int ka = up ? PX - k : k;
            float2 A = mk2(0.f, 0.f), B = mk2(0.f, 0.f);
            if (k == 0 || k == PX / 2) {
                const bool nyq = k != 0;
                if (sa_) { const float2 v = sa_[0]; A = mk2(nyq ? v.y : v.x, 0.f); }
                if (sb_) { const float2 v = sb_[0]; B = mk2(nyq ? v.y : v.x, 0.f); }
            } else {
                if (sa_) { A = sa_[ka]; if (up) A.y = -A.y; }
                if (sb_) { B = sb_[ka]; if (up) B.y = -B.y; }
            }
            z[i] = mk2(A.x - B.y, A.y + B.x);
        }
    }
    __syncthreads();   // twiddles and staged rows
    if (p.demag_on) {
        F::template run<true>(z, scr + gi * R::SC, tw, lg);
        if (kind == 2) {
#pragma unroll
            for (int i = 0; i < IC; ++i) {
                const int x = lg + P * i;
                if (x < nx) { xch[pair * 2 * PX + x] = z[i].x; xch[pair * 2 * PX + PX + x] = z[i].y; }
            }
        }
    }
    __syncthreads();

    // ---- per cell: field, torque (kinds 0 and 1: rows r0 and r0+1)
    const int rr = kind & 1;
    const int r = r0 + rr;
    const bool vr = kind < 2 && (rr == 0 ? v0 : v1);
    const int q = 2 * pair + rr + 1;              // staged row of this lane's cells
    const int y = r % ny;
    const float* rc = mrow + q * 3 * NXM;
    const float* rm = (y > 0 || g.pbc[1]) ? rc - 3 * NXM : nullptr;
    const float* rp = (y < ny - 1 || g.pbc[1]) ? rc + 3 * NXM : nullptr;
    if (ny == 1) { rm = nullptr; rp = nullptr; }
    float kx[IC], ky[IC], kz[IC];
    bool bad = false;
#pragma unroll
    for (int i = 0; i < IC; ++i) {
        kx[i] = ky[i] = kz[i] = 0.f;
        const int x = lg + P * i;
        if (!(vr && x < nx)) continue;
        float hx = 0.f, hy = 0.f, hz = 0.f;
        if (p.demag_on) { hx = z[i].x; hy = z[i].y; hz = xch[pair * 2 * PX + rr * PX + x]; }
        local_field_lds(g, p, rm, rc, rp, r, x, step, hx, hy, hz);
        if (sa.mode == ROW_EVAL) {
            float* h = sa.h_out;
            const long long qq = (long long)r * nx + x;
            h[qq] = hx * p.Ms; h[cs + qq] = hy * p.Ms; h[2 * cs + qq] = hz * p.Ms;
            bad |= !(isfinite(hx) && isfinite(hy) && isfinite(hz));
            continue;
        }
        ll_torque(p, rc[x], rc[nx + x], rc[2 * nx + x], hx, hy, hz, kx[i], ky[i], kz[i]);
        bad |= !(isfinite(kx[i]) && isfinite(ky[i]) && isfinite(kz[i]));
    }
    if (bad) atomicOr(&st->health, 1);
    if (sa.mode == ROW_EVAL) return;

    // ---- combination with the earlier stages: one pass over the cells per
    // earlier k, all loads of a pass independent of each other
    float ax[IC], ay[IC], az[IC];
    const float cl = stage ? dtau * sa.a[sa.nk - 1] : sa.e[sa.nk - 1];
#pragma unroll
    for (int i = 0; i < IC; ++i) {
        const int x = lg + P * i;
        const bool ok = vr && x < nx;
        const float* m0r = m0row + (2 * pair + rr) * 3 * NXM;
        ax[i] = cl * kx[i] + ((stage && ok) ? m0r[x] : 0.f);
        ay[i] = cl * ky[i] + ((stage && ok) ? m0r[nx + x] : 0.f);
        az[i] = cl * kz[i] + ((stage && ok) ? m0r[2 * nx + x] : 0.f);
    }
    if (sa.mode == ROW_STAGE || sa.mode == ROW_ERROR) {
        for (int j = 0; j + 1 < sa.nk; ++j) {
            const float c = stage ? dtau * sa.a[j] : sa.e[j];
            if (c == 0.f) continue;
            const float* __restrict__ kj = resolve(sa.kprev[j], cur);
            float vx[IC], vy[IC], vz[IC];
#pragma unroll
            for (int i = 0; i < IC; ++i) {
                const int x = lg + P * i;
                const long long qq = (long long)r * nx + x;
                const bool ok = vr && x < nx;
                vx[i] = ok ? kj[qq] : 0.f;
                vy[i] = ok ? kj[cs + qq] : 0.f;
                vz[i] = ok ? kj[2 * cs + qq] : 0.f;
            }
#pragma unroll
            for (int i = 0; i < IC; ++i) { ax[i] += c * vx[i]; ay[i] += c * vy[i]; az[i] += c * vz[i]; }
        }
    }
    // ---- stores
    float errmax = 0.f;
    float nmx[E], nmy[E], nmz[E];
#pragma unroll
    for (int i = 0; i < E; ++i) nmx[i] = nmy[i] = nmz[i] = 0.f;
#pragma unroll
    for (int i = 0; i < IC; ++i) {
        const int x = lg + P * i;
        if (!(vr && x < nx)) continue;
        const long long qq = (long long)r * nx + x;
        if (ko) { ko[qq] = kx[i]; ko[cs + qq] = ky[i]; ko[2 * cs + qq] = kz[i]; }
        if (stage) {
            const float inv = rsqrtf(ax[i] * ax[i] + ay[i] * ay[i] + az[i] * az[i]);
            nmx[i] = ax[i] * inv; nmy[i] = ay[i] * inv; nmz[i] = az[i] * inv;
            mo[qq] = nmx[i]; mo[cs + qq] = nmy[i]; mo[2 * cs + qq] = nmz[i];
        } else if (sa.mode == ROW_ERROR) {
            errmax = fmaxf(errmax, dtau * sqrtf(ax[i] * ax[i] + ay[i] * ay[i] + az[i] * az[i]));
        }
    }
    if (sa.mode == ROW_ERROR) {
        for (int off = 32; off > 0; off >>= 1) errmax = fmaxf(errmax, __shfl_xor(errmax, off));
        if ((tid & 63) == 0) wmax[tid >> 6] = errmax;
        __syncthreads();
        if (tid == 0) {
            float m = wmax[0];
            for (int w = 1; w < FRT / 64; ++w) m = fmaxf(m, wmax[w]);
            atomicMax(&st->err_bits, __float_as_uint(m));
        }
        return;
    }
    if (stage && p.demag_on) {
        __syncthreads();   // everyone has read xch
        R::forward_store(g, S, scr + gi * R::SC, tw, xch + pair * 2 * PX, nmx, nmy, nmz, kind, lg, gbase, r0, v0, v1);
    }
}

template <int PX, int E, bool XPER>
__global__ __launch_bounds__(FRT) void row_inv_fast(Grid g, Phys p, const float2* __restrict__ twx,
                                                    float2* __restrict__ S, StageArgs sa,
                                                    DevState* __restrict__ st) {
    extern __shared__ char dyn_lds[];
    row_inv_body<PX, E, XPER>(g, p, twx, S, sa, st, blockIdx.x, dyn_lds);
}

// ---------------------------------------------------------------------------
// columns (2D): y transform, product with the kernel spectrum, inverse
// ---------------------------------------------------------------------------
template <int L, int E, bool SPLIT>
struct ColFast {
    static constexpr int P = L / E;
    static constexpr int NH = SPLIT ? 2 : 1;
    static constexpr int W = (512 / (2 * NH * P)) > 0 ? 512 / (2 * NH * P) : 1;
    static constexpr int UNITS = W * NH * 2;
    static constexpr int NT = UNITS * P;
    static_assert(NT == 512, "column blocks have 512 threads");
    static constexpr int TM = SPLIT ? 2 : 1;
    using F = LaneFFT<L, E, TM, float2>;
    static constexpr int SC = LfScratch<L>::size;
    static constexpr int O_TW = 0;
    static constexpr int O_SCR = lds_align(O_TW + L * TM * 8);
    static constexpr int O_COMB = lds_align(O_SCR + UNITS * SC * 8);
    static constexpr int bytes() { return lds_align(O_COMB + (SPLIT ? W * 3 * L * 8 : 16)); }
};

template <int L, int E, bool SPLIT>
__device__ __forceinline__ void col2d_body(const Col2dArgs& a, DevState* __restrict__ st, int lb, char* lds) {
    using CF = ColFast<L, E, SPLIT>;
    using F = typename CF::F;
    constexpr int P = CF::P, NH = CF::NH, W = CF::W, NT = CF::NT;
    constexpr int TL = L * CF::TM;       // twiddle table length (= Py)
    float2* tw = (float2*)(lds + CF::O_TW);
    float2* scr = (float2*)(lds + CF::O_SCR);
    float2* comb = (float2*)(lds + CF::O_COMB);
    if (st->done) return;
    const int tid = threadIdx.x;
    const int u = tid / P, lg = tid % P;
    const int gbase = (tid & 63) - lg;
    const int grp = u % 2;               // 0: x and y components, 1: z
    const int h = (u / 2) % NH;          // frequency half
    const int w = u / (2 * NH);
    const int kx = lb * W + w;
    const bool packed = kx == 0;
    for (int m = tid; m < TL; m += NT) tw[m] = a.tw[m];
    const int ny = a.ny, Py = a.Py;
    const long long cs = (long long)ny * a.nkxp;
    const long long kcs = (long long)a.nkx_full * (Py / 2 + 1);
    const float* K = a.K;
    // kernel values of this lane's elements (mirror compressed along y;
    // the xy component is odd in ky)
    float ka0[E], ka1[E], ka2[E], kn0[E], kn1[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int pos = lg + P * i;
        const int ky = SPLIT ? 2 * pos + h : pos;
        const bool flip = ky > Py - ky;
        const int iy = flip ? Py - ky : ky;
        const long long o = (long long)kx * (Py / 2 + 1) + iy;
        const long long oN = (long long)(a.nkx_full - 1) * (Py / 2 + 1) + iy;
        if (grp == 0) {
            ka0[i] = K[o];                  // xx
            ka1[i] = K[kcs + o];            // yy
            const float kxy = K[3 * kcs + o];
            ka2[i] = flip ? -kxy : kxy;     // xy
            kn0[i] = packed ? K[oN] : 0.f;
            kn1[i] = packed ? K[kcs + oN] : 0.f;
        } else {
            ka0[i] = K[2 * kcs + o];        // zz
            kn0[i] = packed ? K[2 * kcs + oN] : 0.f;
            ka1[i] = ka2[i] = kn1[i] = 0.f;
        }
    }
    // input columns
    float2 x0[E], x1[E];
    const float2* c0 = a.S + (grp == 0 ? 0 : 2) * cs + kx;
    const float2* c1p = a.S + cs + kx;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int y = lg + P * i;
        x0[i] = mk2(0.f, 0.f);
        x1[i] = mk2(0.f, 0.f);
        if (y < ny) {
            x0[i] = c0[(long long)y * a.nkxp];
            if (grp == 0) x1[i] = c1p[(long long)y * a.nkxp];
        }
    }
    __syncthreads();   // twiddle table
    if (SPLIT && h == 1) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int y = lg + P * i;
            const float2 t = tw[y];
            x0[i] = cmul(x0[i], t);
            x1[i] = cmul(x1[i], t);
        }
    }
    float2* sc = scr + u * CF::SC;
    F::template run<false>(x0, sc, tw, lg);
    if (grp == 0) F::template run<false>(x1, sc, tw, lg);

    if (!packed) {
        if (grp == 0) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const float2 Mx = x0[i], My = x1[i];
                x0[i] = mk2(ka0[i] * Mx.x + ka2[i] * My.x, ka0[i] * Mx.y + ka2[i] * My.y);
                x1[i] = mk2(ka2[i] * Mx.x + ka1[i] * My.x, ka2[i] * Mx.y + ka1[i] * My.y);
            }
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i) x0[i] = mk2(ka0[i] * x0[i].x, ka0[i] * x0[i].y);
        }
    } else {
        // column 0 carries (kx = 0) + i (kx = Px/2): separate with the
        // Hermitian symmetry in ky, apply each column's (diagonal) kernel,
        // pack again.  The partner of ky is -ky: in the odd half of a split
        // axis it is position L-1-pos, otherwise (L-pos) mod L.
        float2 p0[E], p1[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            if (SPLIT && h == 1) {
                p0[i] = partner_odd<E, P>(x0, i, lg, gbase);
                p1[i] = partner_odd<E, P>(x1, i, lg, gbase);
            } else {
                p0[i] = partner_mirror<E, P>(x0, i, lg, gbase);
                p1[i] = partner_mirror<E, P>(x1, i, lg, gbase);
            }
        }
#pragma unroll
        for (int i = 0; i < E; ++i) {
            // A = (Z + conj Zp)/2 (kx = 0), B = (Z - conj Zp)/(2i) (kx = Px/2)
            const float2 z0 = x0[i], q0 = p0[i];
            float2 A = mk2(0.5f * (z0.x + q0.x), 0.5f * (z0.y - q0.y));
            float2 B = mk2(0.5f * (z0.y + q0.y), -0.5f * (z0.x - q0.x));
            A = mk2(ka0[i] * A.x, ka0[i] * A.y);
            B = mk2(kn0[i] * B.x, kn0[i] * B.y);
            x0[i] = mk2(A.x - B.y, A.y + B.x);
            if (grp == 0) {
                const float2 z1 = x1[i], q1 = p1[i];
                float2 C = mk2(0.5f * (z1.x + q1.x), 0.5f * (z1.y - q1.y));
                float2 D = mk2(0.5f * (z1.y + q1.y), -0.5f * (z1.x - q1.x));
                C = mk2(ka1[i] * C.x, ka1[i] * C.y);
                D = mk2(kn1[i] * D.x, kn1[i] * D.y);
                x1[i] = mk2(C.x - D.y, C.y + D.x);
            }
        }
    }
    F::template run<true>(x0, sc, tw, lg);
    if (grp == 0) F::template run<true>(x1, sc, tw, lg);

    const int cA = grp == 0 ? 0 : 2;
    if (SPLIT) {
        if (h == 1) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int y = lg + P * i;
                if (y < ny) {
                    const float2 t = cconj(tw[y]);
                    comb[(w * 3 + cA) * L + y] = cmul(x0[i], t);
                    if (grp == 0) comb[(w * 3 + 1) * L + y] = cmul(x1[i], t);
                }
            }
        }
        __syncthreads();
        if (h == 1) return;
    }
    float2* o0 = a.S + cA * cs + kx;
    float2* o1 = a.S + cs + kx;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int y = lg + P * i;
        if (y < ny) {
            float2 v0 = x0[i], v1 = x1[i];
            if (SPLIT) {
                const float2 c0v = comb[(w * 3 + cA) * L + y];
                v0 = mk2(v0.x + c0v.x, v0.y + c0v.y);
                if (grp == 0) { const float2 c1v = comb[(w * 3 + 1) * L + y]; v1 = mk2(v1.x + c1v.x, v1.y + c1v.y); }
            }
            o0[(long long)y * a.nkxp] = v0;
            if (grp == 0) o1[(long long)y * a.nkxp] = v1;
        }
    }
}

template <int L, int E, bool SPLIT>
__global__ __launch_bounds__(512) void col2d_fast(Col2dArgs a, DevState* __restrict__ st) {
    extern __shared__ char dyn_lds[];
    col2d_body<L, E, SPLIT>(a, st, xcd_remap_blocks(blockIdx.x, gridDim.x), dyn_lds);
}

// ---------------------------------------------------------------------------
// grouped launches: one launch runs a pass for many films of different
// sizes; block b works on film map[b].x, local block map[b].y
// ---------------------------------------------------------------------------
#define ROW_GROUP_SIZES(X) X(64, 8) X(128, 8) X(192, 12) X(256, 8) X(384, 12) X(512, 8) X(768, 12) X(1024, 16)
#define COL_GROUP_SIZES(X) X(32, 8) X(64, 8) X(96, 12) X(128, 8) X(192, 12) X(256, 8) X(384, 12) X(512, 8)

__global__ __launch_bounds__(FRT) void row_fwd_group(const FilmRow* __restrict__ films,
                                                     const int2* __restrict__ map) {
    extern __shared__ char dyn_lds[];
    const int2 m = map[blockIdx.x];
    const FilmRow& f = films[m.x];
    switch (f.g.Px) {
#define CASE(PX, E) case PX: row_fwd_body<PX, E>(f.g, f.twx, f.S, f.fa, f.st, m.y, dyn_lds); break;
        ROW_GROUP_SIZES(CASE)
#undef CASE
        default: break;
    }
}

__global__ __launch_bounds__(FRT) void row_inv_group(const FilmRow* __restrict__ films,
                                                     const int2* __restrict__ map) {
    extern __shared__ char dyn_lds[];
    const int2 m = map[blockIdx.x];
    const FilmRow& f = films[m.x];
    switch (f.g.Px) {
#define CASE(PX, E) case PX: row_inv_body<PX, E, false>(f.g, f.p, f.twx, f.S, f.sa, f.st, m.y, dyn_lds); break;
        ROW_GROUP_SIZES(CASE)
#undef CASE
        default: break;
    }
}

__global__ __launch_bounds__(512) void col_group(const FilmCol* __restrict__ films, const int2* __restrict__ map) {
    extern __shared__ char dyn_lds[];
    const int2 m = map[blockIdx.x];
    const FilmCol& f = films[m.x];
    switch (f.a.Py / 2) {
#define CASE(LL, E) case LL: col2d_body<LL, E, true>(f.a, f.st, m.y, dyn_lds); break;
        COL_GROUP_SIZES(CASE)
#undef CASE
        default: break;
    }
}

// kernels whose dynamic LDS may exceed 64 KB need the limit raised once
static hipError_t allow_lds(const void* kernel, int bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
#define ROW_SIZES(X) X(64, 8) X(128, 8) X(192, 12) X(256, 8) X(384, 12) X(512, 8) X(768, 12) X(1024, 16)
#define COL_SIZES(X) X(32, 8) X(64, 8) X(96, 12) X(128, 8) X(192, 12) X(256, 8) X(384, 12) X(512, 8)

bool fast2d_row_ok(int Px) {
#define CASE(PX, E) if (Px == PX) return true;
    ROW_SIZES(CASE)
#undef CASE
    return false;
}

bool fast2d_col_ok(int L, int split) {
    if (!split) return false;
#define CASE(LL, E) if (L == LL) return true;
    COL_SIZES(CASE)
#undef CASE
    return false;
}

hipError_t launch_row_fwd_fast(const Grid& g, const float2* twx, float2* S, const FwdArgs& fa,
                               DevState* st, hipStream_t s) {
    if (g.nx > g.Px || g.nkxp < g.Px / 2) return hipErrorInvalidValue;
#define CASE(PX, E)                                                                       \
    if (g.Px == PX) {                                                                     \
        constexpr int rows = 2 * RowFast<PX, E>::RP;                                      \
        constexpr int lds = RowFast<PX, E>::fwd_bytes();                                  \
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&row_fwd_fast<PX, E>), lds); \
        if (e_ != hipSuccess) return e_;                                                  \
        hipLaunchKernelGGL((row_fwd_fast<PX, E>), dim3((g.nrows + rows - 1) / rows), dim3(FRT), \
                           lds, s, g, twx, S, fa, st);                                    \
        return hipGetLastError();                                                         \
    }
    ROW_SIZES(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

hipError_t launch_row_inv_fast(const Grid& g, const Phys& p, const float2* twx, float2* S,
                               const StageArgs& sa, DevState* st, hipStream_t s) {
    if (g.nx > g.Px || g.nkxp < g.Px / 2 || sa.nk > kMaxK) return hipErrorInvalidValue;
    if ((sa.mode == ROW_STAGE || sa.mode == ROW_ERROR) && sa.nk < 1) return hipErrorInvalidValue;
#define CASE(PX, E)                                                                       \
    if (g.Px == PX) {                                                                     \
        constexpr int rows = 2 * RowFast<PX, E>::RP;                                      \
        const dim3 grid((g.nrows + rows - 1) / rows);                                     \
        constexpr int lds_p = RowFast<PX, E>::template inv_bytes<true>();                 \
        constexpr int lds_o = RowFast<PX, E>::template inv_bytes<false>();                \
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&row_inv_fast<PX, E, true>), lds_p); \
        if (e_ == hipSuccess) e_ = allow_lds(reinterpret_cast<const void*>(&row_inv_fast<PX, E, false>), lds_o); \
        if (e_ != hipSuccess) return e_;                                                  \
        if (g.nx == PX)                                                                   \
            hipLaunchKernelGGL((row_inv_fast<PX, E, true>), grid, dim3(FRT),              \
                               lds_p, s, g, p, twx, S, sa, st);                           \
        else if (2 * g.nx <= PX)                                                          \
            hipLaunchKernelGGL((row_inv_fast<PX, E, false>), grid, dim3(FRT),             \
                               lds_o, s, g, p, twx, S, sa, st);                           \
        else                                                                              \
            return hipErrorInvalidValue;                                                  \
        return hipGetLastError();                                                         \
    }
    ROW_SIZES(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

hipError_t launch_col2d_fast(const Col2dArgs& a, DevState* st, hipStream_t s) {
    if (a.Py % 2 || a.ny > a.Py / 2 || a.nkx_full != a.nkx + 1) return hipErrorInvalidValue;
    const int L = a.Py / 2;
#define CASE(LL, E)                                                                       \
    if (L == LL) {                                                                        \
        using CF = ColFast<LL, E, true>;                                                  \
        if (a.nkx % CF::W) return hipErrorInvalidValue;                                   \
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&col2d_fast<LL, E, true>), CF::bytes());                  \
        if (e_ != hipSuccess) return e_;                                                  \
        hipLaunchKernelGGL((col2d_fast<LL, E, true>), dim3(a.nkx / CF::W), dim3(CF::NT), CF::bytes(), s, a, st); \
        return hipGetLastError();                                                         \
    }
    COL_SIZES(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

// ---- grouped launchers ------------------------------------------------------------
int fast2d_row_rows_per_block(int Px) {
#define CASE(PX, E) if (Px == PX) return 2 * RowFast<PX, E>::RP;
    ROW_GROUP_SIZES(CASE)
#undef CASE
    return 0;
}
int fast2d_row_fwd_lds(int Px) {
#define CASE(PX, E) if (Px == PX) return RowFast<PX, E>::fwd_bytes();
    ROW_GROUP_SIZES(CASE)
#undef CASE
    return 0;
}
int fast2d_row_inv_lds(int Px) {
#define CASE(PX, E) if (Px == PX) return RowFast<PX, E>::template inv_bytes<false>();
    ROW_GROUP_SIZES(CASE)
#undef CASE
    return 0;
}
int fast2d_col_width(int L) {
#define CASE(LL, E) if (L == LL) return ColFast<LL, E, true>::W;
    COL_GROUP_SIZES(CASE)
#undef CASE
    return 0;
}
int fast2d_col_lds(int L) {
#define CASE(LL, E) if (L == LL) return ColFast<LL, E, true>::bytes();
    COL_GROUP_SIZES(CASE)
#undef CASE
    return 0;
}

hipError_t launch_row_fwd_group(const FilmRow* films, const int2* map, int nblocks, int lds, hipStream_t s) {
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&row_fwd_group), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(row_fwd_group, dim3(nblocks), dim3(FRT), lds, s, films, map);
    return hipGetLastError();
}
hipError_t launch_row_inv_group(const FilmRow* films, const int2* map, int nblocks, int lds, hipStream_t s) {
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&row_inv_group), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(row_inv_group, dim3(nblocks), dim3(FRT), lds, s, films, map);
    return hipGetLastError();
}
hipError_t launch_col_group(const FilmCol* films, const int2* map, int nblocks, int lds, hipStream_t s) {
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&col_group), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(col_group, dim3(nblocks), dim3(512), lds, s, films, map);
    return hipGetLastError();
}

}  // namespace llg
