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

#include <atomic>
#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>

#include "cell_physics.hpp"
#include "internal.hpp"
#include "lane_fft.hpp"

namespace llg {

namespace {

constexpr int kRowThreads = 768;   // launch bound of the row kernels (at most twelve wavefronts)

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
// rows: every length-PX row transform is split into NQ frequency classes
// (NQ = 2 or 4) of length LQ = PX/NQ, each computed by its own lane group,
// so a row pair occupies 3 NQ groups: (mx + i my of the first row, of the
// second row, mz of the first + i mz of the second) x (class q).  With
// W = exp(-2 pi i / PX) and w = exp(-2 pi i / NQ):
//   forward:  X[NQ j + q] = FFT_LQ( W^{nq} sum_r w^{rq} a_{n + r LQ} )[j]
//             (a_{n + r LQ} = 0 for r >= NQ/2 unless x is periodic)
//   inverse:  x_{n + r LQ} = sum_q w^{-rq} W^{-nq} IFFT_LQ(X[NQ j + q])[n]
// Spectrum columns kx < PX/2 are stored in the order col = q QC + j <->
// kx = NQ j + q, QC = PX/(2 NQ).  The Hermitian partner X[PX - k] of class q
// lies in class (NQ - q) mod NQ: within the group for q = 0 and q = NQ/2,
// in the partner group (through LDS) otherwise.  The per-cell work (fields,
// torque, stage combination) is spread over all threads of the block, cell
// by cell in row order.
// ---------------------------------------------------------------------------
constexpr int lds_align(int b) { return (b + 15) / 16 * 16; }
// the largest divisor of n that is at most c (chunks that tile n exactly)
constexpr int divisor_upto(int n, int c) {
    int d = c < n ? c : n;
    while (n % d != 0) --d;
    return d;
}

// first row of row block blk.  2D: blocks in row order.  3D (NAT) with whole
// blocks per z plane: z fastest, so the blocks one XCD runs one after
// another hold the same y rows of consecutive planes, and the z neighbours
// a block reads from global memory are the rows its neighbours stage at
// about the same time (L2 hits instead of a second pass over m)
template <bool NAT>
__device__ __forceinline__ int row_block_start(const Grid& g, int blk, int rows_per_block) {
    if (NAT && g.nz > 1 && g.ny % rows_per_block == 0) {
        const int z = blk % g.nz, yb = blk / g.nz;
        return z * g.ny + yb * rows_per_block;
    }
    return rows_per_block * blk;
}

// (row, x) of flat cell index e of rows of length nx, without an integer
// division: rnx = 1/nx in FP32 gives the row within one, fixed up exactly
// (e < 2^24)
__device__ __forceinline__ void split_cell(int e, int nx, float rnx, int& ri, int& x) {
    ri = (int)((float)e * rnx);
    x = e - ri * nx;
    if (x >= nx) { ++ri; x -= nx; }
    else if (x < 0) { --ri; x += nx; }
}

// a * exp(-2 pi i m / 4) (m taken mod 4)
__device__ __forceinline__ float2 rot4(float2 a, int m) {
    switch (m & 3) {
        case 0: return a;
        case 1: return mk2(a.y, -a.x);
        case 2: return mk2(-a.x, -a.y);
        default: return mk2(-a.y, a.x);
    }
}

template <int PX, int E2, int NQ>
struct RowSplit {
    static_assert(NQ == 2 || NQ == 4, "two or four frequency classes");
    static constexpr int LQ = PX / NQ;             // length of a class transform
    static constexpr int H = PX / 2;               // largest open-axis row length
    static constexpr int P = LQ / E2;              // lanes per class transform
    static constexpr int RP = 64 / P;              // row pairs per block
    static constexpr int NG = 3 * NQ * RP;         // lane groups per block
    static constexpr int NT = NG * P;              // threads per block
    static constexpr int QC = PX / (2 * NQ);       // stored columns per class
    static_assert(NT <= kRowThreads, "row blocks fit the launch bound");
    static constexpr int SC = LfScratch<LQ>::size;
    using F = LaneFFT<LQ, E2, NQ, float2>;
    // LDS (bytes): twiddles W^m (m < PX); the stage twiddle tables of the
    // class transforms; FFT scratch; the exchange of the inverse transforms
    // (inverse kernel only); staged m rows (with the y neighbours), which the
    // inverse kernel overwrites with the new m rows once every cell has its
    // field; reduction slots
    //
    // BIG (4096-point rows): there is no room for staged rows beside the
    // scratch.  The rows the forward transform reads and the new rows the
    // inverse kernel hands to it alias the scratch (behind a barrier), the
    // exchange aliases it too, and the inverse kernel reads the stage input
    // m and its neighbours from global memory instead of staged rows.
    static constexpr bool BIG = PX >= 4096;
    static constexpr int O_TW = 0;
    static constexpr int O_TWS = lds_align(PX * 8);
    static constexpr int O_SCR = lds_align(O_TWS + F::TWS_ALLOC * 8);
    static constexpr int SCR_BYTES = NG * SC * 8;
    static constexpr int O_M = BIG ? O_SCR : lds_align(O_SCR + SCR_BYTES);   // forward kernel: no exchange
    static constexpr int NR = 2 * RP + 2;
    // the exchange gets its own region unless that would not fit the LDS
    // (then it aliases the scratch, behind one more barrier)
    static constexpr int SEP_BYTES = lds_align(O_M + NG * LQ * 8) + NR * 3 * PX * 4 + 64;
    static constexpr bool XALIAS = BIG || SEP_BYTES > 160 * 1024;
    static constexpr int O_XCH = XALIAS ? O_SCR : O_M;
    static_assert(NG * LQ * 8 <= SCR_BYTES, "the exchange fits the scratch");
    static constexpr int O_MI = BIG ? O_SCR : XALIAS ? O_M : lds_align(O_M + NG * LQ * 8);
    template <bool XPER> static constexpr int nxm() { return XPER ? PX : H; }
    static constexpr int imax(int a, int b) { return a > b ? a : b; }
    template <bool XPER> static constexpr int fwd_bytes() {
        return BIG ? lds_align(O_SCR + imax(SCR_BYTES, 2 * RP * 3 * nxm<XPER>() * 4))
                   : lds_align(O_M + 2 * RP * 3 * nxm<XPER>() * 4);
    }
    template <bool XPER> static constexpr int o_nm() { return O_MI; }
    template <bool XPER> static constexpr int o_wmax() {
        return BIG ? lds_align(O_SCR + imax(SCR_BYTES, 2 * RP * 3 * nxm<XPER>() * 4))
                   : lds_align(O_MI + NR * 3 * nxm<XPER>() * 4);
    }
    template <bool XPER> static constexpr int inv_bytes() { return lds_align(o_wmax<XPER>() + 16 * 4); }

    // group gi -> (kind, class, pair), the pair fastest: the groups of one
    // wavefront share kind and class
    static __device__ __forceinline__ void group(int gi, int& kind, int& q, int& pair) {
        pair = gi % RP;
        const int kq = gi / RP;
        q = kq % NQ;
        kind = kq / NQ;
    }
    static __device__ __forceinline__ int group_of(int kind, int q, int pair) { return (kind * NQ + q) * RP + pair; }

    // forward transform of the block's rows, whose magnetisation sits in LDS
    // nm[row][c][x] (row stride 3 NXM), and store of the columns kx < PX/2;
    // scr is the block's scratch (every group calls this).  NAT: natural
    // layout instead (row-major rows of PX/2 + 1 columns kx = 0 ... PX/2, as
    // the 3D column passes read them)
    template <int NXM, bool NAT>
    static __device__ __forceinline__ void forward(const Grid& g, float2* __restrict__ S, float2* scr,
                                                   const float2* tw, const float2* tws, const float* nm, int kind, int q,
                                                   int pair, int lg, int gbase, int rb) {
        const int nx = g.nx;
        const int r0 = rb + 2 * pair;
        const bool v0 = r0 < g.nrows, v1 = r0 + 1 < g.nrows;
        const float* ra = nm + (2 * pair + (kind == 1 ? 1 : 0)) * 3 * NXM;
        const float* rz0 = nm + (2 * pair) * 3 * NXM + 2 * NXM;
        const float* rz1 = rz0 + 3 * NXM;
        const bool va = kind == 1 ? v1 : v0;
        auto at = [&](int n) -> float2 {
            if (n >= nx) return mk2(0.f, 0.f);
            if (kind < 2) return va ? mk2(ra[n], ra[NXM + n]) : mk2(0.f, 0.f);
            return mk2(v0 ? rz0[n] : 0.f, v1 ? rz1[n] : 0.f);
        };
        constexpr int NRIN = NXM == PX ? NQ : NQ / 2;    // nonzero input blocks of length LQ
        float2 z[E2];
#pragma unroll
        for (int i = 0; i < E2; ++i) {
            const int n = lg + P * i;
            float2 acc = at(n);
#pragma unroll
            for (int r = 1; r < NRIN; ++r) {
                const float2 v = rot4(at(n + r * LQ), (r * q * (4 / NQ)));
                acc.x += v.x; acc.y += v.y;
            }
            z[i] = q ? cmul(acc, tw[n * q]) : acc;
        }
        if constexpr (BIG) __syncthreads();   // every group has read the rows, which alias the scratch
        float2* own = scr + group_of(kind, q, pair) * SC;
        F::template run<false>(z, own, tws, lg);
        // partners in another class go through LDS (four classes only)
        const float2* pz = nullptr;
        if constexpr (NQ == 4) {
            __syncthreads();   // every class transform has left the scratch
#pragma unroll
            for (int i = 0; i < E2; ++i) own[lg + P * i] = z[i];
            __syncthreads();
            pz = scr + group_of(kind, (NQ - q) % NQ, pair) * SC;
        }
        const int cs = g.nrows * g.nkxp;
        const float2 zN = z[E2 / 2];   // X[PX/2]: class 0, lane 0
        float2* s0 = NAT ? S + r0 * g.nkxp : S + (r0 << g.tsh);
        float2* s1 = NAT ? s0 + g.nkxp : s0 + (1 << g.tsh);
#pragma unroll
        for (int i = 0; i < E2 / 2; ++i) {
            const int j = lg + P * i;
            const float2 zk = z[i];
            float2 zm;
            if (q == 0) zm = partner_mirror<E2, P>(z, i, lg, gbase);
            else if (2 * q == NQ) zm = partner_odd<E2, P>(z, i, lg, gbase);
            else zm = pz[LQ - 1 - j];
            float2 A = mk2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
            float2 B = mk2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
            if (!NAT && q == 0 && j == 0) {   // pack the real DC and Nyquist coefficients
                A = mk2(zk.x, zN.x);
                B = mk2(zk.y, zN.y);
            }
            const int col = NAT ? NQ * j + q : tile_index(0, q * QC + j, g.nrows, g.tsh);
            if (kind == 0) {
                if (v0) { s0[col] = A; s0[cs + col] = B; }
            } else if (kind == 1) {
                if (v1) { s1[col] = A; s1[cs + col] = B; }
            } else {
                if (v0) s0[2 * cs + col] = A;
                if (v1) s1[2 * cs + col] = B;
            }
        }
        if (NAT && q == 0 && lg == 0) {   // the real Nyquist coefficients, column PX/2
            const float2 A = mk2(zN.x, 0.f), B = mk2(zN.y, 0.f);
            const int col = PX / 2;
            if (kind == 0) {
                if (v0) { s0[col] = A; s0[cs + col] = B; }
            } else if (kind == 1) {
                if (v1) { s1[col] = A; s1[cs + col] = B; }
            } else {
                if (v0) s0[2 * cs + col] = A;
                if (v1) s1[2 * cs + col] = B;
            }
        }
    }
};

template <int PX, int E2, int NQ, bool XPER, bool NAT>
__device__ __forceinline__ void row_fwd_body(const Grid& g, const float2* __restrict__ twx,
                                             float2* __restrict__ S, const FwdArgs& fa,
                                             DevState* __restrict__ st, int blk, char* lds) {
    using R = RowSplit<PX, E2, NQ>;
    constexpr int NXM = R::template nxm<XPER>();
    constexpr int NT = R::NT;
    float2* tw = (float2*)(lds + R::O_TW);
    float2* tws = (float2*)(lds + R::O_TWS);
    float2* scr = (float2*)(lds + R::O_SCR);
    float* nm = (float*)(lds + R::O_M);
    if (st->done) return;
    const int tid = threadIdx.x;
    const int gi = R::P == 64 ? __builtin_amdgcn_readfirstlane(tid / R::P) : tid / R::P;
    const int lg = tid % R::P;
    int kind, q, pair;
    R::group(gi, kind, q, pair);
    const int gbase = (tid & 63) - lg;
    const int rb = row_block_start<NAT>(g, blk, 2 * R::RP);
    // the twiddle reads go out with the magnetisation reads below (one
    // memory round trip); their LDS stores follow those of the rows
    StagedCopy<PX, NT, float2> twc;
    twc.load(twx, tid);
    typename R::F::template TwFill<NT> twf;
    twf.load(twx, tid);
    const int cur = st->cur;
    const float c1 = st->dtau * fa.a1;
    const int cs = g.ncells;
    const float* mi = resolve(fa.m_in, cur);
    const float* m0 = resolve(fa.m0, cur);
    const float* k1 = resolve(fa.k1, cur);
    float* mo = resolve(fa.m_out, cur);
    const int nx = g.nx;
    const float rnx = 1.0f / (float)nx;
    const int nrow = min(2 * R::RP, g.nrows - rb);
    // one cell: the stage state (m0 + c1 k1, normalised) or m itself
    auto cell = [&](int qq, float& ax, float& ay, float& az) {
        if (fa.combine) {
            ax = m0[qq] + c1 * k1[qq];
            ay = m0[cs + qq] + c1 * k1[cs + qq];
            az = m0[2 * cs + qq] + c1 * k1[2 * cs + qq];
            const float inv = rsqrtf(ax * ax + ay * ay + az * az);
            ax *= inv; ay *= inv; az *= inv;
        } else {
            ax = mi[qq]; ay = mi[cs + qq]; az = mi[2 * cs + qq];
        }
    };
    if ((nx & 3) == 0 && (cs & 3) == 0) {
        // four consecutive cells per thread, 16-byte loads and stores (rows
        // and components start 16-byte aligned); the same arithmetic per
        // cell as `cell`
        const int n4 = nx >> 2;
        auto ld4 = [](const float* p, float (&o)[4]) {
            const float4 w = *reinterpret_cast<const float4*>(p);
            o[0] = w.x; o[1] = w.y; o[2] = w.z; o[3] = w.w;
        };
        for (int t = tid; t < nrow * n4; t += NT) {
            const int ri = t / n4, x = 4 * (t - ri * n4);
            const int qq = (rb + ri) * nx + x;
            float v[3][4];
            if (fa.combine) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float a[4], k[4];
                    ld4(m0 + c * cs + qq, a);
                    ld4(k1 + c * cs + qq, k);
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[c][i] = a[i] + c1 * k[i];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float inv = rsqrtf(v[0][i] * v[0][i] + v[1][i] * v[1][i] + v[2][i] * v[2][i]);
                    v[0][i] *= inv; v[1][i] *= inv; v[2][i] *= inv;
                }
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float a[4];
                    ld4(mi + c * cs + qq, a);
#pragma unroll
                    for (int i = 0; i < 4; ++i) v[c][i] = a[i];
                }
            }
            float* row = nm + ri * 3 * NXM;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float4 w = make_float4(v[c][0], v[c][1], v[c][2], v[c][3]);
                if (fa.combine) *reinterpret_cast<float4*>(mo + c * cs + qq) = w;
                *reinterpret_cast<float4*>(row + c * NXM + x) = w;
            }
        }
    } else {
        for (int e = tid; e < nrow * nx; e += NT) {
            int ri, x;
            split_cell(e, nx, rnx, ri, x);
            const int qq = (rb + ri) * nx + x;
            float ax, ay, az;
            cell(qq, ax, ay, az);
            if (fa.combine) { mo[qq] = ax; mo[cs + qq] = ay; mo[2 * cs + qq] = az; }
            float* row = nm + ri * 3 * NXM;
            row[x] = ax; row[NXM + x] = ay; row[2 * NXM + x] = az;
        }
    }
    twc.store(tw, tid);
    twf.store(tws, tid);
    __syncthreads();
    R::template forward<NXM, NAT>(g, S, scr, tw, tws, nm, kind, q, pair, lg, gbase, rb);
}

template <int PX, int E2, int NQ, bool XPER, bool NAT>
__global__ __launch_bounds__((RowSplit<PX, E2, NQ>::NT)) void row_fwd_fast(Grid g, const float2* __restrict__ twx,
                                                            float2* __restrict__ S, FwdArgs fa,
                                                            DevState* __restrict__ st) {
    extern __shared__ char dyn_lds[];
    row_fwd_body<PX, E2, NQ, XPER, NAT>(g, twx, S, fa, st, xcd_remap_blocks(blockIdx.x, gridDim.x), dyn_lds);
}

// exchange + anisotropy + applied + thermal field of cell x of a row whose
// magnetisation and that of its y neighbours sit in LDS (rm, rc, rp: rows
// y-1, y, y+1, component stride cstr; null where the neighbour is missing)
__device__ __forceinline__ void local_field_lds(const Grid& g, const Phys& p, const float* rm,
                                                const float* rc, const float* rp, int cstr, int r, int x,
                                                uint64_t step, float& hx, float& hy, float& hz) {
    const int nx = g.nx;
    const float mx = rc[x], my = rc[cstr + x], mz = rc[2 * cstr + x];
    float sx = 0.f, sy = 0.f, sz = 0.f;
    auto nb = [&](const float* row, int xx, float c) {
        sx += c * (row[xx] - mx);
        sy += c * (row[cstr + xx] - my);
        sz += c * (row[2 * cstr + xx] - mz);
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
    if (p.kc1 != 0.f || p.kc2 != 0.f) cubic_field(p, mx, my, mz, hx, hy, hz);
    hx += p.hz[0]; hy += p.hz[1]; hz += p.hz[2];
    if (p.sig_th != 0.f) {
        float ex, ey, ez;
        thermal_eta((uint32_t)((long long)r * nx + x), step, p.seed_lo, p.seed_hi, ex, ey, ez);
        hx += p.sig_th * ex; hy += p.sig_th * ey; hz += p.sig_th * ez;
    }
}

// the z neighbours of cell x of row r (in plane z) of a 3D grid (below:
// bit 0 of the returned mask, above: bit 1; absent at an open z face),
// loaded from global memory (component stride ncells) ahead of their use
__device__ __forceinline__ unsigned z_neighbours(const Grid& g, const Phys& p, const float* __restrict__ m, int r,
                                                 int z, int x, float (&lo)[3], float (&up)[3]) {
    if (p.cex[2] == 0.f || g.nz < 2) return 0u;
    const long long cs = g.ncells;
    const long long i = (long long)r * g.nx + x, sl = (long long)g.ny * g.nx;
    long long il = -1, iu = -1;
    if (z > 0) il = i - sl; else if (g.pbc[2]) il = i + (long long)(g.nz - 1) * sl;
    if (z < g.nz - 1) iu = i + sl; else if (g.pbc[2]) iu = i - (long long)(g.nz - 1) * sl;
    unsigned mask = 0u;
    if (il >= 0) { lo[0] = m[il]; lo[1] = m[cs + il]; lo[2] = m[2 * cs + il]; mask |= 1u; }
    if (iu >= 0) { up[0] = m[iu]; up[1] = m[cs + iu]; up[2] = m[2 * cs + iu]; mask |= 2u; }
    return mask;
}

// exchange terms of a 3D grid that the staged rows of a block do not hold:
// the periodic y wrap at the edges of a z plane (read from global memory)
// and the z neighbours (from z_neighbours)
__device__ __forceinline__ void exchange_wrap_z(const Grid& g, const Phys& p, const float* __restrict__ m, int r,
                                                int x, int y, float mx, float my, float mz, const float (&lo)[3],
                                                const float (&up)[3], unsigned zmask, float& hx, float& hy,
                                                float& hz) {
    const long long cs = g.ncells;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    auto nb = [&](int rr, float c) {
        const long long i = (long long)rr * g.nx + x;
        sx += c * (m[i] - mx);
        sy += c * (m[cs + i] - my);
        sz += c * (m[2 * cs + i] - mz);
    };
    if (p.cex[1] != 0.f && g.ny > 1 && g.pbc[1]) {
        if (y == 0) nb(r + g.ny - 1, p.cex[1]);
        if (y == g.ny - 1) nb(r - (g.ny - 1), p.cex[1]);
    }
    const float c = p.cex[2];
    if (zmask & 1u) { sx += c * (lo[0] - mx); sy += c * (lo[1] - my); sz += c * (lo[2] - mz); }
    if (zmask & 2u) { sx += c * (up[0] - mx); sy += c * (up[1] - my); sz += c * (up[2] - mz); }
    hx += sx; hy += sy; hz += sz;
}

// XPER: the x axis is periodic (nx == PX), else nx <= PX/2
template <int PX, int E2, int NQ, bool XPER, bool NAT>
__device__ __forceinline__ void row_inv_body(const Grid& g, const Phys& p, const float2* __restrict__ twx,
                                             float2* __restrict__ S, const StageArgs& sa,
                                             DevState* __restrict__ st, int blk, char* lds) {
    using R = RowSplit<PX, E2, NQ>;
    using F = typename R::F;
    constexpr bool BIG = R::BIG;
    static_assert(!(BIG && NAT), "4096-point rows serve 2D films only");
    constexpr int P = R::P, RP = R::RP, LQ = R::LQ, QC = R::QC, NT = R::NT;
    constexpr int NXM = R::template nxm<XPER>();
    float2* tw = (float2*)(lds + R::O_TW);
    float2* tws = (float2*)(lds + R::O_TWS);
    float2* scr = (float2*)(lds + R::O_SCR);
    float2* xch = (float2*)(lds + R::O_XCH);
    float* mrow = (float*)(lds + R::O_MI);
    float* nm = (float*)(lds + R::template o_nm<XPER>());   // aliases mrow
    float* wmax = (float*)(lds + R::template o_wmax<XPER>());
    if (st->done) return;
    const int tid = threadIdx.x;
    // a group that fills its wavefront: the group index is wave-uniform
    const int gi = P == 64 ? __builtin_amdgcn_readfirstlane(tid / P) : tid / P;
    const int lg = tid % P;
    int kind, q, pair;
    R::group(gi, kind, q, pair);
    const int gbase = (tid & 63) - lg;
    const int rb = row_block_start<NAT>(g, blk, 2 * RP);   // first row of the block
    const int r0 = rb + 2 * pair;
    const bool v0 = r0 < g.nrows, v1 = r0 + 1 < g.nrows;
    const int cur = st->cur;
    const float dtau = st->dtau;
    const uint64_t step = (uint64_t)st->step;
    const int nx = g.nx, ny = g.ny;
    // (y, z) of the block's row rb + ri: one division per block, then steps
    const int y0 = rb % ny, z0 = rb / ny;
    auto plane_of = [&](int ri, int& y, int& z) {
        y = y0 + ri;
        z = z0;
        while (y >= ny) { y -= ny; ++z; }
    };
    const int cs = g.ncells;
    const float* mi = resolve(sa.m_in, cur);
    const float* m0 = resolve(sa.m0, cur);
    float* mo = resolve(sa.m_out, cur);
    float* ko = resolve(sa.k_out, cur);
    const bool stage = sa.mode == ROW_STAGE;
    const bool errm = sa.mode == ROW_ERROR || ((stage || sa.mode == ROW_KONLY) && sa.with_err);

    // ---- global reads.  Every read of the prologue is issued before the
    // first one is used (one memory round trip): the twiddles; the staged m
    // rows rb-1 .. rb+2RP (y neighbours wrap on a periodic y axis); this
    // group's class of the spectrum; m0 and the first round of the earlier
    // stages' k at this thread's cells; the 3D z neighbours.  Then the LDS
    // stores, the spectrum fix-ups and the k sums.
    StagedCopy<PX, NT, float2> twc;
    twc.load(twx, tid);
    typename F::template TwFill<NT> twf;
    twf.load(twx, tid);
    // staged row rq holds grid row rb - 1 + rq; NAT (3D): the halo rows serve
    // only as in-plane neighbours, the periodic y wrap and the z neighbours
    // come from global memory
    auto staged_row = [&](int rq, bool& ok) {
        int row = rb - 1 + rq;
        ok = row >= 0 && row < g.nrows;
        if (!NAT && g.pbc[1]) { row = row < 0 ? row + ny : (row >= ny ? row - ny : row); ok = true; }
        return row;
    };
    // 16-byte loads where every (row, component) run of nx floats starts
    // 16-byte aligned; BIG: no staged rows (the per-cell work reads m from
    // global memory)
    const bool vec4 = !BIG && (nx & 3) == 0 && (cs & 3) == 0;
    const int n4 = nx >> 2;
    constexpr int ITR = BIG ? 1 : (R::NR * 3 * (NXM / 4) + NT - 1) / NT;
    constexpr bool ROW1 = ITR <= 8;   // the staged rows in the first round
    auto row_load = [&](int t, float4& v, int& d) {
        d = -1;
        if (t >= R::NR * 3 * n4) return;
        const int rq = t / (3 * n4), rem = t - rq * 3 * n4;
        const int c = rem / n4, x4 = rem - c * n4;
        bool ok;
        const int row = staged_row(rq, ok);
        v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ok) v = *reinterpret_cast<const float4*>(mi + (size_t)c * cs + (size_t)row * nx + 4 * x4);
        d = rq * 3 * NXM + c * NXM + 4 * x4;
    };
    float4 rv[ROW1 ? ITR : 1];
    int rd[ROW1 ? ITR : 1];
    if (ROW1 && vec4) {
#pragma unroll
        for (int it = 0; it < (ROW1 ? ITR : 1); ++it) row_load(tid + it * NT, rv[it], rd[it]);
    }
    // X[k], k = NQ j + q, from the stored columns kx < PX/2 and the
    // Hermitian symmetry X[PX - k] = conj X[k] of a real row (class
    // (NQ - q) mod NQ, index LQ - j for q = 0, LQ - 1 - j otherwise): the
    // loads (in the first round unless E2 > 8), then the conjugations and
    // the packed DC / Nyquist column
    const int scs = g.nrows * g.nkxp;
    const float2* sa_ = nullptr;
    const float2* sb_ = nullptr;
    if (p.demag_on) {
        const int rs0 = NAT ? r0 * g.nkxp : (r0 << g.tsh);
        const int rs1 = NAT ? (r0 + 1) * g.nkxp : ((r0 + 1) << g.tsh);
        if (kind == 0) { if (v0) { sa_ = S + rs0; sb_ = sa_ + scs; } }
        else if (kind == 1) { if (v1) { sa_ = S + rs1; sb_ = sa_ + scs; } }
        else {
            if (v0) sa_ = S + 2 * scs + rs0;
            if (v1) sb_ = S + 2 * scs + rs1;
        }
    }
    auto spec_col = [&](int i) {
        const int j = lg + P * i;
        const int k = NQ * j + q;
        const bool up = k > PX / 2;
        if (NAT) return up ? PX - k : k;   // natural layout: kx = 0 ... PX/2 stored, the rest conjugate
        if (k == 0 || k == PX / 2) return 0;
        const int sc = q == 0 ? (up ? LQ - j : j) : (up ? (NQ - q) * QC + LQ - 1 - j : q * QC + j);
        return tile_index(0, sc, g.nrows, g.tsh);
    };
    auto spec_fix = [&](int i, float2 A, float2 B) {
        const int k = NQ * (lg + P * i) + q;
        if (!NAT && (k == 0 || k == PX / 2)) {
            const bool nyq = k != 0;
            A = mk2(nyq ? A.y : A.x, 0.f);
            B = mk2(nyq ? B.y : B.x, 0.f);
        } else if (k > PX / 2) {
            A.y = -A.y;
            B.y = -B.y;
        }
        return mk2(A.x - B.y, A.y + B.x);
    };
    constexpr int CZ = divisor_upto(E2, 8);
    constexpr bool Z1 = CZ == E2;
    float2 za[CZ], zb[CZ];
    auto spec_load = [&](int i0) {
#pragma unroll
        for (int ii = 0; ii < CZ; ++ii) {
            const int col = spec_col(i0 + ii);
            za[ii] = sa_ ? sa_[col] : mk2(0.f, 0.f);
            zb[ii] = sb_ ? sb_[col] : mk2(0.f, 0.f);
        }
    };
    if (p.demag_on) spec_load(0);
    // the parts of the stage combination that do not depend on this stage's
    // k: m0 + dtau sum_{j<s} a_j k_j and sum_{j<s} e_j k_j at this thread's
    // cells.  Up to eight cells per thread: KB of the k's for ITC cells per
    // memory round trip (at most KBUD values in flight), accumulated in
    // stage order.  More cells (4096-point periodic rows): one after another.
    constexpr int MAXIT = (2 * RP * NXM + NT - 1) / NT;
    const int nrow = min(2 * RP, g.nrows - rb);
    const int ncb = nrow * nx;
    const float rnx = 1.0f / (float)nx;
    float px_[MAXIT], py_[MAXIT], pz_[MAXIT], ex_[MAXIT], ey_[MAXIT], ez_[MAXIT];
    float mnx[MAXIT], mny[MAXIT], mnz[MAXIT];   // the new stage state, held until the staged rows are free
    constexpr int KP = kMaxK - 1;
    const int nprev = (stage || errm) ? sa.nk - 1 : 0;
    auto used = [&](int j) {
        return j < nprev && ((stage && dtau * sa.a[j] != 0.f) || (errm && sa.e[j] != 0.f));
    };
    constexpr bool KSER = MAXIT > 8;
    // values in flight per round: fewer in 3D, whose blocks share a compute
    // unit three at a time (and whose integrators combine few stages)
    constexpr int KBUD = NAT ? 3 * MAXIT : 36;
    constexpr int ITC = KSER ? 1 : (MAXIT * 3 <= KBUD ? MAXIT : KBUD / 3);
    constexpr int KB0 = KBUD / (3 * ITC);
    constexpr int KB = KB0 < 1 ? 1 : (KB0 > KP ? KP : KB0);
    int qq_[KSER ? 1 : MAXIT];   // this thread's cells (-1: none)
    auto k_load = [&](int i0, int j0, float (&kv)[KB][ITC][3]) {
#pragma unroll
        for (int jj = 0; jj < KB && j0 + jj < KP; ++jj) {
            const int j = j0 + jj;
            if (!used(j)) continue;
            const float* __restrict__ kj = resolve(sa.kprev[j], cur);
#pragma unroll
            for (int ii = 0; ii < ITC && i0 + ii < MAXIT; ++ii) {
                const int qq = qq_[KSER ? 0 : i0 + ii];
                if (qq < 0) continue;
                kv[jj][ii][0] = kj[qq]; kv[jj][ii][1] = kj[cs + qq]; kv[jj][ii][2] = kj[2 * cs + qq];
            }
        }
    };
    auto k_add = [&](int i0, int j0, const float (&kv)[KB][ITC][3]) {
#pragma unroll
        for (int jj = 0; jj < KB && j0 + jj < KP; ++jj) {
            const int j = j0 + jj;
            if (!used(j)) continue;
            const float ca = stage ? dtau * sa.a[j] : 0.f;
            const float ce = errm ? sa.e[j] : 0.f;
#pragma unroll
            for (int ii = 0; ii < ITC && i0 + ii < MAXIT; ++ii) {
                const int it = i0 + ii;
                if (qq_[KSER ? 0 : it] < 0) continue;
                const float vx = kv[jj][ii][0], vy = kv[jj][ii][1], vz = kv[jj][ii][2];
                if (ca != 0.f) { px_[it] += ca * vx; py_[it] += ca * vy; pz_[it] += ca * vz; }
                if (ce != 0.f) { ex_[it] += ce * vx; ey_[it] += ce * vy; ez_[it] += ce * vz; }
            }
        }
    };
    // with the spectrum in several rounds (E2 > 8) the stage combination is
    // read after it instead
    constexpr bool EARLYK = Z1 && !KSER;
    float kv0[KB][ITC][3];
    auto m0_load = [&]() {
#pragma unroll
        for (int it = 0; it < MAXIT; ++it) {
            px_[it] = py_[it] = pz_[it] = ex_[it] = ey_[it] = ez_[it] = 0.f;
            qq_[it] = -1;
            const int e = tid + it * NT;
            if (e >= ncb || !(stage || errm)) continue;
            int ri, x;
            split_cell(e, nx, rnx, ri, x);
            const int qq = (rb + ri) * nx + x;
            qq_[it] = qq;
            if (stage) { px_[it] = m0[qq]; py_[it] = m0[cs + qq]; pz_[it] = m0[2 * cs + qq]; }
        }
    };
    if constexpr (KSER) {
#pragma unroll
        for (int it = 0; it < MAXIT; ++it) {
            px_[it] = py_[it] = pz_[it] = ex_[it] = ey_[it] = ez_[it] = 0.f;
            const int e = tid + it * NT;
            if (e >= ncb || !(stage || errm)) continue;
            int ri, x;
            split_cell(e, nx, rnx, ri, x);
            const int qq = (rb + ri) * nx + x;
            if (stage) { px_[it] = m0[qq]; py_[it] = m0[cs + qq]; pz_[it] = m0[2 * cs + qq]; }
            for (int j = 0; j < nprev; ++j) {
                if (!used(j)) continue;
                const float ca = stage ? dtau * sa.a[j] : 0.f;
                const float ce = errm ? sa.e[j] : 0.f;
                const float* __restrict__ kj = resolve(sa.kprev[j], cur);
                const float vx = kj[qq], vy = kj[cs + qq], vz = kj[2 * cs + qq];
                if (ca != 0.f) { px_[it] += ca * vx; py_[it] += ca * vy; pz_[it] += ca * vz; }
                if (ce != 0.f) { ex_[it] += ce * vx; ey_[it] += ce * vy; ez_[it] += ce * vz; }
            }
        }
    } else if constexpr (EARLYK) {
        m0_load();
        k_load(0, 0, kv0);
    }
    // 3D: the z neighbours of this thread's cells
    float zlo[MAXIT][3], zup[MAXIT][3];
    unsigned zmask[MAXIT];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        zmask[it] = 0u;
        if constexpr (NAT) {
            const int e = tid + it * NT;
            if (e < ncb) {
                int ri, x;
                split_cell(e, nx, rnx, ri, x);
                int yr, zr;
                plane_of(ri, yr, zr);
                zmask[it] = z_neighbours(g, p, mi, rb + ri, zr, x, zlo[it], zup[it]);
            }
        }
    }
    // ---- LDS stores and fix-ups
    twc.store(tw, tid);
    twf.store(tws, tid);
    if (ROW1 && vec4) {
#pragma unroll
        for (int it = 0; it < (ROW1 ? ITR : 1); ++it)
            if (rd[it] >= 0) *reinterpret_cast<float4*>(mrow + rd[it]) = rv[it];
    } else if (vec4) {
        // longest staged rows: rounds of eight loads
#pragma unroll
        for (int i0 = 0; i0 < ITR; i0 += 8) {
            float4 v[8];
            int d[8];
#pragma unroll
            for (int ii = 0; ii < 8; ++ii) {
                d[ii] = -1;
                if (i0 + ii < ITR) row_load(tid + (i0 + ii) * NT, v[ii], d[ii]);
            }
#pragma unroll
            for (int ii = 0; ii < 8; ++ii)
                if (d[ii] >= 0) *reinterpret_cast<float4*>(mrow + d[ii]) = v[ii];
        }
    } else if (!BIG) {
        for (int rq = 0; rq < R::NR; ++rq) {
            bool ok;
            const int row = staged_row(rq, ok);
            const float* src = mi + row * nx;
            float* dst = mrow + rq * 3 * NXM;
            for (int t = tid; t < 3 * nx; t += NT) {
                const int c = t >= nx ? (t >= 2 * nx ? 2 : 1) : 0;
                const int x = t - c * nx;
                dst[c * NXM + x] = ok ? src[c * cs + x] : 0.f;
            }
        }
    }
    float2 z[E2];
#pragma unroll
    for (int i = 0; i < E2; ++i) z[i] = mk2(0.f, 0.f);
    if (p.demag_on) {
#pragma unroll
        for (int i0 = 0; i0 < E2; i0 += CZ) {
            if (i0 > 0) spec_load(i0);   // the first round was read above
#pragma unroll
            for (int ii = 0; ii < CZ; ++ii) z[i0 + ii] = spec_fix(i0 + ii, za[ii], zb[ii]);
        }
    }
    // the earlier stages' k: the first round (read above), then the rest
    if constexpr (!KSER) {
        if constexpr (!EARLYK) m0_load();
#pragma unroll
        for (int i0 = 0; i0 < MAXIT; i0 += ITC) {
#pragma unroll
            for (int j0 = 0; j0 < KP; j0 += KB) {
                if (EARLYK && i0 == 0 && j0 == 0) {
                    k_add(0, 0, kv0);
                    continue;
                }
                if (j0 >= nprev) break;
                float kv[KB][ITC][3];
                k_load(i0, j0, kv);
                k_add(i0, j0, kv);
            }
        }
    }
    __syncthreads();   // twiddles and staged rows
    if (p.demag_on) F::template run<true>(z, scr + gi * R::SC, tws, lg);
    if constexpr (R::XALIAS) __syncthreads();   // every transform has left the scratch
    if (p.demag_on) {
        float2* xo = xch + ((pair * 3 + kind) * NQ + q) * LQ;
#pragma unroll
        for (int i = 0; i < E2; ++i) {
            const int n = lg + P * i;
            xo[n] = q ? cmul(z[i], cconj(tw[n * q])) : z[i];
        }
    }
    __syncthreads();

    // ---- per cell: field, torque, stage combination
    float errmax = 0.f;
    bool bad = false;
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int e = tid + it * NT;
        if (e >= ncb) continue;
        int ri, x;
        split_cell(e, nx, rnx, ri, x);
        const int pr = ri >> 1, rr = ri & 1;
        const int r = rb + ri;
        int y, zpl;
        plane_of(ri, y, zpl);
        // the cell's row (component stride cstr) and its y neighbours: staged
        // rows, or (BIG) the stage input in global memory
        const int cstr = BIG ? cs : NXM;
        const float* rc = BIG ? mi + (size_t)r * nx : mrow + (ri + 1) * 3 * NXM;
        const float* rm = nullptr;
        const float* rp = nullptr;
        if (BIG) {
            if (ny > 1 && y > 0) rm = rc - nx; else if (ny > 1 && g.pbc[1]) rm = rc + (size_t)(ny - 1) * nx;
            if (ny > 1 && y < ny - 1) rp = rc + nx; else if (ny > 1 && g.pbc[1]) rp = rc - (size_t)(ny - 1) * nx;
        } else {
            rm = (ny > 1 && (y > 0 || g.pbc[1])) ? rc - 3 * NXM : nullptr;
            rp = (ny > 1 && (y < ny - 1 || g.pbc[1])) ? rc + 3 * NXM : nullptr;
        }
        float hx = 0.f, hy = 0.f, hz = 0.f;
        if (p.demag_on) {
            // x = n + r LQ: sum over the classes of w^{-rq} times the
            // pre-twiddled class results
            const int r = x / LQ, n = x - r * LQ;
            const float2* xa = xch + ((pr * 3 + rr) * NQ) * LQ;
            const float2* xz = xch + ((pr * 3 + 2) * NQ) * LQ;
            float2 sa2 = xa[n], sz2 = xz[n];
#pragma unroll
            for (int cq = 1; cq < NQ; ++cq) {
                const int m = -(r * cq * (4 / NQ));
                const float2 u = rot4(xa[cq * LQ + n], m), v = rot4(xz[cq * LQ + n], m);
                sa2.x += u.x; sa2.y += u.y; sz2.x += v.x; sz2.y += v.y;
            }
            hx = sa2.x; hy = sa2.y;
            hz = rr ? sz2.y : sz2.x;
        }
        if constexpr (NAT) {
            // x and in-plane y neighbours from the staged rows (the block's
            // rows and one halo row each side, consecutive in memory)
            const float* rmn = (ny > 1 && y > 0) ? rc - 3 * NXM : nullptr;
            const float* rpn = (ny > 1 && y < ny - 1) ? rc + 3 * NXM : nullptr;
            local_field_lds(g, p, rmn, rc, rpn, NXM, r, x, step, hx, hy, hz);
            exchange_wrap_z(g, p, mi, r, x, y, rc[x], rc[NXM + x], rc[2 * NXM + x], zlo[it], zup[it], zmask[it], hx,
                            hy, hz);
        } else {
            local_field_lds(g, p, rm, rc, rp, cstr, r, x, step, hx, hy, hz);
        }
        const int qq = r * nx + x;
        if (sa.mode == ROW_EVAL) {
            float* h = sa.h_out;
            h[qq] = hx * p.Ms; h[cs + qq] = hy * p.Ms; h[2 * cs + qq] = hz * p.Ms;
            bad |= !(isfinite(hx) && isfinite(hy) && isfinite(hz));
            continue;
        }
        float kx, ky, kz;
        ll_torque(p, rc[x], rc[cstr + x], rc[2 * cstr + x], hx, hy, hz, kx, ky, kz);
        if (p.stt_on) {
            // D = (j . grad) m from the staged rows: x neighbours in the row,
            // y neighbours in the rows above and below (the cell itself where
            // a free surface has none)
            const float mx = rc[x], my = rc[cstr + x], mz = rc[2 * cstr + x];
            float Dx = 0.f, Dy = 0.f, Dz = 0.f;
            if (NAT) {
                stt_gradient(g, p, mi, r, x, mx, my, mz, Dx, Dy, Dz);
            } else if (p.cj[0] != 0.f && nx > 1) {
                const int xu = x < nx - 1 ? x + 1 : (g.pbc[0] ? 0 : x);
                const int xd = x > 0 ? x - 1 : (g.pbc[0] ? nx - 1 : x);
                Dx += p.cj[0] * (rc[xu] - rc[xd]);
                Dy += p.cj[0] * (rc[cstr + xu] - rc[cstr + xd]);
                Dz += p.cj[0] * (rc[2 * cstr + xu] - rc[2 * cstr + xd]);
            }
            if (!NAT && p.cj[1] != 0.f && ny > 1) {
                const float* ru = rp ? rp : rc;
                const float* rd = rm ? rm : rc;
                Dx += p.cj[1] * (ru[x] - rd[x]);
                Dy += p.cj[1] * (ru[cstr + x] - rd[cstr + x]);
                Dz += p.cj[1] * (ru[2 * cstr + x] - rd[2 * cstr + x]);
            }
            stt_torque(p, mx, my, mz, Dx, Dy, Dz, kx, ky, kz);
        }
        bad |= !(isfinite(kx) && isfinite(ky) && isfinite(kz));
        if (ko) { ko[qq] = kx; ko[cs + qq] = ky; ko[2 * cs + qq] = kz; }
        if (sa.mode == ROW_KONLY) {
            if (errm) errmax = fmaxf(errmax, sqrtf(kx * kx + ky * ky + kz * kz));
            continue;
        }
        // combination with the earlier stages (stage input and/or error)
        float ax = 0.f, ay = 0.f, az = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
        if (stage) {
            const float c = dtau * sa.a[sa.nk - 1];
            ax = px_[it] + c * kx; ay = py_[it] + c * ky; az = pz_[it] + c * kz;
        }
        if (errm) {
            const float c = sa.e[sa.nk - 1];
            ex = ex_[it] + c * kx; ey = ey_[it] + c * ky; ez = ez_[it] + c * kz;
        }
        if (stage) {
            const float inv = rsqrtf(ax * ax + ay * ay + az * az);
            ax *= inv; ay *= inv; az *= inv;
            mo[qq] = ax; mo[cs + qq] = ay; mo[2 * cs + qq] = az;
            mnx[it] = ax; mny[it] = ay; mnz[it] = az;
        }
        if (errm) errmax = fmaxf(errmax, dtau * sqrtf(ex * ex + ey * ey + ez * ez));
    }
    if (bad) atomicOr(&st->health, 1);
    if (errm) {
        for (int off = 32; off > 0; off >>= 1) errmax = fmaxf(errmax, __shfl_xor(errmax, off));
        if ((tid & 63) == 0) wmax[tid >> 6] = errmax;
        __syncthreads();
        if (tid == 0) {
            float m = wmax[0];
            for (int w = 1; w < NT / 64; ++w) m = fmaxf(m, wmax[w]);
            atomicMax(&st->err_bits, __float_as_uint(m));
        }
        if (!stage) return;
    }
    if (stage && p.demag_on && !sa.skip_fwd) {
        __syncthreads();   // staged rows and exchange no longer read
#pragma unroll
        for (int it = 0; it < MAXIT; ++it) {
            const int e = tid + it * NT;
            if (e >= ncb) continue;
            int ri, x;
            split_cell(e, nx, rnx, ri, x);
            float* row = nm + ri * 3 * NXM;
            row[x] = mnx[it]; row[NXM + x] = mny[it]; row[2 * NXM + x] = mnz[it];
        }
        __syncthreads();   // new rows complete
        R::template forward<NXM, NAT>(g, S, scr, tw, tws, nm, kind, q, pair, lg, gbase, rb);
    }
}

template <int PX, int E2, int NQ, bool XPER, bool NAT>
__global__ __launch_bounds__((RowSplit<PX, E2, NQ>::NT)) void row_inv_fast(Grid g, Phys p, const float2* __restrict__ twx,
                                                            float2* __restrict__ S, StageArgs sa,
                                                            DevState* __restrict__ st) {
    extern __shared__ char dyn_lds[];
    row_inv_body<PX, E2, NQ, XPER, NAT>(g, p, twx, S, sa, st, xcd_remap_blocks(blockIdx.x, gridDim.x), dyn_lds);
}

// ---------------------------------------------------------------------------
// columns (2D): y transform, product with the kernel spectrum, inverse.
// The y axis is zero padded (Py = 2L, ny <= L), so every column transform
// is split into NQ frequency classes of length LC = Py/NQ (class q holds
// ky = NQ j + q), as the rows are.  One lane group per (component, class,
// column): the x and y groups of a class swap their spectra through LDS
// for the off-diagonal xy term, the packed column finds its Hermitian
// partners (class (NQ - q) mod NQ) there too; after the inverse every class
// leaves W^{-nq} times its result in LDS and the groups of the first NQ/2
// classes each assemble and store one block of LC outputs.
// ---------------------------------------------------------------------------
constexpr int kColThreads = 768;   // launch bound of the column kernels

template <int L, int E, int NQ>
struct ColSplit {
    static_assert(NQ == 2 || NQ == 4, "two or four frequency classes");
    static constexpr int PY = 2 * L;
    static constexpr int LC = PY / NQ;              // length of a class transform
    static constexpr int P = LC / E;                // lanes per class transform
    static constexpr int W = 64 / P;                // columns per block
    static constexpr int SC = LfScratch<LC>::size;
    static constexpr int KL = L + 1;                // kernel entries per column (ky = 0 .. L)
    // BIG (half lengths of 2048: 16 or more elements per lane, one column
    // per wavefront group): the three components of a column do not share a
    // block.  A block holds either the x and y components of one column
    // (they meet in the xy product) or the z components of two columns, so
    // that blocks stay at 2 NQ wavefronts and a wavefront may use 256
    // registers.  No block-shared copies of the spectrum and kernel columns
    // (every lane reads its own values from global memory), and the spectrum
    // exchange aliases the FFT scratch behind extra barriers.
    static constexpr bool BIG = L >= 2048;
    static_assert(!BIG || W == 1, "one column per lane group on the longest columns");
    static constexpr int NG = BIG ? 2 * NQ : 3 * NQ * W;   // lane groups per block
    static constexpr int NT = NG * P;               // threads per block
    static_assert(W >= 1 && NT <= kColThreads, "column blocks fit the launch bound");
    using F = LaneFFT<LC, E, NQ, float2>;
    static_assert(SC >= LC, "the exchange fits the scratch");
    // blocks of a launch over nkx stored columns
    static constexpr int blocks(int nkx) { return BIG ? nkx + nkx / 2 : nkx / W; }
    // LDS (bytes): the stage twiddle tables; the block's kernel columns
    // [w][xx, yy, zz, xy][ky] and the Nyquist column's [xx, yy, zz][ky]
    // (block 0 only: the packed column); its spectrum columns [c][w][y]
    // (y < ny); FFT scratch; the spectrum exchange (reused for the inverse
    // results after a barrier)
    static constexpr int O_TWS = 0;
    static constexpr int O_KST = lds_align(F::TWS_ALLOC * 8);
    static constexpr int O_XST = BIG ? O_KST : lds_align(O_KST + (W * 4 + 3) * KL * 4);
    static constexpr int O_SCR = BIG ? O_KST : lds_align(O_XST + 3 * W * L * 8);
    static constexpr int O_XCH = BIG ? O_SCR : lds_align(O_SCR + NG * SC * 8);
    static constexpr int bytes() { return BIG ? lds_align(O_SCR + NG * SC * 8) : lds_align(O_XCH + NG * LC * 8); }
    // exchange slot of group (component c, class q, column w); BIG blocks
    // number their own groups (component or column, then class)
    static __device__ __forceinline__ int slot(int c, int q, int w) {
        return BIG ? ((c < 2 ? c : w) * NQ + q) : (c * NQ + q) * W + w;
    }
};

template <int L, int E, int NQ>
__device__ __forceinline__ void col2d_body(const Col2dArgs& a, DevState* __restrict__ st, int lb, char* lds) {
    using CF = ColSplit<L, E, NQ>;
    using F = typename CF::F;
    constexpr int P = CF::P, W = CF::W, LC = CF::LC, NT = CF::NT, KL = CF::KL;
    constexpr bool BIG = CF::BIG;
    float2* tws = (float2*)(lds + CF::O_TWS);
    float* kst = (float*)(lds + CF::O_KST);
    float2* xst = (float2*)(lds + CF::O_XST);
    float2* scr = (float2*)(lds + CF::O_SCR);
    float2* xch = (float2*)(lds + CF::O_XCH);
    if (st->done) return;
    const int tid = threadIdx.x;
    // a group that fills its wavefront: the group index is wave-uniform
    const int gi = P == 64 ? __builtin_amdgcn_readfirstlane(tid / P) : tid / P;
    const int lg = tid % P;
    int w, q, c, scol;
    if (BIG) {
        // blocks [0, nkx): x and y of column lb; then z of columns 2j, 2j+1
        q = gi % NQ;
        const bool zb = lb >= a.nkx;
        c = zb ? 2 : gi / NQ;
        w = zb ? gi / NQ : 0;
        scol = zb ? 2 * (lb - a.nkx) + w : lb;
    } else {
        w = gi % W;
        q = (gi / W) % NQ;               // frequency class
        c = gi / (NQ * W);               // component
        scol = lb * W + w;
    }
    // stored column -> kx: columns are kept in the class order of the rows
    const int kq = a.nkx / a.nq;
    auto kx_of = [&](int sc) { return a.nq * (sc % kq) + sc / kq; };
    const int kx = kx_of(scol);
    const bool packed = scol == 0;
    const int ny = a.ny, Py = a.Py;
    const int cs = ny * a.nkxp;
    const int kcs = a.nkx_full * KL;
    // kernel values at ky = NQ pos + q (mirror compressed along y; xy is
    // odd in ky): diagonal kd, off-diagonal ko (x, y), Nyquist column kn
    float kd[E], ko[E], kn[E];
    float2 x[E];
    float2 twb = mk2(1.f, 0.f);   // BIG: the lane's twiddle W^(lg q)
    const float2* src = a.S + c * cs + tile_index(0, scol, ny, a.tsh);
    if constexpr (BIG) {
        // ---- global reads, per lane: this group's column (zero beyond ny;
        // blocks n + r LC for r < NQ/2) and its pre-twiddles, combined into
        // the class input as they arrive; the kernel values follow the
        // forward transform (fewer live registers through it)
        // (the pre-twiddle W^(yq), y = lg + P i, as W^(lg q) W^(P i q): one
        // read per lane, the second factor the same for the whole wavefront)
        float2 v0[E], v1[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int y = lg + P * i;
            v0[i] = y < ny ? src[y << a.tsh] : mk2(0.f, 0.f);
            v1[i] = (NQ == 4 && y + LC < ny) ? src[(y + LC) << a.tsh] : mk2(0.f, 0.f);
        }
        twb = q ? a.tw[lg * q] : mk2(1.f, 0.f);
#pragma unroll
        for (int i = 0; i < E; ++i) {
            float2 v = v0[i];
            if (NQ == 4) { const float2 t = rot4(v1[i], q); v.x += t.x; v.y += t.y; }
            x[i] = q ? cmul(v, cmul(twb, a.tw[P * i * q])) : v;
        }
    }
    // not BIG: the global reads shared by the block through LDS, its W
    // spectrum columns (the classes of a column read the same values; W
    // consecutive stored columns are contiguous within a tile row) and its
    // kernel columns (contiguous in ky); the stage twiddles; per lane, the
    // pre/post twiddles W^(nq) of its elements.  Every load is issued before
    // the first LDS store (one memory round trip).
    constexpr int ITX = BIG ? 1 : (3 * W * L + NT - 1) / NT;
    constexpr int ITK = BIG ? 1 : (W * 4 * KL + NT - 1) / NT;
    constexpr int ITN = BIG ? 1 : (3 * KL + NT - 1) / NT;
    float2 xv[ITX];
    float kv[ITK], nv[ITN];
    int xd[ITX];
    float2 twq[BIG ? 1 : E];
    typename F::template TwFill<NT> twf;
    twf.load(a.tw, tid);
    if constexpr (!BIG) {
#pragma unroll
        for (int it = 0; it < ITX; ++it) {
            const int e = tid + it * NT;
            xd[it] = -1;
            if (e < 3 * W * L) {   // zeros at y >= ny
                const int ww = e % W, t = e / W;
                const int y = t % L, cc = t / L;
                xv[it] = y < ny ? a.S[cc * cs + tile_index(y, lb * W + ww, ny, a.tsh)] : mk2(0.f, 0.f);
                xd[it] = (cc * W + ww) * L + y;
            }
        }
#pragma unroll
        for (int it = 0; it < ITK; ++it) {
            const int e = tid + it * NT;
            if (e < W * 4 * KL) {
                const int j = e % KL, t = e / KL;
                const int comp = t % 4, ww = t / 4;
                kv[it] = a.K[comp * kcs + kx_of(lb * W + ww) * KL + j];
            }
        }
        if (lb == 0) {   // the packed column also needs the Nyquist column kx = Px/2
#pragma unroll
            for (int it = 0; it < ITN; ++it) {
                const int e = tid + it * NT;
                if (e < 3 * KL) {
                    const int j = e % KL, comp = e / KL;
                    nv[it] = a.K[comp * kcs + (a.nkx_full - 1) * KL + j];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < E; ++i) twq[i] = q ? a.tw[(lg + P * i) * q] : mk2(1.f, 0.f);
    }
    twf.store(tws, tid);
    if constexpr (!BIG) {
#pragma unroll
        for (int it = 0; it < ITX; ++it)
            if (xd[it] >= 0) xst[xd[it]] = xv[it];
#pragma unroll
        for (int it = 0; it < ITK; ++it) {
            const int e = tid + it * NT;
            if (e < W * 4 * KL) kst[e] = kv[it];   // [w][comp][ky]
        }
        if (lb == 0) {
#pragma unroll
            for (int it = 0; it < ITN; ++it) {
                const int e = tid + it * NT;
                if (e < 3 * KL) kst[W * 4 * KL + e] = nv[it];
            }
        }
    }
    __syncthreads();   // stage twiddles (and the staged columns)
    if constexpr (!BIG) {
        // every LDS read first (the staged columns hold zeros at y >= ny;
        // with four classes n + LC < L), then the class inputs and signs
        const float2* col = xst + (c * W + w) * L;
        const float* kc = kst + w * 4 * KL;
        const float* kl = kst + W * 4 * KL;
        float2 va[E], vb[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int n = lg + P * i;
            va[i] = col[n];
            vb[i] = NQ == 4 ? col[n + LC] : mk2(0.f, 0.f);
            const int ky = NQ * n + q;
            const int iy = ky > Py - ky ? Py - ky : ky;
            kd[i] = kc[c * KL + iy];
            ko[i] = c < 2 ? kc[3 * KL + iy] : 0.f;
            kn[i] = packed ? kl[c * KL + iy] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int n = lg + P * i;
            float2 v = va[i];
            if (NQ == 4) { const float2 t = rot4(vb[i], q); v.x += t.x; v.y += t.y; }
            x[i] = q ? cmul(v, twq[i]) : v;
            const int ky = NQ * n + q;
            if (ky > Py - ky) ko[i] = -ko[i];
        }
    }
    F::template run<false>(x, scr + gi * CF::SC, tws, lg);
    if constexpr (BIG) {
        // every load first, the odd-symmetry signs after them
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int ky = NQ * (lg + P * i) + q;
            const int iy = ky > Py - ky ? Py - ky : ky;
            const int o = kx * KL + iy;
            kd[i] = a.K[c * kcs + o];
            ko[i] = c < 2 ? a.K[3 * kcs + o] : 0.f;
            kn[i] = packed ? a.K[c * kcs + (a.nkx_full - 1) * KL + iy] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int ky = NQ * (lg + P * i) + q;
            if (ky > Py - ky) ko[i] = -ko[i];
        }
        __syncthreads();   // every transform has left the scratch (the exchange aliases it)
    }
    // every class spectrum to LDS
    {
        float2* xo = xch + CF::slot(c, q, w) * LC;
#pragma unroll
        for (int i = 0; i < E; ++i) xo[lg + P * i] = x[i];
    }
    __syncthreads();
    if (!packed) {
        // H_x = Kxx M_x + Kxy M_y, H_y = Kxy M_x + Kyy M_y, H_z = Kzz M_z
        if (c < 2) {
            const float2* xp = xch + CF::slot(1 - c, q, w) * LC;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const float2 o = xp[lg + P * i];
                x[i] = mk2(kd[i] * x[i].x + ko[i] * o.x, kd[i] * x[i].y + ko[i] * o.y);
            }
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i) x[i] = mk2(kd[i] * x[i].x, kd[i] * x[i].y);
        }
    } else {
        // column 0 carries (kx = 0) + i (kx = Px/2): separate with the
        // Hermitian symmetry in ky, apply each column's (diagonal) kernel,
        // pack again.  The partner of ky is -ky: class (NQ - q) mod NQ,
        // position (LC - pos) mod LC for q = 0, LC - 1 - pos otherwise.
        const float2* xp = xch + CF::slot(c, (NQ - q) % NQ, w) * LC;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int pos = lg + P * i;
            const float2 z = x[i];
            const float2 zp = xp[q == 0 ? (LC - pos) % LC : LC - 1 - pos];
            float2 A = mk2(0.5f * (z.x + zp.x), 0.5f * (z.y - zp.y));
            float2 B = mk2(0.5f * (z.y + zp.y), -0.5f * (z.x - zp.x));
            A = mk2(kd[i] * A.x, kd[i] * A.y);
            B = mk2(kn[i] * B.x, kn[i] * B.y);
            x[i] = mk2(A.x - B.y, A.y + B.x);
        }
    }
    if constexpr (BIG) __syncthreads();   // every group has read the exchange before the scratch is reused
    F::template run<true>(x, scr + gi * CF::SC, tws, lg);
    __syncthreads();   // every group has read the exchange (and left the scratch)
    {
        float2* xo = xch + CF::slot(c, q, w) * LC;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const float2 t = BIG ? cmul(twb, a.tw[P * i * q]) : twq[BIG ? 0 : i];
            xo[lg + P * i] = q ? cmul(x[i], cconj(t)) : x[i];
        }
    }
    __syncthreads();
    // outputs y = n + r LC: the group of class r (r < NQ/2) assembles them
    if (2 * q >= NQ) return;
    const int r = q;
    float2* dst = a.S + c * cs + tile_index(0, scol, ny, a.tsh);
    // (the LDS reads of four elements issued before their sums)
    constexpr int CE = divisor_upto(E, 4);
#pragma unroll
    for (int i0 = 0; i0 < E; i0 += CE) {
        float2 u[CE][NQ];
#pragma unroll
        for (int ii = 0; ii < CE; ++ii)
#pragma unroll
            for (int cq = 0; cq < NQ; ++cq) u[ii][cq] = xch[CF::slot(c, cq, w) * LC + lg + P * (i0 + ii)];
#pragma unroll
        for (int ii = 0; ii < CE; ++ii) {
            const int y = lg + P * (i0 + ii) + r * LC;
            float2 s = u[ii][0];
#pragma unroll
            for (int cq = 1; cq < NQ; ++cq) {
                const float2 t = rot4(u[ii][cq], -(r * cq * (4 / NQ)));
                s.x += t.x; s.y += t.y;
            }
            if (y < ny) dst[y << a.tsh] = s;
        }
    }
}

template <int L, int E, int NQ>
__global__ __launch_bounds__((ColSplit<L, E, NQ>::NT)) void col2d_fast(Col2dArgs a, DevState* __restrict__ st) {
    extern __shared__ char dyn_lds[];
    col2d_body<L, E, NQ>(a, st, xcd_remap_blocks(blockIdx.x, gridDim.x), dyn_lds);
}

// ---------------------------------------------------------------------------
// compiled variants: (length, elements per lane, variant index).  Rows are
// keyed by the padded x length Px, columns by the half length L = Py/2; the
// variant in use for a length comes from a process-wide table that
// llg_autotune fills (variant 0 until then).
// ---------------------------------------------------------------------------
// rows: (Px, elements per lane, frequency classes, variant)
#define ROW_VARIANTS(X) X(64, 4, 2, 0) X(64, 8, 2, 1) X(128, 4, 2, 0) X(128, 4, 4, 1) X(192, 12, 2, 0)    \
    X(192, 6, 2, 1) X(256, 4, 2, 0) X(256, 4, 4, 1) X(384, 12, 2, 0) X(384, 6, 4, 1) X(512, 4, 2, 0)    \
    X(512, 4, 4, 1) X(768, 12, 2, 0) X(768, 6, 4, 1) X(1024, 8, 2, 0) X(1024, 4, 4, 1) X(2048, 8, 4, 0)  \
    X(2048, 16, 2, 1) X(4096, 16, 4, 0) X(4096, 32, 2, 1)
// columns: (L = Py/2, elements per lane, frequency classes, variant)
#define COL_VARIANTS(X) X(32, 4, 2, 0) X(32, 8, 2, 1) X(64, 4, 2, 0) X(64, 4, 4, 1) X(96, 12, 2, 0)        \
    X(96, 6, 2, 1) X(128, 4, 2, 0) X(128, 4, 4, 1) X(192, 12, 2, 0) X(192, 6, 4, 1) X(256, 4, 2, 0)       \
    X(256, 4, 4, 1) X(384, 12, 2, 0) X(384, 6, 4, 1) X(512, 8, 2, 0) X(512, 4, 4, 1) X(1024, 16, 2, 0)    \
    X(1024, 8, 4, 1) X(2048, 16, 4, 0) X(2048, 32, 2, 1)

// grouped launches: one launch runs a pass for all films of one length
// class (same compiled variant); block b works on film map[b].x, local
// block map[b].y of that film
template <int PX, int E2, int NQ>
__global__ __launch_bounds__((RowSplit<PX, E2, NQ>::NT)) void row_fwd_group(const FilmRow* __restrict__ films,
                                                             const int2* __restrict__ map) {
    extern __shared__ char dyn_lds[];
    const int2 m = map[blockIdx.x];
    const FilmRow& f = films[m.x];
    row_fwd_body<PX, E2, NQ, false, false>(f.g, f.twx, f.S, f.fa, f.st, m.y, dyn_lds);
}

template <int PX, int E2, int NQ>
__global__ __launch_bounds__((RowSplit<PX, E2, NQ>::NT)) void row_inv_group(const FilmRow* __restrict__ films,
                                                             const int2* __restrict__ map) {
    extern __shared__ char dyn_lds[];
    const int2 m = map[blockIdx.x];
    const FilmRow& f = films[m.x];
    row_inv_body<PX, E2, NQ, false, false>(f.g, f.p, f.twx, f.S, f.sa, f.st, m.y, dyn_lds);
}

template <int L, int E, int NQ>
__global__ __launch_bounds__((ColSplit<L, E, NQ>::NT)) void col_group(const FilmCol* __restrict__ films,
                                                         const int2* __restrict__ map) {
    extern __shared__ char dyn_lds[];
    const int2 m = map[blockIdx.x];
    const FilmCol& f = films[m.x];
    col2d_body<L, E, NQ>(f.a, f.st, m.y, dyn_lds);
}

// LDS of one workgroup on gfx950
constexpr int kMaxLds = 160 * 1024;

// kernels whose dynamic LDS may exceed 64 KB need the limit raised once
static hipError_t allow_lds(const void* kernel, int bytes) { return raise_lds_limit(kernel, bytes); }

// the variant table: lengths up to 4096 in steps of 32
std::atomic<int> g_row_var[129], g_col_var[129];
int slot(int len) { return (len % 32 == 0 && len >= 32 && len <= 4096) ? len / 32 : 0; }

}  // namespace

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
int fast2d_row_variant(int Px) { return g_row_var[slot(Px)].load(); }

// tile width of the 2D spectrum (log2); LLG_TILE_LOG2 overrides it for
// layout experiments
int fast2d_tile_shift() {
    const char* e = getenv("LLG_TILE_LOG2");
    if (e && e[0] >= '0' && e[0] <= '5' && e[1] == 0) return e[0] - '0';
    return 2;
}
int fast2d_col_variant(int L) { return g_col_var[slot(L)].load(); }
bool fast2d_set_row_variant(int Px, int var, bool xper) {
    if (!fast2d_row_ok(Px, var, xper)) return false;
    g_row_var[slot(Px)].store(var);
    return true;
}
bool fast2d_set_col_variant(int L, int var) {
    if (!fast2d_col_ok(L, 1, var)) return false;
    g_col_var[slot(L)].store(var);
    return true;
}
bool fast2d_set_variants(int Px, int rv, int L, int cv, bool xper) {
    if (!fast2d_row_ok(Px, rv, xper) || !fast2d_col_ok(L, 1, cv)) return false;
    g_row_var[slot(Px)].store(rv);
    g_col_var[slot(L)].store(cv);
    return true;
}

bool fast2d_row_ok(int Px, int var, bool xper) {
    if (var < 0) var = fast2d_row_variant(Px);
#define CASE(PX, E, NQ, V)                                                                \
    if (Px == PX && var == V)                                                             \
        return (xper ? RowSplit<PX, E, NQ>::template inv_bytes<true>()                    \
                     : RowSplit<PX, E, NQ>::template inv_bytes<false>()) <= kMaxLds;
    ROW_VARIANTS(CASE)
#undef CASE
    return false;
}

bool fast2d_col_ok(int L, int split, int var) {
    if (!split) return false;
    if (var < 0) var = fast2d_col_variant(L);
#define CASE(LL, E, NQ, V) if (L == LL && var == V) return ColSplit<LL, E, NQ>::bytes() <= kMaxLds;
    COL_VARIANTS(CASE)
#undef CASE
    return false;
}

// the fast row kernels of one compiled variant: periodic x (XPER) or
// zero-padded, packed 2D (NAT false) or natural 3D (NAT true) spectrum
template <int PX, int E, int NQ, bool NAT>
hipError_t launch_row_fwd_t(const Grid& g, const float2* twx, float2* S, const FwdArgs& fa, DevState* st,
                            hipStream_t s) {
    using R_ = RowSplit<PX, E, NQ>;
    constexpr int rows = 2 * R_::RP;
    const dim3 grid((g.nrows + rows - 1) / rows);
    constexpr int lds_p = R_::template fwd_bytes<true>();
    constexpr int lds_o = R_::template fwd_bytes<false>();
    if (g.nx == PX) {
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&row_fwd_fast<PX, E, NQ, true, NAT>), lds_p);
        if (e_ != hipSuccess) return e_;
        hot_launch(row_fwd_fast<PX, E, NQ, true, NAT>, grid, dim3(R_::NT), lds_p, s, g, twx, S, fa, st);
    } else if (2 * g.nx <= PX) {
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&row_fwd_fast<PX, E, NQ, false, NAT>), lds_o);
        if (e_ != hipSuccess) return e_;
        hot_launch(row_fwd_fast<PX, E, NQ, false, NAT>, grid, dim3(R_::NT), lds_o, s, g, twx, S, fa, st);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int PX, int E, int NQ, bool NAT>
hipError_t launch_row_inv_t(const Grid& g, const Phys& p, const float2* twx, float2* S, const StageArgs& sa,
                            DevState* st, hipStream_t s) {
    using R_ = RowSplit<PX, E, NQ>;
    constexpr int rows = 2 * R_::RP;
    const dim3 grid((g.nrows + rows - 1) / rows);
    constexpr int lds_p = R_::template inv_bytes<true>();
    constexpr int lds_o = R_::template inv_bytes<false>();
    if (g.nx == PX) {
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&row_inv_fast<PX, E, NQ, true, NAT>), lds_p);
        if (e_ != hipSuccess) return e_;
        hot_launch(row_inv_fast<PX, E, NQ, true, NAT>, grid, dim3(R_::NT), lds_p, s, g, p, twx, S, sa, st);
    } else if (2 * g.nx <= PX) {
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&row_inv_fast<PX, E, NQ, false, NAT>), lds_o);
        if (e_ != hipSuccess) return e_;
        hot_launch(row_inv_fast<PX, E, NQ, false, NAT>, grid, dim3(R_::NT), lds_o, s, g, p, twx, S, sa,
                           st);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// one compiled variant, packed 2D (nat false) or natural 3D layout; the
// 4096-point rows serve 2D films only
template <int PX, int E, int NQ>
hipError_t launch_row_fwd_v(const Grid& g, const float2* twx, float2* S, const FwdArgs& fa, DevState* st,
                            hipStream_t s, bool nat) {
    if constexpr (RowSplit<PX, E, NQ>::BIG) {
        if (nat) return hipErrorInvalidValue;
        return launch_row_fwd_t<PX, E, NQ, false>(g, twx, S, fa, st, s);
    } else {
        return nat ? launch_row_fwd_t<PX, E, NQ, true>(g, twx, S, fa, st, s)
                   : launch_row_fwd_t<PX, E, NQ, false>(g, twx, S, fa, st, s);
    }
}
template <int PX, int E, int NQ>
hipError_t launch_row_inv_v(const Grid& g, const Phys& p, const float2* twx, float2* S, const StageArgs& sa,
                            DevState* st, hipStream_t s, bool nat) {
    if constexpr (RowSplit<PX, E, NQ>::BIG) {
        if (nat) return hipErrorInvalidValue;
        return launch_row_inv_t<PX, E, NQ, false>(g, p, twx, S, sa, st, s);
    } else {
        return nat ? launch_row_inv_t<PX, E, NQ, true>(g, p, twx, S, sa, st, s)
                   : launch_row_inv_t<PX, E, NQ, false>(g, p, twx, S, sa, st, s);
    }
}

// 2D (nz = 1): the packed, tiled spectrum of the column kernel; 3D: the
// natural layout [c][row][nkxp] of the 3D column passes
hipError_t launch_row_fwd_fast(const Grid& g, const float2* twx, float2* S, const FwdArgs& fa,
                               DevState* st, hipStream_t s) {
    if (g.nx > g.Px || g.nkxp < g.Px / 2 || g.tsh < 0 || (g.Px / 2) % (1 << g.tsh)) return hipErrorInvalidValue;
    const bool nat = g.nz > 1;
    if (nat && (g.nkxp < g.Px / 2 + 1 || g.nkx != g.Px / 2 + 1)) return hipErrorInvalidValue;
    const int var = g.rvar;
#define CASE(PX, E, NQ, V) \
    if (g.Px == PX && var == V) return launch_row_fwd_v<PX, E, NQ>(g, twx, S, fa, st, s, nat);
    ROW_VARIANTS(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

hipError_t launch_row_inv_fast(const Grid& g, const Phys& p, const float2* twx, float2* S,
                               const StageArgs& sa, DevState* st, hipStream_t s) {
    if (g.nx > g.Px || g.nkxp < g.Px / 2 || sa.nk > kMaxK || g.tsh < 0 || (g.Px / 2) % (1 << g.tsh))
        return hipErrorInvalidValue;
    if ((sa.mode == ROW_STAGE || sa.mode == ROW_ERROR) && sa.nk < 1) return hipErrorInvalidValue;
    const bool nat = g.nz > 1;
    if (nat && (g.nkxp < g.Px / 2 + 1 || g.nkx != g.Px / 2 + 1)) return hipErrorInvalidValue;
    const int var = g.rvar;
#define CASE(PX, E, NQ, V) \
    if (g.Px == PX && var == V) return launch_row_inv_v<PX, E, NQ>(g, p, twx, S, sa, st, s, nat);
    ROW_VARIANTS(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

hipError_t launch_col2d_fast(const Col2dArgs& a, DevState* st, hipStream_t s) {
    if (a.Py % 2 || a.ny > a.Py / 2 || a.nkx_full != a.nkx + 1 || a.nkx % 2) return hipErrorInvalidValue;
    if (a.tsh < 0 || a.nkx % (1 << a.tsh) || (a.nq != 2 && a.nq != 4) || a.nkx % a.nq) return hipErrorInvalidValue;
    const int L = a.Py / 2;
    const int var = a.var;
#define CASE(LL, E, NQ, V)                                                                \
    if (L == LL && var == V) {                                                            \
        using CF = ColSplit<LL, E, NQ>;                                                   \
        if (a.nkx % CF::W) return hipErrorInvalidValue;                                   \
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&col2d_fast<LL, E, NQ>), CF::bytes()); \
        if (e_ != hipSuccess) return e_;                                                  \
        hot_launch(col2d_fast<LL, E, NQ>, dim3(CF::blocks(a.nkx)), dim3(CF::NT), CF::bytes(), s, a, st); \
        return hipGetLastError();                                                         \
    }
    COL_VARIANTS(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

// ---- grouped launchers ------------------------------------------------------------
int fast2d_row_rows_per_block(int Px, int var) {
#define CASE(PX, E, NQ, V) if (Px == PX && var == V) return 2 * RowSplit<PX, E, NQ>::RP;
    ROW_VARIANTS(CASE)
#undef CASE
    return 0;
}
bool fast2d_variant_shape(int kind, int len, int var, int* elems, int* classes) {
    if (kind == 0) {
#define CASE(PX, E, NQ, V) if (len == PX && var == V) { *elems = E; *classes = NQ; return true; }
        ROW_VARIANTS(CASE)
#undef CASE
    } else if (kind == 1) {
#define CASE(LL, E, NQ, V) if (len == LL && var == V) { *elems = E; *classes = NQ; return true; }
        COL_VARIANTS(CASE)
#undef CASE
    }
    return false;
}

int fast2d_row_classes(int Px, int var) {
    if (var < 0) var = fast2d_row_variant(Px);
#define CASE(PX, E, NQ, V) if (Px == PX && var == V) return NQ;
    ROW_VARIANTS(CASE)
#undef CASE
    return 0;
}
// smallest compiled row length Px >= n, and column half length L >= n
// (0 if there is none): zero padding beyond 2 n - 1 leaves the convolution
// unchanged, so a film may use a longer compiled transform
int fast2d_row_len_at_least(int n) {
    int best = 0;
#define CASE(PX, E, NQ, V) if (V == 0 && PX >= n && (best == 0 || PX < best)) best = PX;
    ROW_VARIANTS(CASE)
#undef CASE
    return best;
}
int fast2d_col_len_at_least(int n) {
    int best = 0;
#define CASE(LL, E, NQ, V) if (V == 0 && LL >= n && (best == 0 || LL < best)) best = LL;
    COL_VARIANTS(CASE)
#undef CASE
    return best;
}

int fast2d_col_blocks(int L, int var, int nkx) {
    if (var < 0) var = fast2d_col_variant(L);
#define CASE(LL, E, NQ, V) if (L == LL && var == V) return ColSplit<LL, E, NQ>::blocks(nkx);
    COL_VARIANTS(CASE)
#undef CASE
    return 0;
}

int fast2d_col_width(int L, int var) {
    if (var < 0) var = fast2d_col_variant(L);
#define CASE(LL, E, NQ, V) if (L == LL && var == V) return ColSplit<LL, E, NQ>::W;
    COL_VARIANTS(CASE)
#undef CASE
    return 0;
}

hipError_t launch_row_fwd_group(int Px, int var, const FilmRow* films, const int2* map, int nblocks,
                                hipStream_t s) {
#define CASE(PX, E, NQ, V)                                                                \
    if (Px == PX && var == V) {                                                           \
        using R_ = RowSplit<PX, E, NQ>;                                                   \
        constexpr int lds = R_::template fwd_bytes<false>();                              \
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&row_fwd_group<PX, E, NQ>), lds); \
        if (e_ != hipSuccess) return e_;                                                  \
        hipLaunchKernelGGL((row_fwd_group<PX, E, NQ>), dim3(nblocks), dim3(R_::NT), lds, s, films, map); \
        return hipGetLastError();                                                         \
    }
    ROW_VARIANTS(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

hipError_t launch_row_inv_group(int Px, int var, const FilmRow* films, const int2* map, int nblocks,
                                hipStream_t s) {
#define CASE(PX, E, NQ, V)                                                                \
    if (Px == PX && var == V) {                                                           \
        using R_ = RowSplit<PX, E, NQ>;                                                   \
        constexpr int lds = R_::template inv_bytes<false>();                              \
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&row_inv_group<PX, E, NQ>), lds); \
        if (e_ != hipSuccess) return e_;                                                  \
        hipLaunchKernelGGL((row_inv_group<PX, E, NQ>), dim3(nblocks), dim3(R_::NT), lds, s, films, map); \
        return hipGetLastError();                                                         \
    }
    ROW_VARIANTS(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

hipError_t launch_col_group(int L, int var, const FilmCol* films, const int2* map, int nblocks, hipStream_t s) {
#define CASE(LL, E, NQ, V)                                                                \
    if (L == LL && var == V) {                                                            \
        using CF = ColSplit<LL, E, NQ>;                                                   \
        constexpr int lds = CF::bytes();                                                  \
        hipError_t e_ = allow_lds(reinterpret_cast<const void*>(&col_group<LL, E, NQ>), lds); \
        if (e_ != hipSuccess) return e_;                                                  \
        hipLaunchKernelGGL((col_group<LL, E, NQ>), dim3(nblocks), dim3(CF::NT), lds, s, films, map); \
        return hipGetLastError();                                                         \
    }
    COL_VARIANTS(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

// sizes beyond the hardware are refused before any runtime call; a failed
// call leaves no error behind for later calls
hipError_t raise_lds_limit(const void* fn, int bytes) {
    if (bytes > kMaxLds) return hipErrorInvalidValue;
    if (bytes <= 65536) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, int> raised;
    const std::pair<int, const void*> key(dev, fn);
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = raised.find(key);
        if (it != raised.end() && it->second >= bytes) return hipSuccess;
    }
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    std::lock_guard<std::mutex> lock(mu);
    int& v = raised[key];
    if (v < bytes) v = bytes;
    return hipSuccess;
}

}  // namespace llg
