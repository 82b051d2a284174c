// FP32 hot-path kernels of the effective-field evaluation and time step.
//
// One H_eff evaluation of an nx x ny x nz grid is (Sec. 3.2 of the paper:
// forward transform of the zero-padded magnetisation, point-wise product
// with the transformed kernel, inverse transform):
//
//   row_fwd   r2c of each x-row, zero padded to Px          (2 rows / block)
//   col       2D: y transform, product with K, inverse y    (W columns / block)
//             3D: y forward, z transform + product + inverse z, y inverse
//   row_inv   c2r of each x-row -> demag field, + exchange (Eq. 3),
//             anisotropy (Eq. 4), applied and thermal (Eq. 6) fields,
//             then the LL torque (Eq. 1) and the Runge-Kutta stage
//             combination (Sec. 2.2), then the r2c of the next stage input
//
// Zero-padded input rows/columns are never stored: the x transforms fill
// the padding in LDS, and the open-axis column transforms are split into
// even and odd frequency halves of length P/2, which only ever see the n
// non-zero inputs.  Two real rows share one complex transform (z = a + i b),
// separated afterwards with the Hermitian symmetry of real signals.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "cell_physics.hpp"

namespace llg {

constexpr int RT = 256;   // threads of the row kernels
constexpr int CT = 256;   // threads of the column kernel

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 f2(float x, float y) { float2 r; r.x = x; r.y = y; return r; }

// Forward x transform of the two rows r0, r0+1 whose values sit in the
// per-thread slots nm[q] (slot q covers cell e = tid + q*RT, row e / nx),
// then separation of the three packed transforms and the store of the
// Px/2+1 retained frequencies of each row and component into S.
template <int MAXE>
__device__ __forceinline__ void row_forward_store(const Grid& g, const FftPlan& px,
                                                  const float2* __restrict__ twx, float2* __restrict__ S,
                                                  float2* lds, const float (*nm)[3], int r0, bool has1) {
    constexpr int MAXC = (MAXE + 2) / 3;
    const int tid = threadIdx.x;
    const int Px = g.Px, nx = g.nx;
    float2* Z0 = lds;
    float2* Z1 = lds + Px;
    float2* Z2 = lds + 2 * Px;
    const int ncell2 = (has1 ? 2 : 1) * nx;
    for (int x = tid; x < Px; x += RT) {
        if (x >= nx) { Z0[x] = f2(0.f, 0.f); Z1[x] = f2(0.f, 0.f); Z2[x] = f2(0.f, 0.f); }
        else if (!has1) { Z1[x] = f2(0.f, 0.f); Z2[x].y = 0.f; }
    }
#pragma unroll
    for (int q = 0; q < MAXC; ++q) {
        const int e = tid + q * RT;
        if (e < ncell2) {
            const int rr = e / nx, x = e - rr * nx;
            if (rr == 0) { Z0[x] = f2(nm[q][0], nm[q][1]); Z2[x].x = nm[q][2]; }
            else { Z1[x] = f2(nm[q][0], nm[q][1]); Z2[x].y = nm[q][2]; }
        }
    }
    __syncthreads();
    lds_fft<MAXE>(lds, px, 3, twx, 1, false, tid, RT);
    const long long cs = (long long)g.nrows * g.nkxp;
    float2* s0 = S + (long long)r0 * g.nkxp;
    float2* s1 = s0 + g.nkxp;
    for (int k = tid; k < g.nkx; k += RT) {
        const int km = k == 0 ? 0 : Px - k;
        float2 A[3], B[3];
        const float2* Zs[3] = {Z0, Z1, Z2};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const float2 zk = Zs[t][k], zm = Zs[t][km];   // Z[k], Z[Px-k]
            // a = (Z[k] + conj Z[-k]) / 2,  b = (Z[k] - conj Z[-k]) / (2i)
            const float sx = zk.x + zm.x, sy = zk.y - zm.y;
            const float dx = zk.x - zm.x, dy = zk.y + zm.y;
            A[t] = f2(0.5f * sx, 0.5f * sy);
            B[t] = f2(0.5f * dy, -0.5f * dx);
        }
        s0[k] = A[0];
        s0[cs + k] = B[0];
        s0[2 * cs + k] = A[2];
        if (has1) {
            s1[k] = A[1];
            s1[cs + k] = B[1];
            s1[2 * cs + k] = B[2];
        }
    }
}

// ---------------------------------------------------------------------------
// forward x pass: S <- r2c(m) of rows (2 per block); optional prologue
// m_out = normalize(m0 + dtau a1 k1) (first stage of an adaptive attempt)
// ---------------------------------------------------------------------------
template <int MAXE>
__global__ __launch_bounds__(RT) void row_fwd_kernel(Grid g, FftPlan px, const float2* __restrict__ twx,
                                                     float2* __restrict__ S, FwdArgs fa,
                                                     DevState* __restrict__ st) {
    extern __shared__ float2 lds[];
    if (st->done) return;
    constexpr int MAXC = (MAXE + 2) / 3;
    const int cur = st->cur;
    const float dtau = st->dtau;
    const int tid = threadIdx.x;
    const int r0 = 2 * blockIdx.x;
    const bool has1 = r0 + 1 < g.nrows;
    const int nx = g.nx;
    const long long cs = g.ncells;
    const int ncell2 = (has1 ? 2 : 1) * nx;
    float nm[MAXC][3];
    const float* mi = resolve(fa.m_in, cur);
    const float* m0 = resolve(fa.m0, cur);
    const float* k1 = resolve(fa.k1, cur);
    float* mo = resolve(fa.m_out, cur);
    const float c1 = dtau * fa.a1;
#pragma unroll
    for (int q = 0; q < MAXC; ++q) {
        const int e = tid + q * RT;
        if (e < ncell2) {
            const int rr = e / nx, x = e - rr * nx;
            const long long i = (long long)(r0 + rr) * nx + x;
            if (fa.combine) {
                float ax = m0[i] + c1 * k1[i];
                float ay = m0[cs + i] + c1 * k1[cs + i];
                float az = m0[2 * cs + i] + c1 * k1[2 * cs + i];
                const float inv = rsqrtf(ax * ax + ay * ay + az * az);
                ax *= inv; ay *= inv; az *= inv;
                mo[i] = ax; mo[cs + i] = ay; mo[2 * cs + i] = az;
                nm[q][0] = ax; nm[q][1] = ay; nm[q][2] = az;
            } else {
                nm[q][0] = mi[i]; nm[q][1] = mi[cs + i]; nm[q][2] = mi[2 * cs + i];
            }
        }
    }
    row_forward_store<MAXE>(g, px, twx, S, lds, nm, r0, has1);
}

// ---------------------------------------------------------------------------
// inverse x pass fused with the local field terms, the torque, the stage
// combination and the next stage's forward x pass
// ---------------------------------------------------------------------------
template <int MAXE>
__global__ __launch_bounds__(RT) void row_inv_kernel(Grid g, Phys p, FftPlan px, const float2* __restrict__ twx,
                                                     float2* __restrict__ S, StageArgs sa,
                                                     DevState* __restrict__ st) {
    extern __shared__ float2 lds[];
    __shared__ float wmax[RT / 64];
    if (st->done) return;
    constexpr int MAXC = (MAXE + 2) / 3;
    const int cur = st->cur;
    const float dtau = st->dtau;
    const uint64_t step = (uint64_t)st->step;
    const int tid = threadIdx.x;
    const int r0 = 2 * blockIdx.x;
    const bool has1 = r0 + 1 < g.nrows;
    const int Px = g.Px, nx = g.nx;
    float2* Z0 = lds;
    float2* Z1 = lds + Px;
    float2* Z2 = lds + 2 * Px;

    if (p.demag_on) {
        const long long cs = (long long)g.nrows * g.nkxp;
        const float2* s0 = S + (long long)r0 * g.nkxp;
        const float2* s1 = s0 + g.nkxp;
        for (int k = tid; k < g.nkx; k += RT) {
            const float2 hx0 = s0[k], hy0 = s0[cs + k], hz0 = s0[2 * cs + k];
            float2 hx1 = f2(0.f, 0.f), hy1 = hx1, hz1 = hx1;
            if (has1) { hx1 = s1[k]; hy1 = s1[cs + k]; hz1 = s1[2 * cs + k]; }
            // packed spectra a + i b of two real signals
            Z0[k] = f2(hx0.x - hy0.y, hx0.y + hy0.x);
            Z1[k] = f2(hx1.x - hy1.y, hx1.y + hy1.x);
            Z2[k] = f2(hz0.x - hz1.y, hz0.y + hz1.x);
            if (k > 0 && k < Px - k) {
                // Hermitian extension: spectrum at Px-k is conj(a) + i conj(b)
                Z0[Px - k] = f2(hx0.x + hy0.y, hy0.x - hx0.y);
                Z1[Px - k] = f2(hx1.x + hy1.y, hy1.x - hx1.y);
                Z2[Px - k] = f2(hz0.x + hz1.y, hz1.x - hz0.y);
            }
        }
        __syncthreads();
        lds_fft<MAXE>(lds, px, 3, twx, 1, true, tid, RT);
    }

    const long long cs = g.ncells;
    const int ncell2 = (has1 ? 2 : 1) * nx;
    const float* mi = resolve(sa.m_in, cur);
    const float* m0 = resolve(sa.m0, cur);
    float* mo = resolve(sa.m_out, cur);
    float* ko = resolve(sa.k_out, cur);
    float nm[MAXC][3];
    float errmax = 0.f;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < MAXC; ++q) {
        const int e = tid + q * RT;
        nm[q][0] = nm[q][1] = nm[q][2] = 0.f;
        if (e < ncell2) {
            const int rr = e / nx, x = e - rr * nx;
            const int r = r0 + rr;
            const long long i = (long long)r * nx + x;
            const float mx = mi[i], my = mi[cs + i], mz = mi[2 * cs + i];
            float hx = 0.f, hy = 0.f, hz = 0.f;
            if (p.demag_on) {
                const float2 a = rr ? Z1[x] : Z0[x];
                const float2 b = Z2[x];
                hx = a.x; hy = a.y; hz = rr ? b.y : b.x;
            }
            local_field(g, p, mi, r, x, mx, my, mz, step, hx, hy, hz);
            if (sa.mode == ROW_EVAL) {
                float* h = sa.h_out;
                h[i] = hx * p.Ms; h[cs + i] = hy * p.Ms; h[2 * cs + i] = hz * p.Ms;
                bad |= !(isfinite(hx) && isfinite(hy) && isfinite(hz));
                continue;
            }
            float kx, ky, kz;
            ll_torque(p, mx, my, mz, hx, hy, hz, kx, ky, kz);
            if (p.stt_on) {
                float Dx, Dy, Dz;
                stt_gradient(g, p, mi, r, x, mx, my, mz, Dx, Dy, Dz);
                stt_torque(p, mx, my, mz, Dx, Dy, Dz, kx, ky, kz);
            }
            bad |= !(isfinite(kx) && isfinite(ky) && isfinite(kz));
            if (ko) { ko[i] = kx; ko[cs + i] = ky; ko[2 * cs + i] = kz; }
            if (sa.mode == ROW_KONLY && sa.with_err) errmax = fmaxf(errmax, sqrtf(kx * kx + ky * ky + kz * kz));
            if (sa.mode == ROW_STAGE) {
                float ax = m0[i], ay = m0[cs + i], az = m0[2 * cs + i];
                for (int j = 0; j + 1 < sa.nk; ++j) {
                    const float c = dtau * sa.a[j];
                    if (c != 0.f) {
                        const float* kj = resolve(sa.kprev[j], cur);
                        ax += c * kj[i]; ay += c * kj[cs + i]; az += c * kj[2 * cs + i];
                    }
                }
                const float c = dtau * sa.a[sa.nk - 1];
                ax += c * kx; ay += c * ky; az += c * kz;
                const float inv = rsqrtf(ax * ax + ay * ay + az * az);
                ax *= inv; ay *= inv; az *= inv;
                mo[i] = ax; mo[cs + i] = ay; mo[2 * cs + i] = az;
                nm[q][0] = ax; nm[q][1] = ay; nm[q][2] = az;
            }
            if (sa.mode == ROW_ERROR || (sa.mode == ROW_STAGE && sa.with_err)) {
                float ex = 0.f, ey = 0.f, ez = 0.f;
                for (int j = 0; j + 1 < sa.nk; ++j) {
                    const float c = sa.e[j];
                    if (c != 0.f) {
                        const float* kj = resolve(sa.kprev[j], cur);
                        ex += c * kj[i]; ey += c * kj[cs + i]; ez += c * kj[2 * cs + i];
                    }
                }
                const float c = sa.e[sa.nk - 1];
                ex += c * kx; ey += c * ky; ez += c * kz;
                const float err = dtau * sqrtf(ex * ex + ey * ey + ez * ez);
                errmax = fmaxf(errmax, err);
            }
        }
    }
    if (bad) atomicOr(&st->health, 1);
    if (sa.mode == ROW_ERROR || ((sa.mode == ROW_STAGE || sa.mode == ROW_KONLY) && sa.with_err)) {
        for (int off = 32; off > 0; off >>= 1) errmax = fmaxf(errmax, __shfl_xor(errmax, off));
        if ((tid & 63) == 0) wmax[tid >> 6] = errmax;
        __syncthreads();
        if (tid == 0) {
            float m = wmax[0];
            for (int w = 1; w < RT / 64; ++w) m = fmaxf(m, wmax[w]);
            atomicMax(&st->err_bits, __float_as_uint(m));
        }
        if (sa.mode != ROW_STAGE) return;
    }
    if (sa.mode == ROW_STAGE && p.demag_on && !sa.skip_fwd) {
        __syncthreads();   // every thread is done reading the inverse transform
        row_forward_store<MAXE>(g, px, twx, S, lds, nm, r0, has1);
    }
}

// ---------------------------------------------------------------------------
// column pass along y (2D, or 3D forward / inverse) or z (3D, with the
// product).  A block owns W adjacent kx columns of one outer index.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_K(const ColArgs& a, int kx, int ka, int ko, float* Kv) {
    bool fa = false, fo = false;
    int ia = ka, io = ko;
    if (ka > a.Pa - ka) { ia = a.Pa - ka; fa = true; }
    if (ko > a.Po - ko) { io = a.Po - ko; fo = true; }
    const long long comp_stride = (long long)a.no_c * a.nkx * a.na_c;
    const long long off = ((long long)io * a.nkx + kx) * a.na_c + ia;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        float v = 0.f;
        if (c < a.ncomp) {
            v = a.K[c * comp_stride + off];
            if (fa && a.sign_a[c] < 0) v = -v;
            if (fo && a.sign_o[c] < 0) v = -v;
        }
        Kv[c] = v;
    }
}

template <int MAXE, int MODE>
__global__ __launch_bounds__(CT) void col_kernel(ColArgs a, DevState* __restrict__ st) {
    extern __shared__ float2 lds[];
    if (st->done) return;
    const int tid = threadIdx.x;
    const int lb = xcd_remap_blocks(blockIdx.x, gridDim.x);
    const int o = lb / a.ntiles;
    const int tile = lb - o * a.ntiles;
    const int kx0 = tile * a.W;
    const int Wt = min(a.W, a.nkx - kx0);
    const int Lh = a.split ? a.P / 2 : a.P;
    const int nh = a.split ? 2 : 1;
    const int tmul = a.split ? 2 : 1;
    const int nbat = 3 * Wt;
    const float2* in = a.in + o * a.os_in + kx0;
    float2* out = a.out + o * a.os_out + kx0;

    float2 xin[MAXE];
    float2 acc[MAXE];
    const int nIn = 3 * Wt * a.n_in;
    const int nOut = 3 * Wt * a.n_out;
    if (MODE != COL_INV) {
#pragma unroll
        for (int q = 0; q < MAXE; ++q) {
            const int e = tid + q * CT;
            if (e < nIn) {
                const int w = e % Wt, t = e / Wt;
                const int pos = t % a.n_in, c = t / a.n_in;
                xin[q] = in[c * a.cs_in + pos * a.as_in + w];
            }
        }
    }
    for (int h = 0; h < nh; ++h) {
        // ---- fill LDS with this half's input
        if (MODE != COL_INV) {
            for (int e = tid; e < nbat * Lh; e += CT) {
                if (e % Lh >= a.n_in) lds[e] = f2(0.f, 0.f);
            }
#pragma unroll
            for (int q = 0; q < MAXE; ++q) {
                const int e = tid + q * CT;
                if (e < nIn) {
                    const int w = e % Wt, t = e / Wt;
                    const int pos = t % a.n_in, c = t / a.n_in;
                    float2 v = xin[q];
                    if (h) v = cmul(v, a.tw[pos]);      // x[n] w_P^n feeds the odd half
                    lds[(c * Wt + w) * Lh + pos] = v;
                }
            }
        } else {
            for (int e = tid; e < nbat * Lh; e += CT) {
                const int w = e % Wt, t = e / Wt;
                const int pos = t % Lh, c = t / Lh;
                lds[(c * Wt + w) * Lh + pos] = in[c * a.cs_in + (h * Lh + pos) * a.as_in + w];
            }
        }
        __syncthreads();
        if (MODE != COL_INV) lds_fft<MAXE>(lds, a.plan, nbat, a.tw, tmul, false, tid, CT);

        if (MODE == COL_FWD) {
            for (int e = tid; e < nbat * Lh; e += CT) {
                const int w = e % Wt, t = e / Wt;
                const int pos = t % Lh, c = t / Lh;
                out[c * a.cs_out + (h * Lh + pos) * a.as_out + w] = lds[(c * Wt + w) * Lh + pos];
            }
            __syncthreads();
            continue;
        }
        if (MODE == COL_FULL) {
            // point-wise product with the real symmetric kernel spectrum
            int ko = 0;
            if (a.Po > 1) {
                if (a.o_split) {
                    const int hp = a.Po / 2;
                    ko = 2 * (o % hp) + o / hp;
                } else {
                    ko = o;
                }
            }
            for (int e = tid; e < Wt * Lh; e += CT) {
                const int pos = e % Lh, w = e / Lh;
                const int ka = a.split ? 2 * pos + h : pos;
                float Kv[6];
                load_K(a, kx0 + w, ka, ko, Kv);
                float2* px = lds + (0 * Wt + w) * Lh + pos;
                float2* py = lds + (1 * Wt + w) * Lh + pos;
                float2* pz = lds + (2 * Wt + w) * Lh + pos;
                const float2 Mx = *px, My = *py, Mz = *pz;
                // K = [xx, yy, zz, xy, xz, yz]
                *px = f2(Kv[0] * Mx.x + Kv[3] * My.x + Kv[4] * Mz.x, Kv[0] * Mx.y + Kv[3] * My.y + Kv[4] * Mz.y);
                *py = f2(Kv[3] * Mx.x + Kv[1] * My.x + Kv[5] * Mz.x, Kv[3] * Mx.y + Kv[1] * My.y + Kv[5] * Mz.y);
                *pz = f2(Kv[4] * Mx.x + Kv[5] * My.x + Kv[2] * Mz.x, Kv[4] * Mx.y + Kv[5] * My.y + Kv[2] * Mz.y);
            }
            __syncthreads();
        }
        lds_fft<MAXE>(lds, a.plan, nbat, a.tw, tmul, true, tid, CT);
        // ---- accumulate the kept outputs: h0[n] + w_P^{-n} h1[n]
#pragma unroll
        for (int q = 0; q < MAXE; ++q) {
            const int e = tid + q * CT;
            if (e < nOut) {
                const int w = e % Wt, t = e / Wt;
                const int pos = t % a.n_out, c = t / a.n_out;
                float2 v = lds[(c * Wt + w) * Lh + pos];
                if (h) {
                    v = cmul(v, cconj(a.tw[pos]));
                    acc[q] = f2(acc[q].x + v.x, acc[q].y + v.y);
                } else {
                    acc[q] = v;
                }
            }
        }
        __syncthreads();
    }
    if (MODE != COL_FWD) {
#pragma unroll
        for (int q = 0; q < MAXE; ++q) {
            const int e = tid + q * CT;
            if (e < nOut) {
                const int w = e % Wt, t = e / Wt;
                const int pos = t % a.n_out, c = t / a.n_out;
                out[c * a.cs_out + pos * a.as_out + w] = acc[q];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// controllers (one thread)
// ---------------------------------------------------------------------------
__global__ void ctrl_fixed_kernel(DevState* st, int evals) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    st->t += st->dt;
    st->cur ^= 1;
    st->step += 1;
    st->nsteps += 1;
    st->nevals += evals;
}

// Fixed tableau with a bounded change of m per step: the first stage of a
// step left max over cells |k_1| in err_bits (k in units of dtau); the
// step is max_dm / that (tol holds max_dm), at most dt_max, and the last
// one lands on t_end.
__global__ void ctrl_dm_kernel(DevState* st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (st->done) return;
    const float kf = __uint_as_float(st->err_bits);
    st->err_bits = 0u;
    st->last_err = (double)kf;
    if (st->health) { st->done = 1; return; }
    double dt = st->dt_max;
    if (kf > 0.f) dt = fmin(dt, st->tol / ((double)kf * st->gms));
    const double rem = st->t_end - st->t;
    if (dt >= rem) { dt = rem; st->clipped = 1; }
    else st->clipped = 0;
    st->dt = dt;
    st->dt_next = dt;
    st->dtau = (float)(dt * st->gms);
}

// end of such a step: the new state is in place
__global__ void ctrl_dm_accept_kernel(DevState* st, int evals) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (st->done) return;
    const long long a = st->nattempt++;
    if (a < st->log_cap && st->log) {
        llg_attempt r;
        r.dt = st->dt;
        r.err = (float)(st->last_err * (double)st->dtau);   // bound on |dm| of the first stage
        r.accepted = 1;
        st->log[a] = r;
    }
    st->nevals += evals;
    if (st->health) { st->done = 1; return; }
    st->t = st->clipped ? st->t_end : st->t + st->dt;
    st->cur ^= 1;
    st->step += 1;
    st->nsteps += 1;
    if (st->clipped) st->done = 1;
}

__global__ void ctrl_fixed_group_kernel(DevState* states, int nfilms, int evals) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nfilms) return;
    DevState* st = states + i;
    st->t += st->dt;
    st->cur ^= 1;
    st->step += 1;
    st->nsteps += 1;
    st->nevals += evals;
}

// Dormand-Prince step control: accept if err <= tol, next step
// dt * clamp(0.9 (tol/err)^(1/5), 0.2, 5), last step lands on t_end.  The
// record is read into registers in one round of loads, updated there and
// written back once (the single thread would otherwise wait on one global
// read after another).
__device__ void dp45_control(DevState* st) {
    DevState h = *st;
    // a finished run is left as it is: the decisions below are computed
    // either way (register arithmetic only) and the stores skipped, so that
    // every load of the record is issued before the first branch
    const bool live = !h.done;
    const float errf = __uint_as_float(h.err_bits);
    const double err = (double)errf;
    const double dt_att = h.dt;
    h.err_bits = 0u;
    h.nevals += h.ev_attempt;
    h.last_err = err;
    const bool ok = (h.health == 0) && (err <= h.tol);
    const long long a = h.nattempt++;
    if (h.health) {
        h.done = 1;
    } else {
        if (ok) {
            h.t = h.clipped ? h.t_end : h.t + dt_att;
            h.cur ^= 1;
            h.step += 1;
            h.nsteps += 1;
        } else {
            h.nrej += 1;
        }
        double f = (err == 0.0) ? 5.0 : 0.9 * pow(h.tol / err, h.ctrl_exp);
        f = fmin(5.0, fmax(0.2, f));
        const double dn = dt_att * f;
        h.dt_next = dn;
        if (dn < h.dt_min) {
            h.health |= 2;
            h.done = 1;
        } else if (ok && h.clipped) {
            h.done = 1;
        } else {
            const double rem = h.t_end - h.t;
            if (dn >= rem) { h.dt = rem; h.clipped = 1; }
            else { h.dt = dn; h.clipped = 0; }
            h.dtau = (float)(h.dt * h.gms);
        }
    }
    if (!live) return;
    if (a < h.log_cap && h.log) {
        llg_attempt r;
        r.dt = dt_att;
        r.err = errf;
        r.accepted = ok ? 1 : 0;
        h.log[a] = r;
    }
    *st = h;
}

__global__ void ctrl_dp45_kernel(DevState* st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    dp45_control(st);
}

// one thread per film of a batch
__global__ void ctrl_dp45_group_kernel(DevState* states, int nfilms) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < nfilms) dp45_control(states + f);
}

__global__ void state_add_evals_kernel(DevState* st, int evals) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st->nevals += evals;
}

// renormalise m in place; flag | |m| - 1 | > 1e-3 or non-finite values
__global__ void normalize_check_kernel(float* m, int ncells, int* bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncells) return;
    const float x = m[i], y = m[ncells + i], z = m[2 * ncells + i];
    const float n = sqrtf(x * x + y * y + z * z);
    if (!isfinite(n) || fabsf(n - 1.f) > 1e-3f) { atomicOr(bad, 1); return; }
    m[i] = x / n; m[ncells + i] = y / n; m[2 * ncells + i] = z / n;
}

// flag | |m| - 1 | > 1e-3 or non-finite values; m itself is left as it is
__global__ void check_unit_kernel(const float* m, int ncells, int* bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncells) return;
    const float x = m[i], y = m[ncells + i], z = m[2 * ncells + i];
    const float n = sqrtf(x * x + y * y + z * z);
    if (!isfinite(n) || fabsf(n - 1.f) > 1e-3f) atomicOr(bad, 1);
}

// FFT self-check: `batch` vectors of length n, forward+inverse (or inverse
// only), scaled by 1/n; one block per group of vectors that fits in LDS.
template <int MAXE>
__global__ __launch_bounds__(CT) void fft_test_kernel(float2* data, int n, int batch, int per_block,
                                                     FftPlan pl, const float2* __restrict__ tw,
                                                     int inverse_only) {
    extern __shared__ float2 lds[];
    const int b0 = blockIdx.x * per_block;
    const int nb = min(per_block, batch - b0);
    if (nb <= 0) return;
    for (int e = threadIdx.x; e < nb * n; e += CT) lds[e] = data[(long long)b0 * n + e];
    __syncthreads();
    if (!inverse_only) lds_fft<MAXE>(lds, pl, nb, tw, 1, false, threadIdx.x, CT);
    lds_fft<MAXE>(lds, pl, nb, tw, 1, true, threadIdx.x, CT);
    const float s = 1.0f / (float)n;
    for (int e = threadIdx.x; e < nb * n; e += CT) {
        const float2 v = lds[e];
        data[(long long)b0 * n + e] = f2(v.x * s, v.y * s);
    }
}

// ---------------------------------------------------------------------------
// launchers: check the shapes the kernels assume before launching
// ---------------------------------------------------------------------------
// smallest instantiation whose per-thread slots hold the three packed
// transforms (3 Px elements) and the cells of two rows (2 nx)
static int row_maxe(int Px, int nx) {
    for (int me : {6, 12, 24})
        if (3 * Px <= me * RT && 2 * nx <= ((me + 2) / 3) * RT) return me;
    return -1;
}

hipError_t launch_row_fwd(const Grid& g, const Phys& p, const FftPlan& px, const float2* twx,
                          float2* S, const FwdArgs& fa, DevState* st, hipStream_t s) {
    (void)p;
    const int me = row_maxe(g.Px, g.nx);
    if (me < 0 || px.L != g.Px || g.nx > g.Px) return hipErrorInvalidValue;
    const dim3 grid((g.nrows + 1) / 2), block(RT);
    const size_t sh = 3 * (size_t)g.Px * sizeof(float2);
    switch (me) {
        case 6: hipLaunchKernelGGL((row_fwd_kernel<6>), grid, block, sh, s, g, px, twx, S, fa, st); break;
        case 12: hipLaunchKernelGGL((row_fwd_kernel<12>), grid, block, sh, s, g, px, twx, S, fa, st); break;
        default: hipLaunchKernelGGL((row_fwd_kernel<24>), grid, block, sh, s, g, px, twx, S, fa, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_row_inv(const Grid& g, const Phys& p, const FftPlan& px, const float2* twx,
                          float2* S, const StageArgs& sa, DevState* st, hipStream_t s) {
    const int me = row_maxe(g.Px, g.nx);
    if (me < 0 || px.L != g.Px || g.nx > g.Px || sa.nk > kMaxK) return hipErrorInvalidValue;
    if ((sa.mode == ROW_STAGE || sa.mode == ROW_ERROR) && sa.nk < 1) return hipErrorInvalidValue;
    const dim3 grid((g.nrows + 1) / 2), block(RT);
    const size_t sh = 3 * (size_t)g.Px * sizeof(float2);
    switch (me) {
        case 6: hipLaunchKernelGGL((row_inv_kernel<6>), grid, block, sh, s, g, p, px, twx, S, sa, st); break;
        case 12: hipLaunchKernelGGL((row_inv_kernel<12>), grid, block, sh, s, g, p, px, twx, S, sa, st); break;
        default: hipLaunchKernelGGL((row_inv_kernel<24>), grid, block, sh, s, g, p, px, twx, S, sa, st); break;
    }
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_col_mode(const ColArgs& a, DevState* st, int me, hipStream_t s) {
    const int nblk = a.nouter * a.ntiles;
    const int Lh = a.split ? a.P / 2 : a.P;
    const size_t sh = 3 * (size_t)a.W * Lh * sizeof(float2);
    const dim3 grid(nblk), block(CT);
    switch (me) {
        case 6: hipLaunchKernelGGL((col_kernel<6, MODE>), grid, block, sh, s, a, st); break;
        case 12: hipLaunchKernelGGL((col_kernel<12, MODE>), grid, block, sh, s, a, st); break;
        default: hipLaunchKernelGGL((col_kernel<24, MODE>), grid, block, sh, s, a, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_col(const ColArgs& a, DevState* st, int mode, hipStream_t s) {
    const int Lh = a.split ? a.P / 2 : a.P;
    if (a.plan.L != Lh || a.W < 1 || a.ntiles != (a.nkx + a.W - 1) / a.W) return hipErrorInvalidValue;
    if (a.split && a.P % 2) return hipErrorInvalidValue;
    // non-zero inputs (forward) and kept outputs (inverse) fit one half
    if (mode != COL_INV && (a.n_in < 1 || a.n_in > Lh)) return hipErrorInvalidValue;
    if (mode != COL_FWD && (a.n_out < 1 || a.n_out > Lh)) return hipErrorInvalidValue;
    if (mode == COL_FULL && a.n_in != a.n_out) return hipErrorInvalidValue;
    // elements per thread: FFT buffer, kept inputs and outputs
    int need = 3 * a.W * Lh;
    if (mode != COL_INV) need = max(need, 3 * a.W * a.n_in);
    if (mode != COL_FWD) need = max(need, 3 * a.W * a.n_out);
    need = (need + CT - 1) / CT;
    int me = need <= 6 ? 6 : need <= 12 ? 12 : need <= 24 ? 24 : -1;
    if (me < 0) return hipErrorInvalidValue;
    switch (mode) {
        case COL_FWD: return launch_col_mode<COL_FWD>(a, st, me, s);
        case COL_FULL: return launch_col_mode<COL_FULL>(a, st, me, s);
        default: return launch_col_mode<COL_INV>(a, st, me, s);
    }
}

hipError_t launch_ctrl_fixed(DevState* st, int evals, double dt, hipStream_t s) {
    (void)dt;
    hipLaunchKernelGGL(ctrl_fixed_kernel, dim3(1), dim3(64), 0, s, st, evals);
    return hipGetLastError();
}

hipError_t launch_ctrl_fixed_group(DevState* states, int nfilms, int evals, hipStream_t s) {
    hipLaunchKernelGGL(ctrl_fixed_group_kernel, dim3((nfilms + 63) / 64), dim3(64), 0, s, states, nfilms, evals);
    return hipGetLastError();
}

hipError_t launch_ctrl_dp45(DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(ctrl_dp45_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_ctrl_dm(DevState* st, hipStream_t s) {
    hipLaunchKernelGGL(ctrl_dm_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_ctrl_dm_accept(DevState* st, int evals, hipStream_t s) {
    hipLaunchKernelGGL(ctrl_dm_accept_kernel, dim3(1), dim3(64), 0, s, st, evals);
    return hipGetLastError();
}

hipError_t launch_ctrl_dp45_group(DevState* states, int nfilms, hipStream_t s) {
    hipLaunchKernelGGL(ctrl_dp45_group_kernel, dim3((nfilms + 63) / 64), dim3(64), 0, s, states, nfilms);
    return hipGetLastError();
}

hipError_t launch_state_add_evals(DevState* st, int evals, hipStream_t s) {
    hipLaunchKernelGGL(state_add_evals_kernel, dim3(1), dim3(64), 0, s, st, evals);
    return hipGetLastError();
}

hipError_t launch_check_unit(const float* m, int ncells, int* bad, hipStream_t s) {
    hipLaunchKernelGGL(check_unit_kernel, dim3((ncells + 255) / 256), dim3(256), 0, s, m, ncells, bad);
    return hipGetLastError();
}

hipError_t launch_normalize_check(float* m, int ncells, int* bad, hipStream_t s) {
    hipLaunchKernelGGL(normalize_check_kernel, dim3((ncells + 255) / 256), dim3(256), 0, s, m, ncells, bad);
    return hipGetLastError();
}

hipError_t launch_fft_test(float2* data, int n, int batch, const FftPlan& pl, const float2* tw,
                           int inverse_only, hipStream_t s) {
    if (pl.L != n || n < 1 || batch < 1) return hipErrorInvalidValue;
    // as many vectors per block as keep the per-thread element count <= 24
    int per_block = (24 * CT) / n;
    if (per_block < 1) return hipErrorInvalidValue;
    per_block = min(per_block, batch);
    const int need = (per_block * n + CT - 1) / CT;
    const int me = need <= 6 ? 6 : need <= 12 ? 12 : 24;
    const dim3 grid((batch + per_block - 1) / per_block), block(CT);
    const size_t sh = (size_t)per_block * n * sizeof(float2);
    switch (me) {
        case 6: hipLaunchKernelGGL((fft_test_kernel<6>), grid, block, sh, s, data, n, batch, per_block, pl, tw, inverse_only); break;
        case 12: hipLaunchKernelGGL((fft_test_kernel<12>), grid, block, sh, s, data, n, batch, per_block, pl, tw, inverse_only); break;
        default: hipLaunchKernelGGL((fft_test_kernel<24>), grid, block, sh, s, data, n, batch, per_block, pl, tw, inverse_only); break;
    }
    return hipGetLastError();
}

}  // namespace llg
