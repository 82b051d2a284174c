// Per-cell physics shared by the fused row kernels: the local effective
// field terms (exchange, Eq. 3; uniaxial anisotropy, Eq. 4; applied field;
// thermal field, Eq. 6) and the Landau-Lifshitz torque (Eq. 1), in reduced
// units (fields / Ms, time * gamma0 Ms).
#pragma once

#include "internal.hpp"

namespace llg {

// cubic anisotropy (Eq. 5): h = -sum_i a_i (kc1 (a_j^2 + a_k^2) + kc2 a_j^2 a_k^2) c_i
// with a_i = m . c_i, in reduced units
__device__ __forceinline__ void cubic_field(const Phys& p, float mx, float my, float mz,
                                            float& hx, float& hy, float& hz) {
    float a[3], a2[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        a[i] = mx * p.c[i][0] + my * p.c[i][1] + mz * p.c[i][2];
        a2[i] = a[i] * a[i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int j = (i + 1) % 3, k = (i + 2) % 3;
        const float f = a[i] * (p.kc1 * (a2[j] + a2[k]) + p.kc2 * a2[j] * a2[k]);
        hx -= f * p.c[i][0]; hy -= f * p.c[i][1]; hz -= f * p.c[i][2];
    }
}

// effective field without the demag term (reduced units), for cell (r, x)
__device__ __forceinline__ void local_field(const Grid& g, const Phys& p, const float* __restrict__ m,
                                            int r, int x, float mx, float my, float mz,
                                            uint64_t step, float& hx, float& hy, float& hz) {
    const long long cs = g.ncells;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    auto nb = [&](int rr, int xx, float c) {
        const long long i = (long long)rr * g.nx + xx;
        sx += c * (m[i] - mx);
        sy += c * (m[cs + i] - my);
        sz += c * (m[2 * cs + i] - mz);
    };
    if (p.cex[0] != 0.f && g.nx > 1) {
        const float c = p.cex[0];
        if (x > 0) nb(r, x - 1, c); else if (g.pbc[0]) nb(r, g.nx - 1, c);
        if (x < g.nx - 1) nb(r, x + 1, c); else if (g.pbc[0]) nb(r, 0, c);
    }
    if (p.cex[1] != 0.f && g.ny > 1) {
        const float c = p.cex[1];
        const int y = r % g.ny;
        if (y > 0) nb(r - 1, x, c); else if (g.pbc[1]) nb(r + g.ny - 1, x, c);
        if (y < g.ny - 1) nb(r + 1, x, c); else if (g.pbc[1]) nb(r - (g.ny - 1), x, c);
    }
    if (p.cex[2] != 0.f && g.nz > 1) {
        const float c = p.cex[2];
        const int z = r / g.ny;
        if (z > 0) nb(r - g.ny, x, c); else if (g.pbc[2]) nb(r + (g.nz - 1) * g.ny, x, c);
        if (z < g.nz - 1) nb(r + g.ny, x, c); else if (g.pbc[2]) nb(r - (g.nz - 1) * g.ny, x, c);
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
        thermal_eta((uint32_t)((long long)r * g.nx + x), step, p.seed_lo, p.seed_hi, ex, ey, ez);
        hx += p.sig_th * ex; hy += p.sig_th * ey; hz += p.sig_th * ez;
    }
}

// Zhang-Li torque (Eq. 7-8) in reduced units, added to k:
// -1/(1+alpha^2) [m x (m x D) + (xi - alpha) m x D], D = (j . grad) m as
// weighted central differences (weights cj fold in b_j / (2 d gamma0 Ms))
__device__ __forceinline__ void stt_torque(const Phys& p, float mx, float my, float mz,
                                           float Dx, float Dy, float Dz, float& kx, float& ky, float& kz) {
    const float ax = my * Dz - mz * Dy, ay = mz * Dx - mx * Dz, az = mx * Dy - my * Dx;
    const float bx = my * az - mz * ay, by = mz * ax - mx * az, bz = mx * ay - my * ax;
    kx += p.llpre * (bx + p.xi_a * ax);
    ky += p.llpre * (by + p.xi_a * ay);
    kz += p.llpre * (bz + p.xi_a * az);
}

// D = (j . grad) m of cell (r, x) from global memory: central differences;
// at a free surface the missing neighbour is the cell itself, a periodic
// axis wraps, an axis one cell long contributes nothing
__device__ __forceinline__ void stt_gradient(const Grid& g, const Phys& p, const float* __restrict__ m, int r,
                                             int x, float mx, float my, float mz, float& Dx, float& Dy, float& Dz) {
    const long long cs = g.ncells;
    Dx = Dy = Dz = 0.f;
    auto diff = [&](long long up, long long dn, float c, bool has_up, bool has_dn) {
        const float ux = has_up ? m[up] : mx, uy = has_up ? m[cs + up] : my, uz = has_up ? m[2 * cs + up] : mz;
        const float vx = has_dn ? m[dn] : mx, vy = has_dn ? m[cs + dn] : my, vz = has_dn ? m[2 * cs + dn] : mz;
        Dx += c * (ux - vx); Dy += c * (uy - vy); Dz += c * (uz - vz);
    };
    const long long i = (long long)r * g.nx + x;
    if (p.cj[0] != 0.f && g.nx > 1) {
        const bool hu = x < g.nx - 1 || g.pbc[0], hd = x > 0 || g.pbc[0];
        diff(x < g.nx - 1 ? i + 1 : i - (g.nx - 1), x > 0 ? i - 1 : i + (g.nx - 1), p.cj[0], hu, hd);
    }
    if (p.cj[1] != 0.f && g.ny > 1) {
        const int y = r % g.ny;
        const bool hu = y < g.ny - 1 || g.pbc[1], hd = y > 0 || g.pbc[1];
        const long long row = g.nx;
        diff(y < g.ny - 1 ? i + row : i - (long long)(g.ny - 1) * row, y > 0 ? i - row : i + (long long)(g.ny - 1) * row,
             p.cj[1], hu, hd);
    }
    if (p.cj[2] != 0.f && g.nz > 1) {
        const int z = r / g.ny;
        const bool hu = z < g.nz - 1 || g.pbc[2], hd = z > 0 || g.pbc[2];
        const long long sl = (long long)g.ny * g.nx;
        diff(z < g.nz - 1 ? i + sl : i - (long long)(g.nz - 1) * sl, z > 0 ? i - sl : i + (long long)(g.nz - 1) * sl,
             p.cj[2], hu, hd);
    }
}

// dm/dtau = -1/(1+alpha^2) (m x h + alpha m x (m x h))
__device__ __forceinline__ void ll_torque(const Phys& p, float mx, float my, float mz,
                                          float hx, float hy, float hz,
                                          float& kx, float& ky, float& kz) {
    const float ax = my * hz - mz * hy, ay = mz * hx - mx * hz, az = mx * hy - my * hx;
    const float bx = my * az - mz * ay, by = mz * ax - mx * az, bz = mx * ay - my * ax;
    kx = p.llpre * (ax + p.alpha * bx);
    ky = p.llpre * (ay + p.alpha * by);
    kz = p.llpre * (az + p.alpha * bz);
}

}  // namespace llg
