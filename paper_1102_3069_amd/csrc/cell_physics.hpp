// Per-cell physics shared by the fused row kernels: the local effective
// field terms (exchange, Eq. 3; uniaxial anisotropy, Eq. 4; applied field;
// thermal field, Eq. 6) and the Landau-Lifshitz torque (Eq. 1), in reduced
// units (fields / Ms, time * gamma0 Ms).
#pragma once

#include "internal.hpp"

namespace llg {

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
    hx += p.hz[0]; hy += p.hz[1]; hz += p.hz[2];
    if (p.sig_th != 0.f) {
        float ex, ey, ez;
        thermal_eta((uint32_t)((long long)r * g.nx + x), step, p.seed_lo, p.seed_hi, ex, ey, ez);
        hx += p.sig_th * ex; hy += p.sig_th * ey; hz += p.sig_th * ez;
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
