// Host-side helpers shared by the single-film runtime (solver.hip) and the
// batched runtime (batch.hip): physical constants, the SI -> reduced-unit
// conversion of the field coefficients, the Butcher tableaux of the
// integrators, and FFT length / plan / twiddle helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <vector>

#include "internal.hpp"
#include "llg.h"

namespace llg {
namespace host {

constexpr double kMu0 = 4.0e-7 * M_PI;
constexpr double kGammaLL = 1.7595e11;
constexpr double kGamma0 = kMu0 * kGammaLL;
constexpr double kBoltzmann = 1.380649e-23;
constexpr double kDtMin = 1e-18;
constexpr int kMaxPx = 2048;
constexpr int kMaxHalf = 2048;

// Butcher tableaux (rows of A for stages 2..S, then b)
struct Tableau {
    int S;
    double A[7][7];
    double b[7];
    double bhat[7];
};

inline Tableau tab_euler() { Tableau t = {}; t.S = 1; t.b[0] = 1.0; return t; }
inline Tableau tab_heun() { Tableau t = {}; t.S = 2; t.A[1][0] = 1.0; t.b[0] = 0.5; t.b[1] = 0.5; return t; }
inline Tableau tab_rk4() {
    Tableau t = {};
    t.S = 4;
    t.A[1][0] = 0.5; t.A[2][1] = 0.5; t.A[3][2] = 1.0;
    t.b[0] = 1.0 / 6.0; t.b[1] = 1.0 / 3.0; t.b[2] = 1.0 / 3.0; t.b[3] = 1.0 / 6.0;
    return t;
}
// Dormand & Prince (1980) RK5(4)7M; row 6 equals b (first same as last)
inline Tableau tab_dp45() {
    Tableau t = {};
    t.S = 7;
    t.A[1][0] = 1.0 / 5.0;
    t.A[2][0] = 3.0 / 40.0; t.A[2][1] = 9.0 / 40.0;
    t.A[3][0] = 44.0 / 45.0; t.A[3][1] = -56.0 / 15.0; t.A[3][2] = 32.0 / 9.0;
    t.A[4][0] = 19372.0 / 6561.0; t.A[4][1] = -25360.0 / 2187.0; t.A[4][2] = 64448.0 / 6561.0;
    t.A[4][3] = -212.0 / 729.0;
    t.A[5][0] = 9017.0 / 3168.0; t.A[5][1] = -355.0 / 33.0; t.A[5][2] = 46732.0 / 5247.0;
    t.A[5][3] = 49.0 / 176.0; t.A[5][4] = -5103.0 / 18656.0;
    t.A[6][0] = 35.0 / 384.0; t.A[6][1] = 0.0; t.A[6][2] = 500.0 / 1113.0; t.A[6][3] = 125.0 / 192.0;
    t.A[6][4] = -2187.0 / 6784.0; t.A[6][5] = 11.0 / 84.0;
    for (int j = 0; j < 6; ++j) t.b[j] = t.A[6][j];
    t.b[6] = 0.0;
    t.bhat[0] = 5179.0 / 57600.0; t.bhat[1] = 0.0; t.bhat[2] = 7571.0 / 16695.0;
    t.bhat[3] = 393.0 / 640.0; t.bhat[4] = -92097.0 / 339200.0; t.bhat[5] = 187.0 / 2100.0;
    t.bhat[6] = 1.0 / 40.0;
    return t;
}

inline bool good_len(int L) {
    if (L < 1) return false;
    for (int f : {2, 3, 5, 7})
        while (L % f == 0) L /= f;
    return L == 1;
}

// smallest even FFT length >= 2n made of 2, 3, 5, 7 (open axis)
inline int pad_len(int n) {
    int L = 2 * n;
    while (!good_len(L)) L += 2;
    return L;
}

inline bool make_plan(int L, FftPlan& p) {
    p.L = L;
    p.ns = 0;
    int n = L;
    const int order[6] = {8, 4, 2, 3, 5, 7};
    for (int r : order)
        while (n % r == 0) {
            if (p.ns >= kMaxStages) return false;
            p.rad[p.ns++] = r;
            n /= r;
        }
    return n == 1;
}


// material and field parameters of one problem (SI)
struct Material {
    double Ms = 0, Aex = 0, alpha = 0;
    double Ku = 0, u[3] = {1, 0, 0};
    double B[3] = {0, 0, 0};
    double d[3] = {0, 0, 0};
    double T = 0;
    uint64_t seed = 0;
    int terms = LLG_TERM_ALL;
};

// coefficients in reduced units (fields / Ms, time * gamma0 Ms)
inline Phys phys_of(const Material& s, double dt_thermal) {
    Phys p = {};
    const double Ms2 = s.Ms * s.Ms;
    for (int a = 0; a < 3; ++a)
        p.cex[a] = (s.terms & LLG_TERM_EXCHANGE) ? (float)(2.0 * s.Aex / (kMu0 * Ms2 * s.d[a] * s.d[a])) : 0.f;
    const double un = sqrt(s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2]);
    p.ku = (s.terms & LLG_TERM_ANISOTROPY) ? (float)(2.0 * s.Ku / (kMu0 * Ms2)) : 0.f;
    for (int a = 0; a < 3; ++a) {
        p.u[a] = (float)(s.u[a] / un);
        p.hz[a] = (s.terms & LLG_TERM_ZEEMAN) ? (float)(s.B[a] / (kMu0 * s.Ms)) : 0.f;
    }
    p.alpha = (float)s.alpha;
    p.llpre = (float)(-1.0 / (1.0 + s.alpha * s.alpha));
    p.sig_th = 0.f;
    if ((s.terms & LLG_TERM_THERMAL) && s.T > 0.0 && dt_thermal > 0.0) {
        const double V = s.d[0] * s.d[1] * s.d[2];
        const double sig = sqrt(2.0 * s.alpha * kBoltzmann * s.T / (kGamma0 * kMu0 * s.Ms * V * dt_thermal));
        p.sig_th = (float)(sig / s.Ms);
    }
    p.Ms = (float)s.Ms;
    p.seed_lo = (uint32_t)(s.seed & 0xffffffffu);
    p.seed_hi = (uint32_t)(s.seed >> 32);
    p.demag_on = (s.terms & LLG_TERM_DEMAG) ? 1 : 0;
    return p;
}

inline hipError_t make_tw(int L, float2** out) {
    std::vector<float2> h(L);
    for (int m = 0; m < L; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)L;
        h[m].x = (float)cos(a);
        h[m].y = (float)sin(a);
    }
    hipError_t e = hipMalloc(out, sizeof(float2) * L);
    if (e == hipSuccess) e = hipMemcpy(*out, h.data(), sizeof(float2) * L, hipMemcpyHostToDevice);
    return e;
}


}  // namespace host
}  // namespace llg
