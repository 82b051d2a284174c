// Host-side helpers shared by the single-film runtime (solver.hip) and the
// batched runtime (batch.hip): physical constants, the SI -> reduced-unit
// conversion of the field coefficients, the Butcher tableaux of the
// integrators, and FFT length / plan / twiddle helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "internal.hpp"
#include "llg.h"

namespace llg {
namespace host {

// A roctx range over a host-side scope (an API call, a kernel build, a pass
// being enqueued); visible with rocprofv3 --marker-trace, free otherwise.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

constexpr double kMu0 = 4.0e-7 * M_PI;
constexpr double kGammaLL = 1.7595e11;
constexpr double kGamma0 = kMu0 * kGammaLL;
constexpr double kBohrMagneton = 9.2740100783e-24;   // J/T
constexpr double kElectronCharge = 1.602176634e-19;  // C
constexpr double kBoltzmann = 1.380649e-23;
constexpr double kDtMin = 1e-18;
constexpr int kMaxPx = 4096;
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

// Kutta's third-order method
inline Tableau tab_rk3() {
    Tableau t = {};
    t.S = 3;
    t.A[1][0] = 0.5; t.A[2][0] = -1.0; t.A[2][1] = 2.0;
    t.b[0] = 1.0 / 6.0; t.b[1] = 2.0 / 3.0; t.b[2] = 1.0 / 6.0;
    return t;
}
// Heun-Euler 2(1): Heun's method, Euler's method as the embedded estimate
inline Tableau tab_rk12() {
    Tableau t = tab_heun();
    t.bhat[0] = 1.0; t.bhat[1] = 0.0;
    return t;
}
// Bogacki & Shampine (1989) 3(2); row 3 equals b (first same as last)
inline Tableau tab_rk23() {
    Tableau t = {};
    t.S = 4;
    t.A[1][0] = 0.5;
    t.A[2][1] = 0.75;
    t.A[3][0] = 2.0 / 9.0; t.A[3][1] = 1.0 / 3.0; t.A[3][2] = 4.0 / 9.0;
    for (int j = 0; j < 3; ++j) t.b[j] = t.A[3][j];
    t.bhat[0] = 7.0 / 24.0; t.bhat[1] = 0.25; t.bhat[2] = 1.0 / 3.0; t.bhat[3] = 0.125;
    return t;
}
// Cash & Karp (1990) 5(4)
inline Tableau tab_rkck() {
    Tableau t = {};
    t.S = 6;
    t.A[1][0] = 0.2;
    t.A[2][0] = 3.0 / 40.0; t.A[2][1] = 9.0 / 40.0;
    t.A[3][0] = 0.3; t.A[3][1] = -0.9; t.A[3][2] = 1.2;
    t.A[4][0] = -11.0 / 54.0; t.A[4][1] = 2.5; t.A[4][2] = -70.0 / 27.0; t.A[4][3] = 35.0 / 27.0;
    t.A[5][0] = 1631.0 / 55296.0; t.A[5][1] = 175.0 / 512.0; t.A[5][2] = 575.0 / 13824.0;
    t.A[5][3] = 44275.0 / 110592.0; t.A[5][4] = 253.0 / 4096.0;
    t.b[0] = 37.0 / 378.0; t.b[2] = 250.0 / 621.0; t.b[3] = 125.0 / 594.0; t.b[5] = 512.0 / 1771.0;
    t.bhat[0] = 2825.0 / 27648.0; t.bhat[2] = 18575.0 / 48384.0; t.bhat[3] = 13525.0 / 55296.0;
    t.bhat[4] = 277.0 / 14336.0; t.bhat[5] = 0.25;
    return t;
}
// an embedded pair: its tableau, the order q of its error estimate, and
// whether its last stage is evaluated at the new state (first same as last)
struct Adaptive {
    Tableau t;
    int q;
    bool fsal;
};
inline bool adaptive_of(int method, Adaptive* out) {
    switch (method) {
        case LLG_RKDP45: *out = {tab_dp45(), 4, true}; return true;
        case LLG_RK23: *out = {tab_rk23(), 2, true}; return true;
        case LLG_RKCK: *out = {tab_rkck(), 4, false}; return true;
        case LLG_RK12: *out = {tab_rk12(), 1, false}; return true;
        default: return false;
    }
}
inline bool fixed_of(int method, Tableau* out) {
    switch (method) {
        case LLG_EULER: *out = tab_euler(); return true;
        case LLG_HEUN: *out = tab_heun(); return true;
        case LLG_RK3: *out = tab_rk3(); return true;
        case LLG_RK4: *out = tab_rk4(); return true;
        default: return false;
    }
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
    double Kc1 = 0, Kc2 = 0, c1[3] = {1, 0, 0}, c2[3] = {0, 1, 0};
    double j[3] = {0, 0, 0}, P = 0, xi = 0;   // current density (A/m^2), polarisation, non-adiabaticity
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
    // cubic axes: c1 and c2 normalised, c3 = c1 x c2
    {
        double a[3], b[3];
        const double na = sqrt(s.c1[0] * s.c1[0] + s.c1[1] * s.c1[1] + s.c1[2] * s.c1[2]);
        const double nb = sqrt(s.c2[0] * s.c2[0] + s.c2[1] * s.c2[1] + s.c2[2] * s.c2[2]);
        for (int k = 0; k < 3; ++k) { a[k] = s.c1[k] / na; b[k] = s.c2[k] / nb; }
        const double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
        for (int k = 0; k < 3; ++k) { p.c[0][k] = (float)a[k]; p.c[1][k] = (float)b[k]; p.c[2][k] = (float)c[k]; }
        const bool on = (s.terms & LLG_TERM_ANISOTROPY) != 0;
        p.kc1 = on ? (float)(2.0 * s.Kc1 / (kMu0 * Ms2)) : 0.f;
        p.kc2 = on ? (float)(2.0 * s.Kc2 / (kMu0 * Ms2)) : 0.f;
    }
    // Zhang-Li torque (Eq. 7-8): b_j = P mu_B / (e Ms (1 + xi^2)), reduced by
    // gamma0 Ms, with the 1/(2 d) of a central difference folded in
    {
        const double bj = s.P * kBohrMagneton / (kElectronCharge * s.Ms * (1.0 + s.xi * s.xi));
        const bool on = (s.terms & LLG_TERM_STT) && (s.j[0] != 0.0 || s.j[1] != 0.0 || s.j[2] != 0.0) && bj != 0.0;
        p.stt_on = on ? 1 : 0;
        for (int a = 0; a < 3; ++a) p.cj[a] = on ? (float)(bj * s.j[a] / (2.0 * s.d[a] * kGamma0 * s.Ms)) : 0.f;
        p.xi_a = (float)(s.xi - s.alpha);
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
