// Host-side logic of the library, exercised without a GPU under the address
// and undefined-behaviour sanitizers (built by tests/test_host_sanitized.py):
// FFT length padding and plans, the Runge-Kutta tableaux the kernels are
// driven with (order conditions of Butcher's theory up to each method's
// order, for the solution and the embedded estimate: Sec. 2.2), and the
// reduced-unit coefficients (finite; the thermal sigma of Eq. 6).
#include <math.h>
#include <stdio.h>

#include "host_common.hpp"

using namespace llg;
using namespace llg::host;

static int failures = 0;
#define CHECK(cond, ...)                      \
    do {                                      \
        if (!(cond)) {                        \
            ++failures;                       \
            fprintf(stderr, "FAIL: " __VA_ARGS__); \
            fputc('\n', stderr);              \
        }                                     \
    } while (0)

// sum_i w_i f_i for a stage vector f
static double dot(const double* w, const double* f, int S) {
    double s = 0.0;
    for (int i = 0; i < S; ++i) s += w[i] * f[i];
    return s;
}
static void matvec(const Tableau& t, const double* f, double* out) {
    for (int i = 0; i < t.S; ++i) {
        out[i] = 0.0;
        for (int j = 0; j < i; ++j) out[i] += t.A[i][j] * f[j];
    }
}

// the order conditions up to order p (p <= 5) of weights w with matrix A
static void order_conditions(const char* name, const Tableau& t, const double* w, int p) {
    const int S = t.S;
    double c[7], c2[7], c3[7], c4[7], Ac[7], Ac2[7], Ac3[7], AAc[7], AAc2[7], AAAc[7], cAc[7], AcAc[7];
    double one[7];
    for (int i = 0; i < S; ++i) one[i] = 1.0;
    matvec(t, one, c);
    for (int i = 0; i < S; ++i) { c2[i] = c[i] * c[i]; c3[i] = c2[i] * c[i]; c4[i] = c3[i] * c[i]; }
    matvec(t, c, Ac);
    matvec(t, c2, Ac2);
    matvec(t, c3, Ac3);
    matvec(t, Ac, AAc);
    matvec(t, Ac2, AAc2);
    matvec(t, AAc, AAAc);
    for (int i = 0; i < S; ++i) cAc[i] = c[i] * Ac[i];
    matvec(t, cAc, AcAc);
    struct Cond { int order; double value, expect; const char* what; };
    double cAcv[7], c2Acv[7], cAc2v[7], cAAcv[7], Ac_sq[7];
    for (int i = 0; i < S; ++i) {
        cAcv[i] = c[i] * Ac[i]; c2Acv[i] = c2[i] * Ac[i]; cAc2v[i] = c[i] * Ac2[i];
        cAAcv[i] = c[i] * AAc[i]; Ac_sq[i] = Ac[i] * Ac[i];
    }
    const Cond conds[] = {
        {1, dot(w, one, S), 1.0, "sum b"},
        {2, dot(w, c, S), 0.5, "b.c"},
        {3, dot(w, c2, S), 1.0 / 3.0, "b.c^2"},
        {3, dot(w, Ac, S), 1.0 / 6.0, "b.Ac"},
        {4, dot(w, c3, S), 0.25, "b.c^3"},
        {4, dot(w, cAcv, S), 0.125, "b.(c Ac)"},
        {4, dot(w, Ac2, S), 1.0 / 12.0, "b.Ac^2"},
        {4, dot(w, AAc, S), 1.0 / 24.0, "b.AAc"},
        {5, dot(w, c4, S), 0.2, "b.c^4"},
        {5, dot(w, c2Acv, S), 0.1, "b.(c^2 Ac)"},
        {5, dot(w, cAc2v, S), 1.0 / 15.0, "b.(c Ac^2)"},
        {5, dot(w, cAAcv, S), 1.0 / 30.0, "b.(c AAc)"},
        {5, dot(w, Ac_sq, S), 0.05, "b.(Ac)^2"},
        {5, dot(w, Ac3, S), 0.05, "b.Ac^3"},
        {5, dot(w, AcAc, S), 1.0 / 40.0, "b.A(c Ac)"},
        {5, dot(w, AAc2, S), 1.0 / 60.0, "b.AAc^2"},
        {5, dot(w, AAAc, S), 1.0 / 120.0, "b.AAAc"},
    };
    for (const Cond& k : conds)
        if (k.order <= p) CHECK(fabs(k.value - k.expect) < 1e-13, "%s: %s = %.17g, expected %.17g", name, k.what, k.value, k.expect);
    // one condition of order p + 1 fails, so the order is exactly p
    if (p < 5) {
        bool all = true;
        for (const Cond& k : conds)
            if (k.order == p + 1 && fabs(k.value - k.expect) >= 1e-13) all = false;
        CHECK(!all, "%s: every order-%d condition also holds", name, p + 1);
    }
}

int main() {
    // padding: the smallest even 2,3,5,7-smooth length >= 2n
    for (int n = 1; n <= 4096; ++n) {
        const int L = pad_len(n);
        CHECK(L >= 2 * n && L % 2 == 0 && good_len(L), "pad_len(%d) = %d", n, L);
        for (int m = 2 * n; m < L; m += 2) CHECK(!good_len(m), "pad_len(%d) = %d skips %d", n, L, m);
    }
    // plans: radices multiply back to the length
    for (int L = 1; L <= 4096; ++L) {
        FftPlan p;
        const bool ok = make_plan(L, p);
        CHECK(ok == good_len(L) || !good_len(L), "make_plan(%d) refused a smooth length", L);
        if (!ok) continue;
        long prod = 1;
        for (int s = 0; s < p.ns; ++s) prod *= p.rad[s];
        CHECK(prod == L && p.L == L, "make_plan(%d): radices give %ld", L, prod);
    }
    // tableaux: the solution weights b to the method's order, the embedded
    // weights to the estimate's order
    order_conditions("euler", tab_euler(), tab_euler().b, 1);
    order_conditions("heun", tab_heun(), tab_heun().b, 2);
    order_conditions("rk3", tab_rk3(), tab_rk3().b, 3);
    order_conditions("rk4", tab_rk4(), tab_rk4().b, 4);
    const int methods[4] = {LLG_RKDP45, LLG_RK23, LLG_RKCK, LLG_RK12};
    const char* names[4] = {"dp45", "rk23", "rkck", "rk12"};
    const int orders[4] = {5, 3, 5, 2};
    for (int k = 0; k < 4; ++k) {
        Adaptive ad;
        CHECK(adaptive_of(methods[k], &ad), "%s is not an adaptive pair", names[k]);
        order_conditions(names[k], ad.t, ad.t.b, orders[k]);
        char emb[32];
        snprintf(emb, sizeof emb, "%s (embedded)", names[k]);
        order_conditions(emb, ad.t, ad.t.bhat, ad.q);
        CHECK(ad.q == orders[k] - 1, "%s: estimate order %d", names[k], ad.q);
        if (ad.fsal) {   // the last row equals b: the last stage is at the new state
            for (int j = 0; j < ad.t.S - 1; ++j)
                CHECK(ad.t.A[ad.t.S - 1][j] == ad.t.b[j], "%s: last row differs from b at %d", names[k], j);
        }
    }
    // reduced units: the coefficients of a full problem are finite, and the
    // thermal sigma is Eq. 6's over Ms
    Material m;
    m.Ms = 8e5; m.Aex = 1.3e-11; m.alpha = 0.1; m.Ku = 5e3; m.u[0] = 1; m.u[1] = 1; m.u[2] = 0;
    m.Kc1 = 1e4; m.Kc2 = -2e3; m.j[0] = 1e12; m.P = 0.4; m.xi = 0.05; m.B[0] = 0.01; m.B[2] = -0.02;
    m.d[0] = 4e-9; m.d[1] = 4e-9; m.d[2] = 3e-9; m.T = 300; m.seed = 0x1234567890abcdefull;
    const Phys p = phys_of(m, 1e-13);
    const float* f = reinterpret_cast<const float*>(&p);
    for (size_t i = 0; i < offsetof(Phys, seed_lo) / sizeof(float); ++i) CHECK(isfinite(f[i]), "Phys field %zu", i);
    const double V = m.d[0] * m.d[1] * m.d[2];
    const double sig = sqrt(2.0 * m.alpha * kBoltzmann * m.T / (kGamma0 * kMu0 * m.Ms * V * 1e-13)) / m.Ms;
    CHECK(fabs(p.sig_th - sig) <= 1e-6 * sig, "thermal sigma %g against %g", p.sig_th, sig);
    CHECK(fabs(p.u[0] * p.u[0] + p.u[1] * p.u[1] + p.u[2] * p.u[2] - 1.f) < 1e-6f, "anisotropy axis not unit");
    CHECK(p.seed_lo == 0x90abcdefu && p.seed_hi == 0x12345678u, "seed split");
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("host logic ok\n");
    return 0;
}
