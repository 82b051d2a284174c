// FP64 construction of the demagnetising kernel and its spectrum.
//
// The paper (Sec. 2.1.1, Eq. 2) convolves M with the kernel of the
// magnetostatic integral and (Sec. 3.2) keeps that kernel symmetric so that
// its Fourier transform is real.  The library uses the cell-averaged tensor
//     N(X) = (1/V) int_cell int_cell -(1/4pi) grad grad 1/|r - r'|,
// evaluated
//   * within 8 cells (max-norm) by the closed form of Newell, Williams &
//     Dunlop (1993): a signed 27-point second difference of f (diagonal) or
//     g (off-diagonal), permuted per component;
//   * beyond, as the point-dipole tensor averaged against the product of
//     per-axis tents (d - |s|)^+ with 3-point Gauss-Legendre on each half
//     axis (216 nodes);
//   * plus, along periodic axes, point-dipole images n = -P..P (n != 0),
//     the Nyquist offset of an even periodic length standing for +n/2 and
//     -n/2 with weight 1/2 each.
// All of this, the FFT of the kernel and the residue check run in FP64; the
// result is scaled by -1/(Px Py Pz) (reduced units, unnormalised FFTs) and
// rounded to FP32 once, mirror-compressed along the two non-x axes.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "internal.hpp"

namespace llg {

namespace {

constexpr int TT = 256;

__device__ double nf(double x, double y, double z) {
    x = fabs(x); y = fabs(y); z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double r = (2.0 * x2 - y2 - z2) * R / 6.0;
    const double rxz = sqrt(x2 + z2);
    if (rxz > 0.0) r += 0.5 * y * (z2 - x2) * asinh(y / rxz);
    const double rxy = sqrt(x2 + y2);
    if (rxy > 0.0) r += 0.5 * z * (y2 - x2) * asinh(z / rxy);
    const double xR = x * R;
    if (xR > 0.0) r -= x * y * z * atan(y * z / xR);
    return r;
}

__device__ double ng(double x, double y, double z) {
    const double sgn = (x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0)) * (y > 0.0 ? 1.0 : (y < 0.0 ? -1.0 : 0.0));
    if (sgn == 0.0) return 0.0;
    x = fabs(x); y = fabs(y); z = fabs(z);
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double r = -x * y * R / 3.0;
    const double rxy = sqrt(x2 + y2);
    if (rxy > 0.0) r += x * y * z * asinh(z / rxy);
    const double ryz = sqrt(y2 + z2);
    if (ryz > 0.0) r += y / 6.0 * (3.0 * z2 - y2) * asinh(x / ryz);
    const double rxz = sqrt(x2 + z2);
    if (rxz > 0.0) r += x / 6.0 * (3.0 * z2 - x2) * asinh(y / rxz);
    const double zR = z * R;
    if (zR > 0.0) r -= z2 * z / 6.0 * atan(x * y / zR);
    const double yR = y * R;
    if (yR > 0.0) r -= z * y2 / 2.0 * atan(x * z / yR);
    const double xR = x * R;
    if (xR > 0.0) r -= z * x2 / 2.0 * atan(y * z / xR);
    return sgn * r;
}

// component order: xx, yy, zz, xy, xz, yz
__device__ double newell(int comp, double X, double Y, double Z, double dx, double dy, double dz) {
    // permute so that the evaluated function is f(a, b, c) (diagonal) or
    // g(a, b, c) (off-diagonal) in its own axis order
    double a, b, c, da, db, dc;
    bool diag = comp < 3;
    switch (comp) {
        case 0: a = X; b = Y; c = Z; da = dx; db = dy; dc = dz; break;
        case 1: a = Y; b = X; c = Z; da = dy; db = dx; dc = dz; break;
        case 2: a = Z; b = Y; c = X; da = dz; db = dy; dc = dx; break;
        case 3: a = X; b = Y; c = Z; da = dx; db = dy; dc = dz; break;
        case 4: a = X; b = Z; c = Y; da = dx; db = dz; dc = dy; break;
        default: a = Y; b = Z; c = X; da = dy; db = dz; dc = dx; break;
    }
    const double w[3] = {-1.0, 2.0, -1.0};
    double acc = 0.0;
    for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q)
            for (int r = 0; r < 3; ++r) {
                const double aa = a + (p - 1) * da, bb = b + (q - 1) * db, cc = c + (r - 1) * dc;
                const double v = diag ? nf(aa, bb, cc) : ng(aa, bb, cc);
                acc += w[p] * w[q] * w[r] * v;
            }
    return acc / (4.0 * M_PI * dx * dy * dz);
}

__device__ double dipole(int comp, double x, double y, double z) {
    const double r2 = x * x + y * y + z * z;
    const double r = sqrt(r2);
    const double i3 = 1.0 / (r2 * r), i5 = i3 / r2;
    const double c = 1.0 / (4.0 * M_PI);
    switch (comp) {
        case 0: return c * (i3 - 3.0 * x * x * i5);
        case 1: return c * (i3 - 3.0 * y * y * i5);
        case 2: return c * (i3 - 3.0 * z * z * i5);
        case 3: return c * (-3.0 * x * y * i5);
        case 4: return c * (-3.0 * x * z * i5);
        default: return c * (-3.0 * y * z * i5);
    }
}

// tent quadrature nodes and weights on [-d, d]: 3-point Gauss-Legendre on
// each half, weight d * w_GL * (d - |s|)
__device__ void tent6(double d, double* s, double* w) {
    const double t[3] = {0.5 - 0.5 * sqrt(0.6), 0.5, 0.5 + 0.5 * sqrt(0.6)};
    const double g[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    for (int i = 0; i < 3; ++i) {
        s[2 * i] = d * t[i];
        s[2 * i + 1] = -d * t[i];
        w[2 * i] = w[2 * i + 1] = d * g[i] * (d - d * t[i]);
    }
}

__device__ double far_avg(int comp, double X, double Y, double Z, double dx, double dy, double dz) {
    double sx[6], wx[6], sy[6], wy[6], sz[6], wz[6];
    tent6(dx, sx, wx);
    tent6(dy, sy, wy);
    tent6(dz, sz, wz);
    double acc = 0.0;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            const double wij = wx[i] * wy[j];
            for (int k = 0; k < 6; ++k) acc += wij * wz[k] * dipole(comp, X + sx[i], Y + sy[j], Z + sz[k]);
        }
    return acc / (dx * dy * dz);
}

__device__ double cell_entry(int comp, int i, int j, int k, const TensorGeom& tg) {
    const double dx = tg.d[0], dy = tg.d[1], dz = tg.d[2];
    const int reach = max(abs(i), max(abs(j), abs(k)));
    const double X = i * dx, Y = j * dy, Z = k * dz;
    if (reach <= 8) return newell(comp, X, Y, Z, dx, dy, dz);
    return far_avg(comp, X, Y, Z, dx, dy, dz);
}

__device__ double periodic_entry(int comp, int i, int j, int k, const TensorGeom& tg) {
    double v = cell_entry(comp, i, j, k, tg);
    if (!(tg.pbc[0] || tg.pbc[1] || tg.pbc[2])) return v;
    const int P = tg.images;
    const int ra = tg.pbc[0] ? P : 0, rb = tg.pbc[1] ? P : 0, rc = tg.pbc[2] ? P : 0;
    const double V = tg.d[0] * tg.d[1] * tg.d[2];
    double im = 0.0;
    for (int a = -ra; a <= ra; ++a)
        for (int b = -rb; b <= rb; ++b)
            for (int c = -rc; c <= rc; ++c) {
                if (a == 0 && b == 0 && c == 0) continue;
                im += dipole(comp, (i + a * tg.n[0]) * tg.d[0], (j + b * tg.n[1]) * tg.d[1],
                             (k + c * tg.n[2]) * tg.d[2]);
            }
    return v + V * im;
}

struct Reps {
    int n;
    int off[2];
    double w[2];
};

// offsets that one FFT-grid index stands for along an axis
__device__ Reps axis_reps(int idx, int n, int P, int periodic) {
    Reps r;
    r.n = 0;
    if (!periodic) {
        if (idx < n) { r.n = 1; r.off[0] = idx; r.w[0] = 1.0; }
        else if (idx > P - n) { r.n = 1; r.off[0] = idx - P; r.w[0] = 1.0; }
        return r;
    }
    int q = idx % n;
    if (n % 2 == 0 && q == n / 2) {
        r.n = 2; r.off[0] = n / 2; r.off[1] = -(n / 2); r.w[0] = r.w[1] = 0.5;
        return r;
    }
    if (q > n / 2) q -= n;
    r.n = 1; r.off[0] = q; r.w[0] = 1.0;
    return r;
}

// periodic reduction of an arbitrary signed offset (for the offset query)
__device__ Reps offset_reps(int d, int n, int periodic) {
    Reps r;
    if (!periodic) { r.n = 1; r.off[0] = d; r.w[0] = 1.0; return r; }
    int q = ((d % n) + n) % n;
    return axis_reps(q, n, n, 1);
}

__device__ double entry_from_reps(int comp, const Reps& rx, const Reps& ry, const Reps& rz,
                                  const TensorGeom& tg) {
    double v = 0.0;
    for (int a = 0; a < rx.n; ++a)
        for (int b = 0; b < ry.n; ++b)
            for (int c = 0; c < rz.n; ++c)
                v += rx.w[a] * ry.w[b] * rz.w[c] * periodic_entry(comp, rx.off[a], ry.off[b], rz.off[c], tg);
    return v;
}

__global__ void tensor_grid_kernel(double2* out, int comp, TensorGeom tg) {
    const long long tot = (long long)tg.P[0] * tg.P[1] * tg.P[2];
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= tot) return;
    const int ix = (int)(id % tg.P[0]);
    const int iy = (int)((id / tg.P[0]) % tg.P[1]);
    const int iz = (int)(id / ((long long)tg.P[0] * tg.P[1]));
    const Reps rx = axis_reps(ix, tg.n[0], tg.P[0], tg.pbc[0]);
    const Reps ry = axis_reps(iy, tg.n[1], tg.P[1], tg.pbc[1]);
    const Reps rz = axis_reps(iz, tg.n[2], tg.P[2], tg.pbc[2]);
    double2 v;
    v.x = (rx.n && ry.n && rz.n) ? entry_from_reps(comp, rx, ry, rz, tg) : 0.0;
    v.y = 0.0;
    out[id] = v;
}

__global__ void tensor_offsets_kernel(const int32_t* offs, long long count, double* out, TensorGeom tg) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= count) return;
    const Reps rx = offset_reps(offs[3 * id], tg.n[0], tg.pbc[0]);
    const Reps ry = offset_reps(offs[3 * id + 1], tg.n[1], tg.pbc[1]);
    const Reps rz = offset_reps(offs[3 * id + 2], tg.n[2], tg.pbc[2]);
    for (int c = 0; c < 6; ++c) out[6 * id + c] = entry_from_reps(c, rx, ry, rz, tg);
}

// batched FP64 FFT of lines of a [Pz][Py][Px] complex array along one axis;
// line l starts at (l / inner) * outer_stride + (l % inner) * inner_stride,
// its elements are `as` apart.  A block owns W consecutive lines.
template <int MAXE>
__global__ __launch_bounds__(TT) void fft_lines_f64(double2* data, int nlines, int inner,
                                                    long long inner_stride, long long outer_stride,
                                                    long long as, int W, FftPlan pl,
                                                    const double2* __restrict__ tw) {
    extern __shared__ double2 lds64[];
    const int L = pl.L;
    const int l0 = blockIdx.x * W;
    const int nl = min(W, nlines - l0);
    const bool pos_fast = (as == 1);
    for (int e = threadIdx.x; e < nl * L; e += TT) {
        const int w = pos_fast ? e / L : e % nl;
        const int pos = pos_fast ? e % L : e / nl;
        const int l = l0 + w;
        const long long addr = (long long)(l / inner) * outer_stride + (long long)(l % inner) * inner_stride + pos * as;
        lds64[w * L + pos] = data[addr];
    }
    __syncthreads();
    lds_fft<MAXE>(lds64, pl, nl, tw, 1, false, threadIdx.x, TT);
    for (int e = threadIdx.x; e < nl * L; e += TT) {
        const int w = pos_fast ? e / L : e % nl;
        const int pos = pos_fast ? e % L : e / nl;
        const int l = l0 + w;
        const long long addr = (long long)(l / inner) * outer_stride + (long long)(l % inner) * inner_stride + pos * as;
        data[addr] = lds64[w * L + pos];
    }
}

// max |Re| and |Im| over the spectrum (bit patterns of non-negative doubles
// order like the values)
__global__ void spectrum_residue_kernel(const double2* spec, long long tot, unsigned long long* mx) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= tot) return;
    const double2 v = spec[id];
    atomicMax(&mx[0], (unsigned long long)__double_as_longlong(fabs(v.x)));
    atomicMax(&mx[1], (unsigned long long)__double_as_longlong(fabs(v.y)));
}

// K[comp][o'][kx][a'] = scale * Re spec(kx, ky, kz); 2D: a = y, o = z (one
// plane); 3D: a = z, o = y.  Compressed indices are the non-negative
// frequencies up to P/2 along a and o.
__global__ void compress_kernel(const double2* spec, float* K, int comp, int Px, int Py, int Pz,
                                int nkx, int na_c, int no_c, int two_d, double scale) {
    const long long tot = (long long)no_c * nkx * na_c;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= tot) return;
    const int ia = (int)(id % na_c);
    const int kx = (int)((id / na_c) % nkx);
    const int io = (int)(id / ((long long)na_c * nkx));
    const int ky = two_d ? ia : io;
    const int kz = two_d ? 0 : ia;
    const double v = spec[((long long)kz * Py + ky) * Px + kx].x;
    K[(long long)comp * tot + id] = (float)(v * scale);
}


}  // namespace

// host helpers -----------------------------------------------------------------
static bool factor_plan(int L, FftPlan& p) {
    p.L = L;
    p.ns = 0;
    int n = L;
    while (n % 8 == 0 && p.ns < kMaxStages) { p.rad[p.ns++] = 8; n /= 8; }
    while (n % 4 == 0 && p.ns < kMaxStages) { p.rad[p.ns++] = 4; n /= 4; }
    while (n % 2 == 0 && p.ns < kMaxStages) { p.rad[p.ns++] = 2; n /= 2; }
    while (n % 3 == 0 && p.ns < kMaxStages) { p.rad[p.ns++] = 3; n /= 3; }
    while (n % 5 == 0 && p.ns < kMaxStages) { p.rad[p.ns++] = 5; n /= 5; }
    while (n % 7 == 0 && p.ns < kMaxStages) { p.rad[p.ns++] = 7; n /= 7; }
    return n == 1;
}

#define TRY(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { err = e_; goto done; } } while (0)

static hipError_t fft_axis_f64(double2* data, int Px, int Py, int Pz, int axis, const double2* tw,
                               hipStream_t s) {
    const int L = axis == 0 ? Px : axis == 1 ? Py : Pz;
    if (L == 1) return hipSuccess;
    FftPlan pl;
    if (!factor_plan(L, pl)) return hipErrorInvalidValue;
    if (L > 4096) return hipErrorInvalidValue;
    int W = 4096 / L;
    if (W > 16) W = 16;
    int nlines, inner;
    long long inner_stride, outer_stride, as;
    if (axis == 0) { nlines = Py * Pz; inner = 1; inner_stride = 0; outer_stride = Px; as = 1; }
    else if (axis == 1) { nlines = Px * Pz; inner = Px; inner_stride = 1; outer_stride = (long long)Px * Py; as = Px; }
    else { nlines = Px * Py; inner = Px * Py; inner_stride = 1; outer_stride = 0; as = (long long)Px * Py; }
    const int nblk = (nlines + W - 1) / W;
    const size_t sh = (size_t)W * L * sizeof(double2);
    hipLaunchKernelGGL((fft_lines_f64<16>), dim3(nblk), dim3(TT), sh, s, data, nlines, inner,
                       inner_stride, outer_stride, as, W, pl, tw);
    return hipGetLastError();
}

static hipError_t make_tw64(int L, double2** out) {
    double2* h = (double2*)malloc(sizeof(double2) * L);
    if (!h) return hipErrorOutOfMemory;
    for (int m = 0; m < L; ++m) {
        const double a = -2.0 * M_PI * (double)m / (double)L;
        h[m].x = cos(a);
        h[m].y = sin(a);
    }
    hipError_t e = hipMalloc(out, sizeof(double2) * L);
    if (e == hipSuccess) e = hipMemcpy(*out, h, sizeof(double2) * L, hipMemcpyHostToDevice);
    free(h);
    return e;
}

hipError_t build_kernel_spectrum(const Grid& g, const TensorGeom& tg, float* K, double* resid_out,
                                 hipStream_t s) {
    hipError_t err = hipSuccess;
    const int Px = g.Px, Py = g.Py, Pz = g.Pz;
    const long long tot = (long long)Px * Py * Pz;
    const bool two_d = g.nz == 1;
    const int ncomp = two_d ? 4 : 6;
    const int nkx = g.nkx;
    const int na_c = two_d ? Py / 2 + 1 : Pz / 2 + 1;
    const int no_c = two_d ? 1 : Py / 2 + 1;
    double2* buf = nullptr;
    double2 *twx = nullptr, *twy = nullptr, *twz = nullptr;
    unsigned long long* mx = nullptr;
    unsigned long long hm[2];
    double worst = 0.0;
    TRY(hipMalloc(&buf, sizeof(double2) * tot));
    TRY(hipMalloc(&mx, 2 * sizeof(unsigned long long)));
    TRY(make_tw64(Px, &twx));
    TRY(make_tw64(Py, &twy));
    TRY(make_tw64(Pz, &twz));
    for (int c = 0; c < ncomp; ++c) {
        const int blocks = (int)((tot + TT - 1) / TT);
        hipLaunchKernelGGL(tensor_grid_kernel, dim3(blocks), dim3(TT), 0, s, buf, c, tg);
        TRY(hipGetLastError());
        TRY(fft_axis_f64(buf, Px, Py, Pz, 0, twx, s));
        TRY(fft_axis_f64(buf, Px, Py, Pz, 1, twy, s));
        TRY(fft_axis_f64(buf, Px, Py, Pz, 2, twz, s));
        TRY(hipMemsetAsync(mx, 0, 2 * sizeof(unsigned long long), s));
        hipLaunchKernelGGL(spectrum_residue_kernel, dim3(blocks), dim3(TT), 0, s, buf, tot, mx);
        TRY(hipGetLastError());
        const long long ctot = (long long)no_c * nkx * na_c;
        hipLaunchKernelGGL(compress_kernel, dim3((int)((ctot + TT - 1) / TT)), dim3(TT), 0, s, buf, K, c,
                           Px, Py, Pz, nkx, na_c, no_c, two_d ? 1 : 0, -1.0 / (double)tot);
        TRY(hipGetLastError());
        TRY(hipMemcpyAsync(hm, mx, sizeof(hm), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        {
            double re, im;
            memcpy(&re, &hm[0], sizeof(double));
            memcpy(&im, &hm[1], sizeof(double));
            if (re > 0.0 && im / re > worst) worst = im / re;
        }
    }
    if (resid_out) *resid_out = worst;
done:
    if (buf) (void)hipFree(buf);
    if (mx) (void)hipFree(mx);
    if (twx) (void)hipFree(twx);
    if (twy) (void)hipFree(twy);
    if (twz) (void)hipFree(twz);
    return err;
}

hipError_t tensor_at_offsets(const TensorGeom& tg, const int32_t* offs_dev, long long count,
                             double* out_dev, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(tensor_offsets_kernel, dim3((int)((count + 127) / 128)), dim3(128), 0, s,
                       offs_dev, count, out_dev, tg);
    return hipGetLastError();
}

}  // namespace llg
