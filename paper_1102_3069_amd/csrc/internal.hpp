// Internal types of the solver library: problem geometry on the FFT grid,
// reduced-unit coefficients, the device-resident integrator state and the
// argument blocks of the hot-path kernels, plus the launchers the host
// runtime calls.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"
#include "llg.h"

namespace llg {

// Kernel timing for llg_profile_evals: while g_kernel_timing holds event
// pairs, each launch of a compiled hot-path kernel (hot_launch) takes the
// next pair and has it recorded around its own execution
// (hipExtLaunchKernelGGL), so that the pair times that kernel alone, as a
// profiler's kernel trace does; otherwise hot_launch is a plain launch.
struct KernelTiming {
    hipEvent_t* ev = nullptr;
    int left = 0;
};
extern thread_local KernelTiming g_kernel_timing;

template <typename F, typename... A>
inline void hot_launch(F kernel, const dim3& grid, const dim3& block, uint32_t shm, hipStream_t s, A... args) {
    if (g_kernel_timing.left > 0) {
        hipEvent_t* e = g_kernel_timing.ev;
        g_kernel_timing.ev += 2;
        g_kernel_timing.left -= 1;
        hipExtLaunchKernelGGL(kernel, grid, block, shm, s, e[0], e[1], 0u, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
    }
}

// Geometry of the cell grid and of the convolution (FFT) grid.
//   rows  = ny*nz x-rows of nx cells, row r = k*ny + j
//   P*    = FFT length per axis (2n or more on open axes, n on periodic ones)
//   nkx   = Px/2 + 1 retained x frequencies (real-to-complex)
//   nkxp  = row stride of the spectrum buffers (nkx rounded up to 16)
struct Grid {
    int nx, ny, nz;
    int nrows, ncells;
    int pbc[3];
    int Px, Py, Pz;
    int nkx, nkxp;
    int split_y, split_z;   // 1 on an open axis: even/odd half transforms
    int tsh;                // 2D compiled path: spectrum columns in tiles of 2^tsh
    int rvar, cvar;         // compiled-length kernels: variant of the row length Px and of
                            // the column half length Py/2, fixed when the solver or batch
                            // is set up (the spectrum layout depends on rvar)
};

// Spectrum layout of the 2D compiled path: per component, stored columns
// are grouped in tiles of 2^tsh; a tile keeps its rows contiguous, so a
// column read walks 2^tsh-element strides and a row read 2^tsh-element runs.
__host__ __device__ inline int tile_index(int row, int col, int nrows, int tsh) {
    return (((col >> tsh) * nrows + row) << tsh) + (col & ((1 << tsh) - 1));
}

// Coefficients in reduced units: fields are divided by Ms, time is scaled by
// gamma0*Ms (so dm/dtau = -1/(1+alpha^2) (m x h + alpha m x (m x h))).
struct Phys {
    float cex[3];     // 2A/(mu0 Ms^2 d_a^2): exchange coupling per axis
    float ku;         // 2Ku/(mu0 Ms^2)
    float u[3];       // anisotropy axis (unit)
    float kc1, kc2;   // cubic anisotropy 2K1/(mu0 Ms^2), 2K2/(mu0 Ms^2)
    int stt_on;       // Zhang-Li spin-transfer torque present
    float cj[3];      // b_j j_a / (2 d_a gamma0 Ms): central-difference weight per axis
    float xi_a;       // xi - alpha
    float c[3][3];    // cubic axes c1, c2, c3 = c1 x c2 (unit)
    float hz[3];      // applied field B/(mu0 Ms)
    float alpha;
    float llpre;      // -1/(1+alpha^2)
    float sig_th;     // thermal sigma/Ms for the current step size (0: off)
    float Ms;         // A/m, for SI output
    uint32_t seed_lo, seed_hi;
    int demag_on;
};

// Integrator state kept on the device so that the adaptive controller and
// the buffer swaps run without the host.
struct DevState {
    int cur;              // which of the two state buffers holds m
    int done;             // adaptive: reached t_end / diverged; kernels exit early
    int health;           // bit 0: NaN/Inf seen; bit 1: step below dt_min
    uint32_t err_bits;    // max error of the current attempt (float bits)
    int clipped;          // the pending attempt was shortened to land on t_end
    int ev_attempt;       // adaptive: H_eff evaluations per attempt
    double t, dt, dt_next, t_end, tol, dt_min, gms;
    double last_err;
    double ctrl_exp;      // adaptive: step-size exponent 1/(q+1)
    double dt_max;        // bounded-change runs: largest step, s
    float dtau;           // dt * gamma0 * Ms
    float pad1;
    long long step;       // accepted steps (thermal draw counter)
    long long nsteps, nrej, nevals, nattempt;
    long long log_cap;
    llg_attempt* log;
};

// A buffer argument that may follow the state-buffer swap:
// sel 0 -> p[0]; sel 1 -> p[cur]; sel 2 -> p[cur ^ 1].
struct BufRef {
    float* p[2];
    int sel;
};
__host__ __device__ inline BufRef bref(float* p) { BufRef r; r.p[0] = p; r.p[1] = p; r.sel = 0; return r; }
__host__ __device__ inline BufRef bref_cur(float* a, float* b, int which) {
    BufRef r; r.p[0] = a; r.p[1] = b; r.sel = which; return r;
}
__device__ __forceinline__ float* resolve(const BufRef& r, int cur) {
    return r.sel == 0 ? r.p[0] : r.p[r.sel == 1 ? cur : (cur ^ 1)];
}

enum RowMode {
    ROW_EVAL = 0,    // write H_eff (A/m)
    ROW_STAGE = 1,   // k_s, next stage input, its forward x transform
    ROW_ERROR = 2,   // k_s (last stage) and the embedded error estimate
    ROW_KONLY = 3    // k_s only
};

constexpr int kMaxK = 7;

// What the inverse x pass does after computing H_eff.
struct StageArgs {
    int mode;
    int nk;                  // number of k's in the combination (incl. the current one)
    float a[kMaxK];          // combination weights of k_1..k_nk (times dtau)
    float e[kMaxK];          // error weights (ROW_ERROR, or ROW_STAGE with with_err)
    int with_err;            // ROW_STAGE: also the embedded error estimate;
                             // ROW_KONLY: also max over cells |k| (into err_bits)
    int skip_fwd;            // ROW_STAGE: no forward transform of the new state
    BufRef m_in;             // stage input m_s
    BufRef m0;               // state at the start of the step
    BufRef m_out;            // next stage input / new state
    BufRef k_out;            // where k_s goes (p[0] == nullptr: nowhere)
    BufRef kprev[kMaxK];     // k_1 .. k_{nk-1}
    float* h_out;            // ROW_EVAL output
};

// Forward x pass prologue: either plain m, or m_out = normalize(m0 + dtau a1 k1).
struct FwdArgs {
    BufRef m_in;             // plain input (combine == 0)
    int combine;
    float a1;
    BufRef m0, k1, m_out;
};

// Column (y or z) pass.
enum ColMode { COL_FWD = 0, COL_FULL = 1, COL_INV = 2 };

struct ColArgs {
    const float2* in;
    float2* out;
    long long cs_in, os_in, as_in;     // strides (complex elements)
    long long cs_out, os_out, as_out;
    int nouter, nkx, W, ntiles;
    int n_in, n_out, P, split;
    FftPlan plan;                      // length P/2 (split) or P
    const float2* tw;                  // exp(-2 pi i m / P), m < P
    // multiply (COL_FULL): kernel spectrum K[comp][o'][kx][a'], mirror
    // compressed along the multiply axis a and the other axis o.
    const float* K;
    int ncomp;                         // 4 (2D: xx,yy,zz,xy) or 6
    int Pa, Po, na_c, no_c;            // lengths and compressed extents
    int o_split;                       // 3D: the outer (y) index is in split order
    int sign_a[6], sign_o[6];
};

// Column pass of the 2D fast path (packed spectrum, see fast2d.hip).
struct Col2dArgs {
    float2* S;              // packed spectrum [3][ny][nkxp], nkx = Px/2 columns
    const float* K;         // kernel spectrum [4][nkx_full][Py/2+1]
    const float2* tw;       // exp(-2 pi i m / Py), m < Py
    int nkx, nkx_full, nkxp;
    int ny, Py;
    int tsh;                // tile width log2 (see tile_index)
    int nq;                 // frequency classes of the row transforms (column order)
    int var;                // compiled variant of the column half length Py/2
};

// Raises the dynamic LDS limit of kernel `fn` to `bytes` (needed above 64
// KB, refused above the 160 KB of a gfx950 workgroup).  The runtime call is
// made once per (device, kernel); later launches find it in a table.
hipError_t raise_lds_limit(const void* fn, int bytes);

// ---- launchers (kernels.hip) ------------------------------------------------
hipError_t launch_row_fwd(const Grid& g, const Phys& p, const FftPlan& px, const float2* twx,
                          float2* S, const FwdArgs& fa, DevState* st, hipStream_t s);
hipError_t launch_row_inv(const Grid& g, const Phys& p, const FftPlan& px, const float2* twx,
                          float2* S, const StageArgs& sa, DevState* st, hipStream_t s);
hipError_t launch_col(const ColArgs& a, DevState* st, int mode, hipStream_t s);
hipError_t launch_ctrl_fixed(DevState* st, int evals, double dt, hipStream_t s);
hipError_t launch_ctrl_dm(DevState* st, hipStream_t s);
hipError_t launch_ctrl_dm_accept(DevState* st, int evals, hipStream_t s);
hipError_t launch_ctrl_dp45(DevState* st, hipStream_t s);
hipError_t launch_state_add_evals(DevState* st, int evals, hipStream_t s);
hipError_t launch_check_unit(const float* m, int ncells, int* bad, hipStream_t s);
hipError_t launch_normalize_check(float* m, int ncells, int* bad, hipStream_t s);
hipError_t launch_fft_test(float2* data, int n, int batch, const FftPlan& pl, const float2* tw,
                           int inverse_only, hipStream_t s);

// ---- 2D fast path (fast2d.hip) ---------------------------------------------------
// compiled variants per length (elements per lane); var < 0 selects the
// variant of the process-wide table of defaults (llg_autotune,
// llg_set_variants, llg_batch_autotune), 0 until tuned.  A solver or batch
// copies its variants into Grid::rvar / cvar when it is set up, and the
// launchers below use those copies, never the table.
bool fast2d_row_ok(int Px, int var = -1, bool xper = false);
bool fast2d_col_ok(int L, int split, int var = -1);
int fast2d_row_variant(int Px);
int fast2d_tile_shift();
int fast2d_col_variant(int L);
bool fast2d_set_variants(int Px, int row_var, int L, int col_var, bool xper = false);
bool fast2d_set_row_variant(int Px, int var, bool xper);   // one table entry (false: no such variant)
bool fast2d_set_col_variant(int L, int var);
hipError_t launch_row_fwd_fast(const Grid& g, const float2* twx, float2* S, const FwdArgs& fa,
                               DevState* st, hipStream_t s);
hipError_t launch_row_inv_fast(const Grid& g, const Phys& p, const float2* twx, float2* S,
                               const StageArgs& sa, DevState* st, hipStream_t s);
hipError_t launch_col2d_fast(const Col2dArgs& a, DevState* st, hipStream_t s);

// grouped (multi-film) launches: per-film arguments of one pass
struct FilmRow {
    Grid g;
    Phys p;
    const float2* twx;
    float2* S;
    DevState* st;
    StageArgs sa;     // row_inv
    FwdArgs fa;       // row_fwd
};
struct FilmCol {
    Col2dArgs a;
    DevState* st;
};
int fast2d_row_rows_per_block(int Px, int var);
int fast2d_row_classes(int Px, int var = -1);
// elements per lane and frequency classes of a compiled variant (kind 0:
// row length Px, kind 1: column half length L); false if there is none
bool fast2d_variant_shape(int kind, int len, int var, int* elems, int* classes);
// tiled column passes of the 3D path for axes of compiled length (fast3d.hip)
bool fast3d_col_ok(int P, int split, bool full);     // full: the pass with the kernel product
int fast3d_col_width(int P, int split, bool full);
hipError_t launch_col3_tiled(const ColArgs& a, int mode, DevState* st, hipStream_t s);
int fast2d_row_len_at_least(int n);
int fast2d_col_len_at_least(int n);
int fast2d_col_width(int L, int var = -1);
// blocks of one column launch of a film with nkx stored columns
int fast2d_col_blocks(int L, int var, int nkx);
hipError_t launch_row_fwd_group(int Px, int var, const FilmRow* films, const int2* map, int nblocks,
                                hipStream_t s);
hipError_t launch_row_inv_group(int Px, int var, const FilmRow* films, const int2* map, int nblocks,
                                hipStream_t s);
hipError_t launch_col_group(int L, int var, const FilmCol* films, const int2* map, int nblocks, hipStream_t s);
hipError_t launch_ctrl_dp45_group(DevState* states, int nfilms, hipStream_t s);
hipError_t launch_ctrl_fixed_group(DevState* states, int nfilms, int evals, hipStream_t s);

// ---- demag tensor (tensor.hip) --------------------------------------------------
struct TensorGeom {
    int n[3];
    int P[3];
    int pbc[3];
    int images;
    double d[3];       // cell edges scaled by the largest one
};
hipError_t build_kernel_spectrum(const Grid& g, const TensorGeom& tg, float* K, double* resid_out,
                                 hipStream_t s);
hipError_t tensor_at_offsets(const TensorGeom& tg, const int32_t* offs_dev, long long count,
                             double* out_dev, hipStream_t s);

}  // namespace llg

// batch internals shared with the surrogate (batch.hip)
llg_status llg_batch_fixed_async_(llg_batch* b, llg_method method, double dt, int64_t nsteps, const float* src,
                                  size_t stride, int nload, hipStream_t producer, float** out);
llg_status llg_batch_then_(llg_batch* b, hipStream_t consumer);
