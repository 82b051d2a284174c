// Host runtime of the solver: the C ABI of llg.h.
//
// The host validates parameters, converts SI input to the reduced units the
// kernels use (fields / Ms, time * gamma0 Ms; Sec. 3.3 of the paper keeps
// FP32 values O(1) this way), sizes the FFT grid, builds the FP64 demag
// spectrum once per geometry, and launches the hot-path kernels on its own
// HIP stream.  Integration steps are captured once into HIP graphs and
// replayed; the adaptive controller, the state-buffer swap and the attempt
// log live on the device, so the host only polls a done flag.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "host_common.hpp"
#include "internal.hpp"

using namespace llg;
using namespace llg::host;

namespace {

struct Graph {
    hipGraphExec_t exec = nullptr;
    int method = -1;
    double dt = 0.0;
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        method = -1;
        dt = 0.0;
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// Device scratch of llg_eval_heff_noalloc: a private device-state record
// followed by the spectrum buffers, in one static array that every GPU the
// library runs on holds from module load to process end.  Host code never
// passes the array's name to a kernel: it looks up the array's device
// address once per device (noalloc_scratch_init) and uses that.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNoAllocBytes = (size_t)32 << 20;   // spectra of films up to 1024 x 1024
constexpr size_t kNoAllocStateBytes = 256;           // the state record, padded
static_assert(sizeof(DevState) <= kNoAllocStateBytes, "state record fits its slot");

static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
char* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

// with `device` current: the address of that device's copy of the array
hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_scratch_dev[device] = (char*)ptr;
    return hipSuccess;
}

char* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
}

// the scratch state record: the solver's record (time, step counter for the
// thermal draw) with the done flag, health word and attempt log cleared, so
// that the evaluation runs whatever the solver's run left and touches none
// of the solver's own state
__global__ void noalloc_state_kernel(DevState* __restrict__ dst, const DevState* __restrict__ src) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    DevState h = *src;
    h.cur = 0;
    h.done = 0;
    h.health = 0;
    h.err_bits = 0u;
    h.log = nullptr;
    h.log_cap = 0;
    *dst = h;
}

}  // namespace

namespace llg {
thread_local KernelTiming g_kernel_timing;
}

struct llg_solver {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t user = nullptr;
    hipEvent_t sync_ev = nullptr;
    std::string err = "";
    // problem
    int nx = 0, ny = 0, nz = 0;
    int pbc[3] = {0, 0, 0};
    int images = 10;
    double dx = 0, dy = 0, dz = 0;
    double Ms = 0, Aex = 0, alpha = 0;
    double Ku = 0, u[3] = {1, 0, 0};
    double Kc1 = 0, Kc2 = 0, c1[3] = {1, 0, 0}, c2[3] = {0, 1, 0};
    double jc[3] = {0, 0, 0}, P = 0, xi = 0;
    double B[3] = {0, 0, 0};
    double T = 0;
    uint64_t seed = 0;
    int terms = LLG_TERM_ALL;
    bool have_geom = false, have_cell = false, have_mat = false, have_m = false;
    // plan
    Grid g = {};
    FftPlan px = {}, py = {}, pz = {};
    float2 *twx = nullptr, *twy = nullptr, *twz = nullptr;
    int wy = 1, wz = 1;       // column tile widths
    bool fast2d = false;      // 2D with compiled FFT lengths: packed spectrum kernels
    bool fastrows = false;    // row passes of compiled length (2D packed or 3D natural layout)
    bool fast3dy = false;     // 3D, y axis of compiled length: tiled y passes
    bool fast3dz = false;     // 3D, z axis of compiled length: tiled z pass
    // device buffers
    float* K = nullptr;
    bool K_valid = false;
    double K_resid = 0.0;
    float2* S = nullptr;
    float2* Sy = nullptr;
    float* mbuf[2] = {nullptr, nullptr};
    float* ms[2] = {nullptr, nullptr};
    float* kb[6] = {};
    float* kfs[2] = {nullptr, nullptr};
    float* hbuf = nullptr;
    DevState* st = nullptr;
    int* dflag = nullptr;
    llg_attempt* log = nullptr;
    long long log_cap = 0;
    bool spec_valid = false;   // S holds the forward x transform of m
    bool k1_valid = false;     // kfs[cur] holds f(m) for the adaptive method
    double last_dt = 0.0;
    Graph gfix, gdp, gdm;
    // the done flag of the last two launched chunks of step graphs, copied to
    // pinned host memory behind each chunk (launch_until_done)
    int* hflag = nullptr;
    hipEvent_t flag_ev[2] = {nullptr, nullptr};
};

namespace {

llg_status fail(llg_solver* s, llg_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    return code;
}

#define HIPCHK(s, x)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess)                                                                     \
            return fail(s, e_ == hipErrorOutOfMemory ? LLG_E_NOMEM : LLG_E_DEVICE, "%s: %s (%s:%d)", \
                        #x, hipGetErrorString(e_), __FILE__, __LINE__);                           \
    } while (0)

void free_dev(void* p) {
    if (p) (void)hipFree(p);
}

void invalidate_graphs(llg_solver* s) {
    s->gfix.reset();
    s->gdp.reset();
    s->gdm.reset();
}

void free_buffers(llg_solver* s) {
    invalidate_graphs(s);
    free_dev(s->K); s->K = nullptr;
    free_dev(s->S); s->S = nullptr;
    free_dev(s->Sy); s->Sy = nullptr;
    for (auto& p : s->mbuf) { free_dev(p); p = nullptr; }
    for (auto& p : s->ms) { free_dev(p); p = nullptr; }
    for (auto& p : s->kb) { free_dev(p); p = nullptr; }
    for (auto& p : s->kfs) { free_dev(p); p = nullptr; }
    free_dev(s->hbuf); s->hbuf = nullptr;
    free_dev(s->twx); s->twx = nullptr;
    free_dev(s->twy); s->twy = nullptr;
    free_dev(s->twz); s->twz = nullptr;
    free_dev(s->log); s->log = nullptr;
    s->K_valid = false;
    s->spec_valid = false;
    s->k1_valid = false;
}

// widest column tile whose FFT buffer and kept values fit 12 elements per
// thread (the 24-element variant is kept for lengths that need it)
int col_width(int Lh, int n) {
    const int m = Lh > n ? Lh : n;
    for (int W : {16, 8, 4, 2, 1})
        if (3 * W * m <= 12 * 256) return W;
    return 3 * m <= 24 * 256 ? 1 : 0;
}

bool two_d(const llg_solver* s) { return s->nz == 1; }

Phys make_phys(const llg_solver* s, double dt_thermal) {
    Material m;
    m.Ms = s->Ms; m.Aex = s->Aex; m.alpha = s->alpha; m.Ku = s->Ku;
    for (int a = 0; a < 3; ++a) { m.u[a] = s->u[a]; m.B[a] = s->B[a]; m.c1[a] = s->c1[a]; m.c2[a] = s->c2[a]; }
    m.Kc1 = s->Kc1; m.Kc2 = s->Kc2;
    for (int a = 0; a < 3; ++a) m.j[a] = s->jc[a];
    m.P = s->P; m.xi = s->xi;
    m.d[0] = s->dx; m.d[1] = s->dy; m.d[2] = s->dz;
    m.T = s->T; m.seed = s->seed; m.terms = s->terms;
    return phys_of(m, dt_thermal);
}

llg_status enter(llg_solver* s) {
    if (!s) return LLG_E_ARG;
    s->err.clear();
    HIPCHK(s, hipSetDevice(s->device));
    if (s->user) {
        HIPCHK(s, hipEventRecord(s->sync_ev, s->user));
        HIPCHK(s, hipStreamWaitEvent(s->stream, s->sync_ev, 0));
    }
    return LLG_OK;
}

llg_status ready(llg_solver* s, bool need_m) {
    if (!s->have_geom) return fail(s, LLG_E_STATE, "geometry not set");
    if (!s->have_cell) return fail(s, LLG_E_STATE, "cell size not set");
    if (!s->have_mat) return fail(s, LLG_E_STATE, "material not set");
    if (need_m && !s->have_m) return fail(s, LLG_E_STATE, "magnetisation not set");
    return LLG_OK;
}

llg_status ensure_kernel(llg_solver* s) {
    if (s->K_valid || !(s->terms & LLG_TERM_DEMAG)) return LLG_OK;
    TraceRange trace_("demag kernel build (FP64)");
    TensorGeom tg = {};
    const double d[3] = {s->dx, s->dy, s->dz};
    const double dm = fmax(d[0], fmax(d[1], d[2]));
    const int n[3] = {s->nx, s->ny, s->nz};
    const int P[3] = {s->g.Px, s->g.Py, s->g.Pz};
    for (int a = 0; a < 3; ++a) {
        tg.n[a] = n[a];
        tg.P[a] = P[a];
        tg.pbc[a] = s->pbc[a];
        tg.d[a] = d[a] / dm;
    }
    tg.images = s->images;
    double resid = 0.0;
    HIPCHK(s, build_kernel_spectrum(s->g, tg, s->K, &resid, s->stream));
    s->K_resid = resid;
    if (!(resid <= 1e-9))
        return fail(s, LLG_E_DEVICE, "demag kernel spectrum is not real (residue %g)", resid);
    s->K_valid = true;
    return LLG_OK;
}

// The buffers an evaluation works in: the spectrum (and, in 3D, the
// y-transformed spectrum) and the device state the kernels consult.  The
// solver's own, or those of the no-allocation evaluation.
struct EvalBufs {
    float2* S;
    float2* Sy;
    DevState* st;
};
EvalBufs own_bufs(const llg_solver* s) { return EvalBufs{s->S, s->Sy, s->st}; }

// row passes: packed fast kernels or the generic ones
hipError_t row_fwd(llg_solver* s, const Phys& p, const FwdArgs& fa, const EvalBufs& b) {
    if (s->fastrows) return launch_row_fwd_fast(s->g, s->twx, b.S, fa, b.st, s->stream);
    return launch_row_fwd(s->g, p, s->px, s->twx, b.S, fa, b.st, s->stream);
}
hipError_t row_inv(llg_solver* s, const Phys& p, const StageArgs& sa, const EvalBufs& b) {
    if (s->fastrows) return launch_row_inv_fast(s->g, p, s->twx, b.S, sa, b.st, s->stream);
    return launch_row_inv(s->g, p, s->px, s->twx, b.S, sa, b.st, s->stream);
}
hipError_t row_fwd(llg_solver* s, const Phys& p, const FwdArgs& fa) { return row_fwd(s, p, fa, own_bufs(s)); }
hipError_t row_inv(llg_solver* s, const Phys& p, const StageArgs& sa) { return row_inv(s, p, sa, own_bufs(s)); }

ColArgs col_base(const llg_solver* s) {
    ColArgs a = {};
    a.nkx = s->g.nkx;
    return a;
}

// the spectral pass(es) between the forward and the inverse x transform
llg_status launch_spectral(llg_solver* s, const EvalBufs& b, hipEvent_t* ev_after_y = nullptr) {
    const Grid& g = s->g;
    const long long nkxp = g.nkxp;
    if (two_d(s) && s->fast2d) {
        Col2dArgs c = {};
        c.S = b.S;
        c.K = s->K;
        c.tw = s->twy;
        c.nkx = g.Px / 2;
        c.nkx_full = g.nkx;
        c.nkxp = g.nkxp;
        c.tsh = g.tsh;
        c.nq = fast2d_row_classes(g.Px, g.rvar);
        c.var = g.cvar;
        c.ny = g.ny;
        c.Py = g.Py;
        HIPCHK(s, launch_col2d_fast(c, b.st, s->stream));
        return LLG_OK;
    }
    if (two_d(s)) {
        ColArgs a = col_base(s);
        a.in = b.S; a.out = b.S;
        a.cs_in = a.cs_out = (long long)g.nrows * nkxp;
        a.os_in = a.os_out = 0;
        a.as_in = a.as_out = nkxp;
        a.nouter = 1;
        a.W = s->wy;
        a.ntiles = (g.nkx + a.W - 1) / a.W;
        a.n_in = a.n_out = g.ny;
        a.P = g.Py; a.split = g.split_y; a.plan = s->py; a.tw = s->twy;
        a.K = s->K; a.ncomp = 4;
        a.Pa = g.Py; a.Po = 1; a.na_c = g.Py / 2 + 1; a.no_c = 1; a.o_split = 0;
        const int sa[6] = {1, 1, 1, -1, 1, -1};
        for (int c = 0; c < 6; ++c) { a.sign_a[c] = sa[c]; a.sign_o[c] = 1; }
        HIPCHK(s, launch_col(a, b.st, COL_FULL, s->stream));
        return LLG_OK;
    }
    // 3D: y forward, z with product, y inverse
    ColArgs y = col_base(s);
    y.W = s->wy;
    y.ntiles = (g.nkx + y.W - 1) / y.W;
    y.P = g.Py; y.split = g.split_y; y.plan = s->py; y.tw = s->twy;
    y.nouter = g.nz;
    ColArgs yf = y;
    yf.in = b.S; yf.out = b.Sy;
    yf.cs_in = (long long)g.nrows * nkxp; yf.os_in = (long long)g.ny * nkxp; yf.as_in = nkxp;
    yf.cs_out = (long long)g.nz * g.Py * nkxp; yf.os_out = (long long)g.Py * nkxp; yf.as_out = nkxp;
    yf.n_in = g.ny; yf.n_out = g.Py;
    if (s->fast3dy) {
        yf.W = fast3d_col_width(g.Py, g.split_y, false);
        yf.ntiles = (g.nkx + yf.W - 1) / yf.W;
        HIPCHK(s, launch_col3_tiled(yf, COL_FWD, b.st, s->stream));
    } else {
        HIPCHK(s, launch_col(yf, b.st, COL_FWD, s->stream));
    }
    if (ev_after_y) HIPCHK(s, hipEventRecord(ev_after_y[0], s->stream));
    ColArgs z = col_base(s);
    z.in = b.Sy; z.out = b.Sy;
    z.cs_in = z.cs_out = (long long)g.nz * g.Py * nkxp;
    z.os_in = z.os_out = nkxp;
    z.as_in = z.as_out = (long long)g.Py * nkxp;
    z.nouter = g.Py;
    z.W = s->wz;
    z.ntiles = (g.nkx + z.W - 1) / z.W;
    z.n_in = z.n_out = g.nz;
    z.P = g.Pz; z.split = g.split_z; z.plan = s->pz; z.tw = s->twz;
    z.K = s->K; z.ncomp = 6;
    z.Pa = g.Pz; z.Po = g.Py; z.na_c = g.Pz / 2 + 1; z.no_c = g.Py / 2 + 1; z.o_split = g.split_y;
    const int sz_[6] = {1, 1, 1, 1, -1, -1};   // along z: xz, yz odd
    const int sy_[6] = {1, 1, 1, -1, 1, -1};   // along y: xy, yz odd
    for (int c = 0; c < 6; ++c) { z.sign_a[c] = sz_[c]; z.sign_o[c] = sy_[c]; }
    if (s->fast3dz) {
        z.W = fast3d_col_width(g.Pz, g.split_z, true);
        z.ntiles = (g.nkx + z.W - 1) / z.W;
        HIPCHK(s, launch_col3_tiled(z, COL_FULL, b.st, s->stream));
    } else {
        HIPCHK(s, launch_col(z, b.st, COL_FULL, s->stream));
    }
    if (ev_after_y) HIPCHK(s, hipEventRecord(ev_after_y[1], s->stream));
    ColArgs yi = y;
    yi.in = b.Sy; yi.out = b.S;
    yi.cs_in = (long long)g.nz * g.Py * nkxp; yi.os_in = (long long)g.Py * nkxp; yi.as_in = nkxp;
    yi.cs_out = (long long)g.nrows * nkxp; yi.os_out = (long long)g.ny * nkxp; yi.as_out = nkxp;
    yi.n_in = g.Py; yi.n_out = g.ny;
    if (s->fast3dy) {
        yi.W = fast3d_col_width(g.Py, g.split_y, false);
        yi.ntiles = (g.nkx + yi.W - 1) / yi.W;
        HIPCHK(s, launch_col3_tiled(yi, COL_INV, b.st, s->stream));
    } else {
        HIPCHK(s, launch_col(yi, b.st, COL_INV, s->stream));
    }
    return LLG_OK;
}

llg_status launch_spectral(llg_solver* s, hipEvent_t* ev_after_y = nullptr) {
    return launch_spectral(s, own_bufs(s), ev_after_y);
}

llg_status launch_fwd_plain(llg_solver* s, int sel) {
    FwdArgs fa = {};
    fa.m_in = bref_cur(s->mbuf[0], s->mbuf[1], sel);
    fa.combine = 0;
    fa.m0 = fa.m_in; fa.k1 = fa.m_in; fa.m_out = bref(nullptr);
    const Phys p = make_phys(s, 0.0);
    HIPCHK(s, row_fwd(s, p, fa));
    return LLG_OK;
}

llg_status sync(llg_solver* s) {
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return LLG_OK;
}

llg_status read_state(llg_solver* s, DevState* h) {
    HIPCHK(s, hipMemcpyAsync(h, s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
    return sync(s);
}

llg_status write_state(llg_solver* s, const DevState* h) {
    HIPCHK(s, hipMemcpyAsync(s->st, h, sizeof(DevState), hipMemcpyHostToDevice, s->stream));
    return sync(s);
}

// The hot-path kernels return at once while the device state says the run
// is done, which an adaptive run that reached t_end leaves set.  The calls
// that only evaluate H_eff lift the flag for their launches and put it back.
llg_status lift_done(llg_solver* s, int* was) {
    DevState h;
    llg_status rc = read_state(s, &h);
    if (rc != LLG_OK) return rc;
    *was = h.done;
    if (!h.done) return LLG_OK;
    h.done = 0;
    return write_state(s, &h);
}

llg_status restore_done(llg_solver* s, int was) {
    if (!was) return LLG_OK;
    DevState h;
    llg_status rc = read_state(s, &h);
    if (rc != LLG_OK) return rc;
    h.done = was;
    return write_state(s, &h);
}

// Launches a captured step graph in chunks of eight until the device state's
// done flag is set or `max_launches` graphs have been launched (< 0: no
// limit), then waits for the stream.  Behind each chunk the flag is copied
// to pinned host memory and an event recorded; the host reads a chunk's
// flag only after the next chunk is queued, so the device never waits for
// the host between chunks.  Graphs launched after the flag was set do
// nothing (every kernel of a step returns at once while it is set).
llg_status launch_until_done(llg_solver* s, hipGraphExec_t exec, long long max_launches) {
    constexpr int kChunk = 8;
    long long launched = 0;
    int pend = -1, slot = 0;
    for (;;) {
        int nl = kChunk;
        if (max_launches >= 0 && max_launches - launched < nl) nl = (int)(max_launches - launched);
        if (max_launches < 0 && launched > (1LL << 32)) nl = 0;
        if (nl > 0) {
            for (int i = 0; i < nl; ++i) HIPCHK(s, hipGraphLaunch(exec, s->stream));
            launched += nl;
            HIPCHK(s, hipMemcpyAsync(&s->hflag[slot], &s->st->done, sizeof(int), hipMemcpyDeviceToHost, s->stream));
            HIPCHK(s, hipEventRecord(s->flag_ev[slot], s->stream));
        }
        if (pend >= 0) {
            HIPCHK(s, hipEventSynchronize(s->flag_ev[pend]));
            if (s->hflag[pend]) break;
        }
        if (nl <= 0) break;
        pend = slot;
        slot ^= 1;
    }
    return sync(s);
}

// H_eff of m (mbuf[cur]) into `out` (device); tracks spectrum validity
llg_status eval_into(llg_solver* s, float* out, const Phys& p) {
    llg_status rc;
    if (p.demag_on) {
        if ((rc = launch_fwd_plain(s, 1)) != LLG_OK) return rc;
        if ((rc = launch_spectral(s)) != LLG_OK) return rc;
    }
    StageArgs sa = {};
    sa.mode = ROW_EVAL;
    sa.m_in = bref_cur(s->mbuf[0], s->mbuf[1], 1);
    sa.m0 = sa.m_in;
    sa.m_out = bref(nullptr);
    sa.k_out = bref(nullptr);
    sa.h_out = out;
    HIPCHK(s, row_inv(s, p, sa));
    // the column pass transformed S in place: it no longer holds X(m)
    s->spec_valid = false;
    return LLG_OK;
}


// one fixed step of tableau t: S x (spectral + fused row pass) + controller
llg_status enqueue_fixed_step(llg_solver* s, const Tableau& t, const Phys& p) {
    llg_status rc;
    for (int st = 1; st <= t.S; ++st) {
        if (p.demag_on && (rc = launch_spectral(s)) != LLG_OK) return rc;
        StageArgs sa = {};
        sa.mode = ROW_STAGE;
        sa.m_in = st == 1 ? bref_cur(s->mbuf[0], s->mbuf[1], 1) : bref(s->ms[st % 2]);
        sa.m0 = bref_cur(s->mbuf[0], s->mbuf[1], 1);
        sa.m_out = st == t.S ? bref_cur(s->mbuf[0], s->mbuf[1], 2) : bref(s->ms[(st + 1) % 2]);
        bool needed = false;
        if (st < t.S) {
            if (t.b[st - 1] != 0.0) needed = true;
            for (int r = st; r < t.S; ++r)
                if (t.A[r][st - 1] != 0.0) needed = true;
        }
        sa.k_out = bref(needed ? s->kb[st - 1] : nullptr);
        sa.nk = st;
        for (int j = 0; j < st; ++j) sa.a[j] = (float)(st < t.S ? t.A[st][j] : t.b[j]);
        for (int j = 0; j + 1 < st; ++j) sa.kprev[j] = bref(s->kb[j]);
        sa.h_out = nullptr;
        HIPCHK(s, row_inv(s, p, sa));
    }
    HIPCHK(s, launch_ctrl_fixed(s->st, t.S, 0.0, s->stream));
    return LLG_OK;
}

// one attempt of an embedded pair whose last stage is evaluated at the new
// state (first same as last: k1 is the previous attempt's last k).  With S
// stages: k1 = kfs[cur], k2..k_{S-1} = kb[1..S-2], k_S -> kfs[cur^1].
llg_status enqueue_fsal_attempt(llg_solver* s, const Tableau& t, const Phys& p) {
    const int S = t.S;
    llg_status rc;
    BufRef kref[7];
    kref[0] = bref_cur(s->kfs[0], s->kfs[1], 1);
    for (int j = 1; j + 1 < S; ++j) kref[j] = bref(s->kb[j]);
    kref[S - 1] = bref_cur(s->kfs[0], s->kfs[1], 2);
    // stage 2 input: m_2 = normalize(m0 + dtau a21 k1)
    FwdArgs fa = {};
    fa.combine = 1;
    fa.a1 = (float)t.A[1][0];
    fa.m0 = bref_cur(s->mbuf[0], s->mbuf[1], 1);
    fa.k1 = kref[0];
    fa.m_in = fa.m0;
    fa.m_out = bref(s->ms[0]);
    HIPCHK(s, row_fwd(s, p, fa));
    for (int st = 2; st <= S; ++st) {
        if (p.demag_on && (rc = launch_spectral(s)) != LLG_OK) return rc;
        StageArgs sa = {};
        sa.m0 = bref_cur(s->mbuf[0], s->mbuf[1], 1);
        sa.m_in = st == S ? bref_cur(s->mbuf[0], s->mbuf[1], 2) : bref(s->ms[st % 2 == 0 ? 0 : 1]);
        sa.k_out = kref[st - 1];
        sa.nk = st;
        for (int j = 0; j + 1 < st; ++j) sa.kprev[j] = kref[j];
        if (st < S) {
            sa.mode = ROW_STAGE;
            sa.m_out = st == S - 1 ? bref_cur(s->mbuf[0], s->mbuf[1], 2) : bref(s->ms[st % 2 == 0 ? 1 : 0]);
            for (int j = 0; j < st; ++j) sa.a[j] = (float)t.A[st][j];
        } else {
            sa.mode = ROW_ERROR;
            sa.m_out = bref(nullptr);
            for (int j = 0; j < S; ++j) sa.e[j] = (float)(t.b[j] - t.bhat[j]);
        }
        HIPCHK(s, row_inv(s, p, sa));
    }
    HIPCHK(s, launch_ctrl_dp45(s->st, s->stream));
    return LLG_OK;
}

// one attempt of an embedded pair without that property: the forward pass
// of the state, S stages (k_j in kb[j-1]), the last one writing the
// candidate state and the error estimate together
llg_status enqueue_plain_attempt(llg_solver* s, const Tableau& t, const Phys& p) {
    const int S = t.S;
    llg_status rc;
    if (p.demag_on && (rc = launch_fwd_plain(s, 1)) != LLG_OK) return rc;
    for (int st = 1; st <= S; ++st) {
        if (p.demag_on && (rc = launch_spectral(s)) != LLG_OK) return rc;
        StageArgs sa = {};
        sa.mode = ROW_STAGE;
        sa.m0 = bref_cur(s->mbuf[0], s->mbuf[1], 1);
        sa.m_in = st == 1 ? sa.m0 : bref(s->ms[st % 2]);
        sa.m_out = st == S ? bref_cur(s->mbuf[0], s->mbuf[1], 2) : bref(s->ms[(st + 1) % 2]);
        sa.k_out = bref(st < S ? s->kb[st - 1] : nullptr);
        sa.nk = st;
        for (int j = 0; j + 1 < st; ++j) sa.kprev[j] = bref(s->kb[j]);
        for (int j = 0; j < st; ++j) sa.a[j] = (float)(st < S ? t.A[st][j] : t.b[j]);
        if (st == S) {
            sa.with_err = 1;
            sa.skip_fwd = 1;
            for (int j = 0; j < S; ++j) sa.e[j] = (float)(t.b[j] - t.bhat[j]);
        }
        HIPCHK(s, row_inv(s, p, sa));
    }
    HIPCHK(s, launch_ctrl_dp45(s->st, s->stream));
    return LLG_OK;
}

// one step of a fixed tableau whose size bounds the change of m per step
// (Sec. 2.2): k_1 with max |k_1|, the step size chosen on the device, the
// input of stage 2 (or, with one stage, the new state) with its forward x
// transform, then the remaining stages as in a fixed step
llg_status enqueue_dm_step(llg_solver* s, const Tableau& t, const Phys& p) {
    llg_status rc;
    const int S = t.S;
    if (p.demag_on && (rc = launch_spectral(s)) != LLG_OK) return rc;
    StageArgs sk = {};
    sk.mode = ROW_KONLY;
    sk.with_err = 1;
    sk.m_in = bref_cur(s->mbuf[0], s->mbuf[1], 1);
    sk.m0 = sk.m_in;
    sk.m_out = bref(nullptr);
    sk.k_out = bref(s->kb[0]);
    HIPCHK(s, row_inv(s, p, sk));
    HIPCHK(s, launch_ctrl_dm(s->st, s->stream));
    FwdArgs fa = {};
    fa.combine = 1;
    fa.a1 = (float)(S > 1 ? t.A[1][0] : t.b[0]);
    fa.m0 = bref_cur(s->mbuf[0], s->mbuf[1], 1);
    fa.k1 = bref(s->kb[0]);
    fa.m_in = fa.m0;
    fa.m_out = S > 1 ? bref(s->ms[0]) : bref_cur(s->mbuf[0], s->mbuf[1], 2);
    HIPCHK(s, row_fwd(s, p, fa));
    for (int st = 2; st <= S; ++st) {
        if (p.demag_on && (rc = launch_spectral(s)) != LLG_OK) return rc;
        StageArgs sa = {};
        sa.mode = ROW_STAGE;
        sa.m0 = bref_cur(s->mbuf[0], s->mbuf[1], 1);
        sa.m_in = bref(s->ms[st % 2 == 0 ? 0 : 1]);
        sa.m_out = st == S ? bref_cur(s->mbuf[0], s->mbuf[1], 2) : bref(s->ms[st % 2 == 0 ? 1 : 0]);
        sa.k_out = bref(st < S ? s->kb[st - 1] : nullptr);
        sa.nk = st;
        for (int j = 0; j + 1 < st; ++j) sa.kprev[j] = bref(s->kb[j]);
        for (int j = 0; j < st; ++j) sa.a[j] = (float)(st < S ? t.A[st][j] : t.b[j]);
        HIPCHK(s, row_inv(s, p, sa));
    }
    HIPCHK(s, launch_ctrl_dm_accept(s->st, S, s->stream));
    return LLG_OK;
}

llg_status capture(llg_solver* s, Graph& gr, llg_status (*body)(llg_solver*, const Tableau&, const Phys&),
                   const Tableau& t, const Phys& p) {
    hipGraph_t graph = nullptr;
    HIPCHK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    llg_status rc = body(s, t, p);
    hipError_t e = hipStreamEndCapture(s->stream, &graph);
    if (rc != LLG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    HIPCHK(s, e);
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(s, e);
    gr.reset();
    gr.exec = exec;
    return LLG_OK;
}

llg_status fsal_body(llg_solver* s, const Tableau& t, const Phys& p) { return enqueue_fsal_attempt(s, t, p); }
llg_status plain_body(llg_solver* s, const Tableau& t, const Phys& p) { return enqueue_plain_attempt(s, t, p); }

llg_status ensure_k1(llg_solver* s, const Phys& p) {
    if (s->k1_valid) return LLG_OK;
    llg_status rc;
    if (p.demag_on) {
        if ((rc = launch_fwd_plain(s, 1)) != LLG_OK) return rc;
        if ((rc = launch_spectral(s)) != LLG_OK) return rc;
    }
    StageArgs sa = {};
    sa.mode = ROW_KONLY;
    sa.m_in = bref_cur(s->mbuf[0], s->mbuf[1], 1);
    sa.m0 = sa.m_in;
    sa.m_out = bref(nullptr);
    sa.k_out = bref_cur(s->kfs[0], s->kfs[1], 1);
    HIPCHK(s, row_inv(s, p, sa));
    HIPCHK(s, launch_state_add_evals(s->st, 1, s->stream));
    s->k1_valid = true;
    return LLG_OK;
}

llg_status run_adaptive(llg_solver* s, int method, double t_end, double max_err, double dt0,
                        long long max_attempts, llg_stats* out);

void fill_stats(const DevState& h, llg_stats* out) {
    out->t = h.t;
    out->dt = h.dt;
    out->dt_next = h.dt_next;
    out->max_err = h.last_err;
    out->steps = h.nsteps;
    out->rejected = h.nrej;
    out->evals = h.nevals;
    out->health = h.health;
    out->done = h.done;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

llg_status llg_create(int device, void* hip_stream, llg_solver** out) {
    if (!out) return LLG_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return LLG_E_DEVICE;
    if (device < 0 || device >= ndev) return LLG_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return LLG_E_DEVICE;
    if (noalloc_scratch_init(device) != hipSuccess) return LLG_E_DEVICE;
    llg_solver* s = new llg_solver();
    s->device = device;
    s->user = (hipStream_t)hip_stream;
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s->sync_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s->flag_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s->flag_ev[1], hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc(&s->hflag, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&s->st, sizeof(DevState)) != hipSuccess ||
        hipMalloc(&s->dflag, sizeof(int)) != hipSuccess) {
        llg_destroy(s);
        return LLG_E_DEVICE;
    }
    DevState h = {};
    if (hipMemcpy(s->st, &h, sizeof h, hipMemcpyHostToDevice) != hipSuccess) {
        llg_destroy(s);
        return LLG_E_DEVICE;
    }
    *out = s;
    return LLG_OK;
}

void llg_destroy(llg_solver* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    free_buffers(s);
    free_dev(s->st);
    free_dev(s->dflag);
    if (s->sync_ev) (void)hipEventDestroy(s->sync_ev);
    for (auto& e : s->flag_ev)
        if (e) (void)hipEventDestroy(e);
    if (s->hflag) (void)hipHostFree(s->hflag);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

const char* llg_last_error(const llg_solver* s) { return s ? s->err.c_str() : "null solver"; }

llg_status llg_set_geometry(llg_solver* s, int nx, int ny, int nz, int pbc_x, int pbc_y, int pbc_z,
                            int pbc_images) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (nx < 1 || ny < 1 || nz < 1 || pbc_images < 0)
        return fail(s, LLG_E_ARG, "invalid geometry %d x %d x %d, images %d", nx, ny, nz, pbc_images);
    const int pb[3] = {pbc_x != 0, pbc_y != 0, pbc_z != 0};
    const int n[3] = {nx, ny, nz};
    int P[3];
    for (int a = 0; a < 3; ++a) {
        if (pb[a]) {
            if (!good_len(n[a])) return fail(s, LLG_E_UNSUPPORTED, "periodic length %d is not a product of 2,3,5,7", n[a]);
            P[a] = n[a];
        } else {
            P[a] = pad_len(n[a]);
        }
    }
    if (nz == 1) P[2] = 1;
    const int split_y = !pb[1], split_z = nz > 1 && !pb[2];
    const int Ly = split_y ? P[1] / 2 : P[1];
    const int Lz = split_z ? P[2] / 2 : P[2];
    if (P[0] > kMaxPx || Ly > kMaxHalf || Lz > kMaxHalf)
        return fail(s, LLG_E_UNSUPPORTED, "FFT lengths %d x %d x %d exceed this build's limits", P[0], P[1], P[2]);
    if (P[0] % 2) return fail(s, LLG_E_UNSUPPORTED, "x FFT length must be even (periodic nx odd)");
    (void)hipStreamSynchronize(s->stream);
    free_buffers(s);
    s->have_geom = false;
    s->have_m = false;
    s->nx = nx; s->ny = ny; s->nz = nz;
    for (int a = 0; a < 3; ++a) s->pbc[a] = pb[a];
    s->images = pbc_images;
    Grid& g = s->g;
    g = Grid{};
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.nrows = ny * nz;
    g.ncells = nx * ny * nz;
    for (int a = 0; a < 3; ++a) g.pbc[a] = pb[a];
    g.Px = P[0]; g.Py = P[1]; g.Pz = P[2];
    g.nkx = P[0] / 2 + 1;
    g.nkxp = (g.nkx + 15) / 16 * 16;
    g.tsh = fast2d_tile_shift();
    g.split_y = split_y;
    g.split_z = split_z;
    if (!make_plan(P[0], s->px) || !make_plan(Ly, s->py) || !make_plan(Lz, s->pz))
        return fail(s, LLG_E_UNSUPPORTED, "cannot factor FFT lengths");
    s->wy = col_width(Ly, ny);
    s->wz = col_width(Lz, nz);
    if (s->wy < 1 || s->wz < 1) return fail(s, LLG_E_UNSUPPORTED, "column pass does not fit");
    // LLG_FORCE_GENERIC=1 selects the runtime-length kernels everywhere (used
    // by the tests to check both implementations against the oracle)
    const char* gen = getenv("LLG_FORCE_GENERIC");
    // compiled variants: the table's defaults where they serve this geometry
    // (else variant 0); kept by this solver until its own llg_autotune or
    // llg_set_variants, whatever later calls do to the table
    g.rvar = fast2d_row_variant(P[0]);
    if (!fast2d_row_ok(P[0], g.rvar, nx == P[0])) g.rvar = 0;
    g.cvar = fast2d_col_variant(Ly);
    if (!fast2d_col_ok(Ly, split_y, g.cvar) || (P[0] / 2) % fast2d_col_width(Ly, g.cvar)) g.cvar = 0;
    s->fast2d = nz == 1 && fast2d_row_ok(P[0], g.rvar, nx == P[0]) && fast2d_col_ok(Ly, split_y, g.cvar) &&
                ny <= Ly && (P[0] / 2) % fast2d_col_width(Ly, g.cvar) == 0 && !(gen && gen[0] == '1');
    s->fastrows = s->fast2d || (nz > 1 && fast2d_row_ok(P[0], g.rvar, nx == P[0]) && (nx == P[0] || 2 * nx <= P[0]) &&
                                !(gen && gen[0] == '1'));
    s->fast3dy = nz > 1 && fast3d_col_ok(P[1], split_y, false) && ny <= Ly && !(gen && gen[0] == '1');
    s->fast3dz = nz > 1 && fast3d_col_ok(P[2], split_z, true) && nz <= Lz && !(gen && gen[0] == '1');
    // x transforms above 2048 points exist only as compiled 2D row kernels
    // (the runtime-length kernels stop at 2048)
    if (P[0] > 2048 && !(s->fast2d && nz == 1))
        return fail(s, LLG_E_UNSUPPORTED,
                    "x FFT length %d runs only on the compiled 2D path (one cell thick, compiled y length)", P[0]);
    const size_t vec = sizeof(float) * 3 * (size_t)g.ncells;
    HIPCHK(s, make_tw(P[0], &s->twx));
    HIPCHK(s, make_tw(P[1], &s->twy));
    HIPCHK(s, make_tw(P[2], &s->twz));
    HIPCHK(s, hipMalloc(&s->S, sizeof(float2) * 3 * (size_t)g.nrows * g.nkxp));
    if (!two_d(s)) HIPCHK(s, hipMalloc(&s->Sy, sizeof(float2) * 3 * (size_t)g.nz * g.Py * g.nkxp));
    const size_t kcount = two_d(s) ? 4 * (size_t)g.nkx * (g.Py / 2 + 1)
                                   : 6 * (size_t)(g.Py / 2 + 1) * g.nkx * (g.Pz / 2 + 1);
    HIPCHK(s, hipMalloc(&s->K, sizeof(float) * kcount));
    for (auto& p : s->mbuf) HIPCHK(s, hipMalloc(&p, vec));
    for (auto& p : s->ms) HIPCHK(s, hipMalloc(&p, vec));
    for (auto& p : s->kb) HIPCHK(s, hipMalloc(&p, vec));
    for (auto& p : s->kfs) HIPCHK(s, hipMalloc(&p, vec));
    HIPCHK(s, hipMalloc(&s->hbuf, vec));
    s->log_cap = 1 << 20;
    HIPCHK(s, hipMalloc(&s->log, sizeof(llg_attempt) * s->log_cap));
    s->have_geom = true;
    return LLG_OK;
}

llg_status llg_set_cellsize(llg_solver* s, double dx, double dy, double dz) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!(dx > 0 && dy > 0 && dz > 0) || !isfinite(dx) || !isfinite(dy) || !isfinite(dz))
        return fail(s, LLG_E_ARG, "cell size must be positive");
    s->dx = dx; s->dy = dy; s->dz = dz;
    s->have_cell = true;
    s->K_valid = false;
    s->spec_valid = false;
    s->k1_valid = false;
    invalidate_graphs(s);
    return LLG_OK;
}

llg_status llg_set_material(llg_solver* s, double Ms, double Aex, double alpha) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!(Ms > 0) || !(Aex >= 0) || !(alpha >= 0) || !isfinite(Ms) || !isfinite(Aex) || !isfinite(alpha))
        return fail(s, LLG_E_ARG, "need Ms > 0, Aex >= 0, alpha >= 0");
    s->Ms = Ms; s->Aex = Aex; s->alpha = alpha;
    s->have_mat = true;
    s->k1_valid = false;
    invalidate_graphs(s);
    return LLG_OK;
}

llg_status llg_set_anisotropy_uniaxial(llg_solver* s, double Ku, const double u[3]) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!u || !isfinite(Ku)) return fail(s, LLG_E_ARG, "invalid anisotropy");
    const double n = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    if (!(n > 0) || !isfinite(n)) return fail(s, LLG_E_ARG, "anisotropy axis must be non-zero");
    s->Ku = Ku;
    for (int a = 0; a < 3; ++a) s->u[a] = u[a];
    s->k1_valid = false;
    invalidate_graphs(s);
    return LLG_OK;
}

llg_status llg_set_anisotropy_cubic(llg_solver* s, double K1, double K2, const double c1[3], const double c2[3]) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!c1 || !c2 || !isfinite(K1) || !isfinite(K2)) return fail(s, LLG_E_ARG, "invalid cubic anisotropy");
    const double n1 = sqrt(c1[0] * c1[0] + c1[1] * c1[1] + c1[2] * c1[2]);
    const double n2 = sqrt(c2[0] * c2[0] + c2[1] * c2[1] + c2[2] * c2[2]);
    if (!(n1 > 0) || !(n2 > 0) || !isfinite(n1) || !isfinite(n2))
        return fail(s, LLG_E_ARG, "cubic axes must be non-zero");
    const double d = (c1[0] * c2[0] + c1[1] * c2[1] + c1[2] * c2[2]) / (n1 * n2);
    if (fabs(d) > 1e-6) return fail(s, LLG_E_ARG, "cubic axes must be orthogonal (cos %g)", d);
    s->Kc1 = K1;
    s->Kc2 = K2;
    for (int a = 0; a < 3; ++a) { s->c1[a] = c1[a]; s->c2[a] = c2[a]; }
    s->k1_valid = false;
    invalidate_graphs(s);
    return LLG_OK;
}

llg_status llg_set_current(llg_solver* s, const double j[3], double P, double xi) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!j || !isfinite(j[0]) || !isfinite(j[1]) || !isfinite(j[2]) || !isfinite(P) || !isfinite(xi))
        return fail(s, LLG_E_ARG, "invalid current");
    for (int a = 0; a < 3; ++a) s->jc[a] = j[a];
    s->P = P;
    s->xi = xi;
    s->k1_valid = false;
    invalidate_graphs(s);
    return LLG_OK;
}

llg_status llg_set_applied_field(llg_solver* s, const double B[3]) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!B || !isfinite(B[0]) || !isfinite(B[1]) || !isfinite(B[2])) return fail(s, LLG_E_ARG, "invalid field");
    for (int a = 0; a < 3; ++a) s->B[a] = B[a];
    s->k1_valid = false;
    invalidate_graphs(s);
    return LLG_OK;
}

llg_status llg_set_temperature(llg_solver* s, double T, uint64_t seed) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!(T >= 0) || !isfinite(T)) return fail(s, LLG_E_ARG, "temperature must be >= 0");
    s->T = T;
    s->seed = seed;
    s->k1_valid = false;
    invalidate_graphs(s);
    return LLG_OK;
}

llg_status llg_set_terms(llg_solver* s, int mask) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (mask & ~LLG_TERM_ALL) return fail(s, LLG_E_ARG, "unknown term bits 0x%x", mask);
    s->terms = mask;
    s->k1_valid = false;
    s->spec_valid = false;
    invalidate_graphs(s);
    return LLG_OK;
}

llg_status llg_set_m(llg_solver* s, const float* m, llg_mem where) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!m) return fail(s, LLG_E_ARG, "null m");
    if (!s->have_geom) return fail(s, LLG_E_STATE, "geometry not set");
    const size_t bytes = sizeof(float) * 3 * (size_t)s->g.ncells;
    HIPCHK(s, hipMemcpyAsync(s->mbuf[0], m, bytes, where == LLG_DEVICE ? hipMemcpyDeviceToDevice
                                                                        : hipMemcpyHostToDevice, s->stream));
    int zero = 0, bad = 0;
    HIPCHK(s, hipMemcpyAsync(s->dflag, &zero, sizeof(int), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, launch_normalize_check(s->mbuf[0], s->g.ncells, s->dflag, s->stream));
    HIPCHK(s, hipMemcpyAsync(&bad, s->dflag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    if ((rc = sync(s)) != LLG_OK) return rc;
    if (bad) {
        s->have_m = false;
        return fail(s, LLG_E_ARG, "m is not a field of unit vectors (| |m| - 1 | > 1e-3 or non-finite)");
    }
    DevState h = {};
    h.cur = 0;
    h.log = s->log;
    h.log_cap = s->log_cap;
    h.gms = kGamma0 * (s->have_mat ? s->Ms : 0.0);
    if ((rc = write_state(s, &h)) != LLG_OK) return rc;
    s->have_m = true;
    s->spec_valid = false;
    s->k1_valid = false;
    return LLG_OK;
}

llg_status llg_get_m(llg_solver* s, float* m, llg_mem where) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!m) return fail(s, LLG_E_ARG, "null m");
    if (!s->have_m) return fail(s, LLG_E_STATE, "magnetisation not set");
    DevState h;
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    const size_t bytes = sizeof(float) * 3 * (size_t)s->g.ncells;
    HIPCHK(s, hipMemcpyAsync(m, s->mbuf[h.cur], bytes, where == LLG_DEVICE ? hipMemcpyDeviceToDevice
                                                                           : hipMemcpyDeviceToHost, s->stream));
    return sync(s);
}

llg_status llg_eval_heff(llg_solver* s, float* h_out, llg_mem where) {
    TraceRange trace_("llg_eval_heff");
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!h_out) return fail(s, LLG_E_ARG, "null output");
    if ((rc = ready(s, true)) != LLG_OK) return rc;
    if ((rc = ensure_kernel(s)) != LLG_OK) return rc;
    const Phys p = make_phys(s, s->last_dt);
    float* dst = where == LLG_DEVICE ? h_out : s->hbuf;
    int was = 0;
    if ((rc = lift_done(s, &was)) != LLG_OK) return rc;
    if ((rc = eval_into(s, dst, p)) != LLG_OK) return rc;
    if (where != LLG_DEVICE)
        HIPCHK(s, hipMemcpyAsync(h_out, s->hbuf, sizeof(float) * 3 * (size_t)s->g.ncells,
                                 hipMemcpyDeviceToHost, s->stream));
    if ((rc = sync(s)) != LLG_OK) return rc;
    return restore_done(s, was);
}

llg_status llg_eval_heff_noalloc(llg_solver* s, const float* m_dev, float* h_dev) {
    TraceRange trace_("llg_eval_heff_noalloc");
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!m_dev || !h_dev) return fail(s, LLG_E_ARG, "null m or h");
    if ((rc = ready(s, false)) != LLG_OK) return rc;
    const Phys p = make_phys(s, s->last_dt);
    if (p.demag_on && !s->K_valid)
        return fail(s, LLG_E_STATE, "demag kernel spectrum not built yet (its build allocates): "
                                    "call llg_eval_heff, llg_step or llg_run once first");
    const Grid& g = s->g;
    const size_t sbytes = (sizeof(float2) * 3 * (size_t)g.nrows * g.nkxp + 255) / 256 * 256;
    const size_t sybytes = two_d(s) ? 0 : sizeof(float2) * 3 * (size_t)g.nz * g.Py * g.nkxp;
    const size_t need = kNoAllocStateBytes + sbytes + sybytes;
    if (need > kNoAllocBytes)
        return fail(s, LLG_E_UNSUPPORTED, "this geometry needs %zu bytes of scratch, above the %zu-byte "
                                          "static array of the no-allocation evaluation", need, kNoAllocBytes);
    char* base = noalloc_scratch(s->device);
    if (!base) return fail(s, LLG_E_DEVICE, "no scratch address for device %d", s->device);
    EvalBufs b;
    b.st = (DevState*)base;
    b.S = (float2*)(base + kNoAllocStateBytes);
    b.Sy = two_d(s) ? nullptr : (float2*)(base + kNoAllocStateBytes + sbytes);
    hipLaunchKernelGGL(noalloc_state_kernel, dim3(1), dim3(64), 0, s->stream, b.st, (const DevState*)s->st);
    HIPCHK(s, hipGetLastError());
    if (p.demag_on) {
        FwdArgs fa = {};
        fa.m_in = bref(const_cast<float*>(m_dev));
        fa.combine = 0;
        fa.m0 = fa.m_in; fa.k1 = fa.m_in; fa.m_out = bref(nullptr);
        HIPCHK(s, row_fwd(s, make_phys(s, 0.0), fa, b));
        if ((rc = launch_spectral(s, b)) != LLG_OK) return rc;
    }
    StageArgs sa = {};
    sa.mode = ROW_EVAL;
    sa.m_in = bref(const_cast<float*>(m_dev));
    sa.m0 = sa.m_in;
    sa.m_out = bref(nullptr);
    sa.k_out = bref(nullptr);
    sa.h_out = h_dev;
    HIPCHK(s, row_inv(s, p, sa, b));
    return sync(s);
}

llg_status llg_step(llg_solver* s, llg_method method, double dt, int64_t nsteps) {
    TraceRange trace_("llg_step");
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    Tableau tf;
    if (!fixed_of(method, &tf)) return fail(s, LLG_E_ARG, "llg_step takes Euler, Heun, RK3 or RK4");
    if (!(dt > 0) || !isfinite(dt) || nsteps < 0) return fail(s, LLG_E_ARG, "need dt > 0, nsteps >= 0");
    if ((rc = ready(s, true)) != LLG_OK) return rc;
    if ((rc = ensure_kernel(s)) != LLG_OK) return rc;
    if (nsteps == 0) return LLG_OK;
    const Phys p = make_phys(s, dt);
    // device state: fixed step size
    DevState h;
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    h.dt = dt;
    h.dtau = (float)(dt * kGamma0 * s->Ms);
    h.gms = kGamma0 * s->Ms;
    h.done = 0;
    if ((rc = write_state(s, &h)) != LLG_OK) return rc;
    if (p.demag_on && !s->spec_valid)
        if ((rc = launch_fwd_plain(s, 1)) != LLG_OK) return rc;
    const Tableau t = tf;
    if (!s->gfix.exec || s->gfix.method != (int)method || s->gfix.dt != dt) {
        if ((rc = capture(s, s->gfix, enqueue_fixed_step, t, p)) != LLG_OK) return rc;
        s->gfix.method = (int)method;
        s->gfix.dt = dt;
    }
    for (int64_t i = 0; i < nsteps; ++i) HIPCHK(s, hipGraphLaunch(s->gfix.exec, s->stream));
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    s->spec_valid = p.demag_on != 0;
    s->k1_valid = false;
    s->last_dt = dt;
    if (h.health) return fail(s, LLG_E_DIVERGED, "non-finite field or torque during fixed steps");
    return LLG_OK;
}

llg_status llg_run(llg_solver* s, llg_method method, double t_end, double max_err, double dt0,
                   llg_stats* out) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    return run_adaptive(s, (int)method, t_end, max_err, dt0, -1, out);
}

llg_status llg_run_attempts(llg_solver* s, double t_end, double max_err, double dt0, int64_t max_attempts,
                            llg_stats* out) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (max_attempts < 1) return fail(s, LLG_E_ARG, "max_attempts must be >= 1");
    return run_adaptive(s, LLG_RKDP45, t_end, max_err, dt0, max_attempts, out);
}

llg_status llg_run_dm(llg_solver* s, llg_method method, double t_end, double max_dm, double dt_max,
                      llg_stats* out) {
    TraceRange trace_("llg_run_dm");
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    Tableau tf;
    if (!fixed_of(method, &tf)) return fail(s, LLG_E_ARG, "llg_run_dm takes Euler, Heun, RK3 or RK4");
    if (!(max_dm > 0) || !(dt_max > 0) || !isfinite(t_end) || !isfinite(max_dm) || !isfinite(dt_max))
        return fail(s, LLG_E_ARG, "need max_dm > 0, dt_max > 0");
    if ((rc = ready(s, true)) != LLG_OK) return rc;
    if ((rc = ensure_kernel(s)) != LLG_OK) return rc;
    const Phys p = make_phys(s, 0.0);   // thermal field: fixed steps only
    DevState h;
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    if (h.health) return fail(s, LLG_E_DIVERGED, "state already diverged");
    if (!(t_end > h.t)) {
        if (out) fill_stats(h, out);
        return LLG_OK;
    }
    h.t_end = t_end;
    h.tol = max_dm;
    h.dt_max = dt_max;
    h.gms = kGamma0 * s->Ms;
    h.done = 0;
    h.clipped = 0;
    h.err_bits = 0u;
    if ((rc = write_state(s, &h)) != LLG_OK) return rc;
    if (p.demag_on && !s->spec_valid)
        if ((rc = launch_fwd_plain(s, 1)) != LLG_OK) return rc;
    if (!s->gdm.exec || s->gdm.method != (int)method) {
        if ((rc = capture(s, s->gdm, enqueue_dm_step, tf, p)) != LLG_OK) return rc;
        s->gdm.method = (int)method;
    }
    if ((rc = launch_until_done(s, s->gdm.exec, -1)) != LLG_OK) return rc;
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    s->spec_valid = p.demag_on != 0;
    s->k1_valid = false;
    if (out) fill_stats(h, out);
    if (h.health) return fail(s, LLG_E_DIVERGED, "non-finite field or torque");
    return LLG_OK;
}

llg_status llg_get_state(llg_solver* s, llg_state* out, float* m, llg_mem where) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!out) return fail(s, LLG_E_ARG, "null output");
    if (!s->have_m) return fail(s, LLG_E_STATE, "magnetisation not set");
    DevState h;
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    llg_state o = {};
    o.t = h.t;
    o.dt = h.dt;
    o.dt_next = h.dt_next;
    o.last_err = h.last_err;
    o.step = h.step;
    o.steps = h.nsteps;
    o.rejected = h.nrej;
    o.evals = h.nevals;
    o.health = h.health;
    *out = o;
    if (m) {
        const size_t bytes = sizeof(float) * 3 * (size_t)s->g.ncells;
        HIPCHK(s, hipMemcpyAsync(m, s->mbuf[h.cur], bytes, where == LLG_DEVICE ? hipMemcpyDeviceToDevice
                                                                               : hipMemcpyDeviceToHost, s->stream));
        return sync(s);
    }
    return LLG_OK;
}

llg_status llg_set_state(llg_solver* s, const llg_state* in, const float* m, llg_mem where) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!in || !m) return fail(s, LLG_E_ARG, "null state or m");
    if (!s->have_geom) return fail(s, LLG_E_STATE, "geometry not set");
    if (in->health != 0 || !isfinite(in->t) || !(in->dt >= 0) || !(in->dt_next >= 0) || !isfinite(in->dt) ||
        !isfinite(in->dt_next) || in->step < 0 || in->steps < 0 || in->rejected < 0 || in->evals < 0)
        return fail(s, LLG_E_ARG, "state record is not that of a healthy run");
    const size_t bytes = sizeof(float) * 3 * (size_t)s->g.ncells;
    HIPCHK(s, hipMemcpyAsync(s->mbuf[0], m, bytes, where == LLG_DEVICE ? hipMemcpyDeviceToDevice
                                                                        : hipMemcpyHostToDevice, s->stream));
    int zero = 0, bad = 0;
    HIPCHK(s, hipMemcpyAsync(s->dflag, &zero, sizeof(int), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, launch_check_unit(s->mbuf[0], s->g.ncells, s->dflag, s->stream));
    HIPCHK(s, hipMemcpyAsync(&bad, s->dflag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    if ((rc = sync(s)) != LLG_OK) return rc;
    if (bad) {
        s->have_m = false;
        return fail(s, LLG_E_ARG, "m is not a field of unit vectors (| |m| - 1 | > 1e-3 or non-finite)");
    }
    DevState h = {};
    h.cur = 0;
    h.log = s->log;
    h.log_cap = s->log_cap;
    h.gms = kGamma0 * (s->have_mat ? s->Ms : 0.0);
    h.t = in->t;
    h.dt = in->dt;
    h.dt_next = in->dt_next;
    h.last_err = in->last_err;
    h.step = in->step;
    h.nsteps = in->steps;
    h.nrej = in->rejected;
    h.nevals = in->evals;
    if ((rc = write_state(s, &h)) != LLG_OK) return rc;
    s->have_m = true;
    s->spec_valid = false;
    s->k1_valid = false;
    s->last_dt = in->dt;
    return LLG_OK;
}

llg_status llg_get_stats(llg_solver* s, llg_stats* out) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!out) return fail(s, LLG_E_ARG, "null output");
    DevState h;
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    fill_stats(h, out);
    return LLG_OK;
}

llg_status llg_get_attempts(llg_solver* s, llg_attempt* out, int64_t cap, int64_t* n) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!n || (cap > 0 && !out)) return fail(s, LLG_E_ARG, "null output");
    DevState h;
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    long long have = h.nattempt < s->log_cap ? h.nattempt : s->log_cap;
    if (have > cap) have = cap;
    *n = have;
    if (have > 0) {
        HIPCHK(s, hipMemcpyAsync(out, s->log, sizeof(llg_attempt) * have, hipMemcpyDeviceToHost, s->stream));
        return sync(s);
    }
    return LLG_OK;
}

llg_status llg_profile_evals(llg_solver* s, int n, double* ms_out, int n_kinds, double* total_ms) {
    TraceRange trace_("llg_profile_evals");
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (n < 1 || !ms_out || n_kinds < 5 || !total_ms) return fail(s, LLG_E_ARG, "bad profile arguments");
    if ((rc = ready(s, true)) != LLG_OK) return rc;
    if ((rc = ensure_kernel(s)) != LLG_OK) return rc;
    const Phys p = make_phys(s, s->last_dt);
    if (!p.demag_on) return fail(s, LLG_E_STATE, "profiling needs the demag term");
    int was = 0;
    if ((rc = lift_done(s, &was)) != LLG_OK) return rc;
    // one untimed evaluation first: the first launch of a kernel in a
    // process carries one-time runtime work (code object set-up) that is
    // not the kernel's
    if ((rc = eval_into(s, s->hbuf, p)) != LLG_OK) return rc;
    if ((rc = sync(s)) != LLG_OK) return rc;
    // Every pass one compiled kernel: each kernel's own start and end
    // (events attached to its launch, as a profiler's kernel trace times it).
    const bool exact = s->fastrows && (two_d(s) ? s->fast2d : (s->fast3dy && s->fast3dz));
    if (exact) {
        const int np = two_d(s) ? 3 : 5;    // 2D: fwd, spectral, inv; 3D: fwd, y fwd, z, y inv, inv
        std::vector<hipEvent_t> ev(2 * (size_t)np * n + 2);
        for (auto& e : ev) HIPCHK(s, hipEventCreate(&e));
        struct Guard {
            std::vector<hipEvent_t>& ev;
            ~Guard() {
                g_kernel_timing = KernelTiming{};
                for (auto& e : ev) (void)hipEventDestroy(e);
            }
        } guard{ev};
        hipEvent_t* T = &ev[2 * (size_t)np * n];
        for (int i = 0; i < n; ++i) {
            g_kernel_timing = KernelTiming{&ev[2 * (size_t)np * i], np};
            if ((rc = launch_fwd_plain(s, 1)) != LLG_OK) return rc;
            if ((rc = launch_spectral(s)) != LLG_OK) return rc;
            StageArgs sa = {};
            sa.mode = ROW_EVAL;
            sa.m_in = bref_cur(s->mbuf[0], s->mbuf[1], 1);
            sa.m0 = sa.m_in;
            sa.m_out = bref(nullptr);
            sa.k_out = bref(nullptr);
            sa.h_out = s->hbuf;
            HIPCHK(s, row_inv(s, p, sa));
            if (g_kernel_timing.left != 0) return fail(s, LLG_E_DEVICE, "an evaluation launched fewer kernels than timed");
        }
        g_kernel_timing = KernelTiming{};
        // the wall time of an evaluation from `n` more, launched plainly
        // back to back (the timed launches above carry their events)
        HIPCHK(s, hipEventRecord(T[0], s->stream));
        for (int i = 0; i < n; ++i)
            if ((rc = eval_into(s, s->hbuf, p)) != LLG_OK) return rc;
        HIPCHK(s, hipEventRecord(T[1], s->stream));
        if ((rc = sync(s)) != LLG_OK) return rc;
        // pair index -> kernel kind (0 fwd, 1 spectral / z, 2 inv, 3 y fwd, 4 y inv)
        const int kind2[3] = {0, 1, 2}, kind3[5] = {0, 3, 1, 4, 2};
        double acc[5] = {0, 0, 0, 0, 0};
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < np; ++k) {
                float t = 0.f;
                HIPCHK(s, hipEventElapsedTime(&t, ev[2 * ((size_t)np * i + k)], ev[2 * ((size_t)np * i + k) + 1]));
                acc[two_d(s) ? kind2[k] : kind3[k]] += t;
            }
        float tot = 0.f;
        HIPCHK(s, hipEventElapsedTime(&tot, T[0], T[1]));
        for (int k = 0; k < 5; ++k) ms_out[k] = acc[k] / n;
        for (int k = 5; k < n_kinds; ++k) ms_out[k] = 0.0;
        *total_ms = tot;
        s->spec_valid = false;
        return restore_done(s, was);
    }
    std::vector<hipEvent_t> ev(6 * (size_t)n);
    for (auto& e : ev) HIPCHK(s, hipEventCreate(&e));
    for (int i = 0; i < n; ++i) {
        hipEvent_t* E = &ev[6 * (size_t)i];
        HIPCHK(s, hipEventRecord(E[0], s->stream));
        if ((rc = launch_fwd_plain(s, 1)) != LLG_OK) return rc;
        HIPCHK(s, hipEventRecord(E[1], s->stream));
        if (two_d(s)) {
            if ((rc = launch_spectral(s)) != LLG_OK) return rc;
            HIPCHK(s, hipEventRecord(E[2], s->stream));
            HIPCHK(s, hipEventRecord(E[3], s->stream));
            HIPCHK(s, hipEventRecord(E[4], s->stream));
        } else {
            hipEvent_t mid[2] = {E[2], E[3]};
            if ((rc = launch_spectral(s, mid)) != LLG_OK) return rc;
            HIPCHK(s, hipEventRecord(E[4], s->stream));
        }
        StageArgs sa = {};
        sa.mode = ROW_EVAL;
        sa.m_in = bref_cur(s->mbuf[0], s->mbuf[1], 1);
        sa.m0 = sa.m_in;
        sa.m_out = bref(nullptr);
        sa.k_out = bref(nullptr);
        sa.h_out = s->hbuf;
        HIPCHK(s, row_inv(s, p, sa));
        HIPCHK(s, hipEventRecord(E[5], s->stream));
    }
    if ((rc = sync(s)) != LLG_OK) return rc;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < n; ++i) {
        hipEvent_t* E = &ev[6 * (size_t)i];
        float t01, t12, t23, t34, t45;
        HIPCHK(s, hipEventElapsedTime(&t01, E[0], E[1]));
        HIPCHK(s, hipEventElapsedTime(&t12, E[1], E[2]));
        HIPCHK(s, hipEventElapsedTime(&t23, E[2], E[3]));
        HIPCHK(s, hipEventElapsedTime(&t34, E[3], E[4]));
        HIPCHK(s, hipEventElapsedTime(&t45, E[4], E[5]));
        acc[0] += t01;
        if (two_d(s)) {
            acc[1] += t12;
        } else {
            acc[3] += t12;   // y forward
            acc[1] += t23;   // z pass with the product
            acc[4] += t34;   // y inverse
        }
        acc[2] += t45;
    }
    float tot;
    HIPCHK(s, hipEventElapsedTime(&tot, ev[0], ev[6 * (size_t)(n - 1) + 5]));
    for (int k = 0; k < 5; ++k) ms_out[k] = acc[k] / n;
    for (int k = 5; k < n_kinds; ++k) ms_out[k] = 0.0;
    *total_ms = tot;
    for (auto& e : ev) (void)hipEventDestroy(e);
    s->spec_valid = false;
    return restore_done(s, was);
}

llg_status llg_autotune(llg_solver* s, int iters, double* ms_out, int n_out, int* choice) {
    TraceRange trace_("llg_autotune");
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (iters < 1) return fail(s, LLG_E_ARG, "iters must be >= 1");
    if ((rc = ready(s, true)) != LLG_OK) return rc;
    if ((rc = ensure_kernel(s)) != LLG_OK) return rc;
    if (!s->fast2d) return fail(s, LLG_E_UNSUPPORTED, "no compiled variants for this geometry");
    const Phys p = make_phys(s, s->last_dt);
    if (!p.demag_on) return fail(s, LLG_E_STATE, "tuning needs the demag term");
    int was = 0;
    if ((rc = lift_done(s, &was)) != LLG_OK) return rc;
    const int Px = s->g.Px, L = s->g.Py / 2;
    const int r0 = s->g.rvar, c0 = s->g.cvar;
    double best = 1e300;
    int br = r0, bc = c0;
    hipEvent_t e0, e1;
    HIPCHK(s, hipEventCreate(&e0));
    HIPCHK(s, hipEventCreate(&e1));
    for (int rv = 0; rv < 2; ++rv) {
        for (int cv = 0; cv < 2; ++cv) {
            const int k = rv * 2 + cv;
            if (ms_out && k < n_out) ms_out[k] = -1.0;
            if (!fast2d_row_ok(Px, rv, s->g.nx == Px) || !fast2d_col_ok(L, 1, cv) ||
                (Px / 2) % fast2d_col_width(L, cv))
                continue;
            s->g.rvar = rv;
            s->g.cvar = cv;
            // one untimed evaluation, then `iters` timed ones (H_eff of the
            // current state, kept on the device)
            for (int it = 0; it <= iters; ++it) {
                if (it == 1) HIPCHK(s, hipEventRecord(e0, s->stream));
                if ((rc = launch_fwd_plain(s, 1)) != LLG_OK) break;
                if ((rc = launch_spectral(s)) != LLG_OK) break;
                StageArgs sa = {};
                sa.mode = ROW_EVAL;
                sa.m_in = bref_cur(s->mbuf[0], s->mbuf[1], 1);
                sa.m0 = sa.m_in;
                sa.m_out = bref(nullptr);
                sa.k_out = bref(nullptr);
                sa.h_out = s->hbuf;
                if (row_inv(s, p, sa) != hipSuccess) { rc = LLG_E_DEVICE; break; }
            }
            if (rc != LLG_OK) {
                s->g.rvar = r0;
                s->g.cvar = c0;
                invalidate_graphs(s);
                s->spec_valid = false;
                return fail(s, rc, "tuning launch failed");
            }
            HIPCHK(s, hipEventRecord(e1, s->stream));
            HIPCHK(s, hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(s, hipEventElapsedTime(&ms, e0, e1));
            const double per = ms / iters;
            if (ms_out && k < n_out) ms_out[k] = per;
            if (per < best) { best = per; br = rv; bc = cv; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s->g.rvar = br;
    s->g.cvar = bc;
    (void)fast2d_set_variants(Px, br, L, bc, s->g.nx == Px);   // default for solvers set up later
    invalidate_graphs(s);
    s->spec_valid = false;
    if (choice) { choice[0] = br; choice[1] = bc; }
    return restore_done(s, was);
}

llg_status llg_autotune_attempts(llg_solver* s, double max_err, double dt0, int attempts, double* ms_out,
                                 int n_out, int* choice) {
    TraceRange trace_("llg_autotune_attempts");
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (attempts < 1 || !(max_err > 0) || !isfinite(max_err) || !(dt0 >= 0) || !isfinite(dt0))
        return fail(s, LLG_E_ARG, "need attempts >= 1, max_err > 0, dt0 >= 0");
    if ((rc = ready(s, true)) != LLG_OK) return rc;
    if ((rc = ensure_kernel(s)) != LLG_OK) return rc;
    if (!s->fast2d) return fail(s, LLG_E_UNSUPPORTED, "no compiled variants for this geometry");
    const Phys p = make_phys(s, 0.0);
    if (!p.demag_on) return fail(s, LLG_E_STATE, "tuning needs the demag term");
    DevState h0;
    if ((rc = read_state(s, &h0)) != LLG_OK) return rc;
    if (h0.health) return fail(s, LLG_E_DIVERGED, "state already diverged");
    if (dt0 == 0 && !(h0.dt_next > 0)) return fail(s, LLG_E_STATE, "dt0 = 0 needs an earlier adaptive step");
    const double dt_first = dt0 > 0 ? dt0 : h0.dt_next;
    // every pair starts from the state as it is now: m saved here, the
    // record restored before each run (the attempt log and statistics with
    // it); t_end far enough ahead that no run is clipped
    const double t_end = h0.t + 1e30;
    const size_t bytes = sizeof(float) * 3 * (size_t)s->g.ncells;
    float* msave = nullptr;
    HIPCHK(s, hipMalloc(&msave, bytes));
    struct Free {
        float* p;
        ~Free() { free_dev(p); }
    } free_msave{msave};
    HIPCHK(s, hipMemcpyAsync(msave, s->mbuf[h0.cur], bytes, hipMemcpyDeviceToDevice, s->stream));
    auto restore = [&](bool final) -> llg_status {
        HIPCHK(s, hipMemcpyAsync(s->mbuf[0], msave, bytes, hipMemcpyDeviceToDevice, s->stream));
        DevState h = h0;
        h.cur = 0;
        h.done = final ? h0.done : 0;
        h.err_bits = 0u;
        s->spec_valid = false;
        s->k1_valid = false;
        return write_state(s, &h);
    };
    const int Px = s->g.Px, L = s->g.Py / 2;
    const int r0 = s->g.rvar, c0 = s->g.cvar;
    double best = 1e300;
    int br = r0, bc = c0;
    hipEvent_t e0, e1;
    HIPCHK(s, hipEventCreate(&e0));
    HIPCHK(s, hipEventCreate(&e1));
    for (int rv = 0; rv < 2 && rc == LLG_OK; ++rv) {
        for (int cv = 0; cv < 2 && rc == LLG_OK; ++cv) {
            const int k = rv * 2 + cv;
            if (ms_out && k < n_out) ms_out[k] = -1.0;
            if (!fast2d_row_ok(Px, rv, s->g.nx == Px) || !fast2d_col_ok(L, 1, cv) ||
                (Px / 2) % fast2d_col_width(L, cv))
                continue;
            s->g.rvar = rv;
            s->g.cvar = cv;
            invalidate_graphs(s);
            // untimed: two attempts (the graph capture), then back to the
            // start state and its first stage; timed: `attempts` attempts
            if ((rc = restore(false)) != LLG_OK) break;
            if ((rc = run_adaptive(s, LLG_RKDP45, t_end, max_err, dt_first, 2, nullptr)) != LLG_OK) break;
            if ((rc = restore(false)) != LLG_OK) break;
            if ((rc = ensure_k1(s, p)) != LLG_OK) break;
            if (hipEventRecord(e0, s->stream) != hipSuccess) { rc = fail(s, LLG_E_DEVICE, "event record"); break; }
            if ((rc = run_adaptive(s, LLG_RKDP45, t_end, max_err, dt_first, attempts, nullptr)) != LLG_OK) break;
            float ms = 0.f;
            if (hipEventRecord(e1, s->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = fail(s, LLG_E_DEVICE, "event timing");
                break;
            }
            const double per = ms / attempts;
            if (ms_out && k < n_out) ms_out[k] = per;
            if (per < best) { best = per; br = rv; bc = cv; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s->g.rvar = rc == LLG_OK ? br : r0;
    s->g.cvar = rc == LLG_OK ? bc : c0;
    invalidate_graphs(s);
    const llg_status rr = restore(true);
    if (rc != LLG_OK) return rc;
    if (rr != LLG_OK) return rr;
    (void)fast2d_set_variants(Px, br, L, bc, s->g.nx == Px);   // default for solvers set up later
    if (choice) { choice[0] = br; choice[1] = bc; }
    return LLG_OK;
}

llg_status llg_set_variants(llg_solver* s, int row_var, int col_var) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!s->fast2d) return fail(s, LLG_E_UNSUPPORTED, "no compiled variants for this geometry");
    const int Px = s->g.Px, L = s->g.Py / 2;
    if (!fast2d_row_ok(Px, row_var, s->g.nx == Px) || !fast2d_col_ok(L, 1, col_var) ||
        (Px / 2) % fast2d_col_width(L, col_var))
        return fail(s, LLG_E_ARG, "no compiled variant (%d, %d) for lengths %d, %d", row_var, col_var, Px, L);
    s->g.rvar = row_var;
    s->g.cvar = col_var;
    (void)fast2d_set_variants(Px, row_var, L, col_var, s->g.nx == Px);   // default for solvers set up later
    invalidate_graphs(s);
    s->spec_valid = false;
    return LLG_OK;
}

llg_status llg_variant_shape(int kind, int length, int variant, int* elems, int* classes) {
    if (!elems || !classes) return LLG_E_ARG;
    return fast2d_variant_shape(kind, length, variant, elems, classes) ? LLG_OK : LLG_E_ARG;
}

llg_status llg_get_variants(llg_solver* s, int* row_var, int* col_var) {
    if (!s || !row_var || !col_var) return LLG_E_ARG;
    if (!s->have_geom) return fail(s, LLG_E_STATE, "geometry not set");
    if (!s->fast2d) return fail(s, LLG_E_UNSUPPORTED, "no compiled variants for this geometry");
    *row_var = s->g.rvar;
    *col_var = s->g.cvar;
    return LLG_OK;
}

llg_status llg_kernel_bytes(llg_solver* s, double* bytes_out, int n_kinds) {
    if (!s) return LLG_E_ARG;
    if (!bytes_out || n_kinds < 5) return fail(s, LLG_E_ARG, "bad arguments");
    if (!s->have_geom) return fail(s, LLG_E_STATE, "geometry not set");
    const Grid& g = s->g;
    const double cell_vec = 12.0 * g.ncells;                     // 3 floats per cell
    const double spec_x = 3.0 * 8.0 * g.nrows * g.nkx;          // x-transformed spectrum
    for (int k = 0; k < n_kinds; ++k) bytes_out[k] = 0.0;
    bytes_out[0] = cell_vec + spec_x;                            // read m, write X
    bytes_out[2] = spec_x + 2.0 * cell_vec;                      // read Y and m, write H
    if (two_d(s)) {
        const double K = 4.0 * 4.0 * g.nkx * (g.Py / 2 + 1);
        bytes_out[1] = 2.0 * spec_x + K;                         // read X and K, write Y
    } else {
        const double spec_y = 3.0 * 8.0 * g.nz * g.Py * g.nkx;
        const double K = 6.0 * 4.0 * (g.Py / 2 + 1) * g.nkx * (g.Pz / 2 + 1);
        bytes_out[3] = spec_x + spec_y;
        bytes_out[1] = 2.0 * spec_y + K;
        bytes_out[4] = spec_y + spec_x;
    }
    return LLG_OK;
}

llg_status llg_fft_roundtrip(llg_solver* s, float* data, int n, int batch, int inverse_only) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (!data || n < 1 || n > 4096 || batch < 1 || !good_len(n))
        return fail(s, LLG_E_ARG, "need 1 <= n <= 4096 made of 2,3,5,7 and batch >= 1");
    FftPlan pl;
    if (!make_plan(n, pl)) return fail(s, LLG_E_UNSUPPORTED, "cannot factor %d", n);
    float2* d = nullptr;
    float2* tw = nullptr;
    const size_t bytes = sizeof(float2) * (size_t)n * batch;
    HIPCHK(s, make_tw(n, &tw));
    HIPCHK(s, hipMalloc(&d, bytes));
    HIPCHK(s, hipMemcpyAsync(d, data, bytes, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, launch_fft_test(d, n, batch, pl, tw, inverse_only, s->stream));
    HIPCHK(s, hipMemcpyAsync(data, d, bytes, hipMemcpyDeviceToHost, s->stream));
    rc = sync(s);
    free_dev(d);
    free_dev(tw);
    return rc;
}

llg_status llg_demag_tensor(llg_solver* s, const int32_t* offsets, int64_t count, double* out) {
    llg_status rc = enter(s);
    if (rc != LLG_OK) return rc;
    if (count < 0 || (count > 0 && (!offsets || !out))) return fail(s, LLG_E_ARG, "bad arguments");
    if (!s->have_geom || !s->have_cell) return fail(s, LLG_E_STATE, "geometry and cell size needed");
    const int n[3] = {s->nx, s->ny, s->nz};
    for (int64_t i = 0; i < count; ++i)
        for (int a = 0; a < 3; ++a)
            if (!s->pbc[a] && (offsets[3 * i + a] <= -n[a] || offsets[3 * i + a] >= n[a]))
                return fail(s, LLG_E_ARG, "offset %lld out of range on axis %d", (long long)i, a);
    if (count == 0) return LLG_OK;
    TensorGeom tg = {};
    const double d[3] = {s->dx, s->dy, s->dz};
    const double dm = fmax(d[0], fmax(d[1], d[2]));
    for (int a = 0; a < 3; ++a) {
        tg.n[a] = n[a];
        tg.P[a] = a == 0 ? s->g.Px : a == 1 ? s->g.Py : s->g.Pz;
        tg.pbc[a] = s->pbc[a];
        tg.d[a] = d[a] / dm;
    }
    tg.images = s->images;
    int32_t* od = nullptr;
    double* rd = nullptr;
    HIPCHK(s, hipMalloc(&od, sizeof(int32_t) * 3 * count));
    HIPCHK(s, hipMalloc(&rd, sizeof(double) * 6 * count));
    HIPCHK(s, hipMemcpyAsync(od, offsets, sizeof(int32_t) * 3 * count, hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, tensor_at_offsets(tg, od, count, rd, s->stream));
    HIPCHK(s, hipMemcpyAsync(out, rd, sizeof(double) * 6 * count, hipMemcpyDeviceToHost, s->stream));
    rc = sync(s);
    free_dev(od);
    free_dev(rd);
    return rc;
}

}  // extern "C"

namespace {

llg_status run_adaptive(llg_solver* s, int method, double t_end, double max_err, double dt0,
                        long long max_attempts, llg_stats* out) {
    TraceRange trace_("llg_run (adaptive)");
    llg_status rc;
    Adaptive ad;
    if (!adaptive_of(method, &ad)) return fail(s, LLG_E_ARG, "method %d is not an adaptive pair", method);
    if (!(max_err > 0) || !(dt0 >= 0) || !isfinite(t_end) || !isfinite(max_err) || !isfinite(dt0))
        return fail(s, LLG_E_ARG, "need max_err > 0, dt0 >= 0");
    if ((rc = ready(s, true)) != LLG_OK) return rc;
    if ((rc = ensure_kernel(s)) != LLG_OK) return rc;
    const Phys p = make_phys(s, 0.0);   // thermal field: fixed steps only
    DevState h;
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    if (h.health) return fail(s, LLG_E_DIVERGED, "state already diverged");
    if (!(t_end > h.t)) {
        if (out) fill_stats(h, out);
        return LLG_OK;
    }
    if (ad.fsal) {
        // k1 from the previous attempt is only reusable for the same pair
        if (s->gdp.method != method) s->k1_valid = false;
        if ((rc = ensure_k1(s, p)) != LLG_OK) return rc;
    }
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    if (dt0 == 0) {
        // continue with the step the controller chose last
        if (!(h.dt_next > 0)) return fail(s, LLG_E_STATE, "dt0 = 0 needs an earlier adaptive step");
        dt0 = h.dt_next;
    }
    h.ev_attempt = ad.fsal ? ad.t.S - 1 : ad.t.S;
    h.ctrl_exp = 1.0 / (ad.q + 1);
    h.t_end = t_end;
    h.tol = max_err;
    h.dt_min = kDtMin;
    h.gms = kGamma0 * s->Ms;
    h.done = 0;
    h.err_bits = 0u;
    const double rem = t_end - h.t;
    if (dt0 >= rem) { h.dt = rem; h.clipped = 1; } else { h.dt = dt0; h.clipped = 0; }
    h.dtau = (float)(h.dt * h.gms);
    if ((rc = write_state(s, &h)) != LLG_OK) return rc;
    if (!s->gdp.exec || s->gdp.method != method) {
        if ((rc = capture(s, s->gdp, ad.fsal ? fsal_body : plain_body, ad.t, p)) != LLG_OK) return rc;
        s->gdp.method = method;
    }
    if ((rc = launch_until_done(s, s->gdp.exec, max_attempts > 0 ? max_attempts : -1)) != LLG_OK) return rc;
    if ((rc = read_state(s, &h)) != LLG_OK) return rc;
    // the state buffers now hold the accepted solution; the x spectrum and
    // k1 buffers follow the last accepted attempt only
    s->spec_valid = false;
    s->k1_valid = ad.fsal;
    if (out) fill_stats(h, out);
    if (h.health & 2) return fail(s, LLG_E_DIVERGED, "step size fell below %g s", kDtMin);
    if (h.health) return fail(s, LLG_E_DIVERGED, "non-finite field or torque");
    return LLG_OK;
}

}  // namespace
