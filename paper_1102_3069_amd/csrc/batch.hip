// Batched runtime: many independent 2D films of uneven size (a parameter
// sweep) integrated together with adaptive Dormand-Prince 5(4) or with
// fixed Euler, Heun or RK4 steps.
//
// Every pass of an attempt (the first-stage forward transform, then per
// stage the column pass and the fused row pass, then the step controller)
// is ONE grouped launch that covers all films: its blocks are mapped to
// (film, local tile) by a table, and every block runs the compiled-length
// kernel body of its film's size.  Each film keeps its own device state
// (time, step size, accept/reject, buffer swap, attempt log), so films
// advance with their own steps inside the same launches; a film that has
// reached t_end leaves its blocks idle.  The attempt is captured once into a
// HIP graph and replayed.  The per-film arithmetic is exactly that of the
// single-film solver, so a film's result does not depend on the batch it
// runs in.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <string>
#include <vector>

#include "host_common.hpp"
#include "internal.hpp"

using namespace llg;
using namespace llg::host;

namespace {

struct BatchFilm {
    Material mat;
    Grid g = {};
    float2 *twx = nullptr, *twy = nullptr;
    float* K = nullptr;
    float2* S = nullptr;
    float* mbuf[2] = {nullptr, nullptr};
    float* ms[2] = {nullptr, nullptr};
    float* kb[6] = {};
    float* kfs[2] = {nullptr, nullptr};
    llg_attempt* log = nullptr;
    int row_blocks = 0, col_blocks = 0;   // blocks per pass with the variants g.rvar, g.cvar
};

}  // namespace

struct llg_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<BatchFilm> films;
    DevState* st = nullptr;             // one state per film, contiguous
    long long log_cap = 1 << 16;
    // grouped launch arguments (device arrays, one entry per film)
    FilmRow* d_fwd_plain = nullptr;     // k1 initialisation: forward pass of m
    FilmRow* d_konly = nullptr;         // k1 initialisation: k of m
    FilmRow* d_prep = nullptr;          // stage-2 input and its forward pass
    FilmRow* d_stage[6] = {};           // stages 2..7
    FilmCol* d_col = nullptr;
    // length classes: films of one compiled row (column) variant share a
    // launch; the launches of one pass run as parallel branches
    struct Class {
        int len = 0, var = 0;
        int2* map = nullptr;            // (film, local block) of every block
        int nblocks = 0;
    };
    std::vector<Class> rows, cols;
    std::vector<char> in_map;           // films whose blocks the maps hold
    std::vector<hipStream_t> aux;       // branch streams (default priority)
    std::vector<hipEvent_t> ev;         // fork / join events
    hipGraphExec_t graph = nullptr;
    bool k1_valid = false;
    // fixed steps: per-stage arguments and the captured step of one method
    FilmRow* d_fix[4] = {};
    int fix_method = -1;
    hipGraphExec_t gfix = nullptr;
    hipEvent_t ev_in = nullptr;         // start states ready on the caller's stream
    hipEvent_t ev_out = nullptr;        // end of the last enqueued fixed steps
    // where each film's state sits (mbuf index), known on the host after
    // fixed steps without a state read; hcur_ok is cleared by every call that
    // can move a state otherwise
    std::vector<int> hcur;
    bool hcur_ok = false;
    double fix_dt = 0.0;                // step of the last fixed steps, held in the device states
    bool spec_valid = false;            // S holds the forward x pass of every film's m
};

namespace {

llg_status bfail(llg_batch* b, llg_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) b->err = buf;
    return code;
}

#define BCHK(b, x)                                                                                \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess)                                                                     \
            return bfail(b, e_ == hipErrorOutOfMemory ? LLG_E_NOMEM : LLG_E_DEVICE, "%s: %s (%s:%d)", \
                         #x, hipGetErrorString(e_), __FILE__, __LINE__);                          \
    } while (0)

void bfree(void* p) {
    if (p) (void)hipFree(p);
}

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& v) {
    hipError_t e = hipMalloc(dst, sizeof(T) * v.size());
    if (e == hipSuccess) e = hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
    return e;
}

Col2dArgs col_args(const BatchFilm& f) {
    Col2dArgs c = {};
    c.S = f.S;
    c.K = f.K;
    c.tw = f.twy;
    c.nkx = f.g.Px / 2;
    c.nkx_full = f.g.nkx;
    c.nkxp = f.g.nkxp;
    c.tsh = f.g.tsh;
    c.nq = fast2d_row_classes(f.g.Px, f.g.rvar);
    c.var = f.g.cvar;
    c.ny = f.g.ny;
    c.Py = f.g.Py;
    return c;
}

// the table's default variants where they serve the film's lengths, else
// variant 0 (the rule of the single-film solver); false if even that fails
bool pick_variants(Grid& g) {
    const int L = g.Py / 2;
    g.rvar = fast2d_row_variant(g.Px);
    if (!fast2d_row_ok(g.Px, g.rvar)) g.rvar = 0;
    g.cvar = fast2d_col_variant(L);
    if (!fast2d_col_ok(L, 1, g.cvar) || (g.Px / 2) % fast2d_col_width(L, g.cvar)) g.cvar = 0;
    return fast2d_row_ok(g.Px, g.rvar) && fast2d_col_ok(L, 1, g.cvar) && (g.Px / 2) % fast2d_col_width(L, g.cvar) == 0;
}

FilmRow row_base(const llg_batch* b, int i) {
    const BatchFilm& f = b->films[i];
    FilmRow r = {};
    r.g = f.g;
    r.p = phys_of(f.mat, 0.0);
    r.twx = f.twx;
    r.S = f.S;
    r.st = b->st + i;
    return r;
}

// block maps per length class (largest classes first) over the films
// marked in `active`; the captured graphs, which hold the maps, are dropped
llg_status build_classes(llg_batch* b, const std::vector<char>& active) {
    const int nf = (int)b->films.size();
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    if (b->gfix) (void)hipGraphExecDestroy(b->gfix);
    b->gfix = nullptr;
    b->fix_method = -1;
    for (auto& c : b->rows) bfree(c.map);
    for (auto& c : b->cols) bfree(c.map);
    b->rows.clear();
    b->cols.clear();
    auto build = [&](bool row, std::vector<llg_batch::Class>& out) -> llg_status {
        std::vector<std::pair<int, int>> keys;
        for (int i = 0; i < nf; ++i) {
            if (!active[i]) continue;
            const BatchFilm& f = b->films[i];
            const std::pair<int, int> k = row ? std::make_pair(f.g.Px, f.g.rvar) : std::make_pair(f.g.Py / 2, f.g.cvar);
            if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
        }
        std::sort(keys.begin(), keys.end(), [](const std::pair<int, int>& x, const std::pair<int, int>& y) {
            return x.first > y.first || (x.first == y.first && x.second < y.second);
        });
        for (const auto& k : keys) {
            std::vector<int2> map;
            for (int i = 0; i < nf; ++i) {
                if (!active[i]) continue;
                const BatchFilm& f = b->films[i];
                const bool in = row ? (f.g.Px == k.first && f.g.rvar == k.second)
                                    : (f.g.Py / 2 == k.first && f.g.cvar == k.second);
                if (!in) continue;
                const int nb = row ? f.row_blocks : f.col_blocks;
                for (int j = 0; j < nb; ++j) map.push_back(make_int2(i, j));
            }
            // XCD-aware order: hardware block h runs entry remap(h), so the
            // blocks one XCD runs are contiguous rows or columns of a film
            const int nb = (int)map.size();
            std::vector<int2> order(nb);
            for (int h = 0; h < nb; ++h) {
                const int X = 8, x = h % X, i = h / X, q = nb / X, rmd = nb % X;
                order[h] = map[x * q + std::min(x, rmd) + i];
            }
            llg_batch::Class c;
            c.len = k.first;
            c.var = k.second;
            c.nblocks = nb;
            BCHK(b, upload(&c.map, order));
            out.push_back(c);
        }
        return LLG_OK;
    };
    llg_status rc = build(true, b->rows);
    if (rc == LLG_OK) rc = build(false, b->cols);
    if (rc != LLG_OK) return rc;
    const size_t nbr = std::max(b->rows.size(), b->cols.size());
    while (b->aux.size() + 1 < nbr) {
        hipStream_t st = nullptr;
        BCHK(b, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        b->aux.push_back(st);
    }
    while (b->ev.size() < nbr) {
        hipEvent_t e = nullptr;
        BCHK(b, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->ev.push_back(e);
    }
    b->in_map = active;
    return LLG_OK;
}

// all films in the block maps again (after a run dropped finished ones)
llg_status restore_classes(llg_batch* b) {
    const std::vector<char> all(b->films.size(), 1);
    if (b->in_map == all) return LLG_OK;
    return build_classes(b, all);
}

void free_launch_args(llg_batch* b) {
    bfree(b->d_fwd_plain); b->d_fwd_plain = nullptr;
    bfree(b->d_konly); b->d_konly = nullptr;
    bfree(b->d_prep); b->d_prep = nullptr;
    for (auto& p : b->d_stage) { bfree(p); p = nullptr; }
    bfree(b->d_col); b->d_col = nullptr;
}

// the per-film arguments of every grouped launch of an attempt, for the
// films' current variants (the column pass reads the row variant's
// spectrum order from them), and the block maps; buffer roles follow the
// single-film Dormand-Prince attempt exactly.  Called whenever a variant
// changes: arguments built for other variants would misread the spectrum.
llg_status build_launch_args(llg_batch* b) {
    const int nf = (int)b->films.size();
    (void)hipStreamSynchronize(b->stream);   // no launch still reads the old arguments
    free_launch_args(b);
    for (BatchFilm& f : b->films) {
        f.row_blocks = (f.g.nrows + fast2d_row_rows_per_block(f.g.Px, f.g.rvar) - 1) /
                       fast2d_row_rows_per_block(f.g.Px, f.g.rvar);
        f.col_blocks = fast2d_col_blocks(f.g.Py / 2, f.g.cvar, f.g.Px / 2);
    }
    const Tableau t = tab_dp45();
    std::vector<FilmRow> fwd_plain(nf), konly(nf), prep(nf), stage[6];
    std::vector<FilmCol> col(nf);
    for (auto& v : stage) v.resize(nf);
    for (int i = 0; i < nf; ++i) {
        BatchFilm& f = b->films[i];
        const BufRef mcur = bref_cur(f.mbuf[0], f.mbuf[1], 1);
        const BufRef mnext = bref_cur(f.mbuf[0], f.mbuf[1], 2);
        BufRef kref[7];
        kref[0] = bref_cur(f.kfs[0], f.kfs[1], 1);
        for (int j = 1; j <= 5; ++j) kref[j] = bref(f.kb[j]);
        kref[6] = bref_cur(f.kfs[0], f.kfs[1], 2);

        FilmRow r = row_base(b, i);
        r.fa.m_in = mcur; r.fa.combine = 0; r.fa.m0 = mcur; r.fa.k1 = mcur; r.fa.m_out = bref(nullptr);
        fwd_plain[i] = r;

        r = row_base(b, i);
        r.sa.mode = ROW_KONLY;
        r.sa.m_in = mcur; r.sa.m0 = mcur; r.sa.m_out = bref(nullptr); r.sa.k_out = kref[0];
        konly[i] = r;

        r = row_base(b, i);
        r.fa.combine = 1;
        r.fa.a1 = (float)t.A[1][0];
        r.fa.m0 = mcur; r.fa.k1 = kref[0]; r.fa.m_in = mcur; r.fa.m_out = bref(f.ms[0]);
        prep[i] = r;

        for (int s = 2; s <= 7; ++s) {
            r = row_base(b, i);
            StageArgs& sa = r.sa;
            sa.m0 = mcur;
            sa.m_in = s == 7 ? mnext : bref(f.ms[s % 2 == 0 ? 0 : 1]);
            sa.k_out = kref[s - 1];
            sa.nk = s;
            for (int j = 0; j + 1 < s; ++j) sa.kprev[j] = kref[j];
            if (s < 7) {
                sa.mode = ROW_STAGE;
                sa.m_out = s == 6 ? mnext : bref(f.ms[s % 2 == 0 ? 1 : 0]);
                for (int j = 0; j < s; ++j) sa.a[j] = (float)t.A[s][j];
            } else {
                sa.mode = ROW_ERROR;
                sa.m_out = bref(nullptr);
                for (int j = 0; j < 7; ++j) sa.e[j] = (float)(t.b[j] - t.bhat[j]);
            }
            stage[s - 2][i] = r;
        }
        col[i].a = col_args(f);
        col[i].st = b->st + i;
    }
    BCHK(b, upload(&b->d_fwd_plain, fwd_plain));
    BCHK(b, upload(&b->d_konly, konly));
    BCHK(b, upload(&b->d_prep, prep));
    for (int s = 0; s < 6; ++s) BCHK(b, upload(&b->d_stage[s], stage[s]));
    BCHK(b, upload(&b->d_col, col));
    std::vector<char> all(nf, 1);
    return build_classes(b, all);
}

// one pass over all films: a launch per length class, the classes as
// parallel branches forked from and joined back into the batch stream
enum PassKind { PASS_ROW_FWD, PASS_ROW_INV, PASS_COL };

llg_status pass(llg_batch* b, PassKind kind, const FilmRow* rows) {
    const std::vector<llg_batch::Class>& cl = kind == PASS_COL ? b->cols : b->rows;
    const int n = (int)cl.size();
    if (n > 1) {
        BCHK(b, hipEventRecord(b->ev[0], b->stream));
        for (int i = 1; i < n; ++i) BCHK(b, hipStreamWaitEvent(b->aux[i - 1], b->ev[0], 0));
    }
    for (int i = 0; i < n; ++i) {
        hipStream_t st = i == 0 ? b->stream : b->aux[i - 1];
        const llg_batch::Class& c = cl[i];
        hipError_t e = kind == PASS_ROW_FWD ? launch_row_fwd_group(c.len, c.var, rows, c.map, c.nblocks, st)
                     : kind == PASS_ROW_INV ? launch_row_inv_group(c.len, c.var, rows, c.map, c.nblocks, st)
                                            : launch_col_group(c.len, c.var, b->d_col, c.map, c.nblocks, st);
        BCHK(b, e);
    }
    for (int i = 1; i < n; ++i) {
        BCHK(b, hipEventRecord(b->ev[i], b->aux[i - 1]));
        BCHK(b, hipStreamWaitEvent(b->stream, b->ev[i], 0));
    }
    return LLG_OK;
}

#define PASS(b, kind, rows)                                  \
    do {                                                     \
        llg_status rc_ = pass((b), (kind), (rows));          \
        if (rc_ != LLG_OK) return rc_;                       \
    } while (0)

llg_status enqueue_attempt(llg_batch* b) {
    const int nf = (int)b->films.size();
    PASS(b, PASS_ROW_FWD, b->d_prep);
    for (int s = 0; s < 6; ++s) {
        PASS(b, PASS_COL, nullptr);
        PASS(b, PASS_ROW_INV, b->d_stage[s]);
    }
    BCHK(b, launch_ctrl_dp45_group(b->st, nf, b->stream));
    return LLG_OK;
}

// per-stage arguments of a fixed step; buffer roles follow the single-film
// fixed step exactly (stage inputs alternate between ms[0] and ms[1], k_j
// in kb[j-1], the last stage writes the next state and its forward pass)
llg_status build_fixed_args(llg_batch* b, const Tableau& t) {
    const int nf = (int)b->films.size();
    for (int st = 1; st <= t.S; ++st) {
        std::vector<FilmRow> v(nf);
        bool needed = false;
        if (st < t.S) {
            if (t.b[st - 1] != 0.0) needed = true;
            for (int r = st; r < t.S; ++r)
                if (t.A[r][st - 1] != 0.0) needed = true;
        }
        for (int i = 0; i < nf; ++i) {
            BatchFilm& f = b->films[i];
            FilmRow r = row_base(b, i);
            StageArgs& sa = r.sa;
            sa.mode = ROW_STAGE;
            sa.m_in = st == 1 ? bref_cur(f.mbuf[0], f.mbuf[1], 1) : bref(f.ms[st % 2]);
            sa.m0 = bref_cur(f.mbuf[0], f.mbuf[1], 1);
            sa.m_out = st == t.S ? bref_cur(f.mbuf[0], f.mbuf[1], 2) : bref(f.ms[(st + 1) % 2]);
            sa.k_out = bref(needed ? f.kb[st - 1] : nullptr);
            sa.nk = st;
            for (int j = 0; j < st; ++j) sa.a[j] = (float)(st < t.S ? t.A[st][j] : t.b[j]);
            for (int j = 0; j + 1 < st; ++j) sa.kprev[j] = bref(f.kb[j]);
            v[i] = r;
        }
        bfree(b->d_fix[st - 1]);
        b->d_fix[st - 1] = nullptr;
        BCHK(b, upload(&b->d_fix[st - 1], v));
    }
    return LLG_OK;
}

llg_status enqueue_fixed(llg_batch* b, int nstages) {
    for (int st = 0; st < nstages; ++st) {
        PASS(b, PASS_COL, nullptr);
        PASS(b, PASS_ROW_INV, b->d_fix[st]);
    }
    BCHK(b, launch_ctrl_fixed_group(b->st, (int)b->films.size(), nstages, b->stream));
    return LLG_OK;
}

llg_status read_states(llg_batch* b, std::vector<DevState>& h) {
    h.resize(b->films.size());
    BCHK(b, hipMemcpyAsync(h.data(), b->st, sizeof(DevState) * h.size(), hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    return LLG_OK;
}

llg_status write_states(llg_batch* b, const std::vector<DevState>& h) {
    BCHK(b, hipMemcpyAsync(b->st, h.data(), sizeof(DevState) * h.size(), hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    return LLG_OK;
}

void fill(const DevState& h, llg_stats* o) {
    o->t = h.t; o->dt = h.dt; o->dt_next = h.dt_next; o->max_err = h.last_err;
    o->steps = h.nsteps; o->rejected = h.nrej; o->evals = h.nevals;
    o->health = h.health; o->done = h.done;
}

}  // namespace

extern "C" {

llg_status llg_batch_create(int device, const llg_film_desc* films, int nfilms, llg_batch** out) {
    if (!out || !films || nfilms < 1) return LLG_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return LLG_E_DEVICE;
    if (device < 0 || device >= ndev) return LLG_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return LLG_E_DEVICE;
    llg_batch* b = new llg_batch();
    b->device = device;
    *out = b;
    BCHK(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    b->films.resize(nfilms);
    for (int i = 0; i < nfilms; ++i) {
        const llg_film_desc& d = films[i];
        BatchFilm& f = b->films[i];
        if (d.nx < 1 || d.ny < 1 || !(d.dx > 0 && d.dy > 0 && d.dz > 0) || !(d.Ms > 0) || !(d.Aex >= 0) ||
            !(d.alpha >= 0) || !d.m0)
            return bfail(b, LLG_E_ARG, "film %d: invalid parameters", i);
        const double un = sqrt(d.u[0] * d.u[0] + d.u[1] * d.u[1] + d.u[2] * d.u[2]);
        if (!(un > 0)) return bfail(b, LLG_E_ARG, "film %d: anisotropy axis must be non-zero", i);
        // each axis is padded to the shortest compiled length >= 2 n
        const int Px = fast2d_row_len_at_least(pad_len(d.nx));
        const int L = fast2d_col_len_at_least(pad_len(d.ny) / 2);
        const int Py = 2 * L;
        if (Px == 0 || L == 0)
            return bfail(b, LLG_E_UNSUPPORTED, "film %d: %d x %d exceeds the compiled batched lengths", i, d.nx,
                         d.ny);
        Grid vg = {};
        vg.Px = Px;
        vg.Py = 2 * L;
        if (!pick_variants(vg) || d.ny > L)
            return bfail(b, LLG_E_UNSUPPORTED,
                         "film %d: %d x %d needs FFT lengths %d x %d without a compiled batched kernel", i,
                         d.nx, d.ny, Px, Py);
        f.mat.Ms = d.Ms; f.mat.Aex = d.Aex; f.mat.alpha = d.alpha; f.mat.Ku = d.Ku;
        for (int a = 0; a < 3; ++a) { f.mat.u[a] = d.u[a]; f.mat.B[a] = d.B[a]; }
        f.mat.d[0] = d.dx; f.mat.d[1] = d.dy; f.mat.d[2] = d.dz;
        f.mat.terms = LLG_TERM_ALL & ~LLG_TERM_THERMAL;
        Grid& g = f.g;
        g.nx = d.nx; g.ny = d.ny; g.nz = 1;
        g.nrows = d.ny; g.ncells = d.nx * d.ny;
        g.Px = Px; g.Py = Py; g.Pz = 1;
        g.nkx = Px / 2 + 1;
        g.nkxp = (g.nkx + 15) / 16 * 16;
        g.tsh = fast2d_tile_shift();
        g.split_y = 1; g.split_z = 0;
        g.rvar = vg.rvar;
        g.cvar = vg.cvar;
        const size_t vec = sizeof(float) * 3 * (size_t)g.ncells;
        BCHK(b, make_tw(Px, &f.twx));
        BCHK(b, make_tw(Py, &f.twy));
        BCHK(b, hipMalloc(&f.S, sizeof(float2) * 3 * (size_t)g.nrows * g.nkxp));
        BCHK(b, hipMalloc(&f.K, sizeof(float) * 4 * (size_t)g.nkx * (Py / 2 + 1)));
        for (auto& p : f.mbuf) BCHK(b, hipMalloc(&p, vec));
        for (auto& p : f.ms) BCHK(b, hipMalloc(&p, vec));
        for (auto& p : f.kb) BCHK(b, hipMalloc(&p, vec));
        for (auto& p : f.kfs) BCHK(b, hipMalloc(&p, vec));
        BCHK(b, hipMalloc(&f.log, sizeof(llg_attempt) * b->log_cap));
        // demag kernel spectrum (FP64 build, FP32 store)
        TensorGeom tg = {};
        const double dm = std::max(d.dx, std::max(d.dy, d.dz));
        tg.n[0] = d.nx; tg.n[1] = d.ny; tg.n[2] = 1;
        tg.P[0] = Px; tg.P[1] = Py; tg.P[2] = 1;
        tg.d[0] = d.dx / dm; tg.d[1] = d.dy / dm; tg.d[2] = d.dz / dm;
        tg.images = 0;
        double resid = 0.0;
        BCHK(b, build_kernel_spectrum(g, tg, f.K, &resid, b->stream));
        if (!(resid <= 1e-9)) return bfail(b, LLG_E_DEVICE, "film %d: kernel spectrum not real (%g)", i, resid);
        // initial magnetisation, checked and renormalised
        int* bad = nullptr;
        int hbad = 0;
        BCHK(b, hipMalloc(&bad, sizeof(int)));
        BCHK(b, hipMemsetAsync(bad, 0, sizeof(int), b->stream));
        BCHK(b, hipMemcpyAsync(f.mbuf[0], d.m0, vec, hipMemcpyHostToDevice, b->stream));
        BCHK(b, launch_normalize_check(f.mbuf[0], g.ncells, bad, b->stream));
        BCHK(b, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, b->stream));
        BCHK(b, hipStreamSynchronize(b->stream));
        bfree(bad);
        if (hbad) return bfail(b, LLG_E_ARG, "film %d: m is not a field of unit vectors", i);
    }
    std::vector<DevState> h(nfilms);
    for (int i = 0; i < nfilms; ++i) {
        h[i] = DevState{};
        h[i].log = b->films[i].log;
        h[i].log_cap = b->log_cap;
        h[i].gms = kGamma0 * b->films[i].mat.Ms;
    }
    BCHK(b, hipMalloc(&b->st, sizeof(DevState) * nfilms));
    llg_status rc = write_states(b, h);
    if (rc != LLG_OK) return rc;
    return build_launch_args(b);
}

void llg_batch_destroy(llg_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    if (b->gfix) (void)hipGraphExecDestroy(b->gfix);
    for (auto p : b->d_fix) bfree(p);
    for (auto& f : b->films) {
        bfree(f.twx); bfree(f.twy); bfree(f.K); bfree(f.S); bfree(f.log);
        for (auto p : f.mbuf) bfree(p);
        for (auto p : f.ms) bfree(p);
        for (auto p : f.kb) bfree(p);
        for (auto p : f.kfs) bfree(p);
    }
    bfree(b->st);
    free_launch_args(b);
    for (auto& c : b->rows) bfree(c.map);
    for (auto& c : b->cols) bfree(c.map);
    for (auto st : b->aux) (void)hipStreamDestroy(st);
    for (auto e : b->ev) (void)hipEventDestroy(e);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char* llg_batch_last_error(const llg_batch* b) { return b ? b->err.c_str() : "null batch"; }

llg_status llg_batch_run(llg_batch* b, double t_end, double max_err, double dt0, int64_t max_attempts,
                         llg_stats* per_film) {
    TraceRange trace_("llg_batch_run");
    if (!b) return LLG_E_ARG;
    b->err.clear();
    BCHK(b, hipSetDevice(b->device));
    if (!(max_err > 0) || !(dt0 >= 0) || !isfinite(t_end) || !isfinite(dt0))
        return bfail(b, LLG_E_ARG, "need max_err > 0, dt0 >= 0");
    b->hcur_ok = false;
    const int nf = (int)b->films.size();
    std::vector<DevState> h;
    llg_status rc = restore_classes(b);
    if (rc != LLG_OK) return rc;
    if ((rc = read_states(b, h)) != LLG_OK) return rc;
    if (!b->k1_valid) {
        PASS(b, PASS_ROW_FWD, b->d_fwd_plain);
        PASS(b, PASS_COL, nullptr);
        PASS(b, PASS_ROW_INV, b->d_konly);
        b->k1_valid = true;
        for (auto& s : h) s.nevals += 1;
    }
    b->spec_valid = false;
    for (auto& s : h) {
        if (s.health) return bfail(b, LLG_E_DIVERGED, "a film has already diverged");
        s.t_end = t_end;
        s.tol = max_err;
        s.ev_attempt = 6;          // Dormand-Prince: six evaluations per attempt
        s.ctrl_exp = 0.2;
        s.dt_min = kDtMin;
        s.err_bits = 0u;
        s.done = !(t_end > s.t);
        // dt0 = 0: each film continues with its controller's last choice
        const double first = dt0 > 0 ? dt0 : s.dt_next;
        if (!(first > 0) && !s.done) return bfail(b, LLG_E_STATE, "dt0 = 0 needs an earlier adaptive step");
        const double rem = t_end - s.t;
        if (first >= rem) { s.dt = rem; s.clipped = 1; } else { s.dt = first; s.clipped = 0; }
        s.dtau = (float)(s.dt * s.gms);
    }
    if ((rc = write_states(b, h)) != LLG_OK) return rc;
    auto capture_attempt = [&]() -> llg_status {
        hipGraph_t graph = nullptr;
        BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        llg_status r = enqueue_attempt(b);
        hipError_t e = hipStreamEndCapture(b->stream, &graph);
        if (r != LLG_OK) { if (graph) (void)hipGraphDestroy(graph); return r; }
        BCHK(b, e);
        e = hipGraphInstantiate(&b->graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        BCHK(b, e);
        return LLG_OK;
    };
    if (!b->graph && (rc = capture_attempt()) != LLG_OK) return rc;
    int mapped = nf;
    long long launched = 0;
    for (;;) {
        int nl = 8;
        if (max_attempts > 0) {
            const long long left = max_attempts - launched;
            if (left <= 0) break;
            nl = (int)std::min<long long>(nl, left);
        }
        for (int i = 0; i < nl; ++i) BCHK(b, hipGraphLaunch(b->graph, b->stream));
        launched += nl;
        if ((rc = read_states(b, h)) != LLG_OK) return rc;
        int active = 0;
        for (auto& s : h) active += !s.done;
        if (active == 0) break;
        // once half the mapped films have finished, launch only the others
        // (a finished film's blocks would exit at once; their launch is the
        // cost).  A film's arithmetic does not depend on the maps.
        if (2 * active <= mapped) {
            std::vector<char> act(nf);
            for (int i = 0; i < nf; ++i) act[i] = !h[i].done;
            if ((rc = build_classes(b, act)) != LLG_OK) return rc;
            if ((rc = capture_attempt()) != LLG_OK) return rc;
            mapped = active;
        }
    }
    if (per_film)
        for (int i = 0; i < nf; ++i) fill(h[i], per_film + i);
    for (auto& s : h)
        if (s.health) return bfail(b, LLG_E_DIVERGED, "a film diverged (health %d)", s.health);
    return LLG_OK;
}

llg_status llg_batch_get_m(llg_batch* b, int film, float* m, llg_mem where) {
    if (!b || !m || film < 0 || film >= (int)b->films.size()) return LLG_E_ARG;
    BCHK(b, hipSetDevice(b->device));
    std::vector<DevState> h;
    llg_status rc = read_states(b, h);
    if (rc != LLG_OK) return rc;
    const BatchFilm& f = b->films[film];
    BCHK(b, hipMemcpyAsync(m, f.mbuf[h[film].cur], sizeof(float) * 3 * (size_t)f.g.ncells,
                           where == LLG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    return LLG_OK;
}

llg_status llg_batch_get_attempts(llg_batch* b, int film, llg_attempt* out, int64_t cap, int64_t* n) {
    if (!b || !n || film < 0 || film >= (int)b->films.size() || (cap > 0 && !out)) return LLG_E_ARG;
    BCHK(b, hipSetDevice(b->device));
    std::vector<DevState> h;
    llg_status rc = read_states(b, h);
    if (rc != LLG_OK) return rc;
    long long have = std::min<long long>(h[film].nattempt, b->log_cap);
    have = std::min<long long>(have, cap);
    *n = have;
    if (have > 0) {
        BCHK(b, hipMemcpyAsync(out, b->films[film].log, sizeof(llg_attempt) * have, hipMemcpyDeviceToHost,
                               b->stream));
        BCHK(b, hipStreamSynchronize(b->stream));
    }
    return LLG_OK;
}

}  // extern "C"

namespace {

// nsteps fixed steps of every film.  With src, films 0..nload-1 first take
// new start states src + j * stride (floats), copied on the batch stream once
// `producer` has reached this point, out[j] receives their end-state buffers
// and no film's health is checked (the caller checks the end states it
// uses).  The state block is read twice (two host synchronisations) and
// written without a wait of its own.
llg_status fixed_core(llg_batch* b, llg_method method, double dt, int64_t nsteps, const float* src, size_t stride,
                      int nload, hipStream_t producer, float** out) {
    Tableau t;
    if (!fixed_of(method, &t)) return bfail(b, LLG_E_ARG, "llg_batch_step takes Euler, Heun, RK3 or RK4");
    if (!(dt > 0) || !isfinite(dt) || nsteps < 0) return bfail(b, LLG_E_ARG, "need dt > 0, nsteps >= 0");
    if (src && (nload < 1 || nload > (int)b->films.size())) return bfail(b, LLG_E_ARG, "bad start-state count");
    if (nsteps == 0 && !src) return LLG_OK;
    b->hcur_ok = false;
    std::vector<DevState> h;
    llg_status rc = restore_classes(b);
    if (rc != LLG_OK) return rc;
    if ((rc = read_states(b, h)) != LLG_OK) return rc;
    const int nchk = src ? 0 : (int)h.size();
    if (src) {
        if (!b->ev_in) BCHK(b, hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
        BCHK(b, hipEventRecord(b->ev_in, producer));
        BCHK(b, hipStreamWaitEvent(b->stream, b->ev_in, 0));
        for (int j = 0; j < nload; ++j) {
            const BatchFilm& f = b->films[j];
            BCHK(b, hipMemcpyAsync(f.mbuf[h[j].cur], src + (size_t)j * stride, sizeof(float) * 3 * (size_t)f.g.ncells,
                                   hipMemcpyDeviceToDevice, b->stream));
            h[j].health = 0;
        }
        b->spec_valid = false;
        b->k1_valid = false;
    }
    for (size_t i = 0; i < h.size(); ++i) {
        if ((int)i < nchk && h[i].health) return bfail(b, LLG_E_DIVERGED, "film %d has already diverged", (int)i);
        h[i].dt = dt;
        h[i].dtau = (float)(dt * kGamma0 * b->films[i].mat.Ms);
        h[i].gms = kGamma0 * b->films[i].mat.Ms;
        h[i].done = 0;
    }
    BCHK(b, hipMemcpyAsync(b->st, h.data(), sizeof(DevState) * h.size(), hipMemcpyHostToDevice, b->stream));
    // every return from here on leaves the stream drained, so h (the copy's
    // source) is never released under a pending transfer
    struct Drain {
        hipStream_t s;
        ~Drain() { (void)hipStreamSynchronize(s); }
    } drain{b->stream};
    if (!b->spec_valid)
        PASS(b, PASS_ROW_FWD, b->d_fwd_plain);
    if (!b->gfix || b->fix_method != (int)method) {
        if (b->gfix) (void)hipGraphExecDestroy(b->gfix);
        b->gfix = nullptr;
        b->fix_method = -1;
        if ((rc = build_fixed_args(b, t)) != LLG_OK) return rc;
        hipGraph_t graph = nullptr;
        BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        rc = enqueue_fixed(b, t.S);
        hipError_t e = hipStreamEndCapture(b->stream, &graph);
        if (rc != LLG_OK) { if (graph) (void)hipGraphDestroy(graph); return rc; }
        BCHK(b, e);
        e = hipGraphInstantiate(&b->gfix, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        BCHK(b, e);
        b->fix_method = (int)method;
    }
    for (int64_t i = 0; i < nsteps; ++i) BCHK(b, hipGraphLaunch(b->gfix, b->stream));
    b->spec_valid = true;
    b->k1_valid = false;
    if ((rc = read_states(b, h)) != LLG_OK) return rc;
    b->hcur.resize(h.size());
    for (size_t i = 0; i < h.size(); ++i) b->hcur[i] = h[i].cur;
    b->hcur_ok = true;
    b->fix_dt = dt;
    for (int i = 0; i < nchk; ++i)
        if (h[i].health) return bfail(b, LLG_E_DIVERGED, "film %d: non-finite field or torque", i);
    if (out)
        for (int j = 0; j < nload; ++j) out[j] = b->films[j].mbuf[h[j].cur];
    return LLG_OK;
}

__global__ void clear_health_kernel(DevState* st, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) st[i].health = 0;
}

}  // namespace

extern "C" {

llg_status llg_batch_step(llg_batch* b, llg_method method, double dt, int64_t nsteps) {
    TraceRange trace_("llg_batch_step");
    if (!b) return LLG_E_ARG;
    b->err.clear();
    BCHK(b, hipSetDevice(b->device));
    return fixed_core(b, method, dt, nsteps, nullptr, 0, 0, nullptr, nullptr);
}

llg_status llg_batch_autotune(llg_batch* b, int iters, llg_tune_entry* out, int cap, int* n_out) {
    TraceRange trace_("llg_batch_autotune");
    if (!b || iters < 1 || cap < 0 || (cap > 0 && !out)) return LLG_E_ARG;
    b->err.clear();
    BCHK(b, hipSetDevice(b->device));
    const int nf = (int)b->films.size();
    llg_status rc = restore_classes(b);
    if (rc != LLG_OK) return rc;
    std::vector<DevState> h0;
    if ((rc = read_states(b, h0)) != LLG_OK) return rc;
    {
        // finished films skip their launches: time every film
        std::vector<DevState> ht = h0;
        for (DevState& s : ht) s.done = 0;
        if ((rc = write_states(b, ht)) != LLG_OK) return rc;
    }
    // the lengths in use, largest first
    std::vector<int> lens[2];
    for (const BatchFilm& f : b->films) {
        const int l[2] = {f.g.Px, f.g.Py / 2};
        for (int k = 0; k < 2; ++k)
            if (std::find(lens[k].begin(), lens[k].end(), l[k]) == lens[k].end()) lens[k].push_back(l[k]);
    }
    for (auto& v : lens) std::sort(v.begin(), v.end(), std::greater<int>());
    // every film takes the table's variants; every launch argument and
    // block map rebuilt for them
    auto apply = [&]() -> llg_status {
        for (BatchFilm& f : b->films) (void)pick_variants(f.g);
        return build_launch_args(b);
    };
    // a variant serves a length if every film of that length can use it
    auto usable = [&](int kind, int len, int var) {
        for (const BatchFilm& f : b->films) {
            if (kind == 0 && f.g.Px == len && !fast2d_row_ok(len, var)) return false;
            if (kind == 1 && f.g.Py / 2 == len &&
                (!fast2d_col_ok(len, 1, var) || (f.g.Px / 2) % fast2d_col_width(len, var) != 0))
                return false;
        }
        return true;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BCHK(b, hipEventCreate(&e0));
    BCHK(b, hipEventCreate(&e1));
    struct Events {
        hipEvent_t a, b;
        ~Events() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } evs{e0, e1};
    auto time_evals = [&](double& ms) -> llg_status {
        for (int it = 0; it <= iters; ++it) {   // the first evaluation warms up
            if (it == 1) BCHK(b, hipEventRecord(e0, b->stream));
            PASS(b, PASS_ROW_FWD, b->d_fwd_plain);
            PASS(b, PASS_COL, nullptr);
            PASS(b, PASS_ROW_INV, b->d_konly);
        }
        BCHK(b, hipEventRecord(e1, b->stream));
        BCHK(b, hipEventSynchronize(e1));
        float t = 0.f;
        BCHK(b, hipEventElapsedTime(&t, e0, e1));
        ms = t / iters;
        return LLG_OK;
    };
    std::vector<llg_tune_entry> res;
    auto tune = [&]() -> llg_status {
        for (int kind = 0; kind < 2; ++kind) {
            for (int len : lens[kind]) {
                llg_tune_entry t = {};
                t.kind = kind;
                t.length = len;
                t.variant = kind == 0 ? fast2d_row_variant(len) : fast2d_col_variant(len);
                // two rounds in alternating order, the faster of each
                // variant's two timings kept (drift and noise hit both)
                t.ms[0] = t.ms[1] = -1.0;
                for (int round = 0; round < 2; ++round) {
                    for (int v = 0; v < 2; ++v) {
                        if (!usable(kind, len, v)) continue;
                        if (kind == 0) (void)fast2d_set_row_variant(len, v, false);
                        else (void)fast2d_set_col_variant(len, v);
                        double ms = 0.0;
                        if ((rc = apply()) != LLG_OK || (rc = time_evals(ms)) != LLG_OK) return rc;
                        if (t.ms[v] < 0 || ms < t.ms[v]) t.ms[v] = ms;
                    }
                }
                if (t.ms[0] >= 0 || t.ms[1] >= 0)
                    t.variant = (t.ms[1] >= 0 && (t.ms[0] < 0 || t.ms[1] < t.ms[0])) ? 1 : 0;
                if (kind == 0) (void)fast2d_set_row_variant(len, t.variant, false);
                else (void)fast2d_set_col_variant(len, t.variant);
                res.push_back(t);
            }
        }
        return apply();
    };
    rc = tune();
    // the evaluations wrote only scratch (spectra, k1 buffers, the error
    // word): put every film's state back, also after a failure, and
    // recompute k1 and the spectrum before the next step
    const llg_status rw = write_states(b, h0);
    b->k1_valid = false;
    b->spec_valid = false;
    if (rc != LLG_OK) return rc;
    if (rw != LLG_OK) return rw;
    for (int i = 0; i < (int)res.size() && i < cap; ++i) out[i] = res[i];
    if (n_out) *n_out = (int)res.size();
    return LLG_OK;
}

llg_status llg_batch_set_variant(llg_batch* b, int kind, int length, int variant) {
    if (!b) return LLG_E_ARG;
    b->err.clear();
    BCHK(b, hipSetDevice(b->device));
    if (kind != 0 && kind != 1) return bfail(b, LLG_E_ARG, "kind must be 0 (row) or 1 (column)");
    int hits = 0;
    for (const BatchFilm& f : b->films) {
        const bool row = kind == 0;
        if ((row ? f.g.Px : f.g.Py / 2) != length) continue;
        ++hits;
        const bool ok = row ? fast2d_row_ok(length, variant)
                            : fast2d_col_ok(length, 1, variant) && (f.g.Px / 2) % fast2d_col_width(length, variant) == 0;
        if (!ok) return bfail(b, LLG_E_ARG, "variant %d does not serve %s length %d", variant, row ? "row" : "column", length);
    }
    if (!hits) return bfail(b, LLG_E_ARG, "no film uses %s length %d", kind == 0 ? "row" : "column", length);
    for (BatchFilm& f : b->films) {
        if (kind == 0 && f.g.Px == length) f.g.rvar = variant;
        if (kind == 1 && f.g.Py / 2 == length) f.g.cvar = variant;
    }
    llg_status rc = build_launch_args(b);
    if (rc != LLG_OK) return rc;
    // the spectra and first-stage k's were made with the old variants
    b->k1_valid = false;
    b->spec_valid = false;
    b->hcur_ok = false;
    return LLG_OK;
}

llg_status llg_batch_set_m(llg_batch* b, int film, const float* m, llg_mem where) {
    if (!b || !m || film < 0 || film >= (int)b->films.size()) return LLG_E_ARG;
    b->err.clear();
    BCHK(b, hipSetDevice(b->device));
    b->hcur_ok = false;
    std::vector<DevState> h;
    llg_status rc = read_states(b, h);
    if (rc != LLG_OK) return rc;
    BatchFilm& f = b->films[film];
    const size_t vec = sizeof(float) * 3 * (size_t)f.g.ncells;
    float* dst = f.mbuf[h[film].cur];
    BCHK(b, hipMemcpyAsync(dst, m, vec, where == LLG_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           b->stream));
    int* bad = nullptr;
    int hbad = 0;
    BCHK(b, hipMalloc(&bad, sizeof(int)));
    BCHK(b, hipMemsetAsync(bad, 0, sizeof(int), b->stream));
    BCHK(b, launch_normalize_check(dst, f.g.ncells, bad, b->stream));
    BCHK(b, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    bfree(bad);
    b->spec_valid = false;
    b->k1_valid = false;
    DevState& s = h[film];
    s.t = 0.0; s.step = 0; s.nsteps = 0; s.nrej = 0; s.nevals = 0; s.nattempt = 0;
    s.health = 0; s.done = 0; s.err_bits = 0u;
    if ((rc = write_states(b, h)) != LLG_OK) return rc;
    if (hbad) return bfail(b, LLG_E_ARG, "film %d: m is not a field of unit vectors", film);
    return LLG_OK;
}

}  // extern "C"

// ---- shared with the surrogate's speculative verification ------------------

// films 0..nload-1 restart from src + j * stride (device floats, ready once
// `producer` reaches this call) and every film takes nsteps fixed steps;
// out[j] names film j's end state.  The first call (and any call after
// another batch operation or with another method or step) goes through the
// synchronous path, which also checks health; later calls only enqueue work
// (no host synchronisation, health not checked: a caller that needs the
// end states finite checks them).  llg_batch_then_ orders a consumer stream
// after the enqueued steps.
llg_status llg_batch_fixed_async_(llg_batch* b, llg_method method, double dt, int64_t nsteps, const float* src,
                                  size_t stride, int nload, hipStream_t producer, float** out) {
    if (!b || !src || !out || nsteps < 1 || nload < 1 || nload > (int)b->films.size()) return LLG_E_ARG;
    b->err.clear();
    BCHK(b, hipSetDevice(b->device));
    if (!b->hcur_ok || !b->gfix || b->fix_method != (int)method || b->fix_dt != dt) {
        const llg_status rc = fixed_core(b, method, dt, nsteps, src, stride, nload, producer, out);
        if (rc != LLG_OK) return rc;
    } else {
        const llg_status rc = restore_classes(b);
        if (rc != LLG_OK) return rc;
        if (!b->ev_in) BCHK(b, hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
        BCHK(b, hipEventRecord(b->ev_in, producer));
        BCHK(b, hipStreamWaitEvent(b->stream, b->ev_in, 0));
        for (int j = 0; j < nload; ++j) {
            const BatchFilm& f = b->films[j];
            BCHK(b, hipMemcpyAsync(f.mbuf[b->hcur[j]], src + (size_t)j * stride,
                                   sizeof(float) * 3 * (size_t)f.g.ncells, hipMemcpyDeviceToDevice, b->stream));
        }
        hipLaunchKernelGGL(clear_health_kernel, dim3((nload + 63) / 64), dim3(64), 0, b->stream, b->st, nload);
        BCHK(b, hipGetLastError());
        b->spec_valid = false;
        b->k1_valid = false;
        PASS(b, PASS_ROW_FWD, b->d_fwd_plain);
        for (int64_t i = 0; i < nsteps; ++i) BCHK(b, hipGraphLaunch(b->gfix, b->stream));
        b->spec_valid = true;
        if (nsteps & 1)
            for (auto& c : b->hcur) c ^= 1;
        for (int j = 0; j < nload; ++j) out[j] = b->films[j].mbuf[b->hcur[j]];
    }
    if (!b->ev_out) BCHK(b, hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
    BCHK(b, hipEventRecord(b->ev_out, b->stream));
    return LLG_OK;
}

// makes `consumer` wait for the fixed steps last enqueued on the batch
llg_status llg_batch_then_(llg_batch* b, hipStream_t consumer) {
    if (!b) return LLG_E_ARG;
    if (b->ev_out) BCHK(b, hipStreamWaitEvent(consumer, b->ev_out, 0));
    return LLG_OK;
}
