/*
 * llg.h -- C ABI of the MI355X finite-difference Landau-Lifshitz solver.
 *
 * The library evaluates the effective field of a finite-difference
 * micromagnetic model and integrates the Landau-Lifshitz equation
 * (Vansteenkiste & Van de Wiele, "MuMax: a new high-performance
 * micromagnetic simulation tool", Sec. 2, Eq. 1) on one AMD Instinct MI355X
 * (gfx950).  The magnetostatic field is a zero-padded FFT convolution of the
 * magnetisation with the cell-averaged demagnetising tensor (Sec. 2.1.1,
 * Eq. 2; Sec. 3.2), computed by the library's own FFT kernels.
 *
 * Units: every quantity crossing this interface is SI (m, A/m, J/m, J/m^3,
 * tesla for applied fields given as mu0*H, K, s).  Internally the library
 * works in reduced units (field / Ms, time * gamma0 * Ms), as Sec. 3.3
 * recommends; the conversion is hidden.
 *
 * Arrays: a vector field is float32, component-major, x fastest:
 *     v[c][k][j][i]  at  v + c*nx*ny*nz + (k*ny + j)*nx + i,
 * c = 0,1,2 for x,y,z.  Where an argument says llg_mem, LLG_HOST means a
 * host pointer (the call copies synchronously) and LLG_DEVICE a device
 * pointer on the solver's device (the call is ordered on the solver's stream
 * and returns once its work is complete).  The caller owns every buffer it
 * passes; the library never keeps a caller pointer after a call returns.
 *
 * Errors: every call returns an llg_status; LLG_OK is 0.  The text of the
 * last error of a solver is available through llg_last_error.  A solver is
 * not thread-safe; separate solvers are independent.
 */
#ifndef LLG_H
#define LLG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct llg_solver llg_solver;

typedef enum {
    LLG_OK = 0,
    LLG_E_ARG = 1,          /* invalid argument (size, sign, range, null)         */
    LLG_E_STATE = 2,        /* call out of order (e.g. eval before set_m)         */
    LLG_E_NOMEM = 3,        /* device allocation failed                           */
    LLG_E_DEVICE = 4,       /* HIP runtime error                                  */
    LLG_E_UNSUPPORTED = 5,  /* size or option this build does not handle          */
    LLG_E_DIVERGED = 6      /* NaN/Inf in the state or the step fell below dt_min */
} llg_status;

/* Time integrators of Sec. 2.2.  Fixed steps: RK1 Euler, RK2 Heun, RK3
 * Kutta, RK4 classical.  Adaptive embedded pairs: Dormand-Prince 5(4)
 * (RKDP), Bogacki-Shampine 3(2) (RK23), Cash-Karp 5(4) (RKCK), Heun-Euler
 * 2(1) (RK12). */
typedef enum {
    LLG_EULER = 0,
    LLG_HEUN = 1,
    LLG_RK4 = 2,
    LLG_RKDP45 = 3,
    LLG_RK12 = 4,
    LLG_RK3 = 5,
    LLG_RK23 = 6,
    LLG_RKCK = 7
} llg_method;

typedef enum { LLG_HOST = 0, LLG_DEVICE = 1 } llg_mem;

/* Field terms (Sec. 2.1); a bit mask for llg_set_terms. */
enum {
    LLG_TERM_DEMAG = 1,       /* magnetostatic, Sec. 2.1.1 Eq. 2      */
    LLG_TERM_EXCHANGE = 2,    /* exchange, Sec. 2.1.2 Eq. 3           */
    LLG_TERM_ANISOTROPY = 4,  /* uniaxial anisotropy, Sec. 2.1.3 Eq. 4 */
    LLG_TERM_ZEEMAN = 8,      /* applied field, Sec. 2.1.3            */
    LLG_TERM_THERMAL = 16,    /* thermal field, Sec. 2.1.3 Eq. 6      */
    LLG_TERM_STT = 32,        /* Zhang-Li spin-transfer torque, Eq. 7 */
    LLG_TERM_ALL = 63
};

/* Run statistics. */
typedef struct {
    double t;            /* simulated time, s                                  */
    double dt;           /* last attempted step (fixed: the step), s           */
    double dt_next;      /* adaptive: the controller's next step, s            */
    double max_err;      /* adaptive: error estimate of the last attempt       */
    int64_t steps;       /* accepted steps since llg_set_m                     */
    int64_t rejected;    /* rejected attempts since llg_set_m                  */
    int64_t evals;       /* effective-field evaluations since llg_set_m        */
    int32_t health;      /* bit 0: NaN/Inf seen; bit 1: dt below dt_min        */
    int32_t done;        /* adaptive: 1 once t reached t_end                   */
} llg_stats;

/* One attempted adaptive step, as recorded on the device. */
typedef struct {
    double dt;           /* attempted step, s             */
    float err;           /* error estimate (dimensionless) */
    int32_t accepted;    /* 1 accepted, 0 rejected          */
} llg_attempt;

/* ---- lifetime -------------------------------------------------------------
 * llg_create: makes a solver on HIP device `device`.  `hip_stream` is a
 * hipStream_t to order all work on, or NULL for a stream the solver creates
 * and owns.  The solver owns all its device memory; llg_destroy frees it.
 */
llg_status  llg_create(int device, void *hip_stream, llg_solver **out);
void        llg_destroy(llg_solver *s);
/* Text of the last error on this solver; owned by the solver, valid until the
 * next call on it.  Never NULL. */
const char *llg_last_error(const llg_solver *s);

/* ---- problem (Sec. 2: FD grid of cuboid cells; Sec. 2.1.1: periodic
 * boundary conditions) ------------------------------------------------------
 * llg_set_geometry: nx, ny, nz >= 1 cells.  pbc_* != 0 makes that axis
 * periodic (its length must then be a product of 2, 3, 5, 7);
 * `pbc_images` (>= 0) periodic images are added per periodic axis on each
 * side.  Open axes are zero padded to an FFT length >= 2n made of the
 * factors 2, 3, 5, 7 (Sec. 3.3).  Invalidates m and the demag kernel.
 * LLG_E_UNSUPPORTED if a padded length exceeds the library's limits
 * (x: 2048, y and z: 4096; x up to 4096 for one-cell-thick films whose
 * padded y length has a compiled column kernel, e.g. 2048 x 2048).
 */
llg_status llg_set_geometry(llg_solver *s, int nx, int ny, int nz,
                            int pbc_x, int pbc_y, int pbc_z, int pbc_images);
/* Cell edges dx, dy, dz > 0, metres.  Invalidates the demag kernel. */
llg_status llg_set_cellsize(llg_solver *s, double dx, double dy, double dz);
/* Saturation magnetisation Ms > 0 (A/m), exchange stiffness Aex >= 0 (J/m),
 * damping alpha >= 0 (Eq. 1 and Eq. 3). */
llg_status llg_set_material(llg_solver *s, double Ms, double Aex, double alpha);
/* Uniaxial anisotropy Ku (J/m^3; energy density Ku sin^2 theta, Eq. 4) along
 * the axis u[3] (need not be normalised; must be non-zero). */
llg_status llg_set_anisotropy_uniaxial(llg_solver *s, double Ku, const double u[3]);
/* Cubic anisotropy (Eq. 5): energy density K1 (a1^2 a2^2 + a2^2 a3^2 +
 * a1^2 a3^2) + K2 a1^2 a2^2 a3^2 (J/m^3) with a_i = m . c_i, c3 = c1 x c2;
 * c1 and c2 need not be normalised but must be non-zero and orthogonal
 * (|cos| <= 1e-6), else LLG_E_ARG.  Part of LLG_TERM_ANISOTROPY; adds to the
 * uniaxial term.  Default K1 = K2 = 0. */
llg_status llg_set_anisotropy_cubic(llg_solver *s, double K1, double K2, const double c1[3],
                                    const double c2[3]);
/* Uniform current density j[3] (A/m^2), polarisation P and non-adiabaticity
 * xi of the Zhang-Li spin-transfer torque (Eq. 7-8):
 * -b_j/(1+alpha^2) [m x (m x (j.grad) m) + (xi - alpha) m x (j.grad) m],
 * b_j = P mu_B / (e Ms (1 + xi^2)).  (j.grad) m is a central difference;
 * at a free surface the missing neighbour is the cell itself.  It is a torque,
 * not a field: llg_eval_heff does not include it.  Default j = 0. */
llg_status llg_set_current(llg_solver *s, const double j[3], double P, double xi);
/* Uniform applied field B[3] = mu0 H in tesla. */
llg_status llg_set_applied_field(llg_solver *s, const double B[3]);
/* Temperature T >= 0 (K) and the 64-bit seed of the thermal field of Eq. 6.
 * The Gaussian vector eta of a cell at a step comes from Philox4x32-10
 * (Salmon et al., SC'11) with key (seed lo, seed hi) and counter
 * (cell index, step lo, step hi, 0), Box-Muller on 24-bit uniforms; it is
 * drawn once per step and held across the stages of that step.  The thermal
 * field is only applied by fixed-step integration (llg_step). */
llg_status llg_set_temperature(llg_solver *s, double T, uint64_t seed);
/* Mask of LLG_TERM_* bits that H_eff includes (default LLG_TERM_ALL). */
llg_status llg_set_terms(llg_solver *s, int mask);

/* ---- state ------------------------------------------------------------------
 * llg_set_m: unit vectors, layout above.  LLG_E_ARG if some | |m| - 1 | > 1e-3
 * or a value is not finite; otherwise the vectors are renormalised.  Resets
 * time, step counters and statistics.
 */
llg_status llg_set_m(llg_solver *s, const float *m, llg_mem where);
llg_status llg_get_m(llg_solver *s, float *m, llg_mem where);
/* Effective field H_eff (A/m) of the current m, layout above (Sec. 2.1).
 * The thermal term, if enabled, uses the step size of the last llg_step
 * call and the current step counter. */
llg_status llg_eval_heff(llg_solver *s, float *h_out, llg_mem where);
/* llg_eval_heff_noalloc: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same evaluation as llg_eval_heff, same kernels and same
 * result bit for bit, of the field m_dev given by the caller (device memory,
 * layout above; read only, not checked or renormalised) into h_dev (device,
 * A/m, same layout).  The solver's own m, spectrum and run state are left as
 * they are.  The spectrum and a private copy of the device state live in a
 * static device array of 32 MiB per GPU (held until the process ends), so no
 * call allocates or frees anything: films up to 1024 x 1024 cells in 2D;
 * LLG_E_UNSUPPORTED where a geometry's spectra would not fit.  LLG_E_STATE
 * until the demag kernel spectrum exists (its build allocates: call
 * llg_eval_heff, llg_step or llg_run once first).  Every call on one GPU
 * shares that array: calls that overlap on one GPU (several solvers on
 * different streams or threads) race and must be serialised by the caller.
 * Returns after the result is in h_dev. */
llg_status llg_eval_heff_noalloc(llg_solver *s, const float *m_dev, float *h_dev);

/* ---- time integration (Sec. 2.2) --------------------------------------------
 * llg_step: `nsteps` fixed steps of size dt (s) with LLG_EULER, LLG_HEUN,
 * LLG_RK3 or LLG_RK4.  Every stage input and every new state is
 * renormalised.  LLG_E_DIVERGED if a NaN/Inf appears.
 */
llg_status llg_step(llg_solver *s, llg_method method, double dt, int64_t nsteps);
/* llg_run: adaptive integration with an embedded pair (LLG_RKDP45,
 * LLG_RK23, LLG_RKCK or LLG_RK12) from the current time to t_end (s).  An
 * attempt is accepted when err = max over cells |dt sum_j (b_j - bhat_j)
 * k_j| <= max_err; the next step is dt * clamp(0.9 (max_err/err)^(1/(q+1)),
 * 0.2, 5), q the order of the embedded estimate (4, 2, 4, 1); the last step
 * lands on t_end; dt0 is the first attempted step.  The controller runs on
 * the device: attempts are replayed from a captured HIP graph and the host
 * only polls the done flag.  dt0 = 0 continues with the step the controller
 * chose last (the dt_next of llg_get_stats, or of a state restored by
 * llg_set_state; LLG_E_STATE if there is none).  LLG_E_DIVERGED if the step
 * falls below 1e-18 s or a NaN/Inf appears.  `out` may be NULL. */
llg_status llg_run(llg_solver *s, llg_method method, double t_end, double max_err,
                   double dt0, llg_stats *out);
/* As llg_run with LLG_RKDP45 but stops after at most `max_attempts`
 * attempts (for timing a fixed amount of work); t may then be < t_end. */
llg_status llg_run_attempts(llg_solver *s, double t_end, double max_err, double dt0,
                            int64_t max_attempts, llg_stats *out);
/* llg_run_dm: integration to t_end (s) with a fixed tableau (LLG_EULER,
 * LLG_HEUN, LLG_RK3 or LLG_RK4) whose step size bounds the variation of m per
 * step (Sec. 2.2): before each step, dt = max_dm / max over cells |dm/dt|
 * of the step's first stage (so the first-order change of every cell is at
 * most max_dm, dimensionless), at most dt_max (s), and the last step lands
 * on t_end.  The step size is chosen on the device inside a captured HIP
 * graph; each step is recorded in the attempt log (dt, err = the first-order
 * bound dt |dm/dt|max, accepted = 1).  The thermal field is not applied.
 * LLG_E_ARG unless max_dm > 0 and dt_max > 0; LLG_E_DIVERGED if a NaN/Inf
 * appears.  `out` may be NULL. */
llg_status llg_run_dm(llg_solver *s, llg_method method, double t_end, double max_dm, double dt_max,
                      llg_stats *out);
llg_status llg_get_stats(llg_solver *s, llg_stats *out);
/* Copies up to `cap` recorded adaptive attempts (oldest first, since the last
 * llg_set_m) into `out` (host memory) and stores their number in *n. */
llg_status llg_get_attempts(llg_solver *s, llg_attempt *out, int64_t cap, int64_t *n);

/* ---- checkpoint and resume ---------------------------------------------------
 * The integration state besides m: simulated time, the last and the next
 * step of the controller, the thermal draw counter (the Philox step counter
 * of Eq. 6's noise) and the statistics.  llg_get_state copies it into *out
 * and, if m is not NULL, the current m (layout above; host or device per
 * `where`).  llg_set_state restores both into a solver with the same
 * problem: m is taken bit for bit (no renormalisation; LLG_E_ARG if some
 * | |m| - 1 | > 1e-3 or a value is not finite), and the attempt log starts
 * empty.  A run resumed this way (llg_step with the same dt, llg_run_dm, or
 * llg_run with dt0 = 0) takes exactly the steps the uninterrupted run would
 * have taken, with the same results; a pair whose first stage is the last
 * stage of the previous attempt (LLG_RKDP45, LLG_RK23) evaluates that stage
 * once more on resuming, which the evaluation count shows.  LLG_E_ARG for a record with health != 0,
 * a non-finite time or negative steps or counters.
 */
typedef struct {
    double t;            /* simulated time, s                                */
    double dt;           /* last step or attempted step, s                   */
    double dt_next;      /* the controller's next step, s (0: none)          */
    double last_err;     /* error estimate of the last adaptive attempt      */
    int64_t step;        /* accepted steps: the thermal draw counter         */
    int64_t steps;       /* statistics: accepted steps, rejected attempts,   */
    int64_t rejected;    /*   effective-field evaluations                   */
    int64_t evals;
    int32_t health;      /* must be 0 for llg_set_state                      */
    int32_t reserved;
} llg_state;
llg_status llg_get_state(llg_solver *s, llg_state *out, float *m, llg_mem where);
llg_status llg_set_state(llg_solver *s, const llg_state *in, const float *m, llg_mem where);

/* ---- measurement -------------------------------------------------------------
 * llg_profile_evals: runs `n` H_eff evaluations back to back on the solver's
 * stream (forward x pass, spectral pass(es), inverse x pass with the local
 * terms; output kept on the device) and reports the mean duration in
 * milliseconds of each kernel kind in ms_out[0..n_kinds-1] (0: forward x
 * pass, 1: spectral pass incl. multiply (2D) or the z pass (3D), 2: inverse
 * x pass with local terms, 3: y forward pass (3D), 4: y inverse pass (3D)).
 * Where every pass is one compiled kernel (2D, and 3D with compiled y and z
 * lengths) the HIP events are attached to each kernel's launch
 * (hipExtLaunchKernelGGL) and time that kernel's own execution, and
 * *total_ms is the wall time of `n` further evaluations launched plainly;
 * otherwise the events are recorded on the stream between the launches
 * (each interval then also holds the launch of its kernel) and *total_ms
 * spans the timed evaluations.  `n_kinds` must be >= 5.
 */
llg_status llg_profile_evals(llg_solver *s, int n, double *ms_out, int n_kinds, double *total_ms);
/* Algorithmic HBM bytes per evaluation of each kernel kind (same order as
 * llg_profile_evals), from the sizes of what it must read and write. */
llg_status llg_kernel_bytes(llg_solver *s, double *bytes_out, int n_kinds);

/* ---- tuning -------------------------------------------------------------------
 * The 2D path has two compiled variants (elements per lane, hence lanes and
 * wavefronts per transform) for every row length and every column length.
 * A process-wide table holds the default variant of each length (variant 0
 * at start).  llg_set_geometry and llg_batch_create copy the defaults of
 * their lengths (variant 0 where the default cannot serve the geometry);
 * a solver or batch then keeps its variants until its own llg_autotune,
 * llg_set_variants, llg_batch_autotune or llg_batch_set_variant call,
 * whatever later calls do to the table.
 * llg_autotune times `iters` H_eff evaluations of the solver's current state
 * with each of the four (row, column) variant pairs of its lengths, keeps the
 * fastest for this solver and as the table's default, and returns the mean
 * milliseconds per evaluation of pair (r, c) in ms_out[2r + c] (-1 if that
 * pair cannot serve this geometry; ms_out may be NULL, n_out its length) and
 * the chosen pair in choice[0..1] (may be NULL).  Results of different
 * variants differ by FP32 rounding (each is checked against the FP64 oracle
 * to 1e-5).  LLG_E_UNSUPPORTED unless the geometry is 2D with compiled
 * lengths.  llg_set_variants sets the solver's pair, and the table's
 * defaults for its lengths, directly (LLG_E_ARG if the pair cannot serve the
 * geometry). */
llg_status llg_autotune(llg_solver *s, int iters, double *ms_out, int n_out, int *choice);
/* As llg_autotune, but each pair is timed on what llg_run with LLG_RKDP45
 * does (Sec. 2.2's adaptive Dormand-Prince 5(4), whose stage kernels also
 * take the Runge-Kutta combinations and the next forward transform): from
 * the solver's current state, two untimed attempts (graph capture), then
 * `attempts` timed ones with tolerance max_err, the first of step dt0 (s;
 * 0: the controller's next step, LLG_E_STATE if there is none).  Every pair
 * starts from the same state, and afterwards the solver holds that state
 * again (m, time, controller, statistics and attempt log as before the
 * call; the next run evaluates its first stage anew).  ms_out[2r + c]
 * receives milliseconds per attempt (-1 if the pair cannot serve this
 * geometry).  Allocates one device copy of m for the duration of the call.
 * LLG_E_ARG unless attempts >= 1, max_err > 0 and dt0 >= 0; other errors as
 * llg_autotune. */
llg_status llg_autotune_attempts(llg_solver *s, double max_err, double dt0, int attempts, double *ms_out,
                                 int n_out, int *choice);
llg_status llg_set_variants(llg_solver *s, int row_var, int col_var);
/* The solver's (row, column) variant pair.  LLG_E_UNSUPPORTED unless the
 * geometry is 2D with compiled lengths. */
llg_status llg_get_variants(llg_solver *s, int *row_var, int *col_var);
/* Shape of a compiled variant: kind 0 a row length Px, kind 1 a column half
 * length L = Py/2; *elems receives the elements each lane holds in a
 * transform, *classes the number of frequency classes each padded
 * transform is split into (2 or 4; one lane group per class).  LLG_E_ARG if
 * there is no such variant.  Needs no device. */
llg_status llg_variant_shape(int kind, int length, int variant, int *elems, int *classes);

/* ---- diagnostics ------------------------------------------------------------
 * llg_fft_roundtrip: forward then inverse FP32 FFT, by the library's own FFT
 * kernels, of `batch` complex vectors of length n (interleaved re, im float32
 * in host memory, overwritten in place, result divided by n).  n must be a
 * product of 2, 3, 5, 7 not above 4096.  For checking the FFT alone.
 */
llg_status llg_fft_roundtrip(llg_solver *s, float *data, int n, int batch, int inverse_only);
/* llg_demag_tensor: the FP64 real-space kernel entries (the cell-averaged
 * tensor plus periodic images) the library built, for `count` integer cell
 * offsets (di, dj, dk) given in host memory; writes 6*count doubles (xx, yy,
 * zz, xy, xz, yz per offset) to `out` (host).  Offsets must lie within the
 * convolution range (|d| < n along open axes). */
llg_status llg_demag_tensor(llg_solver *s, const int32_t *offsets, int64_t count, double *out);

/* ---- batched films ----------------------------------------------------------
 * Many independent 2D films (nz = 1, open boundaries, no thermal field) of
 * uneven size, e.g. a parameter sweep, integrated together with adaptive
 * Dormand-Prince 5(4).  Every pass of an attempt is one grouped launch over
 * all films; each film keeps its own step size, accept/reject decisions,
 * time and attempt log on the device, and its arithmetic is that of the
 * single-film solver (same kernels, same order), so results do not depend
 * on the batch composition.  Each axis of a film is zero padded to the
 * shortest compiled FFT length >= 2 n (x: 64, 128, 192, 256, 384, 512, 768,
 * 1024, 2048, 4096; y: twice 32, 64, 96, 128, 192, 256, 384, 512, 1024,
 * 2048), which leaves the convolution unchanged (Sec. 3.2 needs only
 * >= 2 n - 1); where that is also the single-film solver's padding (sides
 * 32, 64, 96, 128, 192, 256, 384, 512, 1024, 2048) a batched film equals
 * the single-film run bit for bit.  Sides beyond 2048 give
 * LLG_E_UNSUPPORTED.
 */
typedef struct llg_batch llg_batch;

typedef struct {
    int nx, ny;               /* cells                                   */
    double dx, dy, dz;        /* cell edges, m                           */
    double Ms, Aex, alpha;    /* A/m, J/m, 1                             */
    double Ku;                /* uniaxial anisotropy, J/m^3              */
    double u[3];              /* anisotropy axis (non-zero)              */
    double B[3];              /* applied field mu0 H, tesla              */
    const float *m0;          /* host, [3][ny][nx] unit vectors; copied  */
} llg_film_desc;

/* Builds every film's demag kernel (FP64) and uploads its initial state.
 * LLG_E_ARG for invalid parameters or m0 not of unit vectors. */
llg_status  llg_batch_create(int device, const llg_film_desc *films, int nfilms, llg_batch **out);
void        llg_batch_destroy(llg_batch *b);
const char *llg_batch_last_error(const llg_batch *b);
/* Advances every film toward t_end (s) with tolerance max_err; dt0 is each
 * film's first attempted step of this call (dt0 = 0: each film's controller's
 * last choice, LLG_E_STATE if a film has none).  Stops when all films are done
 * or after max_attempts attempts (<= 0: no limit).  per_film (host, nfilms
 * entries) may be NULL.  LLG_E_DIVERGED if any film diverged. */
llg_status  llg_batch_run(llg_batch *b, double t_end, double max_err, double dt0,
                          int64_t max_attempts, llg_stats *per_film);
/* Fixed steps (LLG_EULER, LLG_HEUN, LLG_RK3 or LLG_RK4, Sec. 2.2) of size dt (s) for
 * every film, one grouped launch per stage; the per-film arithmetic is that
 * of llg_step on a single-film solver.  LLG_E_DIVERGED if a film's state
 * becomes non-finite. */
llg_status  llg_batch_step(llg_batch *b, llg_method method, double dt, int64_t nsteps);
/* Replaces the state of one film (layout of llg_film_desc.m0; host or
 * device memory on the batch's device), checked and renormalised as by
 * llg_set_m; that film's time, counters and attempt log restart at 0. */
llg_status  llg_batch_set_m(llg_batch *b, int film, const float *m, llg_mem where);
/* Current state of one film into host or device memory. */
llg_status  llg_batch_get_m(llg_batch *b, int film, float *m, llg_mem where);
llg_status  llg_batch_get_attempts(llg_batch *b, int film, llg_attempt *out, int64_t cap, int64_t *n);

/* One tuned length of llg_batch_autotune. */
typedef struct {
    int kind;                 /* 0: row (x) length Px, 1: column half length L = Py/2 */
    int length;
    int variant;              /* chosen compiled variant (0 or 1)                     */
    double ms[2];             /* ms per H_eff evaluation of every film with variant   */
                              /* 0 and 1 for this length (-1: not usable)             */
} llg_tune_entry;
/* The batch's own autotuner: for every padded row length and every column
 * length its films use, largest first, times `iters` H_eff evaluations of
 * all films (forward row pass, column pass, inverse row pass, no state
 * change) with each compiled variant of that length, twice in alternating
 * order, the other lengths held, and keeps the faster (by the better of its
 * two timings) for this batch's films and as the table's default (the table
 * llg_autotune fills; solvers and batches set up afterwards copy it).  Every
 * launch argument of the batch is rebuilt for the new variants (the column
 * pass reads the spectrum in the order the row variant writes it); film
 * states, times and controllers are left as they were, and the first stage
 * is evaluated anew on the next step.  Results of different variants differ
 * by FP32 rounding (each checked against the FP64 oracle to 1e-5).
 * out (host, cap entries, may be NULL with cap = 0) receives one entry per
 * length, *n_out their number (may be NULL). */
llg_status  llg_batch_autotune(llg_batch *b, int iters, llg_tune_entry *out, int cap, int *n_out);
/* Sets the compiled variant (0 or 1) of one padded length of this batch:
 * kind 0 the row (x) length Px, kind 1 the column half length L = Py/2, for
 * every film of that length; the table of defaults is not changed.  Launch
 * arguments are rebuilt and the first stage is evaluated anew on the next
 * step.  LLG_E_ARG if no film uses the length or the variant cannot serve
 * one of them. */
llg_status  llg_batch_set_variant(llg_batch *b, int kind, int length, int variant);

/* ---- learned surrogate ------------------------------------------------------
 * Not part of the paper's method: a small convolutional network that
 * proposes the state of a film `seg_steps` fixed RK4 steps (Sec. 2.2) ahead,
 * so that the plain solver can check many proposals at once instead of
 * advancing one segment after another.  Every committed state comes from the
 * plain solver; the network only decides how far a round may jump.
 *
 * Network: six 3x3 convolutions with zero ("same") padding,
 *   9 -> 32, four times 32 -> 32, 32 -> 3, SiLU after all but the last;
 *   input per cell: m as a BF16 pair, hi = bf16(m) and lo = bf16(256 (m - hi))
 *   (3 + 3 channels, so the first layer resolves m to about 16 bits), and
 *   B / 50 mT (3)
 *   per cell, output z; dm = scale * z (llg_sur_set_output_scale, default
 *   1); proposal m' = (base + dm) / |base + dm|, where the
 *   base is m itself (LLG_SUR_BASE_STATE) or one coarse step of the whole
 *   segment length T by the plain solver: Euler (LLG_SUR_BASE_EULER, one
 *   H_eff evaluation) or classical RK4 (LLG_SUR_BASE_RK4, four).  A coarse
 *   step carries the bulk of the motion, including the long-range demag
 *   field the network's 13 x 13-cell receptive field cannot see, and leaves
 *   the network the correction.  Chained Euler steps of T = 1 ps amplify the
 *   stiff exchange modes, so long chains of proposals need the RK4 base.
 * Parameters (FP32, host layout of llg_sur_set_params): per layer the
 * weights [cout][cin][3][3] (cross-correlation: out[o][y][x] = b[o] +
 * sum w[o][c][u][v] in[c][y+u-1][x+v-1]) followed by the bias [cout].
 * Arithmetic: BF16 operands (round to nearest even) on MFMA with FP32
 * accumulation; FP32 master weights, Adam (beta1 0.9, beta2 0.999, eps
 * 1e-8, bias corrected) on the device.  States use the layout of
 * llg_film_desc.m0 ([3][H][W] float); batches of states are contiguous.
 */
typedef struct llg_sur llg_sur;

enum { LLG_SUR_BASE_STATE = 0, LLG_SUR_BASE_EULER = 1, LLG_SUR_BASE_RK4 = 2 };

typedef struct {
    int64_t rounds;          /* verification rounds (one batched plain launch each) */
    int64_t proposals;       /* proposals compared with a plain segment             */
    int64_t accepted;        /* proposals accepted                                  */
    int64_t segments;        /* segments advanced                                   */
    double max_dm_accepted;  /* largest max-cell |m' - m_plain| that was accepted   */
    double max_dm_seen;      /* largest max-cell |m' - m_plain| compared            */
} llg_sur_stats;

/* A network for films of H x W cells and batches of up to max_batch states;
 * parameters must be set before use. */
llg_status  llg_sur_create(int device, int H, int W, int max_batch, llg_sur **out);
void        llg_sur_destroy(llg_sur *s);
const char *llg_sur_last_error(const llg_sur *s);
/* Number of FP32 parameters (40,483). */
int64_t     llg_sur_num_params(void);
/* Host arrays of llg_sur_num_params() floats.  set_params also clears the
 * Adam moments and step count. */
llg_status  llg_sur_set_params(llg_sur *s, const float *params, int64_t n);
llg_status  llg_sur_get_params(llg_sur *s, float *params, int64_t n);
/* Scale > 0 of the network output: dm = scale * z.  A base that already
 * lands close (a coarse RK4 step leaves ~1e-4) needs a small scale so that
 * the BF16 activations resolve the correction.  LLG_E_ARG otherwise. */
llg_status  llg_sur_set_output_scale(llg_sur *s, double scale);
/* Gradient of the last llg_sur_train_step, parameter layout. */
llg_status  llg_sur_get_grads(llg_sur *s, float *grads, int64_t n);
/* Loss L = mean over cells, components and states of (z - (m_target -
 * base) / scale)^2 and its gradient for `batch` triples (m_in, m_target, m_base)
 * with applied fields B[batch][3] (tesla, host); m_base NULL means base =
 * m_in.  Then, if lr > 0, one Adam step with learning rate lr.  The state
 * arrays are in host or device memory per `where`.  *loss (host, may be
 * NULL) receives L. */
llg_status  llg_sur_train_step(llg_sur *s, const float *m_in, const float *m_target, const float *m_base,
                               const float *B, int batch, llg_mem where, float lr, float *loss);
/* Proposals m' = normalize(base + scale z(m_in)) for `batch` states (host or
 * device memory per `where`; m_base NULL means base = m_in). */
llg_status  llg_sur_predict(llg_sur *s, const float *m_in, const float *m_base, const float *B, int batch,
                            llg_mem where, float *m_out);
/* Pre-activation of layer `layer` (0..5) for host inputs, [batch][H][W][32]
 * float into host memory (channels past the layer's width are 0). */
llg_status  llg_sur_forward_raw(llg_sur *s, const float *m_in, const float *B, int batch, int layer,
                                float *z_out);
/* One layer through the training kernels: x and gy [batch][H][W][32] float
 * (host), rounded to BF16 on the device; y = conv(x) + bias and, if gy is not
 * NULL, the weight, bias and input gradients of sum(gy * y) (host). */
llg_status  llg_sur_conv_check(llg_sur *s, int layer, const float *x, const float *gy, int batch,
                               float *y, float *gx, float *gw, float *gb);
/* Advances the state m (host or device per `where`, overwritten) of `film`
 * (its m0 is ignored; its size must be the network's) by n_segments
 * segments of seg_steps RK4 steps of dt (s).  A round chains up to `window`
 * proposals m'_1..m'_w from the current state m'_0, each with the base
 * `predictor` (an LLG_SUR_BASE_* value, coarse steps with T = seg_steps dt;
 * LLG_E_ARG otherwise); batched plain launches of up to four start
 * states each (each as soon as its start states exist, running beside the
 * remaining proposals) advance m'_0..m'_{w-1} by a segment each, giving
 * p_1..p_w; d_j = max over cells |m'_j - p_j|
 * (infinite for a non-finite proposal).  With j* the first j where
 * d_j > max_dm (or w + 1), the round commits p_{min(j*, w)} and advances
 * min(j*, w) segments; LLG_E_DIVERGED if that state is not finite.  With
 * max_dm = 0 every round commits p_1, the plain segment.  `out` may be
 * NULL. */
llg_status  llg_sur_advance(llg_sur *s, const llg_film_desc *film, int window, int64_t n_segments,
                            int seg_steps, double dt, int predictor, double max_dm, float *m, llg_mem where,
                            llg_sur_stats *out);
/* Diagnostic: one 16x32 by 32x16 product (row-major float inputs rounded to
 * BF16, host) by a single MFMA instruction, to check its lane layout. */
llg_status  llg_mfma_selftest(int device, const float *A, const float *B, float *C);

#ifdef __cplusplus
}
#endif

#endif /* LLG_H */
