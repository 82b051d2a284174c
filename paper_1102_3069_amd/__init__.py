"""Python binding of the MI355X finite-difference Landau-Lifshitz library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libllg.so`` (built in-tree by ``build.py``); the names follow
the C ABI of ``include/llg.h``.  Arrays are float32 of shape (3, nz, ny, nx),
x fastest, either numpy arrays (host) or torch CUDA tensors (device).  The
library raises if it is not built; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libllg.so")

LLG_OK, LLG_E_ARG, LLG_E_STATE, LLG_E_NOMEM, LLG_E_DEVICE, LLG_E_UNSUPPORTED, LLG_E_DIVERGED = range(7)
LLG_SUR_BASE_STATE, LLG_SUR_BASE_EULER, LLG_SUR_BASE_RK4 = 0, 1, 2
STATUS_NAMES = ["LLG_OK", "LLG_E_ARG", "LLG_E_STATE", "LLG_E_NOMEM", "LLG_E_DEVICE",
                "LLG_E_UNSUPPORTED", "LLG_E_DIVERGED"]
LLG_EULER, LLG_HEUN, LLG_RK4, LLG_RKDP45, LLG_RK12, LLG_RK3, LLG_RK23, LLG_RKCK = range(8)
METHODS = {"euler": LLG_EULER, "heun": LLG_HEUN, "rk3": LLG_RK3, "rk4": LLG_RK4, "rkdp45": LLG_RKDP45,
           "rk12": LLG_RK12, "rk23": LLG_RK23, "rkck": LLG_RKCK}
LLG_HOST, LLG_DEVICE = 0, 1
TERM_DEMAG, TERM_EXCHANGE, TERM_ANISOTROPY, TERM_ZEEMAN, TERM_THERMAL, TERM_STT = 1, 2, 4, 8, 16, 32
TERM_ALL = 63
TERM_BITS = {"demag": TERM_DEMAG, "exchange": TERM_EXCHANGE, "anisotropy": TERM_ANISOTROPY,
             "zeeman": TERM_ZEEMAN, "thermal": TERM_THERMAL, "stt": TERM_STT}
KERNEL_KINDS = ("row_fwd", "spectral", "row_inv", "y_fwd", "y_inv")


class LLGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES[code] if 0 <= code < 7 else code}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("dt_next", ctypes.c_double),
                ("max_err", ctypes.c_double), ("steps", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("evals", ctypes.c_int64), ("health", ctypes.c_int32), ("done", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Attempt(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("err", ctypes.c_float), ("accepted", ctypes.c_int32)]


class State(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("dt_next", ctypes.c_double),
                ("last_err", ctypes.c_double), ("step", ctypes.c_int64), ("steps", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("evals", ctypes.c_int64), ("health", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class SurStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("proposals", ctypes.c_int64), ("accepted", ctypes.c_int64),
                ("segments", ctypes.c_int64), ("max_dm_accepted", ctypes.c_double),
                ("max_dm_seen", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneEntry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("length", ctypes.c_int), ("variant", ctypes.c_int),
                ("ms", ctypes.c_double * 2)]


class FilmDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("Ms", ctypes.c_double), ("Aex", ctypes.c_double), ("alpha", ctypes.c_double),
                ("Ku", ctypes.c_double), ("u", ctypes.c_double * 3), ("B", ctypes.c_double * 3),
                ("m0", ctypes.c_void_p)]


_lib = None

# exported symbols of include/llg.h with their argument and result types
_P = ctypes.c_void_p
_SIGNATURES = {
    "llg_create": ([ctypes.c_int, _P, ctypes.POINTER(_P)], ctypes.c_int),
    "llg_destroy": ([_P], None),
    "llg_last_error": ([_P], ctypes.c_char_p),
    "llg_set_geometry": ([_P] + [ctypes.c_int] * 7, ctypes.c_int),
    "llg_set_cellsize": ([_P] + [ctypes.c_double] * 3, ctypes.c_int),
    "llg_set_material": ([_P] + [ctypes.c_double] * 3, ctypes.c_int),
    "llg_set_anisotropy_uniaxial": ([_P, ctypes.c_double, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "llg_set_anisotropy_cubic": ([_P, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "llg_set_current": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double], ctypes.c_int),
    "llg_set_applied_field": ([_P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "llg_set_temperature": ([_P, ctypes.c_double, ctypes.c_uint64], ctypes.c_int),
    "llg_set_terms": ([_P, ctypes.c_int], ctypes.c_int),
    "llg_set_m": ([_P, _P, ctypes.c_int], ctypes.c_int),
    "llg_get_m": ([_P, _P, ctypes.c_int], ctypes.c_int),
    "llg_eval_heff": ([_P, _P, ctypes.c_int], ctypes.c_int),
    "llg_eval_heff_noalloc": ([_P, _P, _P], ctypes.c_int),
    "llg_step": ([_P, ctypes.c_int, ctypes.c_double, ctypes.c_int64], ctypes.c_int),
    "llg_run": ([_P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                 ctypes.POINTER(Stats)], ctypes.c_int),
    "llg_run_attempts": ([_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                          ctypes.POINTER(Stats)], ctypes.c_int),
    "llg_run_dm": ([_P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                    ctypes.POINTER(Stats)], ctypes.c_int),
    "llg_get_stats": ([_P, ctypes.POINTER(Stats)], ctypes.c_int),
    "llg_get_state": ([_P, ctypes.POINTER(State), _P, ctypes.c_int], ctypes.c_int),
    "llg_set_state": ([_P, ctypes.POINTER(State), _P, ctypes.c_int], ctypes.c_int),
    "llg_get_attempts": ([_P, ctypes.POINTER(Attempt), ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)],
                         ctypes.c_int),
    "llg_profile_evals": ([_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                           ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "llg_kernel_bytes": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.c_int], ctypes.c_int),
    "llg_autotune": ([_P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                      ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "llg_autotune_attempts": ([_P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
                              ctypes.c_int),
    "llg_set_variants": ([_P, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "llg_get_variants": ([_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "llg_variant_shape": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                           ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "llg_fft_roundtrip": ([_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "llg_demag_tensor": ([_P, _P, ctypes.c_int64, _P], ctypes.c_int),
    "llg_batch_create": ([ctypes.c_int, ctypes.POINTER(FilmDesc), ctypes.c_int, ctypes.POINTER(_P)],
                         ctypes.c_int),
    "llg_batch_destroy": ([_P], None),
    "llg_batch_last_error": ([_P], ctypes.c_char_p),
    "llg_batch_run": ([_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                       ctypes.POINTER(Stats)], ctypes.c_int),
    "llg_batch_step": ([_P, ctypes.c_int, ctypes.c_double, ctypes.c_int64], ctypes.c_int),
    "llg_batch_autotune": ([_P, ctypes.c_int, _P, ctypes.c_int, _P], ctypes.c_int),
    "llg_batch_set_variant": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "llg_batch_set_m": ([_P, ctypes.c_int, _P, ctypes.c_int], ctypes.c_int),
    "llg_batch_get_m": ([_P, ctypes.c_int, _P, ctypes.c_int], ctypes.c_int),
    "llg_batch_get_attempts": ([_P, ctypes.c_int, ctypes.POINTER(Attempt), ctypes.c_int64,
                                ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "llg_sur_create": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_P)],
                       ctypes.c_int),
    "llg_sur_destroy": ([_P], None),
    "llg_sur_last_error": ([_P], ctypes.c_char_p),
    "llg_sur_num_params": ([], ctypes.c_int64),
    "llg_sur_set_params": ([_P, _P, ctypes.c_int64], ctypes.c_int),
    "llg_sur_get_params": ([_P, _P, ctypes.c_int64], ctypes.c_int),
    "llg_sur_set_output_scale": ([_P, ctypes.c_double], ctypes.c_int),
    "llg_sur_get_grads": ([_P, _P, ctypes.c_int64], ctypes.c_int),
    "llg_sur_train_step": ([_P, _P, _P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                            ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "llg_sur_predict": ([_P, _P, _P, _P, ctypes.c_int, ctypes.c_int, _P], ctypes.c_int),
    "llg_sur_forward_raw": ([_P, _P, _P, ctypes.c_int, ctypes.c_int, _P], ctypes.c_int),
    "llg_sur_conv_check": ([_P, ctypes.c_int, _P, _P, ctypes.c_int, _P, _P, _P, _P], ctypes.c_int),
    "llg_sur_advance": ([_P, ctypes.POINTER(FilmDesc), ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                         ctypes.c_double, ctypes.c_int, ctypes.c_double, _P, ctypes.c_int,
                         ctypes.POINTER(SurStats)], ctypes.c_int),
    "llg_mfma_selftest": ([ctypes.c_int, _P, _P, _P], ctypes.c_int),
}
EXPORTS = tuple(_SIGNATURES)


def load(path=LIB_PATH):
    """Loads libllg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1102_3069_amd/build.py "
                           "(or __graft_entry__.build()); there is no fallback path")
    # PyTorch ships its own HIP runtime; when both are used in one process,
    # PyTorch's must be loaded first or it cannot find the GPU later
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _arr3(v):
    return (ctypes.c_double * 3)(*[float(x) for x in v])


def _is_torch(x):
    return type(x).__module__.startswith("torch")


class Solver:
    """One solver on one HIP device (see include/llg.h for every call)."""

    def __init__(self, device=0, stream=None):
        self._lib = load()
        h = _P()
        rc = self._lib.llg_create(int(device), _P(stream) if stream else None, ctypes.byref(h))
        if rc != LLG_OK:
            raise LLGError(rc, "llg_create failed")
        self._h = h
        self.n = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.llg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != LLG_OK:
            raise LLGError(rc, self._lib.llg_last_error(self._h).decode())

    # ---- problem ----------------------------------------------------------
    def set_geometry(self, n, pbc=(False, False, False), images=10):
        nx, ny, nz = (int(v) for v in n)
        self._chk(self._lib.llg_set_geometry(self._h, nx, ny, nz, int(bool(pbc[0])), int(bool(pbc[1])),
                                             int(bool(pbc[2])), int(images)))
        self.n = (nx, ny, nz)

    def set_cellsize(self, cell):
        self._chk(self._lib.llg_set_cellsize(self._h, *[float(c) for c in cell]))

    def set_material(self, Ms, Aex, alpha):
        self._chk(self._lib.llg_set_material(self._h, float(Ms), float(Aex), float(alpha)))

    def set_anisotropy_uniaxial(self, Ku, u):
        self._chk(self._lib.llg_set_anisotropy_uniaxial(self._h, float(Ku), _arr3(u)))

    def set_anisotropy_cubic(self, K1, K2, c1=(1.0, 0.0, 0.0), c2=(0.0, 1.0, 0.0)):
        self._chk(self._lib.llg_set_anisotropy_cubic(self._h, float(K1), float(K2), _arr3(c1), _arr3(c2)))

    def set_current(self, j, P, xi):
        self._chk(self._lib.llg_set_current(self._h, _arr3(j), float(P), float(xi)))

    def set_applied_field(self, B):
        self._chk(self._lib.llg_set_applied_field(self._h, _arr3(B)))

    def set_temperature(self, T, seed):
        self._chk(self._lib.llg_set_temperature(self._h, float(T), int(seed) & 0xFFFFFFFFFFFFFFFF))

    def set_terms(self, terms):
        mask = terms if isinstance(terms, int) else sum(TERM_BITS[t] for t in terms)
        self._chk(self._lib.llg_set_terms(self._h, int(mask)))

    def set_problem(self, prob):
        """Applies a problem dict (keys as in workloads.py)."""
        self.set_geometry(prob["n"], prob.get("pbc", (False,) * 3), prob.get("images", 10))
        self.set_cellsize(prob["cell"])
        self.set_material(prob["Ms"], prob["Aex"], prob["alpha"])
        self.set_anisotropy_uniaxial(prob.get("Ku", 0.0), prob.get("u", (1.0, 0.0, 0.0)))
        self.set_anisotropy_cubic(prob.get("Kc1", 0.0), prob.get("Kc2", 0.0), prob.get("c1", (1.0, 0.0, 0.0)),
                                  prob.get("c2", (0.0, 1.0, 0.0)))
        self.set_applied_field(prob.get("B", (0.0, 0.0, 0.0)))
        self.set_current(prob.get("j", (0.0, 0.0, 0.0)), prob.get("P", 0.0), prob.get("xi", 0.0))
        self.set_temperature(prob.get("T", 0.0), prob.get("seed", 0))
        terms = prob.get("terms")
        # the oracle's term names are field terms; the torque follows the current
        self.set_terms(TERM_ALL if terms is None else sum(TERM_BITS[t] for t in terms) | TERM_STT)

    # ---- state --------------------------------------------------------------
    def _shape(self):
        if self.n is None:
            raise LLGError(LLG_E_STATE, "geometry not set")
        nx, ny, nz = self.n
        return (3, nz, ny, nx)

    def set_m(self, m):
        if _is_torch(m) and m.is_cuda:
            assert m.dtype.__str__() == "torch.float32" and m.is_contiguous()
            self._chk(self._lib.llg_set_m(self._h, _P(m.data_ptr()), LLG_DEVICE))
        else:
            a = np.ascontiguousarray(m, dtype=np.float32).reshape(self._shape())
            self._chk(self._lib.llg_set_m(self._h, a.ctypes.data_as(_P), LLG_HOST))

    def get_m(self, out=None):
        if out is not None and _is_torch(out) and out.is_cuda:
            self._chk(self._lib.llg_get_m(self._h, _P(out.data_ptr()), LLG_DEVICE))
            return out
        a = np.empty(self._shape(), dtype=np.float32)
        self._chk(self._lib.llg_get_m(self._h, a.ctypes.data_as(_P), LLG_HOST))
        return a

    def eval_heff(self, out=None):
        if out is not None and _is_torch(out) and out.is_cuda:
            self._chk(self._lib.llg_eval_heff(self._h, _P(out.data_ptr()), LLG_DEVICE))
            return out
        a = np.empty(self._shape(), dtype=np.float32)
        self._chk(self._lib.llg_eval_heff(self._h, a.ctypes.data_as(_P), LLG_HOST))
        return a

    def eval_heff_noalloc(self, m, out):
        """llg_eval_heff_noalloc: H_eff of the device field `m` into the
        device tensor `out` (both torch CUDA float32 tensors of the solver's
        shape); nothing is allocated by the library."""
        for t in (m, out):
            if not (_is_torch(t) and t.is_cuda and t.dtype.is_floating_point and t.element_size() == 4
                    and t.is_contiguous() and tuple(t.shape) == self._shape()):
                raise ValueError("m and out must be contiguous float32 CUDA tensors of the solver's shape")
        self._chk(self._lib.llg_eval_heff_noalloc(self._h, _P(m.data_ptr()), _P(out.data_ptr())))
        return out

    # ---- integration ---------------------------------------------------------
    def step(self, method, dt, nsteps=1):
        self._chk(self._lib.llg_step(self._h, METHODS[method], float(dt), int(nsteps)))

    def run(self, t_end, max_err=1e-5, dt0=1e-14, method="rkdp45"):
        st = Stats()
        self._chk(self._lib.llg_run(self._h, METHODS[method], float(t_end), float(max_err), float(dt0),
                                    ctypes.byref(st)))
        return st.as_dict()

    def run_attempts(self, t_end, max_err, dt0, max_attempts):
        st = Stats()
        self._chk(self._lib.llg_run_attempts(self._h, float(t_end), float(max_err), float(dt0),
                                             int(max_attempts), ctypes.byref(st)))
        return st.as_dict()

    def run_dm(self, method, t_end, max_dm, dt_max):
        """Fixed tableau, step chosen so that max |dm| per step is about max_dm."""
        st = Stats()
        self._chk(self._lib.llg_run_dm(self._h, METHODS[method], float(t_end), float(max_dm), float(dt_max),
                                       ctypes.byref(st)))
        return st.as_dict()

    def get_state(self):
        """(state dict, m) for llg_set_state."""
        st = State()
        a = np.empty(self._shape(), dtype=np.float32)
        self._chk(self._lib.llg_get_state(self._h, ctypes.byref(st), a.ctypes.data_as(_P), LLG_HOST))
        return st.as_dict(), a

    def set_state(self, state, m):
        st = State(**{k: state[k] for k in state})
        a = np.ascontiguousarray(m, dtype=np.float32).reshape(self._shape())
        self._chk(self._lib.llg_set_state(self._h, ctypes.byref(st), a.ctypes.data_as(_P), LLG_HOST))

    def stats(self):
        st = Stats()
        self._chk(self._lib.llg_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def attempts(self, cap=1 << 20):
        buf = (Attempt * cap)()
        n = ctypes.c_int64()
        self._chk(self._lib.llg_get_attempts(self._h, buf, cap, ctypes.byref(n)))
        return [(buf[i].dt, float(buf[i].err), bool(buf[i].accepted)) for i in range(n.value)]

    # ---- measurement and diagnostics -----------------------------------------
    def profile_evals(self, n):
        ms = (ctypes.c_double * 5)()
        tot = ctypes.c_double()
        self._chk(self._lib.llg_profile_evals(self._h, int(n), ms, 5, ctypes.byref(tot)))
        return dict(zip(KERNEL_KINDS, list(ms))), tot.value

    def kernel_bytes(self):
        b = (ctypes.c_double * 5)()
        self._chk(self._lib.llg_kernel_bytes(self._h, b, 5))
        return dict(zip(KERNEL_KINDS, list(b)))

    def autotune(self, iters=20):
        """Times the compiled (row, column) variants on H_eff evaluations of
        the current state; returns ({(r, c): ms per eval}, (r, c) chosen)."""
        ms = (ctypes.c_double * 4)()
        ch = (ctypes.c_int * 2)()
        self._chk(self._lib.llg_autotune(self._h, int(iters), ms, 4, ch))
        return {(r, c): ms[2 * r + c] for r in range(2) for c in range(2)}, (ch[0], ch[1])

    def autotune_attempts(self, max_err, dt0, attempts=50):
        """Times the compiled (row, column) variant pairs on adaptive
        Dormand-Prince attempts from the current state (which is kept);
        returns ({(r, c): ms per attempt}, (r, c) chosen)."""
        ms = (ctypes.c_double * 4)()
        ch = (ctypes.c_int * 2)()
        self._chk(self._lib.llg_autotune_attempts(self._h, float(max_err), float(dt0), int(attempts), ms, 4, ch))
        return {(r, c): ms[2 * r + c] for r in range(2) for c in range(2)}, (ch[0], ch[1])

    def set_variants(self, row_var, col_var):
        self._chk(self._lib.llg_set_variants(self._h, int(row_var), int(col_var)))

    def get_variants(self):
        r, c = ctypes.c_int(), ctypes.c_int()
        self._chk(self._lib.llg_get_variants(self._h, ctypes.byref(r), ctypes.byref(c)))
        return r.value, c.value

    def fft_roundtrip(self, data, inverse_only=False):
        """data: complex64 array (batch, n); returns the library's
        forward+inverse (or inverse only) transform divided by n."""
        a = np.ascontiguousarray(data, dtype=np.complex64)
        batch, n = a.shape
        self._chk(self._lib.llg_fft_roundtrip(self._h, a.ctypes.data_as(_P), int(n), int(batch),
                                              int(bool(inverse_only))))
        return a

    def demag_tensor(self, offsets):
        o = np.ascontiguousarray(offsets, dtype=np.int32).reshape(-1, 3)
        out = np.empty((o.shape[0], 6), dtype=np.float64)
        self._chk(self._lib.llg_demag_tensor(self._h, o.ctypes.data_as(_P), o.shape[0],
                                             out.ctypes.data_as(_P)))
        return out


def film_desc(prob, m0, d=None):
    """Fills an llg_film_desc from a problem dict; returns the float32
    (3, 1, ny, nx) copy of m0 that d.m0 points to (keep it alive)."""
    d = FilmDesc() if d is None else d
    nx, ny, nz = prob["n"]
    if nz != 1:
        raise LLGError(LLG_E_ARG, "batched films are one cell thick")
    a = np.ascontiguousarray(m0, dtype=np.float32).reshape(3, 1, ny, nx)
    d.nx, d.ny = nx, ny
    d.dx, d.dy, d.dz = (float(c) for c in prob["cell"])
    d.Ms, d.Aex, d.alpha = float(prob["Ms"]), float(prob["Aex"]), float(prob["alpha"])
    d.Ku = float(prob.get("Ku", 0.0))
    d.u = (ctypes.c_double * 3)(*[float(v) for v in prob.get("u", (1.0, 0.0, 0.0))])
    d.B = (ctypes.c_double * 3)(*[float(v) for v in prob.get("B", (0.0, 0.0, 0.0))])
    d.m0 = a.ctypes.data
    return a


class Batch:
    """Independent 2D films integrated together (see llg_batch_* in llg.h).
    films: list of (problem dict, m0 float32 array) as made by workloads.py."""

    def __init__(self, films, device=0):
        self._lib = load()
        self.shapes = []
        self._keep = []
        descs = (FilmDesc * len(films))()
        for d, (prob, m0) in zip(descs, films):
            a = film_desc(prob, m0, d)
            self._keep.append(a)
            self.shapes.append(a.shape)
        h = _P()
        rc = self._lib.llg_batch_create(int(device), descs, len(films), ctypes.byref(h))
        if rc != LLG_OK:
            msg = self._lib.llg_batch_last_error(h).decode() if h else "llg_batch_create failed"
            if h:
                self._lib.llg_batch_destroy(h)
            raise LLGError(rc, msg)
        self._h = h
        self.n = len(films)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.llg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != LLG_OK:
            raise LLGError(rc, self._lib.llg_batch_last_error(self._h).decode())

    def run(self, t_end, max_err=1e-5, dt0=1e-14, max_attempts=0):
        st = (Stats * self.n)()
        self._chk(self._lib.llg_batch_run(self._h, float(t_end), float(max_err), float(dt0),
                                          int(max_attempts), st))
        return [s.as_dict() for s in st]

    def step(self, method, dt, nsteps=1):
        self._chk(self._lib.llg_batch_step(self._h, METHODS[method], float(dt), int(nsteps)))

    def autotune(self, iters=10):
        """Tunes the compiled variant of every length the films use (the
        process-wide table); returns [{"kind": "row"|"col", "length",
        "variant", "ms": (variant 0, variant 1)}]."""
        cap = 64
        ent = (TuneEntry * cap)()
        n = ctypes.c_int(0)
        self._chk(self._lib.llg_batch_autotune(self._h, int(iters), ctypes.cast(ent, _P), cap, ctypes.byref(n)))
        return [{"kind": ("row", "col")[e.kind], "length": e.length, "variant": e.variant,
                 "ms": (e.ms[0], e.ms[1])} for e in ent[:min(n.value, cap)]]

    def set_variant(self, kind, length, variant):
        """Compiled variant of one padded length of this batch's films
        (kind "row": Px, "col": Py / 2)."""
        self._chk(self._lib.llg_batch_set_variant(self._h, {"row": 0, "col": 1}[kind], int(length), int(variant)))

    def set_m(self, film, m):
        if _is_torch(m) and m.is_cuda:
            assert str(m.dtype) == "torch.float32" and m.is_contiguous()
            self._chk(self._lib.llg_batch_set_m(self._h, int(film), _P(m.data_ptr()), LLG_DEVICE))
        else:
            a = np.ascontiguousarray(m, dtype=np.float32).reshape(self.shapes[film])
            self._chk(self._lib.llg_batch_set_m(self._h, int(film), a.ctypes.data_as(_P), LLG_HOST))

    def get_m(self, film, out=None):
        if out is not None and _is_torch(out) and out.is_cuda:
            self._chk(self._lib.llg_batch_get_m(self._h, int(film), _P(out.data_ptr()), LLG_DEVICE))
            return out
        a = np.empty(self.shapes[film], dtype=np.float32)
        self._chk(self._lib.llg_batch_get_m(self._h, int(film), a.ctypes.data_as(_P), LLG_HOST))
        return a

    def attempts(self, film, cap=1 << 16):
        buf = (Attempt * cap)()
        n = ctypes.c_int64()
        self._chk(self._lib.llg_batch_get_attempts(self._h, int(film), buf, cap, ctypes.byref(n)))
        return [(buf[i].dt, float(buf[i].err), bool(buf[i].accepted)) for i in range(n.value)]


def _ptr_mem(x):
    """(pointer, llg_mem) of a float32 array: torch CUDA tensor or numpy."""
    if _is_torch(x) and x.is_cuda:
        assert str(x.dtype) == "torch.float32" and x.is_contiguous()
        return _P(x.data_ptr()), LLG_DEVICE
    assert x.dtype == np.float32 and x.flags["C_CONTIGUOUS"]
    return x.ctypes.data_as(_P), LLG_HOST


class Surrogate:
    """The learned multi-step proposer (see llg_sur_* in llg.h).  Parameters
    travel as a flat float32 vector in the layout of llg_sur_set_params; the
    helpers pack()/unpack() convert from/to a list of (w, b) per layer."""

    LAYERS = ((9, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 3))

    def __init__(self, H, W, max_batch=1, device=0):
        self._lib = load()
        h = _P()
        rc = self._lib.llg_sur_create(int(device), int(H), int(W), int(max_batch), ctypes.byref(h))
        if rc != LLG_OK:
            msg = self._lib.llg_sur_last_error(h).decode() if h else "llg_sur_create failed"
            if h:
                self._lib.llg_sur_destroy(h)
            raise LLGError(rc, msg)
        self._h = h
        self.H, self.W, self.max_batch = int(H), int(W), int(max_batch)
        self.nparam = int(self._lib.llg_sur_num_params())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.llg_sur_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc != LLG_OK:
            raise LLGError(rc, self._lib.llg_sur_last_error(self._h).decode())

    @classmethod
    def pack(cls, params):
        return np.concatenate([np.concatenate([np.asarray(w, np.float32).reshape(-1),
                                               np.asarray(b, np.float32).reshape(-1)]) for w, b in params])

    @classmethod
    def unpack(cls, flat):
        out, o = [], 0
        for ci, co in cls.LAYERS:
            w = flat[o:o + co * ci * 9].reshape(co, ci, 3, 3)
            o += co * ci * 9
            b = flat[o:o + co]
            o += co
            out.append((w, b))
        return out

    def set_params(self, params):
        flat = np.ascontiguousarray(params if isinstance(params, np.ndarray) else self.pack(params),
                                    dtype=np.float32)
        self._chk(self._lib.llg_sur_set_params(self._h, flat.ctypes.data_as(_P), flat.size))

    def get_params(self):
        a = np.empty(self.nparam, np.float32)
        self._chk(self._lib.llg_sur_get_params(self._h, a.ctypes.data_as(_P), a.size))
        return a

    def get_grads(self):
        a = np.empty(self.nparam, np.float32)
        self._chk(self._lib.llg_sur_get_grads(self._h, a.ctypes.data_as(_P), a.size))
        return a

    def set_output_scale(self, scale):
        """dm = scale * network output."""
        self._chk(self._lib.llg_sur_set_output_scale(self._h, float(scale)))

    def train_step(self, m_in, m_target, B, lr=0.0, m_base=None):
        """m_in, m_target, m_base: (batch, 3, H, W) float32 (numpy or CUDA
        tensor; m_base None: the loss target is m_target - m_in);
        B: (batch, 3) tesla.  Returns the loss."""
        Bh = np.ascontiguousarray(B, dtype=np.float32).reshape(-1, 3)
        pi, where = _ptr_mem(m_in)
        pt, where2 = _ptr_mem(m_target)
        assert where == where2
        pb = None
        if m_base is not None:
            pb, where3 = _ptr_mem(m_base)
            assert where3 == where
        loss = ctypes.c_float()
        self._chk(self._lib.llg_sur_train_step(self._h, pi, pt, pb, Bh.ctypes.data_as(_P), Bh.shape[0], where,
                                               float(lr), ctypes.byref(loss)))
        return loss.value

    def predict(self, m_in, B, out=None, m_base=None):
        """normalize(base + dm(m_in)), base = m_base or m_in."""
        Bh = np.ascontiguousarray(B, dtype=np.float32).reshape(-1, 3)
        pi, where = _ptr_mem(m_in)
        pb = None
        if m_base is not None:
            pb, where3 = _ptr_mem(m_base)
            assert where3 == where
        if out is None:
            assert where == LLG_HOST
            out = np.empty((Bh.shape[0], 3, self.H, self.W), np.float32)
        po, _ = _ptr_mem(out)
        self._chk(self._lib.llg_sur_predict(self._h, pi, pb, Bh.ctypes.data_as(_P), Bh.shape[0], where, po))
        return out

    def forward_raw(self, m_in, B, layer):
        m = np.ascontiguousarray(m_in, dtype=np.float32)
        Bh = np.ascontiguousarray(B, dtype=np.float32).reshape(-1, 3)
        z = np.empty((Bh.shape[0], self.H, self.W, 32), np.float32)
        self._chk(self._lib.llg_sur_forward_raw(self._h, m.ctypes.data_as(_P), Bh.ctypes.data_as(_P),
                                                Bh.shape[0], int(layer), z.ctypes.data_as(_P)))
        return z

    def conv_check(self, layer, x, gy=None):
        """x, gy: (batch, H, W, 32) float32.  Returns y or (y, gx, gw, gb)."""
        ci, co = self.LAYERS[layer]
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.empty_like(x)
        if gy is None:
            self._chk(self._lib.llg_sur_conv_check(self._h, int(layer), x.ctypes.data_as(_P), None,
                                                   x.shape[0], y.ctypes.data_as(_P), None, None, None))
            return y
        gy = np.ascontiguousarray(gy, dtype=np.float32)
        gx = np.empty_like(x)
        gw = np.empty((co, ci, 3, 3), np.float32)
        gb = np.empty(co, np.float32)
        self._chk(self._lib.llg_sur_conv_check(self._h, int(layer), x.ctypes.data_as(_P),
                                               gy.ctypes.data_as(_P), x.shape[0], y.ctypes.data_as(_P),
                                               gx.ctypes.data_as(_P), gw.ctypes.data_as(_P),
                                               gb.ctypes.data_as(_P)))
        return y, gx, gw, gb

    def advance(self, prob, m, n_segments, window=16, seg_steps=10, dt=1e-13, max_dm=1e-2, predictor="rk4"):
        """Advances m (float32 (3, 1, H, W) numpy array or CUDA tensor, in
        place for a tensor) by n_segments segments; returns (m, stats).
        predictor: the proposal base, "rk4" or "euler" (one plain step of
        that scheme over the whole segment) or "state" (the state itself)."""
        pred = {"state": LLG_SUR_BASE_STATE, "euler": LLG_SUR_BASE_EULER, "rk4": LLG_SUR_BASE_RK4}[predictor]
        d = FilmDesc()
        keep = film_desc(prob, np.zeros((3, 1, self.H, self.W), np.float32), d)
        d.m0 = None
        if _is_torch(m) and m.is_cuda:
            pm, where = _ptr_mem(m)
            out = m
        else:
            out = np.ascontiguousarray(m, dtype=np.float32).copy()
            pm, where = _ptr_mem(out)
        st = SurStats()
        self._chk(self._lib.llg_sur_advance(self._h, ctypes.byref(d), int(window), int(n_segments),
                                            int(seg_steps), float(dt), pred, float(max_dm), pm, where,
                                            ctypes.byref(st)))
        del keep
        return out, st.as_dict()


def variant_shape(kind, length, variant):
    """(elements per lane, frequency classes) of a compiled variant; kind
    "row" (length Px) or "col" (length Py / 2)."""
    lib = load()
    e, q = ctypes.c_int(), ctypes.c_int()
    rc = lib.llg_variant_shape({"row": 0, "col": 1}[kind], int(length), int(variant), ctypes.byref(e),
                               ctypes.byref(q))
    if rc != LLG_OK:
        raise LLGError(rc, f"no compiled {kind} variant {variant} of length {length}")
    return e.value, q.value


def mfma_selftest(A, B, device=0):
    """One 16x32 by 32x16 product on a single MFMA instruction (BF16 inputs)."""
    lib = load()
    a = np.ascontiguousarray(A, dtype=np.float32)
    b = np.ascontiguousarray(B, dtype=np.float32)
    assert a.shape == (16, 32) and b.shape == (32, 16)
    c = np.empty((16, 16), np.float32)
    rc = lib.llg_mfma_selftest(int(device), a.ctypes.data_as(_P), b.ctypes.data_as(_P), c.ctypes.data_as(_P))
    if rc != LLG_OK:
        raise LLGError(rc, "llg_mfma_selftest failed")
    return c
