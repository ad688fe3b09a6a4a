"""ctypes binding of libchx (include/chx.h).

Argument marshalling only: every step of the integration runs in the HIP
kernels of libchx.so.  Arrays may be numpy arrays (host memory; the call is
synchronous) or torch tensors on the GPU (device memory; the work is ordered
on torch's current stream).  There is no fallback: if libchx.so is missing
or cannot be loaded the import-time loader raises.
"""
import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchx.so")

# --- constants mirrored from include/chx.h -----------------------------------
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_INTERNAL = range(6)
(SYS_HENON_HEILES, SYS_FPUT, SYS_QUARTIC, SYS_HARMONIC, SYS_DOUBLE_PENDULUM, SYS_CUSTOM,
 SYS_CUSTOM_GENERAL) = (1, 2, 3, 4, 5, 6, 7)
IND_SALI, IND_GALI, IND_LYAP, IND_LD, IND_ENERGY = 1, 2, 4, 8, 16
PTR_DEVICE = 1
INT_YOSHIDA4, INT_DOP853, INT_DOP853_ADAPTIVE = 0, 1, 2
_INTEGRATORS = {"yoshida4": INT_YOSHIDA4, "dop853": INT_DOP853,
                "dop853_adaptive": INT_DOP853_ADAPTIVE}
(ORBIT_OK, ORBIT_MASKED, ORBIT_ESCAPED, ORBIT_NONFINITE, ORBIT_EXITED,
 ORBIT_STEP_FAILED) = range(6)

# Every function include/chx.h declares.
EXPORTS = [
    "chx_options_default", "chx_integrate_ensemble", "chx_sali", "chx_gali",
    "chx_lyap_spectrum", "chx_ld", "chx_ensemble_create", "chx_ensemble_advance",
    "chx_ensemble_results", "chx_ensemble_info", "chx_ensemble_destroy",
    "chx_grid_hh_section", "chx_hh_section_points", "chx_ic_fput_modes", "chx_ic_quartic",
    "chx_last_error", "chx_version", "chx_struct_size", "chx_integrate_batched",
    "chx_ensemble_subset", "chx_gate_create", "chx_gate_destroy", "chx_gate_train",
    "chx_gate_grad", "chx_gate_infer", "chx_gate_get", "chx_gate_set", "chx_gate_features",
    "chx_gate_classify", "chx_ld_indicators", "chx_integrate_ensemble_noalloc", "chx_shutdown",
]
GATE_NFEAT, GATE_NPARAM = 6, 74256


class ChxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libchx status {status}: {msg}")
        self.status = status


class _System(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ndof", C.c_int32),
                ("params", C.POINTER(C.c_double)), ("nparams", C.c_int32),
                ("source", C.c_char_p)]


class _Options(C.Structure):
    _fields_ = [("dt", C.c_double), ("T", C.c_double), ("indicators", C.c_uint32),
                ("renorm_every", C.c_int32), ("n_lyap", C.c_int32), ("gali_kmax", C.c_int32),
                ("ld_p", C.c_double), ("sali_threshold", C.c_double),
                ("early_exit", C.c_int32), ("steps_per_launch", C.c_int32),
                ("seed", C.c_uint64), ("w0", C.c_void_p), ("escape_r2", C.c_double),
                ("flags", C.c_uint32), ("block_size", C.c_int32), ("stream", C.c_void_p),
                ("integrator", C.c_int32), ("rtol", C.c_double), ("atol", C.c_double)]


RESULT_FIELDS = ["x_final", "t_end", "status", "label", "sali_final", "sali_min", "t_chaos",
                 "gali", "lyap", "ld", "energy_err", "ln_growth", "steps", "step_err"]


class _Result(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in RESULT_FIELDS]


class _BatchItem(C.Structure):
    _fields_ = [("sys", _System), ("x0", C.c_void_p), ("mask", C.c_void_p),
                ("n", C.c_int64), ("dt", C.c_double), ("T", C.c_double)]


class _BatchStats(C.Structure):
    _fields_ = [("threads_per_block", C.c_int32), ("blocks", C.c_int32),
                ("launches", C.c_int32), ("from_cache", C.c_int32),
                ("steps_per_launch", C.c_int64), ("integrate_ms", C.c_double),
                ("orbit_steps", C.c_int64 * 4), ("cost_ps", C.c_double * 4)]


class _GateTrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("weight_decay", C.c_float), ("seed", C.c_uint64)]


class _GateStats(C.Structure):
    _fields_ = [("n_active", C.c_int64), ("n_early", C.c_int64), ("n_accepted", C.c_int64),
                ("n_fallback", C.c_int64), ("ms_gate", C.c_double), ("ms_infer", C.c_double),
                ("ms_fallback", C.c_double)]


_lib = None


def lib():
    """The loaded libchx.so; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "python -c 'import __graft_entry__ as g; g.build()'")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, u32, u64, d = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint32,
                                    C.c_uint64, C.c_double)
        S, O, R = C.POINTER(_System), C.POINTER(_Options), C.POINTER(_Result)
        L.chx_options_default.argtypes = [O]
        L.chx_options_default.restype = None
        L.chx_integrate_ensemble.argtypes = [S, P, P, i64, O, R]
        L.chx_integrate_ensemble_noalloc.argtypes = [S, P, P, i64, O, R]
        L.chx_ld_indicators.argtypes = [S, P, P, i64, O, C.POINTER(_LdnOptions),
                                        C.POINTER(_LdnResult)]
        L.chx_sali.argtypes = [S, P, i64, d, d, u64, P, P]
        L.chx_gali.argtypes = [S, P, i64, d, d, i32, u64, P]
        L.chx_lyap_spectrum.argtypes = [S, P, i64, d, d, i32, i32, P]
        L.chx_ld.argtypes = [S, P, i64, d, d, d, P]
        L.chx_ensemble_create.argtypes = [S, P, P, i64, O, C.POINTER(P)]
        L.chx_ensemble_advance.argtypes = [P, i64]
        L.chx_ensemble_results.argtypes = [P, R]
        L.chx_ensemble_info.argtypes = [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
        L.chx_ensemble_destroy.argtypes = [P]
        L.chx_ensemble_destroy.restype = None
        L.chx_grid_hh_section.argtypes = [d, d, d, i32, d, d, i32, P, P, u32, P]
        L.chx_hh_section_points.argtypes = [d, P, P, i64, P, P, u32, P]
        L.chx_ic_fput_modes.argtypes = [S, P, i64, P, u32, P]
        L.chx_ic_quartic.argtypes = [S, P, i64, P, u32, P]
        L.chx_last_error.restype = C.c_char_p
        L.chx_version.restype = C.c_char_p
        L.chx_shutdown.argtypes = []
        L.chx_integrate_batched.argtypes = [C.POINTER(_BatchItem), i32, O, R,
                                            C.POINTER(_BatchStats)]
        L.chx_struct_size.argtypes = [i32]
        L.chx_struct_size.restype = C.c_size_t
        L.chx_ensemble_subset.argtypes = [P, P, C.POINTER(P)]
        L.chx_gate_create.argtypes = [u64, C.POINTER(P)]
        L.chx_gate_destroy.argtypes = [P]
        L.chx_gate_destroy.restype = None
        L.chx_gate_train.argtypes = [P, P, P, i64, C.POINTER(_GateTrainCfg), i32, P, u32, P]
        L.chx_gate_grad.argtypes = [P, P, P, i64, P, P, u32, P]
        L.chx_gate_infer.argtypes = [P, P, i64, P, P, u32, P]
        L.chx_gate_get.argtypes = [P, P, P, P]
        L.chx_gate_set.argtypes = [P, P, P, P]
        L.chx_gate_features.argtypes = [P, P, P, d, i64, P, u32, P]
        L.chx_gate_classify.argtypes = [P, S, P, P, i64, O, d, C.c_float, P, P, P,
                                        C.POINTER(_GateStats)]
        for f in EXPORTS:
            if f not in ("chx_options_default", "chx_ensemble_destroy", "chx_last_error",
                         "chx_version", "chx_struct_size", "chx_gate_destroy"):
                getattr(L, f).restype = C.c_int
        for k, st in enumerate((_System, _Options, _Result, _BatchItem, _BatchStats,
                                _GateTrainCfg, _GateStats, _LdnOptions, _LdnResult)):
            if L.chx_struct_size(k) != C.sizeof(st):
                raise ImportError(f"libchx struct {st.__name__} layout differs from the binding")
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        raise ChxError(status, lib().chx_last_error().decode())


# --- systems -----------------------------------------------------------------

@dataclass
class System:
    kind: int
    ndof: int
    params: tuple = ()
    source: str = None  # SYS_CUSTOM only

    def _c(self):
        arr = (C.c_double * max(1, len(self.params)))(*self.params)
        src = None if self.source is None else self.source.encode()
        s = _System(self.kind, self.ndof, C.cast(arr, C.POINTER(C.c_double)), len(self.params),
                    src)
        s._keep = (arr, src)
        return s


def henon_heiles():
    return System(SYS_HENON_HEILES, 2, ())


def fput(N, k=1.0, alpha=0.0, beta=1.0):
    return System(SYS_FPUT, N, (float(k), float(alpha), float(beta)))


def quartic(N=3, eps=0.1):
    return System(SYS_QUARTIC, N, (float(eps),))


def harmonic(omegas):
    return System(SYS_HARMONIC, len(omegas), tuple(float(w) for w in omegas))


def custom(ndof, source, params=()):
    """A separable system H = |p|^2/2 + V(q) given as HIP device code
    defining chx_potential, chx_force (grad V) and chx_hess (Hess V, upper
    triangle packed row by row); ndof 1..8, up to 16 params (see chx.h)."""
    return System(SYS_CUSTOM, int(ndof), tuple(float(v) for v in params), str(source))


def custom_general(ndof, source, params=()):
    """Any Hamiltonian: HIP device code defining
    template <class T> __device__ void chx_field(const T *x, T *f, const double *prm)
    (Hamilton's equations over a generic number type) and
    __device__ double chx_hamiltonian(const double *x, const double *prm);
    ndof 1..8, up to 16 params; "dop853" or "dop853_adaptive" only."""
    return System(SYS_CUSTOM_GENERAL, int(ndof), tuple(float(v) for v in params), str(source))


def double_pendulum(alpha=1.0, sigma=1.0):
    """x = (theta_1, theta_2, p_1, p_2); alpha the length ratio, sigma the
    mass ratio; integrated with "dop853" or "dop853_adaptive" only."""
    return System(SYS_DOUBLE_PENDULUM, 2, (float(alpha), float(sigma)))


# --- array marshalling -----------------------------------------------------------

def _is_torch(a):
    return type(a).__module__.startswith("torch") and hasattr(a, "data_ptr")


class _Arrays:
    """Host (numpy) or device (torch) arrays for one call."""

    def __init__(self, like):
        self.device = _is_torch(like) and like.is_cuda
        if _is_torch(like) and not like.is_cuda:
            raise TypeError("torch tensors must be on the GPU; use numpy for host memory")
        if self.device:
            import torch
            self.torch = torch
            self.dev = like.device
            self.stream = torch.cuda.current_stream(self.dev).cuda_stream
        else:
            self.stream = None

    @property
    def flags(self):
        return PTR_DEVICE if self.device else 0

    def inp(self, a, dtype):
        if a is None:
            return None, None
        if self.device:
            t = self.torch.as_tensor(a, device=self.dev)
            tdt = {np.float64: self.torch.float64, np.uint8: self.torch.uint8,
                   np.float32: self.torch.float32, np.int8: self.torch.int8}[dtype]
            t = t.to(tdt).contiguous()
            return t, C.c_void_p(t.data_ptr())
        arr = np.ascontiguousarray(a, dtype=dtype)
        return arr, arr.ctypes.data_as(C.c_void_p)

    def out(self, shape, dtype):
        if self.device:
            tdt = {np.float64: self.torch.float64, np.int32: self.torch.int32,
                   np.int8: self.torch.int8, np.uint8: self.torch.uint8,
                   np.float32: self.torch.float32, np.int64: self.torch.int64}[dtype]
            t = self.torch.empty(shape, dtype=tdt, device=self.dev)
            return t, C.c_void_p(t.data_ptr())
        arr = np.empty(shape, dtype=dtype)
        return arr, arr.ctypes.data_as(C.c_void_p)


def make_options(dt, T, indicators, renorm_every=10, n_lyap=0, gali_kmax=0, ld_p=0.5,
                 sali_threshold=1e-8, early_exit=False, steps_per_launch=0, seed=0,
                 escape_r2=0.0, block_size=0, integrator=INT_YOSHIDA4, rtol=0.0, atol=0.0):
    """integrator: INT_YOSHIDA4 / INT_DOP853 / INT_DOP853_ADAPTIVE, or
    "yoshida4" / "dop853" / "dop853_adaptive"; rtol, atol: tolerances of
    the adaptive solver (0 and 0: 1e-10 each)."""
    o = _Options()
    lib().chx_options_default(C.byref(o))
    o.dt, o.T, o.indicators = float(dt), float(T), int(indicators)
    o.renorm_every, o.n_lyap, o.gali_kmax = int(renorm_every), int(n_lyap), int(gali_kmax)
    o.ld_p, o.sali_threshold = float(ld_p), float(sali_threshold)
    o.early_exit, o.steps_per_launch = int(bool(early_exit)), int(steps_per_launch)
    o.seed, o.escape_r2, o.block_size = int(seed) & (2**64 - 1), float(escape_r2), int(block_size)
    o.integrator = _INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
    o.rtol, o.atol = float(rtol), float(atol)
    return o


def _sizes(sys, o):
    N = sys.ndof
    m_s = 2 if o.indicators & IND_SALI else 0
    kmax = (o.gali_kmax or 2) if o.indicators & IND_GALI else 0
    m_s = max(m_s, kmax)
    n_l = (o.n_lyap or 2 * N) if o.indicators & IND_LYAP else 0
    return N, m_s, n_l, kmax


def _alloc_results(arr, sys, o, n, want):
    N, m_s, n_l, kmax = _sizes(sys, o)
    spec = {"x_final": ((n, 2 * N), np.float64), "t_end": ((n,), np.float64),
            "status": ((n,), np.int32), "label": ((n,), np.int8),
            "sali_final": ((n,), np.float64), "sali_min": ((n,), np.float64),
            "t_chaos": ((n,), np.float64), "gali": ((n, max(kmax - 1, 0)), np.float64),
            "lyap": ((n, n_l), np.float64), "ld": ((n,), np.float64),
            "energy_err": ((n,), np.float64), "ln_growth": ((n, m_s), np.float64),
            "steps": ((n, 2), np.int64), "step_err": ((n, 2), np.float64)}
    ind = o.indicators
    avail = {"x_final", "t_end", "status"}
    if ind & IND_SALI:
        avail |= {"label", "sali_final", "sali_min", "t_chaos"}
    if ind & IND_GALI:
        avail.add("gali")
    if ind & IND_LYAP:
        avail.add("lyap")
    if ind & IND_LD:
        avail.add("ld")
    if ind & IND_ENERGY:
        avail.add("energy_err")
    if m_s:
        avail.add("ln_growth")
    if o.integrator == INT_DOP853_ADAPTIVE:
        avail |= {"steps", "step_err"}
    want = avail if want is None else (set(want) & avail)
    res = _Result()
    out = {}
    for f in RESULT_FIELDS:
        if f in want:
            a, p = arr.out(*spec[f])
            out[f] = a
            setattr(res, f, p)
    return res, out


class Ensemble:
    """A resumable device-resident ensemble (chx_ensemble_*)."""

    def __init__(self, sys, x0, mask=None, w0=None, outputs=None, **opts):
        self.sys = sys
        self.arr = _Arrays(x0)
        self.o = make_options(**opts)
        self.o.flags = self.arr.flags
        self.o.stream = self.arr.stream
        self._x0, px0 = self.arr.inp(x0, np.float64)
        self.n = int(self._x0.shape[0]) if self._x0.ndim else 0
        self._mask, pm = self.arr.inp(mask, np.uint8)
        self._w0, pw = self.arr.inp(w0, np.float64)
        self.o.w0 = pw
        self.outputs = outputs
        self.h = C.c_void_p()
        cs = sys._c()
        _check(lib().chx_ensemble_create(C.byref(cs), px0, pm, self.n, C.byref(self.o),
                                         C.byref(self.h)))

    def info(self):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().chx_ensemble_info(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    @property
    def n_total(self):
        return self.info()[0]

    def advance(self, s_end=None):
        if s_end is None:
            s_end = self.n_total
        _check(lib().chx_ensemble_advance(self.h, int(s_end)))

    def results(self, outputs=None):
        res, out = _alloc_results(self.arr, self.sys, self.o, self.n,
                                  outputs if outputs is not None else self.outputs)
        _check(lib().chx_ensemble_results(self.h, C.byref(res)))
        return out

    def subset(self, keep):
        """chx_ensemble_subset: a new Ensemble continuing the active orbits
        with keep[i] != 0 (numbered 0..n2-1 in increasing i)."""
        k, pk = self.arr.inp(keep, np.uint8)
        if int(k.shape[0]) != self.n:
            raise ValueError("keep must have one entry per orbit")
        h = C.c_void_p()
        _check(lib().chx_ensemble_subset(self.h, pk, C.byref(h)))
        e = Ensemble.__new__(Ensemble)
        e.sys, e.arr, e.o, e.outputs, e.h = self.sys, self.arr, self.o, self.outputs, h
        e._x0 = e._mask = e._w0 = None
        e.n = e.info()[2]
        return e

    def close(self):
        if self.h:
            lib().chx_ensemble_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def integrate_ensemble(sys, x0, mask=None, w0=None, outputs=None, **opts):
    """chx_integrate_ensemble: returns a dict of the requested outputs."""
    arr = _Arrays(x0)
    o = make_options(**opts)
    o.flags, o.stream = arr.flags, arr.stream
    x0a, px0 = arr.inp(x0, np.float64)
    n = int(x0a.shape[0])
    ma, pm = arr.inp(mask, np.uint8)
    w0a, pw = arr.inp(w0, np.float64)
    o.w0 = pw
    res, out = _alloc_results(arr, sys, o, n, outputs)
    keep = (x0a, ma, w0a)  # noqa: F841 -- alive until the call returns
    cs = sys._c()
    _check(lib().chx_integrate_ensemble(C.byref(cs), px0, pm, n, C.byref(o), C.byref(res)))
    return out


def integrate_ensemble_noalloc(sys, x0, mask=None, w0=None, outputs=None, **opts):
    """chx_integrate_ensemble_noalloc: chx_integrate_ensemble on device
    tensors with the library's fixed workspace (no device allocation by the
    library; the output tensors are allocated here, by the caller)."""
    arr = _Arrays(x0)
    if not arr.device:
        raise TypeError("the allocation-free entry takes device (torch) tensors only")
    o = make_options(**opts)
    o.flags, o.stream = arr.flags, arr.stream
    x0a, px0 = arr.inp(x0, np.float64)
    n = int(x0a.shape[0])
    ma, pm = arr.inp(mask, np.uint8)
    w0a, pw = arr.inp(w0, np.float64)
    o.w0 = pw
    res, out = _alloc_results(arr, sys, o, n, outputs)
    keep = (x0a, ma, w0a)  # noqa: F841 -- alive until the call returns
    cs = sys._c()
    _check(lib().chx_integrate_ensemble_noalloc(C.byref(cs), px0, pm, n, C.byref(o),
                                                C.byref(res)))
    return out


class _LdnOptions(C.Structure):
    _fields_ = [("dirs", C.c_uint32), ("sigma", C.c_double), ("two_sided", C.c_int32)]


LDN_FIELDS = ["ld", "D", "R", "S", "status"]


class _LdnResult(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in LDN_FIELDS]


def ld_indicators(sys, x0, sigma, dirs=None, two_sided=True, mask=None, outputs=None, **opts):
    """chx_ld_indicators: the difference D, ratio R and second derivative S
    of the (two-sided) LDs of each initial condition and its neighbours at
    +/- sigma along the coordinates in dirs (a list of indices into the 2N
    phase-space coordinates, or None for all); opts as for
    integrate_ensemble (indicators defaults to the LD).  Returns a dict of
    the requested outputs among LDN_FIELDS."""
    arr = _Arrays(x0)
    opts.setdefault("indicators", IND_LD)
    o = make_options(**opts)
    o.flags, o.stream = arr.flags, arr.stream
    x0a, px0 = arr.inp(x0, np.float64)
    n = int(x0a.shape[0])
    ma, pm = arr.inp(mask, np.uint8)
    lo = _LdnOptions()
    lo.dirs = 0 if dirs is None else sum(1 << int(c) for c in dirs)
    lo.sigma, lo.two_sided = float(sigma), int(bool(two_sided))
    want = set(LDN_FIELDS if outputs is None else outputs)
    res, out = _LdnResult(), {}
    for f in LDN_FIELDS:
        if f in want:
            a, p = arr.out((n,), np.int32 if f == "status" else np.float64)
            out[f] = a
            setattr(res, f, p)
    keep = (x0a, ma)  # noqa: F841 -- alive until the call returns
    cs = sys._c()
    _check(lib().chx_ld_indicators(C.byref(cs), px0, pm, n, C.byref(o), C.byref(lo),
                                   C.byref(res)))
    return out


# --- convenience calls (host memory) -----------------------------------------------

def _host(x0, sys):
    x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1, 2 * sys.ndof)
    return x0, x0.ctypes.data_as(C.c_void_p), len(x0)


def sali(sys, x0, dt, T, seed):
    x0, p, n = _host(x0, sys)
    smin, lab = np.empty(n), np.empty(n, np.int8)
    cs = sys._c()
    _check(lib().chx_sali(C.byref(cs), p, n, dt, T, seed, smin.ctypes.data_as(C.c_void_p),
                          lab.ctypes.data_as(C.c_void_p)))
    return smin, lab


def gali(sys, x0, dt, T, kmax, seed):
    x0, p, n = _host(x0, sys)
    g = np.empty((n, kmax - 1))
    cs = sys._c()
    _check(lib().chx_gali(C.byref(cs), p, n, dt, T, kmax, seed, g.ctypes.data_as(C.c_void_p)))
    return g


def lyap_spectrum(sys, x0, dt, T, n_exp, renorm_every=10):
    x0, p, n = _host(x0, sys)
    out = np.empty((n, n_exp))
    cs = sys._c()
    _check(lib().chx_lyap_spectrum(C.byref(cs), p, n, dt, T, n_exp, renorm_every,
                                   out.ctypes.data_as(C.c_void_p)))
    return out


def ld(sys, x0, dt, T, p=0.5):
    x0, px, n = _host(x0, sys)
    out = np.empty(n)
    cs = sys._c()
    _check(lib().chx_ld(C.byref(cs), px, n, dt, T, p, out.ctypes.data_as(C.c_void_p)))
    return out


# --- initial conditions -------------------------------------------------------------

def grid_hh_section(E, ny, npy, y0=-0.4, y1=0.7, py0=-0.45, py1=0.45, device=None):
    """Henon-Heiles section grid; device=None -> numpy, else a torch device."""
    like = None
    if device is not None:
        import torch
        like = torch.empty(0, device=device)
    arr = _Arrays(like if like is not None else np.empty(0))
    x0, px = arr.out((ny * npy, 4), np.float64)
    m, pm = arr.out((ny * npy,), np.uint8)
    _check(lib().chx_grid_hh_section(E, y0, y1, ny, py0, py1, npy, px, pm, arr.flags,
                                     arr.stream))
    return x0, m


def hh_section_points(E, y, py):
    arr = _Arrays(y)
    ya, p1 = arr.inp(y, np.float64)
    pa, p2 = arr.inp(py, np.float64)
    n = int(ya.shape[0])
    x0, px = arr.out((n, 4), np.float64)
    m, pm = arr.out((n,), np.uint8)
    _check(lib().chx_hh_section_points(E, p1, p2, n, px, pm, arr.flags, arr.stream))
    return x0, m


def ic_fput_modes(sys, u):
    arr = _Arrays(u)
    ua, pu = arr.inp(u, np.float64)
    n = int(ua.shape[0])
    x0, px = arr.out((n, 2 * sys.ndof), np.float64)
    cs = sys._c()
    _check(lib().chx_ic_fput_modes(C.byref(cs), pu, n, px, arr.flags, arr.stream))
    return x0


def ic_quartic(sys, draws):
    arr = _Arrays(draws)
    da, pd = arr.inp(draws, np.float64)
    n = int(da.shape[0])
    x0, px = arr.out((n, 2 * sys.ndof), np.float64)
    cs = sys._c()
    _check(lib().chx_ic_quartic(C.byref(cs), pd, n, px, arr.flags, arr.stream))
    return x0


def integrate_batched(items, outputs=None, **opts):
    """chx_integrate_batched.  items: list of dicts with keys sys, x0,
    mask (optional), dt, T.  Returns (list of per-item output dicts, stats
    dict).  All arrays numpy (host) or all torch CUDA tensors (device)."""
    if not items:
        raise ValueError("no items")
    arr = _Arrays(items[0]["x0"])
    o = make_options(dt=items[0]["dt"], T=items[0]["T"], **opts)
    o.flags, o.stream = arr.flags, arr.stream
    c_items = (_BatchItem * len(items))()
    results = (_Result * len(items))()
    keep, outs = [], []
    for k, it in enumerate(items):
        sys = it["sys"]
        xa, px = arr.inp(it["x0"], np.float64)
        ma, pm = arr.inp(it.get("mask"), np.uint8)
        n = int(xa.shape[0])
        cs = sys._c()
        keep += [xa, ma, cs]
        c_items[k].sys = cs
        c_items[k].x0, c_items[k].mask, c_items[k].n = px, pm, n
        c_items[k].dt, c_items[k].T = float(it["dt"]), float(it["T"])
        oi = make_options(dt=it["dt"], T=it["T"], **opts)
        res, out = _alloc_results(arr, sys, oi, n, outputs)
        results[k] = res
        outs.append(out)
    st = _BatchStats()
    _check(lib().chx_integrate_batched(c_items, len(items), C.byref(o), results, C.byref(st)))
    stats = {f: getattr(st, f) for f, _ in _BatchStats._fields_}
    stats["orbit_steps"] = list(st.orbit_steps)[:len(items)]
    stats["cost_ps"] = list(st.cost_ps)[:len(items)]
    return outs, stats


# --- learned gate -----------------------------------------------------------------

def gate_features(x0, ld, ln_growth, t):
    """chx_gate_features: [n][6] float32 features at time t."""
    arr = _Arrays(x0)
    xa, px = arr.inp(x0, np.float64)
    la, pl = arr.inp(ld, np.float64)
    ga, pg = arr.inp(ln_growth, np.float64)
    n = int(xa.shape[0])
    out, po = arr.out((n, GATE_NFEAT), np.float32)
    _check(lib().chx_gate_features(px, pl, pg, float(t), n, po, arr.flags, arr.stream))
    return out


class Gate:
    """The learned gate (chx_gate_*): a 6-256-256-2 GELU perceptron trained and
    evaluated by the library's kernels on the current GPU."""

    def __init__(self, seed=0):
        self.h = C.c_void_p()
        _check(lib().chx_gate_create(int(seed) & (2**64 - 1), C.byref(self.h)))

    def close(self):
        if self.h:
            lib().chx_gate_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def train(self, features, labels, epochs=1, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999,
              eps=1e-8, weight_decay=0.0, seed=0, reset_stats=False):
        """Returns the mean loss of each epoch (numpy float32)."""
        arr = _Arrays(features)
        fa, pf = arr.inp(features, np.float32)
        la, pl = arr.inp(labels, np.int8)
        n = int(fa.shape[0])
        c = _GateTrainCfg(int(epochs), int(batch), float(lr), float(beta1), float(beta2),
                          float(eps), float(weight_decay), int(seed) & (2**64 - 1))
        loss = np.zeros(max(int(epochs), 1), np.float32)
        _check(lib().chx_gate_train(self.h, pf, pl, n, C.byref(c), int(bool(reset_stats)),
                                    loss.ctypes.data_as(C.c_void_p), arr.flags, arr.stream))
        return loss[:int(epochs)]

    def grad(self, features, labels):
        """(mean loss, flat gradient) over up to 65536 rows, no update."""
        arr = _Arrays(features)
        fa, pf = arr.inp(features, np.float32)
        la, pl = arr.inp(labels, np.int8)
        g = np.zeros(GATE_NPARAM, np.float32)
        loss = C.c_float()
        _check(lib().chx_gate_grad(self.h, pf, pl, int(fa.shape[0]), g.ctypes.data_as(C.c_void_p),
                                   C.byref(loss), arr.flags, arr.stream))
        return float(loss.value), g

    def infer(self, features):
        """(p_chaotic, confidence) per row."""
        arr = _Arrays(features)
        fa, pf = arr.inp(features, np.float32)
        n = int(fa.shape[0])
        p, pp = arr.out((n,), np.float32)
        c, pc = arr.out((n,), np.float32)
        _check(lib().chx_gate_infer(self.h, pf, n, pp, pc, arr.flags, arr.stream))
        return p, c

    def get(self):
        p = np.zeros(GATE_NPARAM, np.float32)
        m = np.zeros(GATE_NFEAT, np.float32)
        s = np.zeros(GATE_NFEAT, np.float32)
        _check(lib().chx_gate_get(self.h, p.ctypes.data_as(C.c_void_p),
                                  m.ctypes.data_as(C.c_void_p), s.ctypes.data_as(C.c_void_p)))
        return p, m, s

    def set(self, params=None, mean=None, istd=None):
        ptr = lambda a, n: (None, None) if a is None else (
            lambda x: (x, x.ctypes.data_as(C.c_void_p)))(
                np.ascontiguousarray(a, np.float32).reshape(n))
        pa, pp = ptr(params, GATE_NPARAM)
        ma, pm = ptr(mean, GATE_NFEAT)
        sa, ps = ptr(istd, GATE_NFEAT)
        _check(lib().chx_gate_set(self.h, pp, pm, ps))

    def classify(self, sys, x0, mask=None, t_gate=200.0, conf_min=0.98, **opts):
        """chx_gate_classify: returns ({label, source, confidence}, stats)."""
        arr = _Arrays(x0)
        o = make_options(**opts)
        o.flags, o.stream = arr.flags, arr.stream
        xa, px = arr.inp(x0, np.float64)
        ma, pm = arr.inp(mask, np.uint8)
        n = int(xa.shape[0])
        lab, plab = arr.out((n,), np.int8)
        src, psrc = arr.out((n,), np.uint8)
        cf, pcf = arr.out((n,), np.float32)
        st = _GateStats()
        cs = sys._c()
        _check(lib().chx_gate_classify(self.h, C.byref(cs), px, pm, n, C.byref(o),
                                       float(t_gate), float(conf_min), plab, psrc, pcf,
                                       C.byref(st)))
        stats = {f: getattr(st, f) for f, _ in _GateStats._fields_}
        return {"label": lab, "source": src, "confidence": cf}, stats


def version():
    return lib().chx_version().decode()


def shutdown():
    """Unloads the user-system code objects from the devices (chx_shutdown);
    later calls load them again."""
    _check(lib().chx_shutdown())
