"""ctypes binding of libfd (C ABI in include/fd.h).

Argument marshalling only: every arithmetic step of the apply runs in the HIP
library. Device buffers and streams come from torch (tensors and
``torch.cuda.Stream``); host matrices are numpy FP64 arrays. The library must
be built (``python -m paper_1712_00403_amd.build``); loading fails loudly
otherwise, there is no fallback.
"""
import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfd.so")

FD_OK, FD_E_ARG, FD_E_NOTSPD, FD_E_NOMEM, FD_E_HIP, FD_E_UNSUPPORTED = range(6)
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "bf16_split": 4, "f16_split": 5, "fp8_split": 6}
STATUS_NAMES = {0: "FD_OK", 1: "FD_E_ARG", 2: "FD_E_NOTSPD", 3: "FD_E_NOMEM", 4: "FD_E_HIP",
                5: "FD_E_UNSUPPORTED"}

# every symbol declared in include/fd.h
EXPORTS = ("fd_assemble_1d", "fd_nitsche_stiffness_1d", "fd_mixed_1d", "fd_quadrature_1d", "fd_factor_1d", "fd_geometry_coefficients",
           "fd_separable_factors", "fd_operator_diagonal", "fd_setup", "fd_setup_mass_banded", "fd_destroy",
           "fd_plan_size", "fd_plan_device_bytes", "fd_set_device_limit", "fd_device_bytes_held", "fd_workspace_bytes", "fd_plan_factors", "fd_apply",
           "fd_apply_batched", "fd_batch_create", "fd_batch_apply", "fd_batch_tune", "fd_batch_set_config",
           "fd_batch_info", "fd_batch_signature", "fd_batch_check", "fd_batch_destroy", "fd_apply_persistent_static", "fd_timing_enable", "fd_timing_read", "fd_timing_launches", "fd_last_error")


class FDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class FDLaunchTime(ctypes.Structure):
    _fields_ = [("stage", ctypes.c_int32), ("family", ctypes.c_int32), ("n", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("ms", ctypes.c_double), ("count", ctypes.c_int32)]


class FDWork(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("r", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("nrhs", ctypes.c_int32), ("ld", ctypes.c_int64)]


_lib = None


def lib():
    """Load libfd.so (once). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libfd.so not found at {LIB_PATH}; build it with "
                           "`python -m paper_1712_00403_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    c_dp = ctypes.POINTER(ctypes.c_double)
    L.fd_last_error.restype = ctypes.c_char_p
    L.fd_assemble_1d.argtypes = [ctypes.c_int32] * 5 + [c_dp, c_dp, ctypes.POINTER(ctypes.c_int32), c_dp, c_dp]
    L.fd_quadrature_1d.argtypes = [ctypes.c_int32, ctypes.c_int32, c_dp, c_dp]
    L.fd_mixed_1d.argtypes = [ctypes.c_int32] * 8 + [ctypes.POINTER(ctypes.c_int32)] * 2 + [c_dp]
    L.fd_nitsche_stiffness_1d.argtypes = [ctypes.c_int32] * 3 + [ctypes.c_double, ctypes.POINTER(ctypes.c_int32),
                                                                  c_dp]
    L.fd_factor_1d.argtypes = [ctypes.c_int32, c_dp, c_dp, c_dp, c_dp]
    L.fd_geometry_coefficients.argtypes = [ctypes.c_int32, ctypes.c_int64, c_dp, c_dp, ctypes.c_int32, c_dp, c_dp]
    L.fd_separable_factors.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), c_dp, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_double, c_dp, c_dp]
    L.fd_operator_diagonal.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)] + [ctypes.c_int32] * 5 + \
        [c_dp, c_dp]
    L.fd_setup.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(c_dp),
                           ctypes.POINTER(c_dp), c_dp, c_dp, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    L.fd_setup_mass_banded.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(c_dp),
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    L.fd_destroy.argtypes = [ctypes.c_void_p]
    L.fd_plan_size.argtypes = [ctypes.c_void_p]
    L.fd_plan_size.restype = ctypes.c_int64
    L.fd_plan_device_bytes.argtypes = [ctypes.c_void_p]
    L.fd_plan_device_bytes.restype = ctypes.c_size_t
    L.fd_set_device_limit.argtypes = [ctypes.c_size_t]
    L.fd_set_device_limit.restype = ctypes.c_int
    L.fd_device_bytes_held.argtypes = []
    L.fd_device_bytes_held.restype = ctypes.c_size_t
    L.fd_workspace_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.fd_workspace_bytes.restype = ctypes.c_size_t
    L.fd_plan_factors.argtypes = [ctypes.c_void_p, ctypes.c_int32, c_dp, c_dp]
    L.fd_apply.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                           ctypes.c_int64, ctypes.c_void_p]
    L.fd_apply_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(FDWork), ctypes.c_void_p]
    L.fd_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(FDWork), ctypes.POINTER(ctypes.c_void_p)]
    L.fd_batch_apply.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    L.fd_batch_tune.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    L.fd_batch_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_int32)]
    L.fd_batch_set_config.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    L.fd_batch_set_config.restype = ctypes.c_int
    L.fd_batch_check.argtypes = [ctypes.c_void_p]
    L.fd_batch_signature.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
    L.fd_batch_destroy.argtypes = [ctypes.c_void_p]
    L.fd_apply_persistent_static.argtypes = [ctypes.c_int32, ctypes.POINTER(FDWork), ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p]
    for name in ("fd_batch_create", "fd_batch_apply", "fd_batch_tune", "fd_batch_info", "fd_batch_check",
                 "fd_batch_signature", "fd_batch_destroy", "fd_apply_persistent_static"):
        getattr(L, name).restype = ctypes.c_int
    L.fd_timing_enable.argtypes = [ctypes.c_int32]
    L.fd_timing_read.argtypes = [c_dp, ctypes.POINTER(ctypes.c_int32)]
    L.fd_timing_launches.argtypes = [ctypes.c_int32, ctypes.POINTER(FDLaunchTime), ctypes.POINTER(ctypes.c_int32)]
    L.fd_timing_launches.restype = ctypes.c_int
    for name in ("fd_timing_enable", "fd_timing_read", "fd_assemble_1d", "fd_nitsche_stiffness_1d", "fd_mixed_1d",
                 "fd_quadrature_1d", "fd_factor_1d", "fd_geometry_coefficients", "fd_separable_factors",
                 "fd_operator_diagonal", "fd_setup", "fd_setup_mass_banded", "fd_destroy", "fd_plan_factors", "fd_apply",
                 "fd_apply_batched"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != FD_OK:
        raise FDError(status, lib().fd_last_error().decode())


def set_device_limit(nbytes):
    """Cap the device bytes the library holds at once (0: no cap); setups past it raise FD_E_NOMEM."""
    _check(lib().fd_set_device_limit(int(nbytes)))


def device_bytes_held():
    """Device bytes the library holds now (plans, fixed-batch tables)."""
    return int(lib().fd_device_bytes_held())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64c(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- host-only calls

def assemble_1d(n_el, degree, regularity, dirichlet, npts=0, tau=None, mu=None):
    """Univariate (K, M), column-major FP64 (see fd_assemble_1d)."""
    L = lib()
    m = ctypes.c_int32(0)
    tq = None if tau is None else _f64c(tau).ravel()
    mq = None if mu is None else _f64c(mu).ravel()
    _check(L.fd_assemble_1d(n_el, degree, regularity, int(bool(dirichlet)), npts, _dp(tq), _dp(mq),
                            ctypes.byref(m), None, None))
    K = np.zeros((m.value, m.value), order="F")
    M = np.zeros((m.value, m.value), order="F")
    _check(L.fd_assemble_1d(n_el, degree, regularity, int(bool(dirichlet)), npts, _dp(tq), _dp(mq),
                            ctypes.byref(m), K.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            M.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return np.ascontiguousarray(K), np.ascontiguousarray(M)


def nitsche_stiffness_1d(n_el, degree, regularity, c_pen):
    """The RT blocks' Nitsche-modified stiffness K~ over all functions of the space (fd_nitsche_stiffness_1d)."""
    L = lib()
    m = ctypes.c_int32(0)
    _check(L.fd_nitsche_stiffness_1d(n_el, degree, regularity, float(c_pen), ctypes.byref(m), None))
    K = np.zeros((m.value, m.value), order="F")
    _check(L.fd_nitsche_stiffness_1d(n_el, degree, regularity, float(c_pen), ctypes.byref(m),
                                     K.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return np.ascontiguousarray(K)


def mixed_1d(n_el, deg_a, reg_a, da, deg_b, reg_b, db, npts=0):
    """X[l, m] = int b_{a,l}^(da) b_{b,m}^(db) over all functions of two spaces (fd_mixed_1d)."""
    L = lib()
    ma, mb = ctypes.c_int32(0), ctypes.c_int32(0)
    args = (n_el, deg_a, reg_a, da, deg_b, reg_b, db, npts)
    _check(L.fd_mixed_1d(*args, ctypes.byref(ma), ctypes.byref(mb), None))
    X = np.zeros((ma.value, mb.value), order="F")
    _check(L.fd_mixed_1d(*args, ctypes.byref(ma), ctypes.byref(mb), X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return np.ascontiguousarray(X)


def quadrature_1d(n_el, npts):
    x = np.zeros(n_el * npts)
    w = np.zeros(n_el * npts)
    _check(lib().fd_quadrature_1d(n_el, npts, _dp(x), _dp(w)))
    return x.reshape(n_el, npts), w.reshape(n_el, npts)


def factor_1d(K, M):
    """(U, d) of the pencil (K, M) computed by the library on the host."""
    M = _f64c(M)
    n = M.shape[0]
    Kc = None if K is None else np.asfortranarray(np.asarray(K, dtype=np.float64))
    Mc = np.asfortranarray(M)
    U = np.zeros((n, n), order="F")
    d = np.zeros(n)
    _check(lib().fd_factor_1d(n, None if Kc is None else Kc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              Mc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _dp(d)))
    return np.ascontiguousarray(U), d


def geometry_coefficients(jac, nu, matrices=True, component=None):
    """C (d, d, d, P) with C[k, a, b] = (C_k)_ab at each point, and the pressure weight (P,).

    jac: (P, d, d) Jacobians dG_a/deta_b; nu: (P,) viscosity at the mapped points
    (see fd_geometry_coefficients). ``matrices=False`` returns (None, weight);
    ``component=k`` returns C_k alone as (d, d, P).
    """
    jac = _f64c(jac)
    P, d, _ = jac.shape
    nu = _f64c(nu).ravel()
    if not matrices:
        C = None
    else:
        C = np.empty((d, d, d, P)) if component is None else np.empty((d, d, P))
    qw = np.empty(P)
    _check(lib().fd_geometry_coefficients(d, P, _dp(jac), _dp(nu), -1 if component is None else int(component),
                                          _dp(C), _dp(qw)))
    return C, qw


def separable_factors(Ck, nq, sweeps=20, tol=1e-12):
    """(tau, mu) of one C_k given as (d, d, P) fields on the nq grid (see fd_separable_factors)."""
    Ck = _f64c(Ck)
    d = Ck.shape[0]
    P = Ck.shape[-1]
    tau = np.zeros(int(sum(nq)))
    mu = np.zeros(int(sum(nq)))
    nqa = (ctypes.c_int32 * d)(*[int(x) for x in nq])
    _check(lib().fd_separable_factors(d, nqa, _dp(Ck), (d + 1) * P, int(sweeps), float(tol), _dp(tau), _dp(mu)))
    cuts = np.cumsum([0] + [int(x) for x in nq])
    return ([tau[cuts[i]:cuts[i + 1]] for i in range(d)], [mu[cuts[i]:cuts[i + 1]] for i in range(d)])


def operator_diagonal(n_el, degree, regularity, dirichlet, npts, coef, order):
    """Diagonal of the Galerkin operator with pointwise coefficients (see fd_operator_diagonal).

    order 1: coef (d, d, P); order 0: coef (P,). Returns the diagonal, i_1 fastest.
    """
    d = len(n_el)
    coef = _f64c(coef)
    m = ctypes.c_int32(0)
    N = 1
    for ne in n_el:
        _check(lib().fd_assemble_1d(int(ne), degree, regularity, int(bool(dirichlet)), npts, None, None,
                                    ctypes.byref(m), None, None))
        N *= m.value
    diag = np.zeros(N)
    nea = (ctypes.c_int32 * d)(*[int(x) for x in n_el])
    _check(lib().fd_operator_diagonal(d, nea, degree, regularity, int(bool(dirichlet)), npts, int(order),
                                      _dp(coef), _dp(diag)))
    return diag


# ---------------------------------------------------------------- plans

class Plan:
    """One Kronecker-sum block on the device (fd_setup / fd_destroy)."""

    def __init__(self, Ks, Ms, weights=None, diag_target=None, precision="f64", banded=False):
        """``banded``: a mass-only plan (Ks None, no weights or diag_target) applied by banded
        Cholesky solves per mode (fd_setup_mass_banded) instead of the FD form."""
        L = lib()
        ndim = len(Ms)
        self.ndim = ndim
        self.n = tuple(int(np.asarray(M).shape[0]) for M in Ms)
        self.precision = precision
        self.prec_id = PRECISIONS[precision]
        self.io_dtype = "float64" if precision == "f64" else "float32"
        c_dp = ctypes.POINTER(ctypes.c_double)
        self._Ms = [np.asfortranarray(np.asarray(M, dtype=np.float64)) for M in Ms]
        self._Ks = None if Ks is None else [np.asfortranarray(np.asarray(K, dtype=np.float64)) for K in Ks]
        Marr = (c_dp * ndim)(*[M.ctypes.data_as(c_dp) for M in self._Ms])
        Karr = None if self._Ks is None else (c_dp * ndim)(*[K.ctypes.data_as(c_dp) for K in self._Ks])
        narr = (ctypes.c_int32 * ndim)(*self.n)
        w = None if weights is None else _f64c(weights)
        dt = None if diag_target is None else _f64c(diag_target).ravel()
        h = ctypes.c_void_p(0)
        self.banded = bool(banded)
        if self.banded:
            if Ks is not None or diag_target is not None:
                raise ValueError("a banded plan is mass-only and unscaled")
            _check(L.fd_setup_mass_banded(ndim, narr, Marr, self.prec_id, ctypes.byref(h)))
        else:
            _check(L.fd_setup(ndim, narr, Karr, Marr, _dp(w), _dp(dt), self.prec_id, ctypes.byref(h)))
        self.handle = h.value
        self.device = _current_device()
        self.N = int(L.fd_plan_size(self.handle))
        self.device_bytes = int(L.fd_plan_device_bytes(self.handle))

    def workspace_bytes(self, nrhs=1):
        """Device bytes an apply of nrhs vectors needs beyond the plan, r and z."""
        return int(lib().fd_workspace_bytes(self.handle, int(nrhs)))

    def factors(self, direction):
        n = self.n[direction]
        U = np.zeros((n, n), order="F")
        d = np.zeros(n)
        _check(lib().fd_plan_factors(self.handle, direction,
                                     U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _dp(d)))
        return np.ascontiguousarray(U), d

    def apply_ptr(self, r_ptr, z_ptr, nrhs, ld, stream=0):
        _check(lib().fd_apply(self.handle, r_ptr, z_ptr, int(nrhs), int(ld), stream))

    def apply(self, r, z=None, stream=None):
        """z = P^{-1} r for a torch device tensor r of shape (nrhs, N) or (N,)."""
        import torch
        if z is None:
            check_vectors(r, None, self.N, self.io_dtype, self.device)
            z = torch.empty_like(r)
        check_vectors(r, z, self.N, self.io_dtype, self.device)
        r2 = r.reshape(-1, r.shape[-1])
        nrhs = r2.shape[0]
        ld = r2.stride(0) if nrhs > 1 else r2.shape[-1]
        s = _stream_handle(stream)
        self.apply_ptr(r.data_ptr(), z.data_ptr(), nrhs, ld, s)
        return z

    def close(self):
        if getattr(self, "handle", None):
            lib().fd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _current_device():
    """The current HIP device (the device fd_setup places a plan on) as a torch.device."""
    import torch
    return torch.device("cuda", torch.cuda.current_device())


def check_vectors(r, z, N, io_dtype, device, exact=False):
    """Reject vectors the library would read or write out of bounds, before any pointer is passed.

    r (and z unless None) must be tensors on ``device`` (a torch.device) with dtype
    ``io_dtype``, of shape (nrhs, L) or (L,) with unit stride along the last
    axis and L >= N (L == N and contiguous if ``exact``); z must have r's
    shape and strides. Raises TypeError for a wrong dtype, ValueError
    otherwise.
    """
    import torch
    want = getattr(torch, io_dtype)
    for name, t in (("r", r), ("z", z)):
        if t is None:
            continue
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.dtype != want:
            raise TypeError(f"{name} has dtype {t.dtype}; the plan expects {io_dtype} vectors")
        if t.device != device:
            raise ValueError(f"{name} is on {t.device}; the plan lives on {device}")
        if t.dim() not in (1, 2):
            raise ValueError(f"{name} must have shape (nrhs, L) or (L,)")
        if t.stride(-1) != 1 or (t.dim() == 2 and t.shape[0] > 1 and t.stride(0) < t.shape[-1]):
            raise ValueError(f"{name} must have unit stride along its last axis and non-overlapping rows")
        if exact and (t.shape[-1] != N or not t.is_contiguous()):
            raise ValueError(f"{name} must be contiguous with exactly {N} entries per vector")
        if t.shape[-1] < N:
            raise ValueError(f"{name} has {t.shape[-1]} entries per vector; the plan needs {N}")
    if z is not None and (tuple(z.shape) != tuple(r.shape) or z.stride() != r.stride()):
        raise ValueError(f"z must have r's shape and strides (r {tuple(r.shape)}/{r.stride()}, "
                         f"z {tuple(z.shape)}/{z.stride()})")


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _work_array(works):
    works = list(works)
    arr = (FDWork * len(works))()
    for i, (plan, r, z, nrhs, ld) in enumerate(works):
        arr[i].plan = plan.handle
        arr[i].r = r
        arr[i].z = z
        arr[i].nrhs = nrhs
        arr[i].ld = ld
    return arr


def apply_batched(works, stream=None):
    """works: iterable of (plan, r_ptr, z_ptr, nrhs, ld) -> one fd_apply_batched call."""
    arr = _work_array(works)
    _check(lib().fd_apply_batched(len(arr), arr, _stream_handle(stream)))


class Batch:
    """A fixed batched apply run as one persistent launch (fd_batch_create / fd_batch_apply)."""

    def __init__(self, works):
        arr = _work_array(works)
        h = ctypes.c_void_p(0)
        _check(lib().fd_batch_create(len(arr), arr, ctypes.byref(h)))
        self.handle = h.value

    def apply(self, stream=None):
        _check(lib().fd_batch_apply(self.handle, _stream_handle(stream)))

    WIDE, NARROW, PIPELINED = 0, 1, 2  # body choices of a stage
    # configuration word of the staged route (every work a 3D BF16/FP16
    # slab-route plan): one launch per stage and row-tile group
    STAGED = 1 << 10
    # configuration bit of the segment route: every segment of the persistent
    # layout (with the body choices of bits 0-9) as a launch of its own
    SEGMENTS = 1 << 11

    @staticmethod
    def config_of(choices):
        """Configuration word of per-stage body choices (stage s in bits 2s, 2s + 1)."""
        return sum(int(c) << (2 * s) for s, c in enumerate(choices))

    @staticmethod
    def choices_of(config):
        return [(int(config) >> (2 * s)) & 3 for s in range(5)]

    def tune(self, stream=None, reps=3, cache=None):
        """Choose the body of every stage by timing (greedy), then the staged route if the batch
        has one and it is faster; returns the configuration word.

        ``cache``: None, or the path of a JSON file of configuration words keyed by batch
        signature: a batch whose signature is there takes that word without timing; otherwise
        the tuned word is added to the file."""
        key = None
        table = {}
        if cache is not None:
            key = format(self.signature(), "016x")
            if os.path.exists(cache):
                with open(cache) as fh:
                    table = json.load(fh)
            if key in table:
                self.set_config(int(table[key]))
                return int(table[key])
        c = ctypes.c_int32(0)
        _check(lib().fd_batch_tune(self.handle, _stream_handle(stream), int(reps), ctypes.byref(c)))
        if cache is not None:
            table[key] = c.value
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(table, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return c.value

    def signature(self):
        """64-bit signature of the batch's layout (fd_batch_signature)."""
        s = ctypes.c_uint64(0)
        _check(lib().fd_batch_signature(self.handle, ctypes.byref(s)))
        return s.value

    def set_config(self, config):
        _check(lib().fd_batch_set_config(self.handle, int(config)))

    def info(self):
        t = ctypes.c_int64(0)
        g = ctypes.c_int32(0)
        c = ctypes.c_int32(0)
        _check(lib().fd_batch_info(self.handle, ctypes.byref(t), ctypes.byref(g), ctypes.byref(c)))
        return {"tiles": t.value, "grid": g.value, "config": c.value}

    def check(self):
        _check(lib().fd_batch_check(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            lib().fd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def apply_persistent_static(works, config=0, status=None, stream=None):
    """works: iterable of (plan, r_ptr, z_ptr, nrhs, ld) -> one allocation-free persistent launch.

    ``status``: None or the device address of an int32 the library sets to 0,
    or to 1 if a grid barrier gave up (fd_apply_persistent_static).
    """
    arr = _work_array(works)
    _check(lib().fd_apply_persistent_static(len(arr), arr, int(config), status, _stream_handle(stream)))


STAGE_NAMES = ("mode1_fwd", "mode2_fwd", "last_mode_fused", "mode2_bwd", "mode1_bwd")


def timing_enable(on=True):
    _check(lib().fd_timing_enable(1 if on else 0))


def timing_read():
    """{stage name: (total ms, executions)} since the last read (waits for the events)."""
    ms = (ctypes.c_double * 5)()
    cnt = (ctypes.c_int32 * 5)()
    _check(lib().fd_timing_read(ms, cnt))
    return {STAGE_NAMES[i]: (ms[i], cnt[i]) for i in range(5)}


def timing_launches():
    """Per launch class of the last timing_read: list of dicts (stage, family, n, prec, ms, count)."""
    n = ctypes.c_int32(0)
    _check(lib().fd_timing_launches(0, None, ctypes.byref(n)))
    arr = (FDLaunchTime * max(n.value, 1))()
    _check(lib().fd_timing_launches(n.value, arr, ctypes.byref(n)))
    return [{"stage": STAGE_NAMES[a.stage], "family": a.family, "n": a.n, "prec": a.prec, "ms": a.ms,
             "count": a.count} for a in arr[:n.value]]
