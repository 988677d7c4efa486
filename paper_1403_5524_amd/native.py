"""ctypes binding of librmatrix (include/rmatrix.h), same names as the C ABI.

Argument marshalling only: every step of the sweep runs in the HIP kernels.
PyTorch supplies device memory and the current stream.  If the shared
library is missing the import fails loudly; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librmatrix.so")

RM_OK, RM_ERR_ARG, RM_ERR_NOMEM, RM_ERR_HIP, RM_ERR_NUMERIC, RM_ERR_STATE = \
    range(6)
RM_PREC_FP64, RM_PREC_FP32, RM_PREC_BF16X3 = 0, 1, 2
RM_E_NO_OPEN = 0x01
RM_E_SINGULAR = 0x02
RM_E_CF_NOCONV = 0x04
RM_E_NONFINITE = 0x08
RM_E_ON_THRESHOLD = 0x10
RM_E_REFINE_NOCONV = 0x20
RM_E_ASYM_NOCONV = 0x40
RM_FLAG_AUTOTUNE = 0x1
RM_FLAG_NO_PAIR_PRODUCTS = 0x2
RM_FLAG_PAIR_PRODUCTS = 0x4
RM_FLAG_RADIATION_DAMPING = 0x8

EXPORTED = ("rm_load_poles", "rm_free", "rm_sym_info", "rm_sweep_energies",
            "rm_sweep_energies_noalloc",
            "rm_kmatrix", "rm_collision_strengths", "rm_rmatrix",
            "rm_channel_functions", "rm_profile", "rm_profile_query",
            "rm_mlp_create", "rm_mlp_free", "rm_mlp_n_params",
            "rm_mlp_get_params", "rm_mlp_set_params", "rm_mlp_forward",
            "rm_mlp_grad", "rm_mlp_adam_step", "rm_mesh_from_density",
            "rm_plan_create", "rm_plan_execute", "rm_plan_info",
            "rm_plan_free", "rm_set_propagation", "rm_set_gailitis",
            "rm_load_dipoles",
            "rm_load_widths",
            "rm_photoionization",
            "rm_convolve_gaussian",
            "rm_effective_collision_strengths",
            "rm_group_collision_strengths", "rm_inner_region",
            "rm_inner_region_batch", "rm_last_error")


class RmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("rmatrix error %d: %s" % (code, msg))
        self.code = code


class PolesDesc(ctypes.Structure):
    _fields_ = [("n_chan", ctypes.c_int32), ("n_poles", ctypes.c_int32),
                ("E_pole", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("a", ctypes.c_double), ("e_thr", ctypes.c_void_p),
                ("l", ctypes.c_void_p), ("target", ctypes.c_void_p),
                ("z", ctypes.c_double), ("g", ctypes.c_double)]


class InnerDesc(ctypes.Structure):
    _fields_ = [("n_chan", ctypes.c_int32), ("n_basis", ctypes.c_int32),
                ("n_quad", ctypes.c_int32), ("a", ctypes.c_double),
                ("z", ctypes.c_double), ("e_thr", ctypes.c_void_p),
                ("l", ctypes.c_void_p), ("depth", ctypes.c_void_p),
                ("range", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("near_delta", ctypes.c_double),
                ("solve_fp32", ctypes.c_int32),
                ("refine_iters", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("band_delta", ctypes.c_double)]


_lib = None


def lib():
    """Load librmatrix.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("librmatrix.so not built: run "
                              "python -c 'import __graft_entry__ as g; g.build()'")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.rm_load_poles.argtypes = [ctypes.POINTER(PolesDesc),
                                    ctypes.POINTER(vp), vp]
        L.rm_free.argtypes = [vp]
        L.rm_sym_info.argtypes = [vp, vp, vp, vp]
        L.rm_sweep_energies.argtypes = [vp, i32, i32, vp, i64,
                                        ctypes.POINTER(Opts), vp, vp, vp]
        L.rm_sweep_energies_noalloc.argtypes = [vp, i32, i32, vp, i64,
                                                ctypes.POINTER(Opts), vp, vp,
                                                vp]
        L.rm_kmatrix.argtypes = [vp, vp, i64, ctypes.POINTER(Opts), vp, vp,
                                 vp, vp, vp]
        L.rm_collision_strengths.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp]
        L.rm_rmatrix.argtypes = [vp, vp, i64, ctypes.POINTER(Opts), vp, vp]
        L.rm_channel_functions.argtypes = [vp, vp, i64, vp, vp, vp]
        L.rm_profile.argtypes = [i32]
        L.rm_profile_query.argtypes = [i32, vp, vp]
        f32, f64, u64 = ctypes.c_float, ctypes.c_double, ctypes.c_uint64
        L.rm_mlp_create.argtypes = [i32, i32, i32, i32, u64, ctypes.POINTER(vp)]
        L.rm_mlp_free.argtypes = [vp]
        L.rm_mlp_n_params.argtypes = [vp, ctypes.POINTER(i64)]
        L.rm_mlp_get_params.argtypes = [vp, vp, vp]
        L.rm_mlp_set_params.argtypes = [vp, vp, vp]
        L.rm_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
        L.rm_mlp_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
        L.rm_mlp_adam_step.argtypes = [vp, f32, f32, f32, f32, vp]
        L.rm_mesh_from_density.argtypes = [vp, i32, f64, f64, f64, i64, vp, vp]
        L.rm_plan_create.argtypes = [vp, i32, i32, vp, i64,
                                     ctypes.POINTER(Opts), vp, vp, vp,
                                     ctypes.POINTER(vp)]
        L.rm_plan_execute.argtypes = [vp, vp]
        L.rm_plan_info.argtypes = [vp, vp, vp, vp, i32]
        L.rm_plan_free.argtypes = [vp]
        L.rm_set_propagation.argtypes = [vp, f64, i32, i32, vp, vp]
        L.rm_set_gailitis.argtypes = [vp, i32, vp]
        L.rm_load_dipoles.argtypes = [vp, vp, vp]
        L.rm_load_widths.argtypes = [vp, vp, vp]
        L.rm_photoionization.argtypes = [vp, i32, vp, i64, f64,
                                         ctypes.POINTER(Opts), vp, vp, vp]
        L.rm_convolve_gaussian.argtypes = [vp, i64, vp, i64, f64, vp, vp]
        L.rm_effective_collision_strengths.argtypes = [vp, i64, vp, i32, vp,
                                                       vp, i32, vp, vp]
        L.rm_group_collision_strengths.argtypes = [vp, i64, i32, vp, i32, vp,
                                                   vp]
        L.rm_inner_region.argtypes = [ctypes.POINTER(InnerDesc), vp, vp, vp,
                                      vp, vp]
        L.rm_inner_region_batch.argtypes = [ctypes.POINTER(InnerDesc), i32,
                                            vp, vp, vp, vp, vp]
        L.rm_last_error.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name != "rm_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code):
    if code != RM_OK:
        raise RmError(code, lib().rm_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, numel=None, name="tensor", optional=False):
    """Device pointer of ``t`` after checking what the C ABI cannot: a torch
    tensor of the given dtype, contiguous, with ``numel`` elements (when
    given), on a GPU.  Raises RmError(RM_ERR_ARG) before any library call
    otherwise; ``optional`` admits None (a NULL pointer)."""
    import torch
    if t is None:
        if optional:
            return None
        raise RmError(RM_ERR_ARG, "%s must be a tensor" % name)
    if not isinstance(t, torch.Tensor):
        raise RmError(RM_ERR_ARG, "%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise RmError(RM_ERR_ARG, "%s must be %s, got %s" % (name, dtype,
                                                             t.dtype))
    if not t.is_contiguous():
        raise RmError(RM_ERR_ARG, "%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise RmError(RM_ERR_ARG, "%s must hold %d elements, got %d"
                      % (name, numel, t.numel()))
    if not t.is_cuda:
        raise RmError(RM_ERR_ARG, "%s must be on a GPU" % name)
    return ctypes.c_void_p(t.data_ptr())


def _f64(t, numel=None, name="tensor", optional=False):
    import torch
    return _dev(t, torch.float64, numel, name, optional)


def _i32(t, numel=None, name="tensor", optional=False):
    import torch
    return _dev(t, torch.int32, numel, name, optional)


def _f32(t, numel=None, name="tensor", optional=False):
    import torch
    return _dev(t, torch.float32, numel, name, optional)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_opts(prec=RM_PREC_FP64, near_delta=0.0, solve_fp32=0, refine_iters=0,
              chunk=0, flags=0, band_delta=0.0):
    return Opts(prec, near_delta, solve_fp32, refine_iters, chunk, flags,
                band_delta)


class Symmetry:
    """A loaded symmetry (rm_sym_t); freed with rm_free when released."""

    def __init__(self, handle, n, n_poles, n_target):
        self.handle = handle
        self.n = n
        self.n_poles = n_poles
        self.n_target = n_target

    def free(self):
        if self.handle:
            lib().rm_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def rm_load_poles(E_pole, w, a, e_thr, l, z, g, target=None, stream=None):
    """Host numpy arrays in, device-resident handle out."""
    E_pole = np.ascontiguousarray(E_pole, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    e_thr = np.ascontiguousarray(e_thr, dtype=np.float64)
    l = np.ascontiguousarray(l, dtype=np.int32)
    tg = None if target is None else np.ascontiguousarray(target,
                                                          dtype=np.int32)
    n = int(e_thr.size)
    nh = int(E_pole.size)
    if w.size != n * nh:
        raise RmError(RM_ERR_ARG, "w must hold n_chan*n_poles values")
    d = PolesDesc(n, nh, E_pole.ctypes.data, w.ctypes.data, float(a),
                  e_thr.ctypes.data, l.ctypes.data,
                  None if tg is None else tg.ctypes.data, float(z), float(g))
    h = ctypes.c_void_p()
    st = _stream() if stream is None else stream
    _check(lib().rm_load_poles(ctypes.byref(d), ctypes.byref(h), st))
    nt = ctypes.c_int32()
    _check(lib().rm_sym_info(h, None, None, ctypes.byref(nt)))
    return Symmetry(h, n, nh, int(nt.value))


def load_symmetry(sym):
    """Load a workloads.Symmetry (or mapping with the same keys)."""
    d = sym.as_dict() if hasattr(sym, "as_dict") else sym
    return rm_load_poles(d["E_pole"], d["w"], d["a"], d["e_thr"], d["l"],
                         d["z"], d["g"], d.get("target"))


def rm_sweep_energies(syms, n_target, E, opts=None, omega=None, status=None):
    """E: CUDA float64 tensor [M].  Returns (omega [M, P], status [M])."""
    import torch
    pE = _f64(E, name="E")
    M = int(E.numel())
    P = n_target * (n_target + 1) // 2
    if omega is None:
        omega = torch.empty((M, P), dtype=torch.float64, device=E.device)
    if status is None:
        status = torch.empty((M,), dtype=torch.int32, device=E.device)
    po = _f64(omega, M * P, "omega")
    ps = _i32(status, M, "status")
    arr = (ctypes.c_void_p * len(syms))(*[s.handle for s in syms])
    o = opts if opts is not None else make_opts()
    _check(lib().rm_sweep_energies(arr, len(syms), n_target, pE, M,
                                   ctypes.byref(o), po, ps, _stream()))
    return omega, status


def rm_sweep_energies_noalloc(syms, n_target, E, omega, status, opts=None):
    """rm_sweep_energies with no device allocation inside the library: the
    caller passes E [M], omega [M, P] and status [M] (CUDA tensors)."""
    pE = _f64(E, name="E")
    M = int(E.numel())
    P = n_target * (n_target + 1) // 2
    po = _f64(omega, M * P, "omega")
    ps = _i32(status, M, "status")
    arr = (ctypes.c_void_p * len(syms))(*[s.handle for s in syms])
    o = opts if opts is not None else make_opts()
    _check(lib().rm_sweep_energies_noalloc(arr, len(syms), n_target, pE, M,
                                           ctypes.byref(o), po, ps,
                                           _stream()))
    return omega, status


def rm_kmatrix(sym, E, opts=None, want_R=False):
    """Returns (K [m, n, n], n_open [m], R [m, n, n] or None, status [m])."""
    import torch
    pE = _f64(E, name="E")
    m, n = int(E.numel()), sym.n
    K = torch.empty((m, n, n), dtype=torch.float64, device=E.device)
    no = torch.empty((m,), dtype=torch.int32, device=E.device)
    st = torch.empty((m,), dtype=torch.int32, device=E.device)
    R = torch.empty((m, n, n), dtype=torch.float64, device=E.device) \
        if want_R else None
    o = opts if opts is not None else make_opts()
    _check(lib().rm_kmatrix(sym.handle, pE, m, ctypes.byref(o), _ptr(K),
                            _ptr(no), _ptr(R), _ptr(st), _stream()))
    return K, no, R, st


def rm_collision_strengths(sym, K, n_open, E, n_target, omega):
    """Accumulates into omega [m, P] (device float64)."""
    pE = _f64(E, name="E")
    m = int(E.numel())
    P = n_target * (n_target + 1) // 2
    pK = _f64(K, m * sym.n * sym.n, "K")
    pn = _i32(n_open, m, "n_open")
    po = _f64(omega, m * P, "omega")
    _check(lib().rm_collision_strengths(sym.handle, pK, pn, pE, m, n_target,
                                        po, _stream()))
    return omega


def rm_rmatrix(sym, E, opts=None):
    import torch
    pE = _f64(E, name="E")
    m, n = int(E.numel()), sym.n
    R = torch.empty((m, n, n), dtype=torch.float64, device=E.device)
    o = opts if opts is not None else make_opts()
    _check(lib().rm_rmatrix(sym.handle, pE, m, ctypes.byref(o), _ptr(R),
                            _stream()))
    return R


def rm_channel_functions(sym, E):
    """Returns (out [m, n, 4], status [m])."""
    import torch
    pE = _f64(E, name="E")
    m, n = int(E.numel()), sym.n
    out = torch.empty((m, n, 4), dtype=torch.float64, device=E.device)
    st = torch.empty((m,), dtype=torch.int32, device=E.device)
    _check(lib().rm_channel_functions(sym.handle, pE, m, _ptr(out),
                                      _ptr(st), _stream()))
    return out, st


STAGES = {"chanfn": 0, "polesum": 1, "match": 2, "graph": 3, "convolve": 4,
          "upsilon": 5, "group": 6, "propagate": 7, "jacobi": 8,
          "assemble": 9}


def rm_profile(enable):
    _check(lib().rm_profile(1 if enable else 0))


def rm_profile_query(stage):
    """(total_ms, launches) of a stage recorded since rm_profile(1)."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().rm_profile_query(STAGES.get(stage, stage), ctypes.byref(ms),
                                  ctypes.byref(n)))
    return ms.value, n.value


class Mlp:
    """Device MLP handle (rm_mlp_t)."""

    def __init__(self, d_in, width=256, n_layers=4, prec=0, seed=0):
        h = ctypes.c_void_p()
        _check(lib().rm_mlp_create(d_in, width, n_layers, prec, seed,
                                   ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int64()
        _check(lib().rm_mlp_n_params(h, ctypes.byref(n)))
        self.n_params = int(n.value)
        self.d_in, self.width, self.n_layers = d_in, width, n_layers

    def free(self):
        if self.handle:
            lib().rm_mlp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def get_params(self):
        import torch
        out = torch.empty((self.n_params,), dtype=torch.float32, device="cuda")
        _check(lib().rm_mlp_get_params(self.handle, _ptr(out), _stream()))
        return out

    def set_params(self, p):
        pp = _f32(p, self.n_params, "params")
        _check(lib().rm_mlp_set_params(self.handle, pp, _stream()))

    def forward(self, X):
        import torch
        B = int(X.shape[0]) if X is not None and X.dim() > 0 else 0
        pX = _f32(X, B * self.d_in, "X")
        Y = torch.empty((B,), dtype=torch.float32, device=X.device)
        _check(lib().rm_mlp_forward(self.handle, pX, B, _ptr(Y), _stream()))
        return Y

    def grad(self, X, target, want_grad=False):
        import torch
        B = int(X.shape[0]) if X is not None and X.dim() > 0 else 0
        _f32(X, B * self.d_in, "X")
        _f32(target, B, "target")
        loss = torch.empty((1,), dtype=torch.float32, device=X.device)
        g = torch.empty((self.n_params,), dtype=torch.float32,
                        device=X.device) if want_grad else None
        _check(lib().rm_mlp_grad(self.handle, _ptr(X), _ptr(target),
                                 int(X.shape[0]), _ptr(loss), _ptr(g),
                                 _stream()))
        return loss, g

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().rm_mlp_adam_step(self.handle, lr, beta1, beta2, eps,
                                      _stream()))


def rm_mesh_from_density(dens, lo, hi, floor_frac, M):
    import torch
    pd = _f32(dens, name="dens")
    E = torch.empty((M,), dtype=torch.float64, device=dens.device)
    _check(lib().rm_mesh_from_density(pd, int(dens.numel()), lo, hi,
                                      floor_frac, M, _ptr(E), _stream()))
    return E


class Plan:
    """rm_plan_t: a sweep captured into a hipGraph, bound to E/omega/status."""

    def __init__(self, syms, n_target, E, opts=None, omega=None, status=None):
        import torch
        self.handle = None
        _f64(E, name="E")
        M = int(E.numel())
        P = n_target * (n_target + 1) // 2
        self.E = E
        self.omega = omega if omega is not None else torch.empty(
            (M, P), dtype=torch.float64, device=E.device)
        self.status = status if status is not None else torch.empty(
            (M,), dtype=torch.int32, device=E.device)
        _f64(self.omega, M * P, "omega")
        _i32(self.status, M, "status")
        self._syms = list(syms)
        arr = (ctypes.c_void_p * len(syms))(*[s.handle for s in syms])
        o = opts if opts is not None else make_opts()
        h = ctypes.c_void_p()
        _check(lib().rm_plan_create(arr, len(syms), n_target, _ptr(E), M,
                                    ctypes.byref(o), _ptr(self.omega),
                                    _ptr(self.status), _stream(),
                                    ctypes.byref(h)))
        self.handle = h

    def execute(self):
        _check(lib().rm_plan_execute(self.handle, _stream()))
        return self.omega, self.status

    def info(self):
        c = ctypes.c_int64()
        nc = ctypes.c_int32()
        v = (ctypes.c_int32 * len(self._syms))()
        _check(lib().rm_plan_info(self.handle, ctypes.byref(c),
                                  ctypes.byref(nc), v, len(self._syms)))
        return int(c.value), int(nc.value), list(v)

    def free(self):
        if self.handle:
            lib().rm_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def rm_convolve_gaussian(E, omega, fwhm, out=None):
    """Gaussian smoothing of omega [M, P] (CUDA float64) on the mesh E [M]."""
    import torch
    if not isinstance(omega, torch.Tensor) or omega.dim() != 2:
        raise RmError(RM_ERR_ARG, "omega must be a [M, P] tensor")
    M, P = int(omega.shape[0]), int(omega.shape[1])
    pi = _f64(omega, M * P, "omega")
    pE = _f64(E, M, "E")
    if out is None:
        out = torch.empty_like(omega)
    po = _f64(out, M * P, "out")
    _check(lib().rm_convolve_gaussian(pE, M, pi, P, float(fwhm), po,
                                      _stream()))
    return out


def rm_effective_collision_strengths(E, omega, e_level, n_target, kT):
    """Upsilon [P, nT] (CUDA float64) from omega [M, P]; e_level and kT are
    host sequences."""
    import torch
    lev = np.ascontiguousarray(e_level, dtype=np.float64)
    t = np.ascontiguousarray(np.atleast_1d(kT), dtype=np.float64)
    if lev.size != n_target:
        raise RmError(RM_ERR_ARG, "e_level must hold n_target values")
    P = n_target * (n_target + 1) // 2
    if not isinstance(omega, torch.Tensor) or omega.dim() != 2:
        raise RmError(RM_ERR_ARG, "omega must be a [M, P] tensor")
    M = int(omega.shape[0])
    pom = _f64(omega, M * P, "omega")
    pE = _f64(E, M, "E")
    ups = torch.empty((P, t.size), dtype=torch.float64, device=omega.device)
    _check(lib().rm_effective_collision_strengths(
        pE, M, pom, int(n_target),
        lev.ctypes.data, t.ctypes.data, int(t.size), _ptr(ups), _stream()))
    return ups


def rm_group_collision_strengths(omega, n_target, group, n_group):
    """Omega summed over the level pairs of level groups: [M, Pg]."""
    import torch
    g = np.ascontiguousarray(group, dtype=np.int32)
    if g.size != n_target:
        raise RmError(RM_ERR_ARG, "group must hold n_target values")
    Pg = n_group * (n_group + 1) // 2
    if not isinstance(omega, torch.Tensor) or omega.dim() != 2:
        raise RmError(RM_ERR_ARG, "omega must be a [M, P] tensor")
    M = int(omega.shape[0])
    pom = _f64(omega, M * (n_target * (n_target + 1) // 2), "omega")
    out = torch.empty((M, Pg), dtype=torch.float64, device=omega.device)
    _check(lib().rm_group_collision_strengths(
        pom, M, int(n_target), g.ctypes.data,
        int(n_group), _ptr(out), _stream()))
    return out


def rm_load_dipoles(sym, d):
    """Attach the dipole vector d [n_poles] (host) to a loaded symmetry."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    if d.size != sym.n_poles:
        raise RmError(RM_ERR_ARG, "d must hold n_poles values")
    _check(lib().rm_load_dipoles(sym.handle, d.ctypes.data, _stream()))


def rm_load_widths(sym, gamma):
    """Attach the radiative widths Gamma_k [n_poles] (host, >= 0) to a
    loaded symmetry for the damped photoionization."""
    g = np.ascontiguousarray(gamma, dtype=np.float64)
    if g.size != sym.n_poles:
        raise RmError(RM_ERR_ARG, "gamma must hold n_poles values")
    _check(lib().rm_load_widths(sym.handle, g.ctypes.data, _stream()))


def rm_photoionization(syms, E, e0, opts=None, sigma=None, status=None):
    """sigma [M] in Mb (CUDA float64) and status [M] at the energies E."""
    import torch
    pE = _f64(E, name="E")
    M = int(E.numel())
    if sigma is None:
        sigma = torch.empty((M,), dtype=torch.float64, device=E.device)
    if status is None:
        status = torch.empty((M,), dtype=torch.int32, device=E.device)
    psg = _f64(sigma, M, "sigma")
    pst = _i32(status, M, "status")
    arr = (ctypes.c_void_p * len(syms))(*[s.handle for s in syms])
    o = opts if opts is not None else make_opts()
    _check(lib().rm_photoionization(arr, len(syms), pE, M, float(e0),
                                    ctypes.byref(o), psg, pst, _stream()))
    return sigma, status


def _inner_desc(model, n_basis, n_quad):
    """(InnerDesc, kept arrays, n) for one model dict."""
    e = np.ascontiguousarray(model["e_thr"], dtype=np.float64)
    n = e.size
    l = np.ascontiguousarray(model["l"], dtype=np.int32)
    dep = np.ascontiguousarray(model["depth"], dtype=np.float64)
    rng = np.ascontiguousarray(model["range"], dtype=np.float64)
    if l.shape != (n,) or dep.shape != (n, n) or rng.shape != (n, n):
        raise RmError(RM_ERR_ARG, "model arrays must be [n], [n], [n, n], [n, n]")
    d = InnerDesc(n, int(n_basis), int(n_quad), float(model["a"]),
                  float(model["z"]), e.ctypes.data, l.ctypes.data,
                  dep.ctypes.data, rng.ctypes.data)
    return d, (e, l, dep, rng), n


def rm_inner_region(model, n_basis, n_quad=0):
    """Poles and amplitudes of the model inner-region Hamiltonian (all
    eigenpairs on the device).  model: dict with e_thr [n], l [n], z, a,
    depth [n, n], range [n, n].  Returns (E_pole [n N] ascending, w [n, n N],
    sweeps, rotations), host arrays and counts."""
    d, keep, n = _inner_desc(model, n_basis, n_quad)
    D = n * int(n_basis)
    E = np.zeros(max(D, 0))
    w = np.zeros((n, max(D, 0)))
    sweeps = ctypes.c_int32(0)
    rot = ctypes.c_int64(0)
    _check(lib().rm_inner_region(ctypes.byref(d), E.ctypes.data, w.ctypes.data,
                                 ctypes.byref(sweeps), ctypes.byref(rot),
                                 _stream()))
    return E, w, sweeps.value, rot.value


def rm_inner_region_batch(models, n_basis, n_quad=None):
    """rm_inner_region for several models at once (concurrent on the
    device).  n_basis (and n_quad): one value or one per model.  Returns a
    list of (E_pole, w, sweeps, rotations)."""
    k = len(models)
    nb = list(n_basis) if hasattr(n_basis, "__len__") else [n_basis] * k
    nq = (list(n_quad) if hasattr(n_quad, "__len__")
          else [n_quad or 0] * k)
    descs = (InnerDesc * max(k, 1))()
    keep, Es, ws = [], [], []
    for b, m in enumerate(models):
        d, arrs, n = _inner_desc(m, nb[b], nq[b])
        descs[b] = d
        keep.append(arrs)
        D = n * int(nb[b])
        Es.append(np.zeros(max(D, 0)))
        ws.append(np.zeros((n, max(D, 0))))
    pE = (ctypes.c_void_p * max(k, 1))(*[E.ctypes.data for E in Es])
    pw = (ctypes.c_void_p * max(k, 1))(*[w.ctypes.data for w in ws])
    sw = np.zeros(max(k, 1), dtype=np.int32)
    rot = np.zeros(max(k, 1), dtype=np.int64)
    _check(lib().rm_inner_region_batch(descs, k, pE, pw, sw.ctypes.data,
                                       rot.ctypes.data, _stream()))
    return [(Es[b], ws[b], int(sw[b]), int(rot[b])) for b in range(k)]


def rm_set_propagation(sym, A, n_sec, beta=None):
    """Propagate sym's R-matrix from a to A through n_sec sectors of the
    multipole coupling beta [lmax, n, n] (host; None: no multipoles)."""
    if beta is None:
        beta = np.zeros((0, sym.n, sym.n))
    b = np.ascontiguousarray(beta, dtype=np.float64)
    if b.ndim != 3 or b.shape[1:] != (sym.n, sym.n):
        raise RmError(RM_ERR_ARG, "beta must be [lmax, n, n]")
    _check(lib().rm_set_propagation(sym.handle, float(A), int(n_sec),
                                    int(b.shape[0]),
                                    b.ctypes.data if b.size else None,
                                    _stream()))


def rm_set_gailitis(sym, max_terms):
    """Match sym at A to the coupled asymptotic expansion (at most max_terms
    terms per channel; 0 switches it off); needs rm_set_propagation."""
    _check(lib().rm_set_gailitis(sym.handle if sym is not None else None,
                                 int(max_terms), _stream()))
