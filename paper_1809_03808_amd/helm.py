"""ctypes binding of libhelm.so (C ABI in include/helm.h).

Argument marshalling only: every step of a solve runs in the HIP library.
Device arrays are torch tensors (complex128, contiguous, on the plan's
device); their data_ptr() and the current torch stream are passed through.
If the library has not been built, ``lib()`` raises: there is no fallback.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelm.so")

HELM_OK = 0
HELM_EINVAL = -1
HELM_ENOMEM = -2
HELM_EDEVICE = -3
HELM_ESINGULAR = -4
HELM_ENOCONV = -5
HELM_ENONFINITE = -6
HELM_EUNSUPPORTED = -7

PREC_FP64 = 0
PREC_MIXED = 1
TRANSFORM_AUTO = 0
TRANSFORM_FFT = 1
TRANSFORM_DENSE = 2
DENSE_MAX = 1024
BOUNDARY_AUTO = 0
BOUNDARY_LINES = 1
BOUNDARY_TABLES = 2
EIGEN_AUTO = 0
EIGEN_HOST = 1
EIGEN_DEVICE = 2

# Every symbol declared in include/helm.h.
EXPORTS = (
    "helm_default_options", "helm_setup", "helm_solve", "helm_report_get",
    "helm_residual", "helm_destroy", "helm_strerror", "helm_eig1d", "helm_eig1d_device",
    "helm_setup_general",
    "helm_profile", "helm_kernel_stats_get", "helm_kernel_name",
    "helm_batch_create", "helm_batch_solve", "helm_batch_report_get", "helm_batch_destroy",
    "helm_solve_static",
)

STATIC_SCRATCH_BYTES = 128 << 20
STATIC_MAX_RHS = 1024

NKERNELS = 9


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("check", ctypes.c_int),
                ("transform", ctypes.c_int), ("tune_cache", ctypes.c_char_p),
                ("boundary", ctypes.c_int), ("eigen", ctypes.c_int)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int),
                ("precision", ctypes.c_int), ("nrhs", ctypes.c_int),
                ("rel_residual_max", ctypes.c_double),
                ("rel_residual_first", ctypes.c_double),
                ("transform", ctypes.c_int), ("boundary", ctypes.c_int)]


class KernelStats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 9), ("bytes", ctypes.c_double * 9),
                ("calls", ctypes.c_int * 9)]


class HelmError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def lib():
    """Load libhelm.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} not found: build it with `python -m paper_1809_03808_amd.build`")
    # The library shares the process's HIP runtime with PyTorch (device
    # tensors are passed to it): PyTorch loaded first, the library binds to
    # the runtime PyTorch brought in instead of loading a second copy, which
    # would leave PyTorch without a device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
    L.helm_default_options.argtypes = [ctypes.POINTER(Options)]
    L.helm_default_options.restype = None
    L.helm_setup.argtypes = [ctypes.c_int, i64p, dp, ctypes.c_double, ctypes.c_uint32,
                             ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.helm_setup.restype = ctypes.c_int
    L.helm_setup_general.argtypes = [ctypes.c_int, i64p, dp, ctypes.c_double, dp,
                                     ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.helm_setup_general.restype = ctypes.c_int
    L.helm_solve.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    L.helm_solve.restype = ctypes.c_int
    L.helm_solve_static.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    L.helm_solve_static.restype = ctypes.c_int
    L.helm_report_get.argtypes = [vp, ctypes.POINTER(Report)]
    L.helm_report_get.restype = ctypes.c_int
    L.helm_residual.argtypes = [vp, vp, vp, vp, dp, ctypes.c_int, vp]
    L.helm_residual.restype = ctypes.c_int
    L.helm_destroy.argtypes = [vp]
    L.helm_destroy.restype = None
    L.helm_strerror.argtypes = [ctypes.c_int]
    L.helm_strerror.restype = ctypes.c_char_p
    L.helm_eig1d.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, dp, dp]
    L.helm_eig1d.restype = ctypes.c_int
    L.helm_eig1d_device.argtypes = L.helm_eig1d.argtypes
    L.helm_eig1d_device.restype = ctypes.c_int
    L.helm_profile.argtypes = [vp, ctypes.c_int]
    L.helm_profile.restype = ctypes.c_int
    L.helm_kernel_stats_get.argtypes = [vp, ctypes.POINTER(KernelStats), ctypes.c_int]
    L.helm_kernel_stats_get.restype = ctypes.c_int
    L.helm_kernel_name.argtypes = [ctypes.c_int]
    L.helm_kernel_name.restype = ctypes.c_char_p
    L.helm_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    L.helm_batch_create.restype = ctypes.c_int
    L.helm_batch_solve.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int), vp]
    L.helm_batch_solve.restype = ctypes.c_int
    L.helm_batch_report_get.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Report)]
    L.helm_batch_report_get.restype = ctypes.c_int
    L.helm_batch_destroy.argtypes = [vp]
    L.helm_batch_destroy.restype = None
    _lib = L
    return L


def strerror(code):
    return lib().helm_strerror(int(code)).decode()


def abc_mask(abc):
    """Per-axis (lo, hi) booleans -> face bit mask (bit 2j low, 2j+1 high)."""
    m = 0
    for j, (lo, hi) in enumerate(abc):
        m |= (1 if lo else 0) << (2 * j)
        m |= (1 if hi else 0) << (2 * j + 1)
    return m


def eig1d(n, h, omega, abc_lo=True, abc_hi=True, device=False):
    """Absorbing-boundary eigen-setup (helm_eig1d on the host, or
    helm_eig1d_device on the current HIP device): (lambda[n] complex,
    vb[2][n] complex)."""
    lam = np.zeros(2 * n)
    vb = np.zeros(4 * n)
    fn = lib().helm_eig1d_device if device else lib().helm_eig1d
    rc = fn(int(n), float(h), float(omega), int(bool(abc_lo)), int(bool(abc_hi)),
            lam.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            vb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != HELM_OK:
        raise HelmError(rc, "helm_eig1d_device" if device else "helm_eig1d")
    lam = lam.view(np.complex128)
    vb = vb.view(np.complex128).reshape(2, n)
    return lam, vb


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_tensor(t, grid, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA/HIP tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape[-len(grid):]) != tuple(grid):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, grid is {tuple(grid)}")
    return 1 if t.dim() == len(grid) else int(np.prod(t.shape[:-len(grid)]))


def face_coefficients(omega, faces):
    """gamma array of helm_setup_general from per-axis (lo, hi) faces: a
    boolean face is absorbing (g = -i omega) or Neumann (g = 0), a number is
    the Robin coefficient g itself."""
    out = []
    for pair in faces:
        for face in pair:
            if isinstance(face, (bool, np.bool_)):
                g = complex(0.0, -omega) if face else 0j
            else:
                g = complex(face)
            out += [g.real, g.imag]
    return out


class Plan:
    """A solver plan: ``Plan(grid, h, omega, abc)`` then ``plan.solve(f, u)``.
    With ``c`` given, or ``abc`` holding numeric faces, the plan is built by
    helm_setup_general for -Lap u - c u = f with du/dn + g u = 0 on each face
    (c defaults to omega^2, boolean faces as in helm_setup)."""

    def __init__(self, grid, h, omega, abc=None, precision=PREC_FP64, tol=1e-10, max_iter=8,
                 check=True, transform=None, tune_cache=None, boundary=None, eigen=None, c=None):
        L = lib()
        self.grid = tuple(int(n) for n in grid)
        self.dim = len(self.grid)
        self.h = tuple(float(x) for x in h)
        self.omega = float(omega)
        if abc is None:
            abc = (1 << (2 * self.dim)) - 1
        general = c is not None or (not isinstance(abc, int) and any(
            not isinstance(f, (bool, np.bool_)) for pair in abc for f in pair))
        if general:
            faces = abc if not isinstance(abc, int) else [
                (bool((abc >> (2 * j)) & 1), bool((abc >> (2 * j + 1)) & 1)) for j in range(self.dim)]
            self.faces = tuple(tuple(p) for p in faces)
            self.c = float(self.omega ** 2 if c is None else c)
            self.abc = None
        else:
            self.abc = abc if isinstance(abc, int) else abc_mask(abc)
            self.faces = None
            self.c = self.omega ** 2
        opt = Options()
        L.helm_default_options(ctypes.byref(opt))
        opt.precision = int(precision)
        opt.tol = float(tol)
        opt.max_iter = int(max_iter)
        opt.check = int(bool(check))
        if transform is not None:
            opt.transform = int(transform)
        if boundary is not None:
            opt.boundary = int(boundary)
        if eigen is not None:
            opt.eigen = int(eigen)
        self._tune = tune_cache.encode() if tune_cache else None
        opt.tune_cache = self._tune
        g = (ctypes.c_int64 * self.dim)(*self.grid)
        hh = (ctypes.c_double * self.dim)(*self.h)
        out = ctypes.c_void_p()
        if general:
            gam = (ctypes.c_double * (4 * self.dim))(*face_coefficients(self.omega, self.faces))
            rc = L.helm_setup_general(self.dim, g, hh, self.c, gam, ctypes.byref(opt), ctypes.byref(out))
        else:
            rc = L.helm_setup(self.dim, g, hh, self.omega, ctypes.c_uint32(self.abc), ctypes.byref(opt),
                              ctypes.byref(out))
        if rc != HELM_OK:
            raise HelmError(rc, "helm_setup")
        self._p = out

    def solve(self, f, u, stream=None, raise_on_error=True):
        """u = A^{-1} f (device tensors [nrhs][grid] or [grid]).  Returns the status."""
        nrhs = _check_tensor(f, self.grid, "f")
        if _check_tensor(u, self.grid, "u") != nrhs:
            raise ValueError("f and u hold different numbers of right-hand sides")
        rc = lib().helm_solve(self._p, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                              nrhs, _stream_ptr(stream))
        if rc != HELM_OK and raise_on_error:
            raise HelmError(rc, "helm_solve")
        return rc

    def solve_static(self, f, u, stream=None, raise_on_error=True):
        """helm_solve_static: the same solve with the library's static device
        workspace (nothing allocated).  Returns the status."""
        nrhs = _check_tensor(f, self.grid, "f")
        if _check_tensor(u, self.grid, "u") != nrhs:
            raise ValueError("f and u hold different numbers of right-hand sides")
        rc = lib().helm_solve_static(self._p, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                     nrhs, _stream_ptr(stream))
        if rc != HELM_OK and raise_on_error:
            raise HelmError(rc, "helm_solve_static")
        return rc

    def report(self):
        r = Report()
        rc = lib().helm_report_get(self._p, ctypes.byref(r))
        if rc != HELM_OK:
            raise HelmError(rc, "helm_report_get")
        return {k: getattr(r, k) for k, _ in Report._fields_}

    def residual(self, u, f, r=None, stream=None):
        """FP64 r = f - A u on the device; returns per-RHS ||r||/||f||."""
        nrhs = _check_tensor(f, self.grid, "f")
        _check_tensor(u, self.grid, "u")
        if r is not None:
            _check_tensor(r, self.grid, "r")
        rel = np.zeros(nrhs)
        rc = lib().helm_residual(self._p, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                 ctypes.c_void_p(r.data_ptr() if r is not None else 0),
                                 rel.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nrhs,
                                 _stream_ptr(stream))
        if rc != HELM_OK:
            raise HelmError(rc, "helm_residual")
        return rel

    def profile(self, on=True):
        """Time every kernel launch of later solves with HIP events."""
        rc = lib().helm_profile(self._p, int(bool(on)))
        if rc != HELM_OK:
            raise HelmError(rc, "helm_profile")

    def kernel_stats(self, reset=True):
        """{kernel name: {"ms", "bytes", "calls"}} accumulated since the last reset."""
        st = KernelStats()
        rc = lib().helm_kernel_stats_get(self._p, ctypes.byref(st), int(bool(reset)))
        if rc != HELM_OK:
            raise HelmError(rc, "helm_kernel_stats_get")
        out = {}
        for k in range(NKERNELS):
            name = lib().helm_kernel_name(k)
            if name is None or st.calls[k] == 0:
                continue
            out[name.decode()] = {"ms": st.ms[k], "bytes": st.bytes[k], "calls": st.calls[k]}
        return out

    def close(self):
        if getattr(self, "_p", None):
            lib().helm_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Batch:
    """Independent problems solved by one graph launch.

    ``Batch(plans, max_nrhs)`` then ``batch.solve(fs, us)`` with one
    (f, u) tensor pair per plan.  The plans stay owned by the caller and must
    outlive the batch.
    """

    def __init__(self, plans, max_nrhs=1):
        L = lib()
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._p.value for p in self.plans])
        out = ctypes.c_void_p()
        rc = L.helm_batch_create(arr, len(self.plans), int(max_nrhs), ctypes.byref(out))
        if rc != HELM_OK:
            raise HelmError(rc, "helm_batch_create")
        self._b = out

    def solve(self, fs, us, stream=None, raise_on_error=True):
        n = len(self.plans)
        if len(fs) != n or len(us) != n:
            raise ValueError("one f and one u per plan")
        nr = []
        for p, f, u in zip(self.plans, fs, us):
            k = _check_tensor(f, p.grid, "f")
            if _check_tensor(u, p.grid, "u") != k:
                raise ValueError("f and u hold different numbers of right-hand sides")
            nr.append(k)
        fa = (ctypes.c_void_p * n)(*[f.data_ptr() for f in fs])
        ua = (ctypes.c_void_p * n)(*[u.data_ptr() for u in us])
        na = (ctypes.c_int * n)(*nr)
        rc = lib().helm_batch_solve(self._b, fa, ua, na, _stream_ptr(stream))
        if rc != HELM_OK and raise_on_error:
            raise HelmError(rc, "helm_batch_solve")
        return rc

    def report(self, i):
        r = Report()
        rc = lib().helm_batch_report_get(self._b, int(i), ctypes.byref(r))
        if rc != HELM_OK:
            raise HelmError(rc, "helm_batch_report_get")
        return {k: getattr(r, k) for k, _ in Report._fields_}

    def close(self):
        if getattr(self, "_b", None):
            lib().helm_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
