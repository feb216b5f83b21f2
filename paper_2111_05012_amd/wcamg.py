"""Thin ctypes binding of libwcamg (include/wcamg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Arrays may be torch tensors on the GPU (passed as device pointers) or NumPy
arrays on the host (passed as host pointers); outputs are written in place
into caller-provided arrays of the documented canonical layouts.  There is no
CPU fallback: if the shared library is missing, loading raises.
"""
import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'libwcamg.so')

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, ESTATE, ENUMERIC = 0, 1, -1, -2, -3, -4, -5
DEVICE, HOST = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
PC_AMG, PC_BICG32 = 0, 1
SMOOTH_POST, SMOOTH_PRE, SMOOTH_BOTH = 0, 1, 2
BLOCK_MR, BLOCK_EO_MR = 0, 1
MAX_RHS = 64
NOALLOC_SCRATCH_BYTES = 64 << 20

_c_int4 = ctypes.c_int * 4


class Lattice(ctypes.Structure):
    _fields_ = [('dims', _c_int4), ('block', _c_int4), ('bc', _c_int4), ('kappa', ctypes.c_double),
                ('csw', ctypes.c_double)]


class SetupParams(ctypes.Structure):
    _fields_ = [('nv', ctypes.c_int), ('n_init', ctypes.c_int), ('n_adapt', ctypes.c_int),
                ('sap_sweeps', ctypes.c_int), ('mr_iters', ctypes.c_int), ('coarse_iters', ctypes.c_int),
                ('coarse_tol', ctypes.c_double), ('prec', ctypes.c_int), ('init_vectors', ctypes.c_void_p),
                ('init_where', ctypes.c_int), ('nlevels', ctypes.c_int), ('block1', _c_int4), ('nv1', ctypes.c_int),
                ('mr1_iters', ctypes.c_int), ('init_mr1_iters', ctypes.c_int), ('init_vectors1', ctypes.c_void_p),
                ('seed1', ctypes.c_ulonglong), ('init_net', ctypes.c_int), ('seed', ctypes.c_ulonglong),
                ('smoothing', ctypes.c_int), ('sap_eo', ctypes.c_int), ('vec_chunk', ctypes.c_int)]


class SolveParams(ctypes.Structure):
    _fields_ = [('restart', ctypes.c_int), ('tol', ctypes.c_double), ('max_iters', ctypes.c_int),
                ('rhs_chunk', ctypes.c_int), ('use_graph', ctypes.c_int), ('phase_times', ctypes.c_int),
                ('ortho', ctypes.c_int)]


class BicgParams(ctypes.Structure):
    _fields_ = [('tol', ctypes.c_double), ('max_iters', ctypes.c_int), ('rhs_chunk', ctypes.c_int),
                ('precond', ctypes.c_int), ('inner_iters', ctypes.c_int), ('inner_tol', ctypes.c_double),
                ('phase_times', ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [('iters', ctypes.c_int * MAX_RHS), ('relres', ctypes.c_double * MAX_RHS),
                ('converged', ctypes.c_int * MAX_RHS), ('vcycles', ctypes.c_int), ('t_solve', ctypes.c_double),
                ('t_precond', ctypes.c_double), ('t_coarse', ctypes.c_double), ('t_smoother', ctypes.c_double),
                ('t_rp', ctypes.c_double), ('t_prec_other', ctypes.c_double), ('t_outer', ctypes.c_double)]

    def phases(self):
        """The solve's phase split (seconds) as a dict."""
        return {k: getattr(self, k) for k in ('t_solve', 't_precond', 't_coarse', 't_smoother', 't_rp',
                                               't_prec_other', 't_outer')}


class WcamgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__('wcamg error %d: %s' % (code, msg))
        self.code = code


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
SIGNATURES = {
    'wcamg_create': (_I, [ctypes.POINTER(_P), ctypes.POINTER(Lattice), _P]),
    'wcamg_destroy': (None, [_P]),
    'wcamg_last_error': (ctypes.c_char_p, [_P]),
    'wcamg_sync': (_I, [_P]),
    'wcamg_load_gauge': (_I, [_P, _P, _I]),
    'wcamg_load_clover': (_I, [_P, _P, _I]),
    'wcamg_get_clover': (_I, [_P, _P, _I]),
    'wcamg_apply_D': (_I, [_P, _P, _P, _I, _I, _I]),
    'wcamg_apply_D_noalloc': (_I, [_P, _P, _P, _I, _I]),
    'wcamg_apply_Dsap': (_I, [_P, _P, _P, _I, _I, _I]),
    'wcamg_sap': (_I, [_P, _P, _P, _I, _I, _I, _I, _I, _I]),
    'wcamg_setup': (_I, [_P, ctypes.POINTER(SetupParams)]),
    'wcamg_set_test_vectors': (_I, [_P, _P, ctypes.POINTER(SetupParams), _I]),
    'wcamg_get_test_vectors': (_I, [_P, _P, _I]),
    'wcamg_orthonormalize': (_I, [_P, _P, _P, _I, _I, _I]),
    'wcamg_restrict': (_I, [_P, _P, _P, _I, _I]),
    'wcamg_prolong': (_I, [_P, _P, _P, _I, _I]),
    'wcamg_get_coarse_op': (_I, [_P, _I, _P, _I]),
    'wcamg_set_level1_vectors': (_I, [_P, _P, _I]),
    'wcamg_get_level1_vectors': (_I, [_P, _P, _I]),
    'wcamg_set_coarse_op': (_I, [_P, _I, _P, _I]),
    'wcamg_apply_coarse': (_I, [_P, _I, _P, _P, _I, _I]),
    'wcamg_coarse_solve': (_I, [_P, _I, _P, _P, _I, _I, _D, _I]),
    'wcamg_vcycle': (_I, [_P, _P, _P, _I, _I]),
    'wcamg_solve': (_I, [_P, _P, _P, _I, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveInfo)]),
    'wcamg_solve_bicgstab': (_I, [_P, _P, _P, _I, ctypes.POINTER(BicgParams), ctypes.POINTER(SolveInfo)]),
    'wcamg_net_init': (_I, [_P, _I, _I, _P, _I]),
    'wcamg_net_get_weights': (_I, [_P, _P, _I]),
    'wcamg_net_forward': (_I, [_P, _P, _P, _I]),
    'wcamg_net_gradient': (_I, [_P, _P, _P, ctypes.POINTER(_D), _P, _I]),
    'wcamg_net_train_step': (_I, [_P, _P, _P, _D, ctypes.POINTER(_D), _I]),
    'wcamg_autotune': (_I, [_P, _I, ctypes.c_char_p]),
    'wcamg_autotune_info': (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    'wcamg_kernel_timing': (_I, [_P, _I]),
    'wcamg_kernel_stats': (_I, [_P, ctypes.c_char_p, ctypes.POINTER(_D), ctypes.POINTER(_I), ctypes.POINTER(_D),
                                ctypes.POINTER(_D), ctypes.POINTER(_D)]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libwcamg.so and declare every entry point; raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError('libwcamg.so not built (%s); run __graft_entry__.build()' % path)
    # torch first: its HIP runtime is then the one the library binds to, so
    # that device pointers, streams and the library's device symbols share one
    # runtime (loading the library first would bring in a second one)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    """(pointer, where) for a torch tensor (device or host) or a NumPy array."""
    if isinstance(a, np.ndarray):
        if not a.flags['C_CONTIGUOUS']:
            raise ValueError('arrays must be C-contiguous')
        return a.ctypes.data, HOST
    if not a.is_contiguous():
        raise ValueError('tensors must be contiguous')
    return a.data_ptr(), (DEVICE if a.is_cuda else HOST)


def _same_where(*arrs):
    wh = {_ptr(a)[1] for a in arrs}
    if len(wh) != 1:
        raise ValueError('all arrays of one call must live on the same side (host or device)')
    return wh.pop()


class Context:
    """One library context (lattice, gauge field, hierarchy, workspaces).

    Device work is issued on the library's stream; every method that writes
    a device output synchronises that stream before returning, so results can
    be read from any torch stream."""

    def __init__(self, dims, block, bc, kappa, csw, stream=None):
        self.lib = load_library()
        lat = Lattice(_c_int4(*dims), _c_int4(*block), _c_int4(*bc), float(kappa), float(csw))
        h = _P()
        rc = self.lib.wcamg_create(ctypes.byref(h), ctypes.byref(lat), stream)
        if rc != OK:
            raise WcamgError(rc, 'wcamg_create failed')
        self.h = h
        self.dims, self.block = tuple(dims), tuple(block)

    def _chk(self, rc, allow=(OK,)):
        if rc not in allow:
            raise WcamgError(rc, self.lib.wcamg_last_error(self.h).decode())
        return rc

    def _done(self, rc, *arrs, allow=(OK,)):
        """Check rc; synchronise the library stream if any array is on the device."""
        self._chk(rc, allow)
        if any(_ptr(a)[1] == DEVICE for a in arrs):
            self._chk(self.lib.wcamg_sync(self.h))
        return rc

    def close(self):
        if getattr(self, 'h', None):
            self.lib.wcamg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        self._chk(self.lib.wcamg_sync(self.h))

    def load_gauge(self, U):
        p, w = _ptr(U)
        self._chk(self.lib.wcamg_load_gauge(self.h, p, w))

    def load_clover(self, F):
        p, w = _ptr(F)
        self._chk(self.lib.wcamg_load_clover(self.h, p, w))

    def get_clover(self, F):
        p, w = _ptr(F)
        self._done(self.lib.wcamg_get_clover(self.h, p, w), F)

    def apply_D(self, x, out, nrhs, prec=PREC_FP64):
        w = _same_where(x, out)
        self._done(self.lib.wcamg_apply_D(self.h, _ptr(x)[0], _ptr(out)[0], nrhs, prec, w), out)

    def apply_D_noalloc(self, x, out, nrhs, prec=PREC_FP64):
        """out = D x with the library's fixed scratch area (no allocation);
        device tensors only.  Asynchronous: synchronises like the others."""
        if _ptr(x)[1] != DEVICE or _ptr(out)[1] != DEVICE:
            raise ValueError('apply_D_noalloc takes device tensors')
        self._done(self.lib.wcamg_apply_D_noalloc(self.h, _ptr(x)[0], _ptr(out)[0], nrhs, prec), out)

    def apply_Dsap(self, x, out, nrhs, prec=PREC_FP64):
        w = _same_where(x, out)
        self._done(self.lib.wcamg_apply_Dsap(self.h, _ptr(x)[0], _ptr(out)[0], nrhs, prec, w), out)

    def sap(self, b, x, nrhs, sweeps=4, mr_iters=6, prec=PREC_FP64, block_solve=BLOCK_MR):
        w = _same_where(b, x)
        self._done(self.lib.wcamg_sap(self.h, _ptr(b)[0], _ptr(x)[0], nrhs, sweeps, mr_iters, block_solve, prec, w),
                   x)

    @staticmethod
    def setup_params(nv, prec=PREC_FP64, n_init=3, n_adapt=3, sap_sweeps=4, mr_iters=6, coarse_iters=50,
                     coarse_tol=0.1, init_vectors=None, nlevels=2, block1=(1, 1, 1, 1), nv1=0, mr1_iters=4,
                     init_mr1_iters=8, init_vectors1=None, seed1=1, init_net=0, seed=1, smoothing=SMOOTH_POST,
                     sap_eo=0, vec_chunk=0):
        p = SetupParams(nv, n_init, n_adapt, sap_sweeps, mr_iters, coarse_iters, coarse_tol, prec, None, DEVICE,
                        nlevels, _c_int4(*block1), nv1, mr1_iters, init_mr1_iters, None, seed1, init_net, seed,
                        smoothing, sap_eo, vec_chunk)
        if init_vectors is not None:
            ptr, w = _ptr(init_vectors)
            p.init_vectors = ptr
            p.init_where = w
        if init_vectors1 is not None:
            ptr, w = _ptr(init_vectors1)
            if w != DEVICE:
                raise ValueError('init_vectors1 must be a device tensor')
            p.init_vectors1 = ptr
        return p

    def setup(self, params):
        self._chk(self.lib.wcamg_setup(self.h, ctypes.byref(params)))

    def set_test_vectors(self, V, params):
        p, w = _ptr(V)
        self._chk(self.lib.wcamg_set_test_vectors(self.h, p, ctypes.byref(params), w))

    def get_test_vectors(self, V):
        p, w = _ptr(V)
        self._done(self.lib.wcamg_get_test_vectors(self.h, p, w), V)

    def orthonormalize(self, V, out, nv, prec=PREC_FP64):
        w = _same_where(V, out)
        self._done(self.lib.wcamg_orthonormalize(self.h, _ptr(V)[0], _ptr(out)[0], nv, prec, w), out)

    def restrict(self, x, out, nrhs):
        w = _same_where(x, out)
        self._done(self.lib.wcamg_restrict(self.h, _ptr(x)[0], _ptr(out)[0], nrhs, w), out)

    def prolong(self, xc, out, nrhs):
        w = _same_where(xc, out)
        self._done(self.lib.wcamg_prolong(self.h, _ptr(xc)[0], _ptr(out)[0], nrhs, w), out)

    def get_coarse_op(self, Dc, level=1):
        p, w = _ptr(Dc)
        self._done(self.lib.wcamg_get_coarse_op(self.h, level, p, w), Dc)

    def set_level1_vectors(self, W):
        p, w = _ptr(W)
        self._chk(self.lib.wcamg_set_level1_vectors(self.h, p, w))

    def get_level1_vectors(self, W):
        p, w = _ptr(W)
        self._done(self.lib.wcamg_get_level1_vectors(self.h, p, w), W)

    def set_coarse_op(self, Dc, level=1):
        p, w = _ptr(Dc)
        self._chk(self.lib.wcamg_set_coarse_op(self.h, level, p, w))

    def apply_coarse(self, x, out, nrhs, level=1):
        w = _same_where(x, out)
        self._done(self.lib.wcamg_apply_coarse(self.h, level, _ptr(x)[0], _ptr(out)[0], nrhs, w), out)

    def coarse_solve(self, b, x, nrhs, iters, tol, level=1):
        w = _same_where(b, x)
        self._done(self.lib.wcamg_coarse_solve(self.h, level, _ptr(b)[0], _ptr(x)[0], nrhs, iters, tol, w), x)

    def vcycle(self, v, out, nrhs):
        w = _same_where(v, out)
        self._done(self.lib.wcamg_vcycle(self.h, _ptr(v)[0], _ptr(out)[0], nrhs, w), out)

    def solve(self, b, x, nrhs, restart=16, tol=1e-10, max_iters=2000, rhs_chunk=0, use_graph=1, phase_times=0,
              ortho=0):
        """b, x: device tensors.  Returns (status, SolveInfo)."""
        pb, wb = _ptr(b)
        px, wx = _ptr(x)
        if wb != DEVICE or wx != DEVICE:
            raise ValueError('solve takes device tensors')
        prm = SolveParams(restart, tol, max_iters, rhs_chunk, use_graph, phase_times, ortho)
        info = SolveInfo()
        rc = self._chk(self.lib.wcamg_solve(self.h, pb, px, nrhs, ctypes.byref(prm), ctypes.byref(info)),
                       allow=(OK, NOT_CONVERGED))
        return rc, info

    def solve_bicgstab(self, b, x, nrhs, tol=1e-10, max_iters=1000, rhs_chunk=0, precond=PC_AMG, inner_iters=50,
                       inner_tol=0.1, phase_times=0):
        """The paper's flexible BiCGStab (FP64) preconditioned by the V-cycle
        (PC_AMG) or by an FP32 BiCGStab on D (PC_BICG32, the comparison
        solver).  b, x: device tensors.  Returns (status, SolveInfo)."""
        pb, wb = _ptr(b)
        px, wx = _ptr(x)
        if wb != DEVICE or wx != DEVICE:
            raise ValueError('solve_bicgstab takes device tensors')
        prm = BicgParams(tol, max_iters, rhs_chunk, precond, inner_iters, inner_tol, phase_times)
        info = SolveInfo()
        rc = self._chk(self.lib.wcamg_solve_bicgstab(self.h, pb, px, nrhs, ctypes.byref(prm), ctypes.byref(info)),
                       allow=(OK, NOT_CONVERGED))
        return rc, info

    def net_init(self, weights, layers, channels=16):
        p, w = _ptr(weights)
        self._chk(self.lib.wcamg_net_init(self.h, layers, channels, p, w))

    def net_get_weights(self, out):
        p, w = _ptr(out)
        self._done(self.lib.wcamg_net_get_weights(self.h, p, w), out)

    def net_forward(self, r, out):
        w = _same_where(r, out)
        self._done(self.lib.wcamg_net_forward(self.h, _ptr(r)[0], _ptr(out)[0], w), out)

    def net_gradient(self, r, teacher, grad=None):
        w = _same_where(r, teacher)
        loss = ctypes.c_double()
        gp = _ptr(grad)[0] if grad is not None else None
        self._done(self.lib.wcamg_net_gradient(self.h, _ptr(r)[0], _ptr(teacher)[0], ctypes.byref(loss), gp, w),
                   *([grad] if grad is not None else []))
        return loss.value

    def net_train_step(self, r, teacher, lr):
        w = _same_where(r, teacher)
        loss = ctypes.c_double()
        self._chk(self.lib.wcamg_net_train_step(self.h, _ptr(r)[0], _ptr(teacher)[0], lr, ctypes.byref(loss), w))
        return loss.value

    def autotune(self, enable=True, cache_path=None):
        self._chk(self.lib.wcamg_autotune(self.h, int(enable), cache_path.encode() if cache_path else None))

    def autotune_info(self):
        ms, a, b = ctypes.c_double(), ctypes.c_int(), ctypes.c_int()
        self._chk(self.lib.wcamg_autotune_info(self.h, ctypes.byref(ms), ctypes.byref(a), ctypes.byref(b)))
        return dict(tune_ms=ms.value, keys_tuned=a.value, keys_known=b.value)

    def kernel_timing(self, enable):
        self._chk(self.lib.wcamg_kernel_timing(self.h, int(enable)))

    def kernel_stats(self, name):
        """(total_ms, launches, algorithmic bytes, flops, rhs units) of a class."""
        ms, by, fl, un = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        n = ctypes.c_int()
        self._chk(self.lib.wcamg_kernel_stats(self.h, name.encode(), ctypes.byref(ms), ctypes.byref(n),
                                              ctypes.byref(by), ctypes.byref(fl), ctypes.byref(un)))
        return dict(ms=ms.value, count=n.value, bytes=by.value, flops=fl.value, units=un.value)
