"""ctypes binding of libxdg (include/xdg.h): argument marshalling only.

Device buffers are torch tensors (float64, on the handle's device); host
arrays are numpy.  Every function raises XdgError on a negative status and
returns a positive (warning) status unchanged.  The library must have been
built (paper_2003_02431_amd/build.py); importing this module without it fails
loudly -- there is no fallback.
"""
import ctypes as C
import os

import numpy as np
# torch before libxdg: the process must hold one HIP runtime, and libxdg's
# dependency has to resolve to the one torch brings (loaded the other way
# round, two runtimes coexist and the library's finds no device)
import torch  # noqa: F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libxdg.so")

XDG_OK, XDG_ENOCONV = 0, 1
XDG_EINVAL, XDG_ENOMEM, XDG_EHIP, XDG_ENOTSPD, XDG_EBREAKDOWN = -1, -2, -3, -4, -5
XDG_T_PTRUNC, XDG_T_DENSE = 0, 1
XDG_CG, XDG_FGMRES, XDG_ORTHOMG = 0, 1, 2
XDG_FP64, XDG_MIXED = 0, 1
XDG_JACOBI, XDG_LEARNED, XDG_LEARNED_BF16 = 0, 1, 2

_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_f32p = C.POINTER(C.c_float)
_f64p = C.POINTER(C.c_double)


class XdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libxdg error {code}: {msg}")
        self.code = code


class xdg_matrix(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("np", C.c_int32), ("nnzb", C.c_int32),
                ("row_ptr", _i32p), ("col_idx", _i32p), ("val", _f64p),
                ("n_cells", C.c_int32), ("cell_ptr", _i32p)]


class xdg_transfer(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_rows_c", C.c_int32), ("np_c", C.c_int32),
                ("parent", _i32p), ("R", _f64p), ("n_cells_c", C.c_int32),
                ("cell_ptr_c", _i32p)]


class xdg_projection(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_cols", C.c_int32), ("np", C.c_int32),
                ("nnzb", C.c_int32), ("row_ptr", _i32p), ("col_idx", _i32p), ("val", _f64p)]


class xdg_options(C.Structure):
    _fields_ = [("krylov", C.c_int32), ("restart", C.c_int32), ("maxit", C.c_int32),
                ("nu_pre", C.c_int32), ("nu_post", C.c_int32), ("precision", C.c_int32),
                ("smoother", C.c_int32), ("nrhs", C.c_int32), ("rtol", C.c_double),
                ("omega", C.c_double), ("symmetric", C.c_int32), ("nu_coarse", C.c_int32)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libxdg.so not built at {_LIB_PATH}; run paper_2003_02431_amd/build.py")
    lib = C.CDLL(_LIB_PATH)
    vp = C.c_void_p
    sig = {
        "xdg_create": ([C.POINTER(xdg_matrix), C.c_int32, C.POINTER(xdg_transfer),
                        C.POINTER(xdg_options), vp, C.POINTER(vp)], C.c_int),
        "xdg_spmv": ([vp, C.c_int32, vp, vp], C.c_int),
        "xdg_smooth": ([vp, C.c_int32, vp, vp, C.c_int32], C.c_int),
        "xdg_restrict": ([vp, C.c_int32, vp, vp], C.c_int),
        "xdg_prolong": ([vp, C.c_int32, vp, vp], C.c_int),
        "xdg_vcycle": ([vp, vp, vp], C.c_int),
        "xdg_vcycle_noalloc": ([vp, vp, vp], C.c_int),
        "xdg_solve": ([vp, vp, vp, _f64p, C.c_int32, _i32p, _f64p], C.c_int),
        "xdg_level_info": ([vp, C.c_int32, _i32p, _i32p, _i32p], C.c_int),
        "xdg_get_level_matrix": ([vp, C.c_int32, _i32p, _i32p, _f64p], C.c_int),
        "xdg_get_cell_inverse": ([vp, C.c_int32, C.c_int32, _f64p, C.c_int32, _i32p], C.c_int),
        "xdg_update_matrix": ([vp, vp], C.c_int),
        "xdg_update_cells": ([vp, vp, C.c_int32, _i32p], C.c_int),
        "xdg_spmm": ([vp, C.c_int32, C.c_int32, vp, vp], C.c_int),
        "xdg_setup_time": ([vp, _f64p], C.c_int),
        "xdg_mlp_param_count": ([], C.c_int32),
        "xdg_mlp_set": ([vp, _f32p], C.c_int),
        "xdg_mlp_get": ([vp, _f32p], C.c_int),
        "xdg_mlp_forward": ([vp, C.c_int32, vp, vp], C.c_int),
        "xdg_mlp_gradient": ([vp, C.c_int32, vp, vp, vp, _f32p], C.c_int),
        "xdg_mlp_train": ([vp, C.c_int32, vp, vp, C.c_int32, C.c_int32, C.c_float, _f32p],
                          C.c_int),
        "xdg_set_cell_features": ([vp, _i32p, _f32p], C.c_int),
        "xdg_learned_pairs": ([vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_float, vp, vp, _i32p],
                              C.c_int),
        "xdg_set_tolerance": ([vp, C.c_double, C.c_int32], C.c_int),
        "xdg_set_projection": ([vp, C.POINTER(xdg_projection)], C.c_int),
        "xdg_project": ([vp, vp, vp], C.c_int),
        "xdg_set_smoother": ([vp, C.c_int32, C.c_float], C.c_int),
        "xdg_learned_stats": ([vp, _i64p, _i32p], C.c_int),
        "xdg_destroy": ([vp], None),
        "xdg_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()
EXPORTED = ("xdg_create", "xdg_spmv", "xdg_smooth", "xdg_restrict", "xdg_prolong",
            "xdg_vcycle", "xdg_vcycle_noalloc", "xdg_solve", "xdg_level_info", "xdg_get_level_matrix",
            "xdg_get_cell_inverse", "xdg_update_matrix", "xdg_update_cells", "xdg_spmm", "xdg_setup_time",
            "xdg_mlp_param_count", "xdg_mlp_set", "xdg_mlp_get", "xdg_mlp_forward",
            "xdg_mlp_gradient", "xdg_mlp_train", "xdg_set_cell_features", "xdg_learned_pairs",
            "xdg_set_smoother", "xdg_learned_stats", "xdg_set_tolerance",
            "xdg_set_projection", "xdg_project", "xdg_destroy",
            "xdg_last_error")


def lib():
    return _lib


def _check(rc):
    if rc < 0:
        raise XdgError(rc, _lib.xdg_last_error().decode())
    return rc


def _ptr(t):
    """Device pointer of a contiguous float64 torch tensor."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 device tensor")
    return C.c_void_p(t.data_ptr())


def _ptr32(t):
    """Device pointer of a contiguous float32 torch tensor."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous()):
        raise TypeError("expected a contiguous float32 device tensor")
    return C.c_void_p(t.data_ptr())


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# columns per vector and level-0 smoother cells of every live handle (keyed by
# the handle's address): the device-vector length checks below need them
_HANDLES = {}


def _key(h):
    return h.value if isinstance(h, C.c_void_p) else int(h)


def _need(t, n, what):
    """Refuse a device buffer shorter than the n elements the call touches
    (the library only sees a pointer and would read or write past its end)."""
    if t.numel() < n:
        raise ValueError(f"{what}: device buffer holds {t.numel()} elements, the call needs {n}")


def _vlen(h, level):
    n, npm, _ = xdg_level_info(h, level)
    return n * npm * _HANDLES.get(_key(h), (1, 0))[0]


def _vec(h, level, t, what):
    p = _ptr(t)
    _need(t, _vlen(h, level), what)
    return p


def options(krylov=XDG_CG, restart=30, maxit=500, nu_pre=2, nu_post=2, precision=XDG_FP64,
            smoother=XDG_JACOBI, nrhs=1, rtol=1e-10, omega=0.7, symmetric=1, nu_coarse=0):
    return xdg_options(krylov, restart, maxit, nu_pre, nu_post, precision, smoother, nrhs,
                       rtol, omega, symmetric, nu_coarse)


def xdg_create(row_ptr, col_idx, val, cell_ptr, transfers, opt, stream=None):
    """Build a handle from host arrays (numpy); transfers: list of dicts with
    kind, n_rows_c, np_c, parent, R, cell_ptr_c.  Returns an opaque handle."""
    keep = []
    rp, ci = _np(row_ptr, np.int32), _np(col_idx, np.int32)
    v = _np(val, np.float64)
    cp = _np(cell_ptr, np.int32)
    keep += [rp, ci, v, cp]
    m = xdg_matrix(len(rp) - 1, v.shape[1], len(ci), rp.ctypes.data_as(_i32p),
                   ci.ctypes.data_as(_i32p), v.ctypes.data_as(_f64p), len(cp) - 1,
                   cp.ctypes.data_as(_i32p))
    T = (xdg_transfer * max(1, len(transfers)))()
    for k, t in enumerate(transfers):
        par = _np(t["parent"], np.int32)
        cpc = _np(t["cell_ptr_c"], np.int32)
        keep += [par, cpc]
        Rp = None
        if t["R"] is not None:
            R = _np(t["R"], np.float64)
            keep.append(R)
            Rp = R.ctypes.data_as(_f64p)
        T[k] = xdg_transfer(t["kind"], t["n_rows_c"], t["np_c"], par.ctypes.data_as(_i32p),
                            Rp, len(cpc) - 1, cpc.ctypes.data_as(_i32p))
    h = C.c_void_p()
    _check(_lib.xdg_create(C.byref(m), len(transfers) + 1, T, C.byref(opt),
                           C.c_void_p(stream or 0), C.byref(h)))
    _HANDLES[_key(h)] = (int(opt.nrhs), len(cp) - 1)
    return h


def xdg_spmv(h, level, x, y):
    return _check(_lib.xdg_spmv(h, level, _vec(h, level, x, "x"), _vec(h, level, y, "y")))


def xdg_smooth(h, level, b, x, sweeps):
    return _check(_lib.xdg_smooth(h, level, _vec(h, level, b, "b"), _vec(h, level, x, "x"),
                                  sweeps))


def xdg_restrict(h, level, rf, rc):
    return _check(_lib.xdg_restrict(h, level, _vec(h, level, rf, "rf"),
                                    _vec(h, level + 1, rc, "rc")))


def xdg_prolong(h, level, xc, xf):
    return _check(_lib.xdg_prolong(h, level, _vec(h, level + 1, xc, "xc"),
                                   _vec(h, level, xf, "xf")))


def xdg_vcycle(h, r, z):
    return _check(_lib.xdg_vcycle(h, _vec(h, 0, r, "r"), _vec(h, 0, z, "z")))


def xdg_vcycle_noalloc(h, r, z):
    return _check(_lib.xdg_vcycle_noalloc(h, _vec(h, 0, r, "r"), _vec(h, 0, z, "z")))


def xdg_solve(h, b, x, hist_cap=1000):
    """Returns (status, iterations, final true relres, history array)."""
    hist = np.zeros(hist_cap)
    it = C.c_int32()
    fr = C.c_double()
    rc = _check(_lib.xdg_solve(h, _vec(h, 0, b, "b"), _vec(h, 0, x, "x"),
                               hist.ctypes.data_as(_f64p), hist_cap,
                               C.byref(it), C.byref(fr)))
    return rc, it.value, fr.value, hist[:min(it.value + 1, hist_cap)].copy()


def xdg_level_info(h, level):
    a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
    _check(_lib.xdg_level_info(h, level, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def xdg_get_level_matrix(h, level):
    n, npm, nnzb = xdg_level_info(h, level)
    rp = np.zeros(n + 1, np.int32)
    ci = np.zeros(nnzb, np.int32)
    val = np.zeros((nnzb, npm, npm))
    _check(_lib.xdg_get_level_matrix(h, level, rp.ctypes.data_as(_i32p),
                                     ci.ctypes.data_as(_i32p), val.ctypes.data_as(_f64p)))
    return rp, ci, val


def xdg_get_cell_inverse(h, level, cell, cap=1 << 24):
    out = np.zeros(cap)
    n = C.c_int32()
    _check(_lib.xdg_get_cell_inverse(h, level, cell, out.ctypes.data_as(_f64p), cap,
                                     C.byref(n)))
    return out[:n.value * n.value].reshape(n.value, n.value).copy()


def xdg_spmm(h, level, precision, X, Y):
    return _check(_lib.xdg_spmm(h, level, precision, _vec(h, level, X, "X"),
                                _vec(h, level, Y, "Y")))


def _vals(h, val_dev):
    p = _ptr(val_dev)
    _, npm, nnzb = xdg_level_info(h, 0)
    _need(val_dev, nnzb * npm * npm, "val_dev")
    return p


def xdg_update_matrix(h, val_dev):
    return _check(_lib.xdg_update_matrix(h, _vals(h, val_dev)))


def xdg_update_cells(h, val_dev, cells):
    """New level-0 values changed only in the rows/columns of `cells`."""
    c = np.ascontiguousarray(cells, dtype=np.int32)
    return _check(_lib.xdg_update_cells(h, _vals(h, val_dev), int(c.size),
                                        c.ctypes.data_as(_i32p)))


def xdg_setup_time(h):
    ms = C.c_double()
    _check(_lib.xdg_setup_time(h, C.byref(ms)))
    return ms.value


def xdg_mlp_param_count():
    return int(_lib.xdg_mlp_param_count())


def xdg_mlp_set(h, params):
    p = _np(params, np.float32)
    if p.size != xdg_mlp_param_count():
        raise ValueError("wrong parameter count")
    return _check(_lib.xdg_mlp_set(h, p.ctypes.data_as(_f32p)))


def xdg_mlp_get(h):
    p = np.zeros(xdg_mlp_param_count(), np.float32)
    _check(_lib.xdg_mlp_get(h, p.ctypes.data_as(_f32p)))
    return p


def _samples(X, T, n_in=45, n_out=40):
    n = X.shape[0]
    _need(X, n * n_in, "X")
    _need(T, n * n_out, "T")
    return n


def xdg_mlp_forward(h, X, Y):
    n = _samples(X, Y)
    return _check(_lib.xdg_mlp_forward(h, n, _ptr32(X), _ptr32(Y)))


def xdg_mlp_gradient(h, X, T, grad):
    """Fills grad (float32 device tensor) and returns the loss."""
    loss = C.c_float()
    n = _samples(X, T)
    _need(grad, xdg_mlp_param_count(), "grad")
    _check(_lib.xdg_mlp_gradient(h, n, _ptr32(X), _ptr32(T), _ptr32(grad),
                                 C.byref(loss)))
    return loss.value


def xdg_mlp_train(h, X, T, batch, steps, lr):
    """Returns the minibatch loss history (numpy float32, one per step)."""
    hist = np.zeros(max(steps, 1), np.float32)
    n = _samples(X, T)
    _check(_lib.xdg_mlp_train(h, n, _ptr32(X), _ptr32(T), batch, steps, lr,
                              hist.ctypes.data_as(_f32p)))
    return hist[:steps]


def xdg_set_cell_features(h, row_species, cell_geom):
    rs = _np(row_species, np.int32)
    g = _np(cell_geom, np.float32)
    return _check(_lib.xdg_set_cell_features(h, rs.ctypes.data_as(_i32p),
                                             g.ctypes.data_as(_f32p)))


def xdg_learned_pairs(h, b, xk, xs, cell0, cell_step, X, T, clip=0.0):
    """Writes the pairs into X, T (float32 device tensors); returns the count."""
    n = C.c_int32()
    n_cells = _HANDLES.get(_key(h), (1, 0))[1]
    if cell_step >= 1 and 0 <= cell0 < n_cells:
        m = (n_cells - cell0 + cell_step - 1) // cell_step
        _need(X, m * 45, "X")
        _need(T, m * 40, "T")
    _check(_lib.xdg_learned_pairs(h, _vec(h, 0, b, "b"), _vec(h, 0, xk, "xk"),
                                  _vec(h, 0, xs, "xs"), cell0, cell_step, clip,
                                  _ptr32(X), _ptr32(T), C.byref(n)))
    return n.value


_PROJ = {}     # handle address -> length of the earlier level-0 vector


def xdg_set_projection(h, row_ptr, col_idx, val, n_cols):
    """The L2 re-projection operator from an earlier space of n_cols block
    rows into this handle's level 0 (host arrays, row-major blocks)."""
    rp, ci = _np(row_ptr, np.int32), _np(col_idx, np.int32)
    v = _np(val, np.float64)
    P = xdg_projection(len(rp) - 1, int(n_cols), v.shape[1], len(ci), rp.ctypes.data_as(_i32p),
                       ci.ctypes.data_as(_i32p), v.ctypes.data_as(_f64p))
    rc = _check(_lib.xdg_set_projection(h, C.byref(P)))
    _PROJ[_key(h)] = int(n_cols) * v.shape[1]
    return rc


def xdg_project(h, x_old, x_new):
    p_old = _ptr(x_old)
    _need(x_old, _PROJ.get(_key(h), 0), "x_old")
    return _check(_lib.xdg_project(h, p_old, _vec(h, 0, x_new, "x_new")))


def xdg_set_tolerance(h, rtol, maxit):
    return _check(_lib.xdg_set_tolerance(h, rtol, maxit))


def xdg_set_smoother(h, smoother, guard=4.0):
    return _check(_lib.xdg_set_smoother(h, smoother, guard))


def xdg_learned_stats(h):
    g, f = C.c_int64(), C.c_int32()
    _check(_lib.xdg_learned_stats(h, C.byref(g), C.byref(f)))
    return g.value, f.value


def xdg_destroy(h):
    _HANDLES.pop(_key(h), None)
    _PROJ.pop(_key(h), None)
    _lib.xdg_destroy(h)


def xdg_last_error():
    return _lib.xdg_last_error().decode()


class Solver:
    """Convenience owner of one handle built from a generated problem."""

    def __init__(self, problem, opt=None, stream=None, device="cuda"):
        import torch
        self.torch = torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.opt = opt or options()
        self.h = xdg_create(problem.row_ptr, problem.col_idx, problem.val, problem.cell_ptr,
                            problem.transfers, self.opt, stream)
        self.nlev = len(problem.transfers) + 1
        self.n_cells = len(problem.cell_ptr) - 1
        self.smoother, self.guard = self.opt.smoother, 4.0

    def set_smoother(self, smoother, guard=None):
        self.guard = self.guard if guard is None else guard
        xdg_set_smoother(self.h, smoother, self.guard)
        self.smoother = smoother

    def level_len(self, level):
        n, npm, _ = xdg_level_info(self.h, level)
        return n * npm * self.opt.nrhs

    def vec(self, level=0, data=None):
        t = self.torch
        if data is None:
            return t.zeros(self.level_len(level), dtype=t.float64, device=self.device)
        return t.as_tensor(np.ascontiguousarray(data, dtype=np.float64)).to(self.device)

    def close(self):
        if self.h:
            xdg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
