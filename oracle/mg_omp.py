"""ctypes wrapper of the plain-loop C++17/OpenMP oracle (mg_omp.cpp) -- TEST
INFRASTRUCTURE ONLY (the tests, the smoke check and the benchmark's CPU
baseline use it).

The same solve as `oracle.mg` (scalar CSR levels, Galerkin products,
Cholesky-based cell-block inverses, dense Cholesky on the coarsest level,
symmetric V-cycle, textbook PCG), written as plain loops over all host cores.
It shares no code with the GPU library.  Built by `build()` into
oracle/libmg_omp.so.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mg_omp.cpp")
LIB = os.path.join(HERE, "libmg_omp.so")
FLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-std=c++17", "-shared",
         "-fPIC"]


def build():
    """Compile the oracle library (g++, host code only)."""
    tmp = LIB + ".tmp"
    r = subprocess.run(["g++", *FLAGS, SRC, "-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"g++ failed for mg_omp.cpp:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} not built; run oracle.mg_omp.build()")
        L = C.CDLL(LIB)
        vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        i32p, i64p, f64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_double)
        sig = {
            "mgo_threads": ([], C.c_int),
            "mgo_set_threads": ([C.c_int], None),
            "mgo_set_coarse_sweeps": ([vp, i32], None),
            "mgo_new": ([i32, i32, i32, i32p, i32p, f64p, i32, i32p, f64, i32, i32], vp),
            "mgo_add_transfer": ([vp, i32, i32, i32, i32p, f64p, i32, i32p], None),
            "mgo_setup": ([vp], C.c_int),
            "mgo_levels": ([vp], i32),
            "mgo_level_size": ([vp, i32], i64),
            "mgo_level_nnz": ([vp, i32], i64),
            "mgo_level_csr": ([vp, i32, i64p, i32p, f64p], None),
            "mgo_spmv": ([vp, i32, f64p, f64p], None),
            "mgo_smooth": ([vp, i32, f64p, f64p, i32], None),
            "mgo_vcycle": ([vp, f64p, f64p], None),
            "mgo_pcg": ([vp, f64p, f64p, f64, i32, f64p, i32], i32),
            "mgo_free": ([vp], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def threads():
    return int(lib().mgo_threads())


def set_threads(n):
    lib().mgo_set_threads(int(n))


class OmpHierarchy:
    """The multigrid hierarchy of a generated problem in the C++ oracle."""

    def __init__(self, pr, omega=0.7, nu=2, nu_coarse=0):
        L = lib()
        self._keep = []
        k = lambda a, dt: self._keep.append(np.ascontiguousarray(a, dtype=dt)) or self._keep[-1]
        rp, ci = k(pr.row_ptr, np.int32), k(pr.col_idx, np.int32)
        val, cp = k(pr.val, np.float64), k(pr.cell_ptr, np.int32)
        self.h = C.c_void_p(L.mgo_new(len(rp) - 1, val.shape[1], len(ci), _p(rp, C.c_int32),
                                      _p(ci, C.c_int32), _p(val, C.c_double), len(cp) - 1,
                                      _p(cp, C.c_int32), omega, nu, nu))
        L.mgo_set_coarse_sweeps(self.h, int(nu_coarse))
        for T in pr.transfers:
            par = k(T["parent"], np.int32)
            cpc = k(T["cell_ptr_c"], np.int32)
            R = k(T["R"] if T["R"] is not None else np.zeros(1), np.float64)
            L.mgo_add_transfer(self.h, int(T["kind"]), int(T["n_rows_c"]), int(T["np_c"]),
                               _p(par, C.c_int32), _p(R, C.c_double), len(cpc) - 1,
                               _p(cpc, C.c_int32))
        self._keep = []
        if L.mgo_setup(self.h) != 0:
            raise RuntimeError("C++ oracle: non-positive pivot (matrix not SPD)")
        self.nlev = int(L.mgo_levels(self.h))

    def size(self, l):
        return int(lib().mgo_level_size(self.h, l))

    def level_csr(self, l):
        import scipy.sparse as sp
        n, nnz = self.size(l), int(lib().mgo_level_nnz(self.h, l))
        ptr, col, val = np.zeros(n + 1, np.int64), np.zeros(nnz, np.int32), np.zeros(nnz)
        lib().mgo_level_csr(self.h, l, _p(ptr, C.c_int64), _p(col, C.c_int32), _p(val, C.c_double))
        return sp.csr_matrix((val, col, ptr), shape=(n, n))

    def spmv(self, l, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.size(l))
        lib().mgo_spmv(self.h, l, _p(x, C.c_double), _p(y, C.c_double))
        return y

    def smooth(self, l, b, x, sweeps):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x, dtype=np.float64)
        lib().mgo_smooth(self.h, l, _p(b, C.c_double), _p(x, C.c_double), sweeps)
        return x

    def vcycle(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.size(0))
        lib().mgo_vcycle(self.h, _p(r, C.c_double), _p(z, C.c_double))
        return z

    def pcg(self, b, rtol=1e-10, maxit=500, x0=None):
        """(x, history, iterations) as oracle.mg.pcg."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
        hist = np.zeros(maxit + 1)
        it = int(lib().mgo_pcg(self.h, _p(b, C.c_double), _p(x, C.c_double), rtol, maxit,
                               _p(hist, C.c_double), maxit + 1))
        return x, list(hist[:it + 1]), it

    def close(self):
        if self.h:
            lib().mgo_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
