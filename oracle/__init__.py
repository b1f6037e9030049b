"""FP64 CPU oracle (test infrastructure only).

Plain C implementation of consensus-ADMM calibration written from the paper, loaded through
ctypes.  Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use it; the
GPU library never imports it.  ``build()`` compiles ``oracle.c`` with gcc into ``liboracle.so``
next to this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
OPT_GPA_FIRST = 1
OPT_UNREG_FIRST = 2
SOLVE_CHOLESKY = 0
SOLVE_PCG = 1


def build() -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           os.path.join(HERE, "oracle.c"), "-o", LIB_PATH, "-lm"]
    subprocess.run(cmd, check=True)
    return LIB_PATH


class _Cfg(C.Structure):
    _fields_ = [("N", C.c_int), ("P", C.c_int), ("Q", C.c_int), ("K", C.c_int), ("T", C.c_int),
                ("n_chan", C.POINTER(C.c_int32)), ("n_dirs", C.POINTER(C.c_int32)),
                ("freq", C.POINTER(C.c_double)), ("f0", C.c_double),
                ("rho", C.POINTER(C.c_double)), ("lm_iters", C.c_int),
                ("sage_sweeps", C.c_int), ("options", C.c_uint32), ("lm_tol", C.c_double),
                ("solver", C.c_int), ("cg_tol", C.c_double)]


class _Data(C.Structure):
    _fields_ = [("vis", C.c_void_p), ("coh", C.c_void_p), ("flags", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.c_int, C.POINTER(C.c_double)
        _lib.or_predict.argtypes = [vp, vp, vp, vp]
        _lib.or_subband_cost.argtypes = [vp, vp, vp, vp]
        _lib.or_dir_objective.argtypes = [vp, vp, vp, vp, vp, ip, ip, vp, vp, vp]
        _lib.or_dir_gn_hessian.argtypes = [vp, vp, ip, ip, vp, vp]
        _lib.or_local_step.argtypes = [vp, vp, vp, vp, vp, ip, vp]
        _lib.or_local_step.restype = ip
        _lib.or_gpa.argtypes = [vp, vp, ip]
        _lib.or_consensus.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        _lib.or_consensus.restype = ip
        _lib.or_admm_solve.argtypes = [vp, vp, ip, vp, vp, vp, vp, vp, ip]
        _lib.or_admm_solve.restype = ip
        _lib.or_pcg.argtypes = [ip, vp, vp, C.c_double, vp, vp]
        _lib.or_pcg.restype = ip
        _lib.or_cholesky.argtypes = [ip, vp, vp]
        _lib.or_cholesky.restype = ip
        _lib.or_polar2.argtypes = [vp, vp]
        _lib.or_polar2.restype = ip
        _lib.or_lstsq.argtypes = [ip, ip, vp, ip, vp, vp]
        _lib.or_lstsq.restype = ip
        _lib.or_num_threads.restype = ip
        _lib.or_set_num_threads.argtypes = [ip]
        _lib.or_set_num_threads.restype = None
        del dp
    return _lib


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else C.c_void_p(0)


class Problem:
    """Holds one interval's arrays in the layout the C oracle expects (contiguous copies)."""

    def __init__(self, data: dict, lm_iters: int | None = None, sage_sweeps: int = 1,
                 options: int = OPT_GPA_FIRST, rho=None, lm_tol: float = 0.0,
                 solver: int = SOLVE_CHOLESKY, cg_tol: float = 1e-10):
        self.N, self.P, self.Q, self.K, self.T = (int(data[k]) for k in ("N", "P", "Q", "K", "T"))
        self.n_chan = np.ascontiguousarray(data["n_chan"], np.int32)
        self.n_dirs = np.ascontiguousarray(data["n_dirs"], np.int32)
        self.freq = np.ascontiguousarray(data["freq"], np.float64)
        self.rho = np.ascontiguousarray(data["rho"] if rho is None else rho, np.float64)
        self.vis = np.ascontiguousarray(data["vis"], np.complex128)
        self.coh = np.ascontiguousarray(data["coh"], np.complex128)
        self.flags = np.ascontiguousarray(data["flags"], np.uint8)
        self.lm_iters = int(data.get("lm_iters", 10) if lm_iters is None else lm_iters)
        self.cfg = _Cfg(self.N, self.P, self.Q, self.K, self.T,
                        self.n_chan.ctypes.data_as(C.POINTER(C.c_int32)),
                        self.n_dirs.ctypes.data_as(C.POINTER(C.c_int32)),
                        self.freq.ctypes.data_as(C.POINTER(C.c_double)), float(data["f0"]),
                        self.rho.ctypes.data_as(C.POINTER(C.c_double)), self.lm_iters,
                        int(sage_sweeps), int(options), float(lm_tol), int(solver),
                        float(cg_tol))
        self.dat = _Data(self.vis.ctypes.data, self.coh.ctypes.data, self.flags.ctypes.data)
        self.sage_sweeps = int(sage_sweeps)

    # shapes
    def jshape(self):
        return (self.P, self.K, self.N, 2, 2)

    def zshape(self):
        return (self.K, self.Q, self.N, 2, 2)

    def _c(self):
        return C.byref(self.cfg), C.byref(self.dat)

    def predict(self, J):
        J = np.ascontiguousarray(J, np.complex128)
        out = np.empty_like(self.vis)
        lib().or_predict(*self._c(), _ptr(J), _ptr(out))
        return out

    def subband_cost(self, J):
        J = np.ascontiguousarray(J, np.complex128)
        out = np.empty(self.P)
        lib().or_subband_cost(*self._c(), _ptr(J), _ptr(out))
        return out

    def dir_objective(self, J, Y, BZ, f, k, Jdir=None, grad=True):
        J = np.ascontiguousarray(J, np.complex128)
        Y = np.ascontiguousarray(Y, np.complex128)
        BZ = np.ascontiguousarray(BZ, np.complex128)
        Jdir = np.ascontiguousarray(J[f, k] if Jdir is None else Jdir, np.complex128)
        L = np.zeros(1)
        G = np.zeros((self.N, 2, 2), np.complex128) if grad else None
        lib().or_dir_objective(*self._c(), _ptr(J), _ptr(Y), _ptr(BZ), f, k, _ptr(Jdir),
                               _ptr(L), _ptr(G))
        return (float(L[0]), G) if grad else float(L[0])

    def dir_gn_hessian(self, f, k, Jdir):
        Jdir = np.ascontiguousarray(Jdir, np.complex128)
        H = np.zeros((8 * self.N, 8 * self.N))
        lib().or_dir_gn_hessian(*self._c(), f, k, _ptr(Jdir), _ptr(H))
        return H

    def local_step(self, J, Y, BZ, unregularised=False, trace=False):
        J = np.array(J, np.complex128, copy=True, order="C")
        Y = np.ascontiguousarray(Y, np.complex128)
        BZ = np.ascontiguousarray(BZ, np.complex128)
        tr = np.zeros((self.P, self.sage_sweeps, self.K, self.lm_iters, 3)) if trace else None
        st = lib().or_local_step(*self._c(), _ptr(J), _ptr(Y), _ptr(BZ), int(unregularised),
                                 _ptr(tr))
        assert st == 0
        return (J, tr) if trace else J

    def gpa(self, J, rounds=3):
        J = np.array(J, np.complex128, copy=True, order="C")
        lib().or_gpa(C.byref(self.cfg), _ptr(J), rounds)
        return J

    def consensus(self, J, Y, Z):
        J = np.ascontiguousarray(J, np.complex128)
        Y = np.array(Y, np.complex128, copy=True, order="C")
        Z = np.array(Z, np.complex128, copy=True, order="C")
        BZ = np.zeros(self.jshape(), np.complex128)
        pr, du = np.zeros(1), np.zeros(1)
        st = lib().or_consensus(C.byref(self.cfg), _ptr(J), _ptr(Y), _ptr(Z), _ptr(BZ),
                                _ptr(pr), _ptr(du))
        if st != 0:
            raise ValueError("rank condition violated: fewer subbands than basis terms")
        return Y, Z, BZ, float(pr[0]), float(du[0])

    def admm_solve(self, J0, iters, Y0=None, Z0=None, BZ0=None):
        """C-ADMM from J0 with Y = Z = B_f Z = 0, or (Y0, Z0, BZ0 given) continuing from that
        state, e.g. the previous solution interval's."""
        J = np.array(J0, np.complex128, copy=True, order="C")
        carry = Y0 is not None
        Y = np.array(Y0, np.complex128, copy=True, order="C") if carry else np.zeros(self.jshape(), np.complex128)
        BZ = np.array(BZ0, np.complex128, copy=True, order="C") if carry else np.zeros(self.jshape(), np.complex128)
        Z = np.array(Z0, np.complex128, copy=True, order="C") if carry else np.zeros(self.zshape(), np.complex128)
        tr = np.zeros((iters, 4))
        st = lib().or_admm_solve(*self._c(), iters, _ptr(J), _ptr(Y), _ptr(Z), _ptr(BZ), _ptr(tr),
                                 int(carry))
        if st != 0:
            raise ValueError("rank condition violated: fewer subbands than basis terms")
        return dict(J=J, Y=Y, Z=Z, BZ=BZ, trace=tr)


def cholesky(A):
    A = np.ascontiguousarray(A, np.float64)
    L = np.zeros_like(A)
    st = lib().or_cholesky(A.shape[0], _ptr(A), _ptr(L))
    return L if st == 0 else None


def pcg(M, b, tol):
    """(x, iterations) of the block-Jacobi preconditioned CG on M x = b, or None on breakdown."""
    M = np.ascontiguousarray(M, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros_like(b)
    it = np.zeros(1, np.int32)
    st = lib().or_pcg(M.shape[0], _ptr(M), _ptr(b), float(tol), _ptr(x), _ptr(it))
    return (x, int(it[0])) if st == 0 else None


def polar2(A):
    A = np.ascontiguousarray(A, np.complex128)
    U = np.zeros((2, 2), np.complex128)
    st = lib().or_polar2(_ptr(A), _ptr(U))
    return U if st == 0 else None


def lstsq(A, X):
    A = np.ascontiguousarray(A, np.float64)
    X = np.ascontiguousarray(X, np.complex128)
    m, n = A.shape
    Z = np.zeros((n, X.shape[1]), np.complex128)
    st = lib().or_lstsq(m, n, _ptr(A), X.shape[1], _ptr(X), _ptr(Z))
    return Z if st == 0 else None


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))
