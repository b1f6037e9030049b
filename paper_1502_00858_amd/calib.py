"""Python binding of the C ABI in include/calib.h (argument marshalling only).

Device buffers are torch tensors on the GPU; every step of the computation runs in the HIP
library libcalib_mi355x.so.  There is no fallback: if the library is missing, loading fails.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from .build import LIB_PATH

CALIB_FP64 = 0
CALIB_FP32_MIXED = 1
OPT_GPA_FIRST_ITER = 1
OPT_UNREG_FIRST = 2
OPT_STATS_ONLY = 4
(FIELD_J, FIELD_Z, FIELD_BZ, FIELD_Y, FIELD_MODEL_VIS, FIELD_COST, FIELD_TRACE, FIELD_LM_TRACE,
 FIELD_LM_STEP, FIELD_KERNEL_TIMES, FIELD_STATUS, FIELD_WORK) = range(12)
KERNELS = ["refresh", "lm_begin", "assemble", "chol_solve", "trial", "lm_update", "commit",
           "consensus", "local_step", "pack"]
STATUS = {0: "CALIB_OK", 1: "CALIB_E_INVAL", 2: "CALIB_E_NOMEM", 3: "CALIB_E_DEVICE",
          4: "CALIB_E_RANK", 5: "CALIB_E_NUMERIC", 6: "CALIB_E_STATE"}
EXPORTS = ["calib_init", "admm_local_step", "admm_consensus_update", "admm_solve", "calib_get",
           "calib_set_jones", "calib_set_state", "calib_warmstart_features", "calib_warmstart_target",
           "calib_warmstart_apply", "calib_mlp_create", "calib_mlp_forward", "calib_mlp_train_step", "calib_mlp_get",
           "calib_mlp_destroy", "calib_mlp_last_error", "calib_set_kernel_timing",
           "calib_destroy", "calib_last_error", "calib_consensus_noalloc", "calib_set_data"]
WS_FEATURES = 32
WS_OUTPUTS = 8
WS_SCALE = 10.0


class CalibError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Config(C.Structure):
    _fields_ = [("n_stations", C.c_int32), ("n_subbands", C.c_int32), ("n_basis", C.c_int32),
                ("n_dirs_max", C.c_int32), ("n_times", C.c_int32),
                ("n_chan", C.POINTER(C.c_int32)), ("n_dirs", C.POINTER(C.c_int32)),
                ("freq_hz", C.POINTER(C.c_double)), ("f0_hz", C.c_double),
                ("rho", C.POINTER(C.c_double)), ("precision", C.c_int),
                ("lm_iters", C.c_int32), ("sage_sweeps", C.c_int32), ("options", C.c_uint32),
                ("tile_group", C.c_int32), ("stream_grid", C.c_int32), ("lm_tol", C.c_double),
                ("solver", C.c_int32), ("cg_tol", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch's HIP runtime must be the process's HIP runtime: load it before the library
        # (whose libamdhip64 dependency then resolves to the already-loaded copy)
        import torch  # noqa: F401
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with paper_1502_00858_amd.build.build()")
        lib = C.CDLL(path)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        lib.calib_init.argtypes = [C.POINTER(_Config), vp, vp, vp, vp, vp, C.POINTER(vp)]
        lib.admm_local_step.argtypes = [vp, i32]
        lib.admm_consensus_update.argtypes = [vp, i32]
        lib.admm_solve.argtypes = [vp, i32, dbl, vp, C.POINTER(i32)]
        lib.calib_get.argtypes = [vp, i32, vp]
        lib.calib_set_jones.argtypes = [vp, vp]
        lib.calib_set_state.argtypes = [vp, vp, vp, vp, vp]
        lib.calib_set_data.argtypes = [vp, vp, vp]
        lib.calib_set_kernel_timing.argtypes = [vp, i32]
        lib.calib_destroy.argtypes = [vp]
        lib.calib_destroy.restype = None
        lib.calib_last_error.argtypes = [vp]
        lib.calib_last_error.restype = C.c_char_p
        lib.calib_warmstart_features.argtypes = [vp, vp, vp, vp]
        lib.calib_warmstart_apply.argtypes = [vp, vp, vp]
        lib.calib_warmstart_target.argtypes = [vp, vp, vp]
        lib.calib_mlp_create.argtypes = [i32, vp, vp, C.c_int64, vp, C.POINTER(vp)]
        lib.calib_mlp_forward.argtypes = [vp, vp, C.c_int64, vp]
        lib.calib_mlp_train_step.argtypes = [vp, vp, vp, C.c_int64, C.c_float, i32, vp]
        lib.calib_mlp_get.argtypes = [vp, i32, vp]
        lib.calib_mlp_destroy.argtypes = [vp]
        lib.calib_mlp_destroy.restype = None
        lib.calib_mlp_last_error.argtypes = [vp]
        lib.calib_mlp_last_error.restype = C.c_char_p
        lib.calib_consensus_noalloc.argtypes = [i32, i32, i32, i32, vp, vp, dbl, vp, vp, vp, vp,
                                                vp, vp, vp, vp]
        for name in ("calib_consensus_noalloc", "calib_set_data", "calib_init", "admm_local_step", "admm_consensus_update", "admm_solve",
                     "calib_get", "calib_set_jones", "calib_set_state", "calib_set_kernel_timing",
                     "calib_warmstart_features", "calib_warmstart_target", "calib_warmstart_apply",
                     "calib_mlp_create",
                     "calib_mlp_forward", "calib_mlp_train_step", "calib_mlp_get"):
            getattr(lib, name).restype = C.c_int
        _lib = lib
    return _lib


def _ptr(t) -> C.c_void_p:
    return C.c_void_p(0 if t is None else t.data_ptr())


def device_inputs(data: dict, precision: int = CALIB_FP64, device: str = "cuda"):
    """Move the generator's arrays to the GPU in the element type of the precision mode."""
    import torch
    cdt = torch.complex128 if precision == CALIB_FP64 else torch.complex64
    vis = torch.from_numpy(np.ascontiguousarray(data["vis"])).to(device=device, dtype=cdt)
    coh = torch.from_numpy(np.ascontiguousarray(data["coh"])).to(device=device, dtype=cdt)
    flags = torch.from_numpy(np.ascontiguousarray(data["flags"], np.uint8)).to(device)
    return vis, coh, flags


class Calib:
    """One calibration context (calib_init ... calib_destroy)."""

    def __init__(self, data: dict, vis, coh, flags=None, jones0=None, precision: int = CALIB_FP64,
                 lm_iters: Optional[int] = None, sage_sweeps: int = 1,
                 options: int = OPT_GPA_FIRST_ITER, rho=None, stream=None, tile_group: int = 0,
                 stream_grid: int = 0, lm_tol: float = 0.0, solver: int = 0, cg_tol: float = 0.0):
        import torch
        self.lib = load()
        self.N, self.P, self.Q, self.K, self.T = (int(data[k]) for k in ("N", "P", "Q", "K", "T"))
        self.precision = precision
        self.lm_iters = int(data.get("lm_iters", 10) if lm_iters is None else lm_iters)
        self._n_chan = np.ascontiguousarray(data["n_chan"], np.int32)
        self._n_dirs = np.ascontiguousarray(data["n_dirs"], np.int32)
        self._freq = np.ascontiguousarray(data["freq"], np.float64)
        self._rho = np.ascontiguousarray(data["rho"] if rho is None else rho, np.float64)
        self._vis_shape = tuple(vis.shape)
        self._vis_dtype = vis.dtype
        cfg = _Config(self.N, self.P, self.Q, self.K, self.T,
                      self._n_chan.ctypes.data_as(C.POINTER(C.c_int32)),
                      self._n_dirs.ctypes.data_as(C.POINTER(C.c_int32)),
                      self._freq.ctypes.data_as(C.POINTER(C.c_double)), float(data["f0"]),
                      self._rho.ctypes.data_as(C.POINTER(C.c_double)), int(precision),
                      self.lm_iters, int(sage_sweeps), int(options), int(tile_group),
                      int(stream_grid), float(lm_tol), int(solver), float(cg_tol))
        self.stream = torch.cuda.current_stream() if stream is None else stream
        ctx = C.c_void_p()
        st = self.lib.calib_init(C.byref(cfg), _ptr(vis), _ptr(coh), _ptr(flags), _ptr(jones0),
                                 C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if st != 0:
            raise CalibError(st, self.lib.calib_last_error(None).decode())
        self.ctx = ctx

    def _check(self, st):
        if st != 0:
            raise CalibError(st, self.lib.calib_last_error(self.ctx).decode())

    def local_step(self, admm_iter: int):
        self._check(self.lib.admm_local_step(self.ctx, admm_iter))

    def consensus_update(self, admm_iter: int):
        self._check(self.lib.admm_consensus_update(self.ctx, admm_iter))

    def solve(self, max_iters: int, rel_cost_tol: float = 0.0):
        tr = np.zeros((max(max_iters, 1), 4))
        done = C.c_int32(0)
        self._check(self.lib.admm_solve(self.ctx, max_iters, rel_cost_tol,
                                        C.c_void_p(tr.ctypes.data), C.byref(done)))
        return tr[:done.value]

    def get(self, field: int):
        import torch
        if field == FIELD_KERNEL_TIMES:
            kt = np.zeros((len(KERNELS), 2))
            self._check(self.lib.calib_get(self.ctx, field, C.c_void_p(kt.ctypes.data)))
            return {name: (int(kt[i, 0]), float(kt[i, 1])) for i, name in enumerate(KERNELS)}
        if field == FIELD_TRACE:
            n = 4096
            tr = np.zeros((n, 4))
            self._check(self.lib.calib_get(self.ctx, field, C.c_void_p(tr.ctypes.data)))
            return tr
        shapes = {FIELD_J: (self.P, self.K, self.N, 2, 2), FIELD_Y: (self.P, self.K, self.N, 2, 2),
                  FIELD_BZ: (self.P, self.K, self.N, 2, 2), FIELD_Z: (self.K, self.Q, self.N, 2, 2)}
        if field in shapes:
            out = torch.empty(shapes[field], dtype=torch.complex128, device="cuda")
        elif field == FIELD_MODEL_VIS:
            out = torch.empty(self._vis_shape, dtype=self._vis_dtype, device="cuda")
        elif field == FIELD_COST:
            out = torch.empty(self.P, dtype=torch.float64, device="cuda")
        elif field == FIELD_LM_STEP:
            out = torch.empty((self.P, 2, 8 * self.N), dtype=torch.float64, device="cuda")
        elif field == FIELD_WORK:
            out = torch.empty((self.P, 2), dtype=torch.float64, device="cuda")
        elif field == FIELD_STATUS:
            out = torch.empty(self.P, dtype=torch.int32, device="cuda")
        elif field == FIELD_LM_TRACE:
            out = torch.empty((self.P, self.K, self.lm_iters, 3), dtype=torch.float64, device="cuda")
        else:
            raise ValueError(field)
        self._check(self.lib.calib_get(self.ctx, field, _ptr(out)))
        return out

    def set_kernel_timing(self, enable: bool):
        self._check(self.lib.calib_set_kernel_timing(self.ctx, int(bool(enable))))

    def set_jones(self, J):
        self._check(self.lib.calib_set_jones(self.ctx, _ptr(J)))

    def set_data(self, vis, coh):
        """A new solution interval of the same observation (same shapes, flags and dtype)."""
        if tuple(vis.shape) != self._vis_shape or vis.dtype != self._vis_dtype:
            raise ValueError("calib_set_data needs visibilities of the context's shape and dtype")
        self._check(self.lib.calib_set_data(self.ctx, _ptr(vis), _ptr(coh)))

    def set_state(self, J, Y=None, Z=None, BZ=None):
        self._check(self.lib.calib_set_state(self.ctx, _ptr(J), _ptr(Y), _ptr(Z), _ptr(BZ)))

    def warmstart_features(self, jones_prev2=None, bz_prev=None):
        """Features [P*K*N][32] (float32, device) at the current J."""
        import torch
        out = torch.empty((self.P * self.K * self.N, WS_FEATURES), dtype=torch.float32,
                          device="cuda")
        self._check(self.lib.calib_warmstart_features(self.ctx, _ptr(jones_prev2), _ptr(bz_prev),
                                                      _ptr(out)))
        return out

    def warmstart_target(self, jones_prev):
        """Gauge-aligned training target [P*K*N][8] of the current J against jones_prev."""
        import torch
        out = torch.empty((self.P * self.K * self.N, WS_OUTPUTS), dtype=torch.float32,
                          device="cuda")
        self._check(self.lib.calib_warmstart_target(self.ctx, _ptr(jones_prev), _ptr(out)))
        return out

    def warmstart_apply(self, delta):
        """J += delta / s where that lowers each subband's cost; returns the kept flags [P]."""
        import torch
        kept = torch.empty(self.P, dtype=torch.int32, device="cuda")
        self._check(self.lib.calib_warmstart_apply(self.ctx, _ptr(delta), _ptr(kept)))
        return kept

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.calib_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """The warm-start network (calib_mlp_create ... calib_mlp_destroy)."""

    def __init__(self, dims, params: np.ndarray, max_rows: int, stream=None):
        import torch
        self.lib = load()
        self.dims = [int(d) for d in dims]
        self._dims = np.ascontiguousarray(self.dims, np.int32)
        p = np.ascontiguousarray(params, np.float32)
        if p.size != n_params(self.dims):
            raise ValueError(f"expected {n_params(self.dims)} parameters, got {p.size}")
        self.max_rows = int(max_rows)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = C.c_void_p()
        st = self.lib.calib_mlp_create(len(self.dims) - 1, C.c_void_p(self._dims.ctypes.data),
                                       C.c_void_p(p.ctypes.data), self.max_rows,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != 0:
            raise CalibError(st, self.lib.calib_mlp_last_error(None).decode())
        self.h = h
        self.step = 0

    def _check(self, st):
        if st != 0:
            raise CalibError(st, self.lib.calib_mlp_last_error(self.h).decode())

    def forward(self, x):
        import torch
        y = torch.empty((x.shape[0], self.dims[-1]), dtype=torch.float32, device="cuda")
        self._check(self.lib.calib_mlp_forward(self.h, _ptr(x), int(x.shape[0]), _ptr(y)))
        return y

    def train_step(self, x, target, lr: float, loss=None):
        """One Adam step (lr = 0: gradients only); loss: optional device float32 [1]."""
        if lr > 0:
            self.step += 1
        self._check(self.lib.calib_mlp_train_step(self.h, _ptr(x), _ptr(target), int(x.shape[0]),
                                                  float(lr), max(self.step, 1), _ptr(loss)))

    def params(self) -> np.ndarray:
        out = np.zeros(n_params(self.dims), np.float32)
        self._check(self.lib.calib_mlp_get(self.h, 0, C.c_void_p(out.ctypes.data)))
        return out

    def grads(self) -> np.ndarray:
        out = np.zeros(n_params(self.dims), np.float32)
        self._check(self.lib.calib_mlp_get(self.h, 1, C.c_void_p(out.ctypes.data)))
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.calib_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def consensus_noalloc(N: int, P: int, Q: int, K: int, n_dirs, freq, f0: float, rho, jones, y, z,
                      bz, residuals=None, status=None, stream=None):
    """calib_consensus_noalloc on device tensors (y and z updated in place, bz written)."""
    import torch
    lib = load()
    s = torch.cuda.current_stream() if stream is None else stream
    st = lib.calib_consensus_noalloc(int(N), int(P), int(Q), int(K), _ptr(n_dirs), _ptr(freq),
                                     float(f0), _ptr(rho), _ptr(jones), _ptr(y), _ptr(z), _ptr(bz),
                                     _ptr(residuals), _ptr(status), C.c_void_p(s.cuda_stream))
    if st != 0:
        raise CalibError(st, lib.calib_last_error(None).decode())


def n_params(dims) -> int:
    return int(sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1)))
