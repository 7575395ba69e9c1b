"""ctypes binding of liblsqr.so (include/lsqr.h): argument marshalling only.

Tensors are torch tensors on the GPU; their data pointers go to the C ABI and
every step of the computation runs in the library's HIP kernels. There is no
fallback: if liblsqr.so is missing or fails to load, this module raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsqr.so")

LSQR_OK = 0
LSQR_E_INVALID = -1
LSQR_E_HIP = -2
LSQR_E_NOMEM = -3
LSQR_E_STATE = -4
LSQR_E_UNSUPPORTED = -5
LSQR_F64 = 0
LSQR_F32 = 1

OPTIONS = {"conlim": 1, "tests": 2, "chunk": 3, "graph": 4, "profile": 5, "outer_tol": 6,
           "att_mode": 7, "astro_scan": 8, "ktile": 9, "att_buckets": 10,
           "att_interleave": 11, "fused": 12, "variance": 13, "compact_index": 14,
           "att_rhs": 15, "pipeline": 16, "rhs_lanes": 17}

SYMBOLS = ("lsqr_create", "lsqr_destroy", "lsqr_set_option", "lsqr_aprod1", "lsqr_aprod2",
           "lsqr_aprod1_noalloc", "lsqr_aprod1_f32", "lsqr_aprod2_f32",
           "lsqr_get_precond", "lsqr_get_variance", "lsqr_num_cols", "lsqr_solve",
           "lsqr_solve_refined",
           "lsqr_solve_batched", "lsqr_solve_batched_refined", "lsqr_batch_tuning",
           "lsqr_kernel_times", "lsqr_pass_times",
           "lsqr_last_error")


class LsqrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"lsqr status {status}: {message}")
        self.status = status


class _System(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_stars", ctypes.c_int64),
                ("n_astro", ctypes.c_int32), ("n_axes", ctypes.c_int32),
                ("n_par_axis", ctypes.c_int32), ("n_instr", ctypes.c_int32),
                ("n_dfa", ctypes.c_int64), ("n_instr_cols", ctypes.c_int64),
                ("n_glob", ctypes.c_int32), ("value_type", ctypes.c_int32),
                ("precondition", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("values", ctypes.c_void_p), ("star_of_row", ctypes.c_void_p),
                ("att_start", ctypes.c_void_p), ("instr_idx", ctypes.c_void_p),
                ("stream", ctypes.c_void_p), ("n_con", ctypes.c_int64),
                ("con_rowptr", ctypes.c_void_p), ("con_col", ctypes.c_void_p),
                ("con_val", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("istop", ctypes.c_int32), ("itn", ctypes.c_int32),
                ("outer_steps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("rnorm", ctypes.c_double), ("arnorm", ctypes.c_double),
                ("anorm", ctypes.c_double), ("acond", ctypes.c_double),
                ("xnorm", ctypes.c_double), ("bnorm", ctypes.c_double)]


@dataclass
class Info:
    istop: int
    itn: int
    outer_steps: int
    rnorm: float
    arnorm: float
    anorm: float
    acond: float
    xnorm: float
    bnorm: float


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblsqr.so and declare its signatures (no GPU work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    P, I32, I64, F64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    H = ctypes.c_void_p
    sig = {
        "lsqr_create": ([ctypes.POINTER(_System), ctypes.POINTER(H)], I32),
        "lsqr_destroy": ([H], I32),
        "lsqr_set_option": ([H, I32, F64], I32),
        "lsqr_aprod1": ([H, P, P], I32),
        "lsqr_aprod2": ([H, P, P], I32),
        "lsqr_aprod1_noalloc": ([H, P, P], I32),
        "lsqr_aprod1_f32": ([H, P, P], I32),
        "lsqr_aprod2_f32": ([H, P, P], I32),
        "lsqr_get_precond": ([H, P], I32),
        "lsqr_get_variance": ([H, P], I32),
        "lsqr_num_cols": ([H, ctypes.POINTER(I64)], I32),
        "lsqr_solve": ([H, P, P, I32, F64, F64, ctypes.POINTER(_Info)], I32),
        "lsqr_solve_refined": ([H, P, P, I32, F64, F64, I32, ctypes.POINTER(_Info)], I32),
        "lsqr_solve_batched": ([H, P, P, I32, I32, F64, F64, ctypes.POINTER(_Info)], I32),
        "lsqr_solve_batched_refined": ([H, P, P, I32, I32, F64, F64, I32,
                                        ctypes.POINTER(_Info)], I32),
        "lsqr_batch_tuning": ([H, ctypes.POINTER(I32), ctypes.POINTER(F64)], I32),
        "lsqr_kernel_times": ([H, ctypes.POINTER(F64), ctypes.POINTER(I64),
                               ctypes.POINTER(F64), ctypes.POINTER(I64)], I32),
        "lsqr_pass_times": ([H, ctypes.POINTER(F64), ctypes.POINTER(I64),
                             ctypes.POINTER(I32), ctypes.POINTER(I32)], I32),
        "lsqr_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int):
    if status != LSQR_OK:
        msg = _lib.lsqr_last_error().decode(errors="replace")
        raise LsqrError(status, msg)


def _dev_ptr(t, dtype, shape=None, name="tensor"):
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class LsqrSystem:
    """Handle over a device-resident AVU-GSR system (borrowed tensors).

    values [n_par, m] float64/float32 (n_par = n_astro + 3 x 4 (if n_axes) +
    n_instr + n_glob; 24 for the full layout), star_of_row [m] int64
    (non-decreasing), att_start [m] int64, instr_idx [n_instr, m] int32;
    optional constraint rows below the observations, CSR on the device:
    con_rowptr [n_con + 1] int64, con_col [nnz] int64, con_val [nnz] float64.
    Row vectors (b, y) then have m_obs + n_con entries (self.m)."""

    def __init__(self, values, star_of_row, att_start, instr_idx, n_stars: int, n_dfa: int,
                 n_instr_cols: int, precondition: bool = True, stream=None, n_astro: int = 5,
                 n_axes: int = 3, n_par_axis: int = 4, n_instr: int = 6, n_glob: int = 1,
                 con_rowptr=None, con_col=None, con_val=None):
        import torch

        lib = load_library()
        m = int(values.shape[1])
        n_par = n_astro + n_axes * n_par_axis + n_instr + n_glob
        if values.dtype not in (torch.float64, torch.float32):
            raise TypeError("values must be float64 or float32")
        n_con = 0 if con_rowptr is None else int(con_rowptr.shape[0]) - 1
        con_ptrs = (ctypes.c_void_p(0),) * 3
        if n_con > 0:
            nnz = int(con_col.shape[0])
            con_ptrs = (_dev_ptr(con_rowptr, torch.int64, (n_con + 1,), "con_rowptr"),
                        _dev_ptr(con_col, torch.int64, (nnz,), "con_col"),
                        _dev_ptr(con_val, torch.float64, (nnz,), "con_val"))
        self._keep = (values, star_of_row, att_start, instr_idx, con_rowptr, con_col, con_val)
        self.m_obs = m
        self.n_con = n_con
        self.m = m + n_con
        self.dtype = values.dtype
        self.device = values.device
        stream = stream if stream is not None else torch.cuda.current_stream(values.device)
        self._stream = stream
        desc = _System(
            n_rows=m, n_stars=int(n_stars), n_astro=int(n_astro), n_axes=int(n_axes),
            n_par_axis=int(n_par_axis), n_instr=int(n_instr), n_dfa=int(n_dfa),
            n_instr_cols=int(n_instr_cols), n_glob=int(n_glob),
            value_type=LSQR_F64 if values.dtype == torch.float64 else LSQR_F32,
            precondition=1 if precondition else 0, reserved=0,
            values=_dev_ptr(values, values.dtype, (n_par, m), "values"),
            star_of_row=_dev_ptr(star_of_row, torch.int64, (m,), "star_of_row"),
            att_start=(_dev_ptr(att_start, torch.int64, (m,), "att_start") if n_axes
                       else ctypes.c_void_p(0)),
            instr_idx=(_dev_ptr(instr_idx, torch.int32, (n_instr, m), "instr_idx") if n_instr
                       else ctypes.c_void_p(0)),
            stream=ctypes.c_void_p(stream.cuda_stream), n_con=n_con, con_rowptr=con_ptrs[0],
            con_col=con_ptrs[1], con_val=con_ptrs[2])
        h = ctypes.c_void_p()
        with torch.cuda.device(values.device):
            _check(lib.lsqr_create(ctypes.byref(desc), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        _check(lib.lsqr_num_cols(h, ctypes.byref(n)))
        self.n = int(n.value)

    @classmethod
    def from_host(cls, system, device="cuda:0", precondition=True, con=None):
        """Upload a synth.System (and optional constraint rows with rowptr, col,
        val host arrays) to the GPU and create a handle."""
        import torch

        sp = system.spec
        t = dict(values=torch.from_numpy(system.values).to(device),
                 star_of_row=torch.from_numpy(system.star_of_row).to(device),
                 att_start=torch.from_numpy(system.att_start).to(device),
                 instr_idx=torch.from_numpy(system.instr_idx).to(device))
        if con is not None:
            t.update(con_rowptr=torch.from_numpy(con.rowptr).to(device),
                     con_col=torch.from_numpy(con.col).to(device),
                     con_val=torch.from_numpy(con.val).to(device))
        torch.cuda.synchronize(device)
        return cls(**t, n_stars=sp.n_stars, n_dfa=sp.n_dfa, n_instr_cols=sp.n_instr_cols,
                   precondition=precondition, n_astro=sp.n_astro, n_axes=sp.n_axes,
                   n_par_axis=sp.n_par_axis, n_instr=sp.n_instr, n_glob=sp.n_glob)

    # ------------------------------------------------------------------ API
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lsqr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, name: str, value: float):
        _check(_lib.lsqr_set_option(self._h, OPTIONS[name], float(value)))

    def aprod1(self, x, y):
        """y += A x (in place, asynchronous on the handle's stream)."""
        import torch

        _check(_lib.lsqr_aprod1(self._h, _dev_ptr(x, torch.float64, (self.n,), "x"),
                                _dev_ptr(y, torch.float64, (self.m,), "y")))
        return y

    def aprod1_noalloc(self, x, y):
        """y += A x like aprod1, through the entry point that allocates nothing
        (its scratch is the library's per-GPU array; overlapping calls race)."""
        import torch

        _check(_lib.lsqr_aprod1_noalloc(self._h, _dev_ptr(x, torch.float64, (self.n,), "x"),
                                        _dev_ptr(y, torch.float64, (self.m,), "y")))
        return y

    def aprod1_f32(self, x, y):
        """y += A x with FP32 vectors and accumulation (FP32-stored systems)."""
        import torch

        _check(_lib.lsqr_aprod1_f32(self._h, _dev_ptr(x, torch.float32, (self.n,), "x"),
                                    _dev_ptr(y, torch.float32, (self.m,), "y")))
        return y

    def aprod2_f32(self, x, y):
        """x += A^T y with FP32 vectors and accumulation (FP32-stored systems)."""
        import torch

        _check(_lib.lsqr_aprod2_f32(self._h, _dev_ptr(x, torch.float32, (self.n,), "x"),
                                    _dev_ptr(y, torch.float32, (self.m,), "y")))
        return x

    def aprod2(self, x, y):
        """x += A^T y (in place, asynchronous on the handle's stream)."""
        import torch

        _check(_lib.lsqr_aprod2(self._h, _dev_ptr(x, torch.float64, (self.n,), "x"),
                                _dev_ptr(y, torch.float64, (self.m,), "y")))
        return x

    def precond(self):
        import torch

        p = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(_lib.lsqr_get_precond(self._h, _dev_ptr(p, torch.float64, (self.n,), "p")))
        return p

    def variance(self):
        """p^2 .* sum (w/rho)^2 of the last solve run with option variance = 1."""
        import torch

        var = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(_lib.lsqr_get_variance(self._h, _dev_ptr(var, torch.float64, (self.n,), "var")))
        return var

    @staticmethod
    def _info(ci: _Info) -> Info:
        return Info(**{k: getattr(ci, k) for k, _ in _Info._fields_ if k != "reserved"})

    def solve(self, b, itn_limit: int, atol: float = 1e-12, btol: float = 1e-12, x=None):
        import torch

        x = torch.empty(self.n, dtype=torch.float64, device=self.device) if x is None else x
        ci = _Info()
        _check(_lib.lsqr_solve(self._h, _dev_ptr(b, torch.float64, (self.m,), "b"),
                               _dev_ptr(x, torch.float64, (self.n,), "x"), int(itn_limit),
                               float(atol), float(btol), ctypes.byref(ci)))
        return x, self._info(ci)

    def solve_refined(self, b, itn_limit: int = 200, atol: float = 1e-6, btol: float = 1e-6,
                      outer_limit: int = 10, x=None):
        import torch

        x = torch.empty(self.n, dtype=torch.float64, device=self.device) if x is None else x
        ci = _Info()
        _check(_lib.lsqr_solve_refined(self._h, _dev_ptr(b, torch.float64, (self.m,), "b"),
                                       _dev_ptr(x, torch.float64, (self.n,), "x"),
                                       int(itn_limit), float(atol), float(btol),
                                       int(outer_limit), ctypes.byref(ci)))
        return x, self._info(ci)

    def solve_batched(self, B, itn_limit: int, atol: float = 1e-12, btol: float = 1e-12, X=None):
        """B: [m, k] float64 (row-interleaved); returns X [n, k] and k Info."""
        import torch

        if B.dim() != 2 or B.shape[0] != self.m:
            raise ValueError(f"B must be [m, k] with m={self.m}")
        k = int(B.shape[1])
        X = torch.empty((self.n, k), dtype=torch.float64, device=self.device) if X is None else X
        infos = (_Info * k)()
        _check(_lib.lsqr_solve_batched(self._h, _dev_ptr(B, torch.float64, (self.m, k), "B"),
                                       _dev_ptr(X, torch.float64, (self.n, k), "X"), k,
                                       int(itn_limit), float(atol), float(btol), infos))
        return X, [self._info(ci) for ci in infos]

    def solve_batched_refined(self, B, itn_limit: int = 200, atol: float = 1e-6,
                              btol: float = 1e-6, outer_limit: int = 10, X=None):
        """FP32-stored system: B [m, k] float64; FP64 refinement per RHS around
        FP32 inner solves advancing together. Returns X [n, k] and k Info."""
        import torch

        if B.dim() != 2 or B.shape[0] != self.m:
            raise ValueError(f"B must be [m, k] with m={self.m}")
        k = int(B.shape[1])
        X = torch.empty((self.n, k), dtype=torch.float64, device=self.device) if X is None else X
        infos = (_Info * k)()
        _check(_lib.lsqr_solve_batched_refined(
            self._h, _dev_ptr(B, torch.float64, (self.m, k), "B"),
            _dev_ptr(X, torch.float64, (self.n, k), "X"), k, int(itn_limit), float(atol),
            float(btol), int(outer_limit), infos))
        return X, [self._info(ci) for ci in infos]

    def batch_tuning(self):
        k = ctypes.c_int32()
        ms = (ctypes.c_double * 5)()
        _check(_lib.lsqr_batch_tuning(self._h, ctypes.byref(k), ms))
        return {"k_tile": k.value, "ms_per_rhs_iter": {1 << i: ms[i] for i in range(5)}}

    def kernel_times(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        na, nb = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.lsqr_kernel_times(self._h, ctypes.byref(a), ctypes.byref(na),
                                      ctypes.byref(b), ctypes.byref(nb)))
        return {"aprod1_ms": a.value, "aprod1_n": na.value, "aprod2_ms": b.value,
                "aprod2_n": nb.value}

    def pass_times(self):
        """Profiled milliseconds and iteration counts of the attitude pre-pass,
        the fused (aprod1) pass and the attitude (aprod2) pass, the fused mode
        of the last solve ("mode") and whether its fused passes read the
        compact index copies ("compact")."""
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        mode, compact = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.lsqr_pass_times(self._h, ms, n, ctypes.byref(mode), ctypes.byref(compact)))
        out = {name: (ms[i], n[i]) for i, name in enumerate(("pre", "fused", "attitude"))}
        out["mode"] = mode.value
        out["compact"] = compact.value
        return out
