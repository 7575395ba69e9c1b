"""Oracle for the AVU-GSR LSQR solve: Python access to the plain FP64 C
implementation in oracle.c.

TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's
CPU-baseline leg may use it; the GPU library never imports, links or calls it.
It shares no code with the GPU path; only the seeded input generator (synth)
feeds both.

Pinned by tests/test_oracle_pins.py against dense brute force, the adjoint
identity, LAPACK least squares, SciPy's LSQR, CGLS, closed forms and
invariants. Parity pinned for: aprod1, aprod2, the Eq. (4) norm, the column
norms, the LSQR iterates and estimates, and the variance estimate (loosely, in
its limit), on the full row layout, section subsets and with constraint rows. The physical meaning of the attitude B-spline and instrumental
coefficients is not modelled (synthetic N(0,1) values): parity unpinned there
by construction, since it does not enter the arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# Timing build of the same source (OpenMP, -O3): the CPU baseline only.
OMP_LIB_PATH = os.path.join(_HERE, "liboracle_omp.so")
_lib = None


def build(verbose: bool = False, src: str | None = None, out: str | None = None,
          openmp: bool = False) -> str:
    """Compile liboracle.so: single thread, -O2, no floating-point contraction
    (the pinned reference build). openmp=True compiles the timing build
    liboracle_omp.so from the same source (-O3 -fopenmp).

    src/out let the mutation tests compile a modified copy elsewhere."""
    src = src or os.path.join(_HERE, "oracle.c")
    out = out or (OMP_LIB_PATH if openmp else _LIB_PATH)
    flags = (["-O3", "-fopenmp"] if openmp else ["-O2"]) + ["-ffp-contract=off", "-fno-fast-math"]
    cmd = ["gcc", *flags, "-fPIC", "-shared", "-std=c11", "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def num_threads() -> int:
    """Threads the loaded build runs on (1 for the reference build)."""
    return int(_load().orc_num_threads())


class _Sys(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n_stars", ctypes.c_int64),
                ("n_astro", ctypes.c_int32), ("n_axes", ctypes.c_int32),
                ("n_par_axis", ctypes.c_int32), ("n_dfa", ctypes.c_int64),
                ("n_instr", ctypes.c_int32), ("n_instr_cols", ctypes.c_int64),
                ("n_glob", ctypes.c_int32), ("value_is_f32", ctypes.c_int32),
                ("values", ctypes.c_void_p), ("star", ctypes.c_void_p),
                ("att", ctypes.c_void_p), ("instr", ctypes.c_void_p),
                ("n_con", ctypes.c_int64), ("con_rowptr", ctypes.c_void_p),
                ("con_col", ctypes.c_void_p), ("con_val", ctypes.c_void_p)]


class _Info(ctypes.Structure):
    _fields_ = [("istop", ctypes.c_int32), ("itn", ctypes.c_int32),
                ("rnorm", ctypes.c_double), ("arnorm", ctypes.c_double),
                ("anorm", ctypes.c_double), ("acond", ctypes.c_double),
                ("xnorm", ctypes.c_double), ("bnorm", ctypes.c_double)]


def use_library(path: str | None) -> None:
    """Point the wrapper at another build of oracle.c (None: the default one)."""
    global _lib, _lib_path
    _lib = None
    _lib_path = path or _LIB_PATH


_lib_path = _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_lib_path):
        raise RuntimeError(f"{_lib_path} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(_lib_path)
    P = ctypes.c_void_p
    S = ctypes.POINTER(_Sys)
    lib.orc_ncols.argtypes = [S]
    lib.orc_ncols.restype = ctypes.c_int64
    lib.orc_aprod1.argtypes = [S, P, P]
    lib.orc_aprod1.restype = None
    lib.orc_aprod1_rows.argtypes = [S, P, P, ctypes.c_int64, P]
    lib.orc_aprod1_rows.restype = None
    lib.orc_aprod2.argtypes = [S, P, P]
    lib.orc_aprod2.restype = None
    lib.orc_norm.argtypes = [P, ctypes.c_int64]
    lib.orc_norm.restype = ctypes.c_double
    lib.orc_precond.argtypes = [S, P]
    lib.orc_precond.restype = None
    lib.orc_lsqr.argtypes = [S, P, P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                             ctypes.POINTER(_Info), P]
    lib.orc_lsqr.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int32
    _lib = lib
    return lib


@dataclass
class Info:
    istop: int
    itn: int
    rnorm: float
    arnorm: float
    anorm: float
    acond: float
    xnorm: float
    bnorm: float


class OracleSystem:
    """Host view of a system in the shared SoA layout.

    values [n_par, m_obs] (float64 or float32: float32 is widened on read),
    star_of_row [m_obs] int64, att_start [m_obs] int64, instr_idx [n_instr, m_obs]
    int32; con (optional): constraint rows (rowptr, col, val attributes, CSR)
    appended below the observations. m = m_obs + n_con is the length of b."""

    def __init__(self, values, star_of_row, att_start, instr_idx, n_stars, n_dfa,
                 n_instr_cols, n_astro=5, n_axes=3, n_par_axis=4, n_instr=6, n_glob=1,
                 con=None):
        self._keep = [np.ascontiguousarray(values), np.ascontiguousarray(star_of_row, np.int64),
                      np.ascontiguousarray(att_start, np.int64),
                      np.ascontiguousarray(instr_idx, np.int32)]
        vals, star, att, instr = self._keep
        assert vals.dtype in (np.float64, np.float32)
        self.m_obs = int(vals.shape[1])
        n_con, rp, cc, cv = 0, None, None, None
        if con is not None:
            rp = np.ascontiguousarray(con.rowptr, np.int64)
            cc = np.ascontiguousarray(con.col, np.int64)
            cv = np.ascontiguousarray(con.val, np.float64)
            n_con = int(rp.shape[0] - 1)
            assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and cc.shape == cv.shape == (rp[-1],)
            self._keep += [rp, cc, cv]
        self.n_con = n_con
        self.m = self.m_obs + n_con
        self.c = _Sys(m=self.m_obs, n_stars=n_stars, n_astro=n_astro, n_axes=n_axes,
                      n_par_axis=n_par_axis, n_dfa=n_dfa, n_instr=n_instr,
                      n_instr_cols=n_instr_cols, n_glob=n_glob,
                      value_is_f32=1 if vals.dtype == np.float32 else 0,
                      values=vals.ctypes.data, star=star.ctypes.data, att=att.ctypes.data,
                      instr=instr.ctypes.data, n_con=n_con,
                      con_rowptr=None if rp is None else rp.ctypes.data,
                      con_col=None if cc is None else cc.ctypes.data,
                      con_val=None if cv is None else cv.ctypes.data)
        self.n = int(_load().orc_ncols(ctypes.byref(self.c)))
        if cc is not None and cc.size:
            assert cc.min() >= 0 and cc.max() < self.n

    @classmethod
    def from_synth(cls, system, con=None) -> "OracleSystem":
        sp = system.spec
        return cls(system.values, system.star_of_row, system.att_start, system.instr_idx,
                   n_stars=sp.n_stars, n_dfa=sp.n_dfa, n_instr_cols=sp.n_instr_cols,
                   n_astro=sp.n_astro, n_axes=sp.n_axes, n_par_axis=sp.n_par_axis,
                   n_instr=sp.n_instr, n_glob=sp.n_glob, con=con)

    # -- operators -----------------------------------------------------------
    def aprod1(self, x, y=None):
        """y + A x (y defaults to zeros)."""
        x = np.ascontiguousarray(x, np.float64)
        assert x.shape == (self.n,)
        out = np.zeros(self.m) if y is None else np.array(y, dtype=np.float64, copy=True)
        _load().orc_aprod1(ctypes.byref(self.c), x.ctypes.data, out.ctypes.data)
        return out

    def aprod1_rows(self, x, rows):
        x = np.ascontiguousarray(x, np.float64)
        rows = np.ascontiguousarray(rows, np.int64)
        out = np.zeros(rows.shape[0])
        _load().orc_aprod1_rows(ctypes.byref(self.c), x.ctypes.data, rows.ctypes.data,
                                rows.shape[0], out.ctypes.data)
        return out

    def aprod2(self, y, x=None):
        """x + A^T y (x defaults to zeros)."""
        y = np.ascontiguousarray(y, np.float64)
        assert y.shape == (self.m,)
        out = np.zeros(self.n) if x is None else np.array(x, dtype=np.float64, copy=True)
        _load().orc_aprod2(ctypes.byref(self.c), out.ctypes.data, y.ctypes.data)
        return out

    def precond(self):
        p = np.empty(self.n)
        _load().orc_precond(ctypes.byref(self.c), p.ctypes.data)
        return p

    def lsqr(self, b, itn_limit, atol=1e-12, btol=1e-12, conlim=1e8, precondition=True,
             tests=True, want_var=False):
        b = np.ascontiguousarray(b, np.float64)
        assert b.shape == (self.m,)
        x = np.zeros(self.n)
        var = np.zeros(self.n) if want_var else None
        info = _Info()
        rc = _load().orc_lsqr(ctypes.byref(self.c), b.ctypes.data, x.ctypes.data,
                              int(itn_limit), float(atol), float(btol), float(conlim),
                              1 if precondition else 0, 1 if tests else 0, ctypes.byref(info),
                              None if var is None else var.ctypes.data)
        if rc != 0:
            raise MemoryError("oracle lsqr: allocation failed")
        inf = Info(**{k: getattr(info, k) for k, _ in _Info._fields_})
        return (x, inf, var) if want_var else (x, inf)


def norm(a) -> float:
    """Eq. (4) max-scaled 2-norm."""
    a = np.ascontiguousarray(a, np.float64)
    return float(_load().orc_norm(a.ctypes.data, a.shape[0]))
