"""Seeded synthetic AVU-GSR systems (input plumbing shared by the oracle tests,
the GPU tests and the benchmark).

The row structure follows the paper's description of the coefficient matrix
(Sect. 2): observations grouped by star, per row 5 astrometric coefficients at
the star's columns, 3 attitude axes x 4 consecutive B-spline columns sharing
one start t_i with stride N_DFA between axes, 6 instrumental columns scattered
without pattern, and 1 global column. The real Gaia datasets are not
available; these arrays stand in for them.

Nothing here multiplies by the matrix: callers form b = A x_true + noise with
their own aprod.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile libsynth.so in place (gcc, OpenMP)."""
    import subprocess

    src = os.path.join(_HERE, "synth.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-ffp-contract=off", "-o", _LIB_PATH + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_GPU_LIB_PATH = os.path.join(_HERE, "libsynth_gpu.so")
_gpu_lib = None


def build_gpu(verbose: bool = False) -> str:
    """Compile libsynth_gpu.so (the on-GPU twin of the generator) for gfx950."""
    import subprocess

    src = os.path.join(_HERE, "synth_gpu.hip")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-o", _GPU_LIB_PATH + ".tmp", src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_GPU_LIB_PATH + ".tmp", _GPU_LIB_PATH)
    return _GPU_LIB_PATH


def _load_gpu():
    global _gpu_lib
    if _gpu_lib is not None:
        return _gpu_lib
    if not os.path.exists(_GPU_LIB_PATH):
        raise RuntimeError(f"{_GPU_LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(_GPU_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, u64, u32, f64 = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                               ctypes.c_uint32, ctypes.c_double)
    lib.synth_gpu_star_of_row.argtypes = [P, i64, i64, P, P]
    lib.synth_gpu_rows.argtypes = [u64, i64, i64, i64, P, i32, i32, i32, i64, i32, i64, i32,
                                   f64, f64, f64, i32, P, P, P, P]
    lib.synth_gpu_normals.argtypes = [u64, u32, i64, i64, f64, P, P]
    for f in (lib.synth_gpu_star_of_row, lib.synth_gpu_rows, lib.synth_gpu_normals):
        f.restype = ctypes.c_int
    _gpu_lib = lib
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, u64, u32, f64 = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                               ctypes.c_uint32, ctypes.c_double)
    lib.synth_philox4x32_10.argtypes = [P, P, P]
    lib.synth_philox4x32_10.restype = None
    lib.synth_star_counts.argtypes = [u64, i64, i32, i32, P]
    lib.synth_star_counts.restype = None
    lib.synth_star_of_row.argtypes = [P, i64, i64, i64, P]
    lib.synth_star_of_row.restype = None
    lib.synth_rows.argtypes = [u64, i64, i64, i64, P, i32, i32, i32, i64, i32, i64, i32,
                               f64, f64, f64, i32, P, P, P]
    lib.synth_rows.restype = None
    lib.synth_normals.argtypes = [u64, u32, i64, i64, f64, P]
    lib.synth_normals.restype = None
    lib.synth_test_ln.argtypes = [f64]
    lib.synth_test_ln.restype = f64
    lib.synth_test_exp.argtypes = [f64]
    lib.synth_test_exp.restype = f64
    _lib = lib
    return lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def philox4x32_10(ctr, key) -> tuple:
    """Raw Philox4x32-10 block: four 32-bit words from (counter[4], key[2])."""
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.synth_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return tuple(int(v) for v in out)


@dataclass(frozen=True)
class Spec:
    """Shape of one synthetic system.

    obs_lo == obs_hi gives a fixed number of observations per star; otherwise
    each star draws its count uniformly in [obs_lo, obs_hi]."""
    n_stars: int
    obs_lo: int
    obs_hi: int
    n_dfa: int
    n_instr_cols: int
    seed: int
    value_dtype: str = "f64"  # "f64" or "f32" (values drawn in double, rounded once)
    n_astro: int = 5
    n_axes: int = 3
    n_par_axis: int = 4
    n_instr: int = 6
    n_glob: int = 1
    astro_scale: tuple | None = None  # (lo, hi) exponent range of 10^U(lo,hi)
    # correlation rho in [0, 1) of astrometric coefficients 1.. with the first
    # (harder conditioning: kappa of the scaled per-star blocks ~ 1/sqrt(1-rho))
    astro_corr: float = 0.0
    noise_sigma: float = 1e-6
    n_rhs: int = 1

    def __post_init__(self):
        if not 0.0 <= self.astro_corr < 1.0:
            raise ValueError("astro_corr must be in [0, 1)")

    @property
    def n_par(self) -> int:
        return self.n_astro + self.n_axes * self.n_par_axis + self.n_instr + self.n_glob

    @property
    def n_cols(self) -> int:
        return (self.n_astro * self.n_stars + self.n_axes * self.n_dfa
                + self.n_instr_cols + self.n_glob)

    def scaled(self, **kw) -> "Spec":
        return replace(self, **kw)


BASE_SEED = 20230801

# The five workloads: a parity-sized system, the single-GPU production share,
# the mixed-precision system, the batched system and the largest system.
WORKLOADS = {
    0: Spec(n_stars=1_000, obs_lo=100, obs_hi=100, n_dfa=1_000, n_instr_cols=120,
            seed=BASE_SEED + 0),
    1: Spec(n_stars=1_000_000, obs_lo=100, obs_hi=100, n_dfa=100_000, n_instr_cols=6_000,
            seed=BASE_SEED + 1),
    2: Spec(n_stars=4_000_000, obs_lo=100, obs_hi=100, n_dfa=400_000, n_instr_cols=12_000,
            seed=BASE_SEED + 2, value_dtype="f32", astro_scale=(-2.0, 2.0)),
    3: Spec(n_stars=1_000_000, obs_lo=100, obs_hi=100, n_dfa=100_000, n_instr_cols=6_000,
            seed=BASE_SEED + 3, n_rhs=16),
    4: Spec(n_stars=10_000_000, obs_lo=50, obs_hi=150, n_dfa=1_000_000, n_instr_cols=30_000,
            seed=BASE_SEED + 4, value_dtype="f32", n_rhs=4),
}


def star_layout(spec: Spec) -> np.ndarray:
    """first_row[s] for s in [0, n_stars]; first_row[-1] is the row count."""
    lib = _load()
    counts = np.empty(spec.n_stars, dtype=np.int64)
    lib.synth_star_counts(spec.seed, spec.n_stars, spec.obs_lo, spec.obs_hi, _ptr(counts))
    first = np.zeros(spec.n_stars + 1, dtype=np.int64)
    np.cumsum(counts, out=first[1:])
    return first


@dataclass
class System:
    spec: Spec
    first_row: np.ndarray       # [n_stars + 1]
    values: np.ndarray          # [n_par, m] float64 or float32
    star_of_row: np.ndarray     # [m] int64, non-decreasing
    att_start: np.ndarray       # [m] int64
    instr_idx: np.ndarray       # [n_instr, m] int32
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.first_row[-1])

    @property
    def n(self) -> int:
        return self.spec.n_cols


def rows(spec: Spec, first_row: np.ndarray, r0: int, r1: int, values_out=None,
         star_out=None, att_out=None, instr_out=None):
    """Fill rows [r0, r1) into (optionally preallocated) SoA arrays."""
    lib = _load()
    nr = r1 - r0
    vdt = np.float64 if spec.value_dtype == "f64" else np.float32
    values = values_out if values_out is not None else np.empty((spec.n_par, nr), dtype=vdt)
    star = star_out if star_out is not None else np.empty(nr, dtype=np.int64)
    att = att_out if att_out is not None else np.empty(nr, dtype=np.int64)
    instr = instr_out if instr_out is not None else np.empty((spec.n_instr, nr), dtype=np.int32)
    assert values.dtype == vdt and values.shape == (spec.n_par, nr)
    lib.synth_star_of_row(_ptr(first_row), spec.n_stars, r0, r1, _ptr(star))
    lo, hi = spec.astro_scale if spec.astro_scale else (0.0, 0.0)
    lib.synth_rows(spec.seed, r0, r1, nr, _ptr(star), spec.n_astro, spec.n_axes,
                   spec.n_par_axis, spec.n_dfa, spec.n_instr, spec.n_instr_cols, spec.n_glob,
                   float(lo), float(hi), float(spec.astro_corr), 0 if vdt is np.float64 else 1,
                   _ptr(values), _ptr(att), _ptr(instr))
    return values, star, att, instr


def make_system(spec: Spec) -> System:
    first = star_layout(spec)
    m = int(first[-1])
    values, star, att, instr = rows(spec, first, 0, m)
    return System(spec=spec, first_row=first, values=values, star_of_row=star,
                  att_start=att, instr_idx=instr)


@dataclass
class Constraints:
    """Extra equations appended below the observation rows, in CSR form:
    row r has the coefficients val[rowptr[r]:rowptr[r+1]] at the unknowns
    col[rowptr[r]:rowptr[r+1]]."""
    rowptr: np.ndarray  # [n_con + 1] int64
    col: np.ndarray     # [nnz] int64
    val: np.ndarray     # [nnz] float64

    @property
    def n_con(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def constraints(spec: Spec, n_con: int, nnz=(0, 200), seed: int = 0,
                cols: tuple | None = None, row_norm: float | None = None) -> Constraints:
    """n_con constraint rows: each row draws its length uniformly in
    [nnz[0], nnz[1]] (at most the number of candidate columns), distinct
    columns uniformly from [cols[0], cols[1]) (default: every unknown) in
    ascending order, and N(0, 1) coefficients, rescaled so that every
    non-empty row has 2-norm row_norm when given (sqrt(n_par) weighs a
    constraint like an observation). The paper leaves the content of its
    constraint equations to another work; these rows have its structure (few
    rows at the bottom of the system, long and sparse)."""
    lo_c, hi_c = cols if cols is not None else (0, spec.n_cols)
    span = hi_c - lo_c
    rng = np.random.default_rng([spec.seed, 7, seed])
    lens = rng.integers(nnz[0], nnz[1] + 1, size=n_con)
    lens = np.minimum(lens, span)
    rowptr = np.zeros(n_con + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    col = np.empty(int(rowptr[-1]), dtype=np.int64)
    for r in range(n_con):
        pick = rng.choice(span, size=int(lens[r]), replace=False)
        col[rowptr[r]:rowptr[r + 1]] = np.sort(pick) + lo_c
    val = rng.standard_normal(int(rowptr[-1]))
    if row_norm is not None:
        for r in range(n_con):
            sl = slice(int(rowptr[r]), int(rowptr[r + 1]))
            if sl.stop > sl.start:
                val[sl] *= row_norm / np.linalg.norm(val[sl])
    return Constraints(rowptr=rowptr, col=col, val=val)


def x_true(spec: Spec) -> np.ndarray:
    lib = _load()
    out = np.empty(spec.n_cols, dtype=np.float64)
    lib.synth_normals(spec.seed, 2, 0, spec.n_cols, 1.0, _ptr(out))
    return out


def noise(spec: Spec, m: int, rhs: int = 0, i0: int = 0, i1: int | None = None) -> np.ndarray:
    """N(0, noise_sigma) per row (stream 3 + rhs); the standard deviation is sigma."""
    lib = _load()
    i1 = m if i1 is None else i1
    out = np.empty(i1 - i0, dtype=np.float64)
    lib.synth_normals(spec.seed, 3 + rhs, i0, i1, float(spec.noise_sigma), _ptr(out))
    return out


def tiny(seed: int = 7, n_stars: int = 20, obs=(30, 30), n_dfa: int = 20,
         n_instr_cols: int = 12, value_dtype: str = "f64", **kw) -> Spec:
    """Small systems for brute-force checks."""
    return Spec(n_stars=n_stars, obs_lo=obs[0], obs_hi=obs[1], n_dfa=n_dfa,
                n_instr_cols=n_instr_cols, seed=seed, value_dtype=value_dtype, **kw)


# ------------------------------------------------------------ on-GPU twin
def device_system(spec: Spec, device="cuda:0"):
    """Generate the whole system directly in GPU memory (torch tensors), bit
    for bit the arrays make_system would produce on the host."""
    import torch

    lib = _load_gpu()
    first = star_layout(spec)
    m = int(first[-1])
    dev = torch.device(device)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    vdt = torch.float64 if spec.value_dtype == "f64" else torch.float32
    first_d = torch.from_numpy(first).to(dev)
    star = torch.empty(m, dtype=torch.int64, device=dev)
    att = torch.empty(m, dtype=torch.int64, device=dev)
    instr = torch.empty((spec.n_instr, m), dtype=torch.int32, device=dev)
    values = torch.empty((spec.n_par, m), dtype=vdt, device=dev)
    rc = lib.synth_gpu_star_of_row(first_d.data_ptr(), spec.n_stars, m, star.data_ptr(), stream)
    if rc != 0:
        raise RuntimeError(f"synth_gpu_star_of_row failed ({rc})")
    lo, hi = spec.astro_scale if spec.astro_scale else (0.0, 0.0)
    rc = lib.synth_gpu_rows(spec.seed, 0, m, m, star.data_ptr(), spec.n_astro, spec.n_axes,
                            spec.n_par_axis, spec.n_dfa, spec.n_instr, spec.n_instr_cols,
                            spec.n_glob, float(lo), float(hi), float(spec.astro_corr),
                            0 if vdt == torch.float64 else 1,
                            values.data_ptr(), att.data_ptr(), instr.data_ptr(), stream)
    if rc != 0:
        raise RuntimeError(f"synth_gpu_rows failed ({rc})")
    return dict(values=values, star_of_row=star, att_start=att, instr_idx=instr), first


def device_normals(spec: Spec, stream_id: int, n: int, sigma: float, device="cuda:0",
                   i0: int = 0):
    """sigma * N(0,1) draws i0..i0+n of a stream, generated on the GPU."""
    import torch

    lib = _load_gpu()
    dev = torch.device(device)
    out = torch.empty(n, dtype=torch.float64, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rc = lib.synth_gpu_normals(spec.seed, stream_id, i0, i0 + n, float(sigma), out.data_ptr(),
                               stream)
    if rc != 0:
        raise RuntimeError(f"synth_gpu_normals failed ({rc})")
    return out


def device_x_true(spec: Spec, device="cuda:0"):
    return device_normals(spec, 2, spec.n_cols, 1.0, device)


def device_noise(spec: Spec, m: int, rhs: int = 0, device="cuda:0"):
    return device_normals(spec, 3 + rhs, m, spec.noise_sigma, device)
