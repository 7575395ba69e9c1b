"""Benchmark: LSQR iterations per second on the AVU-GSR system, one MI355X.

Workload (default): 1,000,000 stars x 100 observations = 1e8 rows, FP64
values (19.2 GB), 3 x 100,000 attitude columns, 6,000 instrumental columns,
1 global column (5,306,001 unknowns); synthetic seeded inputs shaped like the
paper's system. A step is one LSQR iteration (aprod1, beta, aprod2, alpha,
Givens rotation, x/w update, stopping tests); the timed region is one
lsqr_solve of exactly `steps` iterations (stopping tests off; its start and
end, one aprod2 and a few vector kernels, included) with HIP events around
every launch of the row passes on the stream they run on: the attitude
pre-pass, the fused pass (the rest of aprod1 with the astrometric,
instrumental and global part of aprod2) and the bucket-order attitude pass.
The same iterations with other pass arrangements are timed for comparison,
then the extra legs: FP32 storage + FP64 refinement (4e8 rows), batched
right-hand sides (1e8 rows, k = 16), the largest system (1e9 rows, FP32,
refined and batched, k = 4), and the oracle on the host cores.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E


def bytes_per_row(vb: int, ub: int):
    """Algorithmic bytes per row and launch of each row pass, for values of vb
    bytes and a row vector u of ub bytes (index layout: int64 star, int64
    attitude start, 6 int32 instrumental indices = 40 B; in bucket order an
    int32 local attitude start):
      aprod1: 24 values + indices + u read and written
      aprod2: 24 values + indices + u read
      fused (fused mode 1): as aprod1, A read once for both products
      attitude_dot (mode 2): 12 attitude values + local start + u read and
        written, in bucket order
      fused_rest (mode 2): the 12 other values + star and instrumental
        indices + u read and written
      attitude: 12 attitude values + local start + u read, in bucket order"""
    return {"aprod1": 24 * vb + 40 + 2 * ub, "aprod2": 24 * vb + 40 + ub,
            "fused": 24 * vb + 40 + 2 * ub, "attitude_dot": 12 * vb + 4 + 2 * ub,
            "fused_rest": 12 * vb + 32 + 2 * ub, "attitude": 12 * vb + 4 + ub}


BYTES_PER_ROW = bytes_per_row(8, 8)      # FP64 values and vectors
# Named variant: with compact index copies (LSQR_OPT_COMPACT_INDEX) the fused
# pass reads an int32 star and six uint16 instrumental indices, 16 bytes less
# per row than the configured layout; the canonical figures keep the
# configured bytes.
COMPACT_SAVING = 16
BYTES_PER_ROW_F32 = bytes_per_row(4, 4)  # the FP32 inner solve of the refinement


def pass_times(g, mode=None):
    """Per-iteration milliseconds of the row passes of the last profiled solve
    (fused mode 2: attitude pre-pass, rest of the fused pass, attitude pass;
    1: fused pass, attitude pass; 0: aprod1, aprod2); mode None: the mode the
    solve ran."""
    pt = g.pass_times()
    mode = pt.pop("mode") if mode is None else mode
    pt.pop("mode", None)
    pt.pop("compact", None)
    per = {k: ms / max(1, n) for k, (ms, n) in pt.items()}
    if mode in (2, 3):
        return {"attitude_dot": per["pre"], "fused_rest": per["fused"],
                "attitude": per["attitude"]}
    a, b = ("fused", "attitude") if mode == 1 else ("aprod1", "aprod2")
    return {a: per["pre"] + per["fused"], b: per["attitude"]}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_fused_c1_fp64.txt")
KERNEL_SOURCES = ("paper_2308_00778_amd/csrc/kernels.hpp", "paper_2308_00778_amd/csrc/lsqr.hip")


def counter_traffic(kernel: str):
    """HBM bytes per launch of `kernel` on the 1e8-row workload, measured with
    rocprofv3 counters (FETCH_SIZE, WRITE_SIZE, calibrated on a device copy) and
    recorded in the committed profile summary; None when the kernel sources
    differ from the ones that were profiled."""
    import hashlib

    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    rec, sha = {}, None
    with open(TRAFFIC_PROFILE) as fh:
        for line in fh:
            w = line.split()
            if len(w) == 3 and w[0] == "traffic_bytes_per_launch":
                rec[w[1]] = float(w[2])
            elif len(w) == 2 and w[0] == "sources_sha256":
                sha = w[1]
    if sha != h.hexdigest():
        return None
    return rec.get(kernel)


def host_ram_gb():
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal:"):
                    return int(line.split()[1]) / 1e6
    except OSError:
        pass
    return None


def cpu_baseline(spec, dev, itn=(1, 6)):
    """The oracle's OpenMP timing build (the same source as the pinned
    single-thread oracle, -O3 -fopenmp) on all host cores, on the full
    workload: the system generated on the GPU and copied to host memory, b
    formed there too; LSQR runs of itn[0] and itn[1] iterations timed, the
    difference per iteration is the figure (set-up excluded)."""
    import torch

    import oracle
    import synth

    if not os.path.exists(oracle.OMP_LIB_PATH):
        oracle.build(openmp=True)
    oracle.use_library(oracle.OMP_LIB_PATH)
    try:
        arrays, first = synth.device_system(spec, dev)
        m = int(first[-1])
        host = {k: v.cpu().numpy() for k, v in arrays.items()}
        del arrays
        torch.cuda.empty_cache()
        o = oracle.OracleSystem(host["values"], host["star_of_row"], host["att_start"],
                                host["instr_idx"], n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                                n_instr_cols=spec.n_instr_cols)
        b = o.aprod1(synth.x_true(spec), synth.noise(spec, m))
        t = []
        for k in itn:
            t0 = time.perf_counter()
            o.lsqr(b, k, atol=0.0, btol=0.0, conlim=0.0, tests=False)
            t.append(time.perf_counter() - t0)
        per_iter = (t[1] - t[0]) / (itn[1] - itn[0])
        threads = oracle.num_threads()
    finally:
        oracle.use_library(None)
    return {"value": 1.0 / per_iter, "unit": "iter/s", "cores": threads, "kind": "oracle",
            "sample": f"the full workload ({m} rows, FP64) in host memory; the oracle's OpenMP "
                      f"timing build, LSQR runs of {itn[0]} and {itn[1]} iterations timed, "
                      f"difference per iteration {per_iter:.3f} s",
            "nproc": os.cpu_count(), "host_ram_GB": host_ram_gb(),
            "build": "gcc -O3 -fopenmp -ffp-contract=off (oracle/oracle.c)",
            "seconds": sum(t)}


def rel_inf(a, b):
    return float((a - b).abs().max() / b.abs().max())


_sc_lib = None


def _stream_lib():
    """libstreamceil.so: hand-written streaming read / write / copy kernels."""
    global _sc_lib
    if _sc_lib is None:
        import ctypes

        path = os.path.join(ROOT, "paper_2308_00778_amd", "libstreamceil.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built: run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        lib.sc_grid.argtypes, lib.sc_grid.restype = [], ctypes.c_int
        lib.sc_read.argtypes, lib.sc_read.restype = [P, I64, P, P], ctypes.c_int
        lib.sc_write.argtypes, lib.sc_write.restype = [P, I64, P], ctypes.c_int
        lib.sc_copy.argtypes, lib.sc_copy.restype = [P, P, I64, P], ctypes.c_int
        _sc_lib = lib
    return _sc_lib


def _time_launch(fn, reps: int):
    """Median milliseconds of `fn` (launches on torch's current stream),
    timed with events on that stream, after one warm-up."""
    import torch

    fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return sorted(ts)[reps // 2]


def read_rate(bufs, reps: int = 5):
    """GB/s of the hand-written streaming read over the given device tensors
    (one launch each, timed together)."""
    import torch

    lib = _stream_lib()
    sink = torch.empty(lib.sc_grid(), dtype=torch.float64, device=bufs[0].device)
    st = torch.cuda.current_stream().cuda_stream
    total = sum(t.numel() * t.element_size() for t in bufs)

    def go():
        for t in bufs:
            rc = lib.sc_read(t.data_ptr(), t.numel() * t.element_size(), sink.data_ptr(), st)
            if rc != 0:
                raise RuntimeError(f"sc_read failed ({rc})")

    ms = _time_launch(go, reps)
    return total / (ms * 1e-3) / 1e9


def stream_ceiling(dev, gib: float = 20.0, reps: int = 5):
    """Practical HBM ceilings on this GPU with hand-written streaming kernels
    (paper_2308_00778_amd/csrc/stream_ceiling.hip: 16-byte nontemporal loads
    and stores, grid-stride): read and write of a `gib` GiB buffer, and a
    copy of half of it into the other half; median of `reps` runs each."""
    import torch

    lib = _stream_lib()
    nbytes = int(gib * 2**30) & ~255
    buf = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
    st = torch.cuda.current_stream(dev).cuda_stream
    p = buf.data_ptr()
    ms_w = _time_launch(lambda: lib.sc_write(p, nbytes, st), reps)
    out = {"read_GBps": read_rate([buf], reps), "write_GBps": nbytes / (ms_w * 1e-3) / 1e9}
    half = nbytes // 2
    ms_c = _time_launch(lambda: lib.sc_copy(p, p + half, half, st), reps)
    out["copy_GBps"] = 2 * half / (ms_c * 1e-3) / 1e9  # bytes read + written
    out["kernels"] = (f"hand-written streaming read / write / copy (stream_ceiling.hip) over "
                      f"{gib:.0f} GiB, median of {reps}")
    del buf
    torch.cuda.empty_cache()
    return out


def _timed(fn):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def refine_leg(cfg: int, dev):
    """FP32 storage + FP64 refinement against plain FP64 on the same GPU, all
    to convergence at atol = btol = 1e-12 (the FP32-rounded values define
    the system): the comparator is the FP64 solve of an FP64-stored copy of
    those values (the same iteration, twice the value bytes); the FP64 solve
    of the FP32-stored values (widened in registers) is reported beside it."""
    import torch

    import synth
    from paper_2308_00778_amd import LsqrSystem

    spec = synth.WORKLOADS[cfg]
    t0 = time.perf_counter()
    arrays, first = synth.device_system(spec, dev)
    m = int(first[-1])
    kw = dict(n_stars=spec.n_stars, n_dfa=spec.n_dfa, n_instr_cols=spec.n_instr_cols)
    g = LsqrSystem(**arrays, **kw)
    b = synth.device_noise(spec, m, 0, dev)
    g.aprod1(synth.device_x_true(spec, dev), b)
    torch.cuda.synchronize()
    log(f"refine leg: m={m} n={g.n} ready in {time.perf_counter() - t0:.1f} s")
    out = {"workload": f"{spec.n_stars} stars x {spec.obs_lo} obs = {m} rows x {g.n} unknowns, "
                       f"FP32 values, astrometric column scale 10^U{spec.astro_scale}"}
    # plain FP64: an FP64-stored copy of the same values, its own handle
    v64 = arrays["values"].double()
    g64 = LsqrSystem(**{**arrays, "values": v64}, **kw)
    g64.solve(b, 2, atol=0.0, btol=0.0)  # bucket order, graphs
    (x64s, i64s), t_fp64s = _timed(lambda: g64.solve(b, 500, atol=1e-12, btol=1e-12))
    g64.close()
    del v64, g64
    torch.cuda.empty_cache()
    # the FP32-stored handle: FP64 arithmetic on the widened values, and the
    # refined solve
    g.solve(b, 2, atol=0.0, btol=0.0)
    g.solve_refined(b, 2, atol=1e-6, btol=1e-6, outer_limit=1)
    (x64, i64), t_fp64 = _timed(lambda: g.solve(b, 500, atol=1e-12, btol=1e-12))
    (x32, i32), t_ref = _timed(lambda: g.solve_refined(b, 200, atol=1e-6, btol=1e-6,
                                                        outer_limit=10))
    # per-iteration kernel times of the FP32 inner loop
    g.set_option("profile", 1)
    g.solve_refined(b, 20, atol=0.0, btol=0.0, outer_limit=1)
    g.set_option("profile", 0)
    ms = pass_times(g)
    out.update({
        "fp64_stored_seconds": t_fp64s, "fp64_stored_itn": i64s.itn,
        "fp64_stored_istop": i64s.istop,
        "fp64_on_fp32_values_seconds": t_fp64, "fp64_on_fp32_values_itn": i64.itn,
        "refined_seconds": t_ref, "refined_inner_itn": i32.itn,
        "refined_outer_steps": i32.outer_steps,
        "speedup_vs_fp64": t_fp64s / t_ref,
        "speedup_vs_fp64_on_fp32_values": t_fp64 / t_ref,
        "rel_inf_err_vs_fp64": rel_inf(x32, x64s),
        "rel_inf_err_vs_fp64_on_fp32_values": rel_inf(x32, x64),
        "inner_kernels": {k: {"ms": ms[k], "GBps": BYTES_PER_ROW_F32[k] * m / (ms[k] * 1e-3) / 1e9,
                              "bytes_per_row": BYTES_PER_ROW_F32[k]} for k in ms},
    })
    log(f"refine leg: fp64-stored {t_fp64s:.2f} s ({i64s.itn} it), fp64 on fp32 values "
        f"{t_fp64:.2f} s ({i64.itn} it), refined {t_ref:.2f} s ({i32.itn} inner, "
        f"{i32.outer_steps} outer), err {out['rel_inf_err_vs_fp64']:.2e}")
    g.close()
    del arrays, b, x64, x32, x64s
    torch.cuda.empty_cache()
    return out


def attitude_ab(dev, cfg: int = 1, itn: int = 20):
    """Row-pass times of the iteration variants on one system: fused pass vs
    separate aprod1 / aprod2, attitude values interleaved or gathered from the
    three axis windows, and for aprod2 the device-atomics attitude scatter vs
    the bucket-order pass, each astrometric reduction; then the attitude
    bucket count."""
    import torch

    import synth
    from paper_2308_00778_amd import LsqrSystem

    spec = synth.WORKLOADS[cfg]
    arrays, first = synth.device_system(spec, dev)
    m = int(first[-1])
    g = LsqrSystem(**arrays, n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                   n_instr_cols=spec.n_instr_cols)
    b = synth.device_noise(spec, m, 0, dev)
    g.aprod1(synth.device_x_true(spec, dev), b)
    out = {}
    for fused, att, scan, il in ((2, 1, 0, 1), (1, 1, 0, 1), (1, 1, 0, 0), (0, 1, 0, 1),
                                 (0, 1, 0, 0), (0, 1, 1, 1), (0, 0, 0, 1)):
        g.set_option("fused", fused)
        g.set_option("att_mode", att)
        g.set_option("astro_scan", scan)
        g.set_option("att_interleave", il)
        g.set_option("tests", 0)
        g.set_option("profile", 1)
        g.solve(b, 2, atol=0.0, btol=0.0)
        x, info = g.solve(b, itn, atol=0.0, btol=0.0)
        ms = pass_times(g, fused if att == 1 else 0)
        key = ("", "fused_", "fused_att_dot_")[fused] + ("atomics", "bucket_pass")[att] + \
            ("_scan" if scan else "_flush") + ("" if il else "_plain_att_gathers")
        out[key] = {**{f"{k}_ms": v for k, v in ms.items()},
                    "iteration_rows_ms": sum(ms.values()), "rnorm": info.rnorm}
        log(f"{key}: " + ", ".join(f"{k} {v:.3f} ms" for k, v in ms.items()))
    g.close()
    # attitude bucket count (fused default path; a fresh handle per count, the
    # option is fixed once the bucket order exists; 0 = the fewest that fit)
    for nbk in (32, 64):
        g = LsqrSystem(**arrays, n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                       n_instr_cols=spec.n_instr_cols)
        g.set_option("att_buckets", nbk)
        g.set_option("tests", 0)
        g.set_option("profile", 1)
        g.solve(b, 2, atol=0.0, btol=0.0)
        x, info = g.solve(b, itn, atol=0.0, btol=0.0)
        ms = pass_times(g)
        key = f"fused_att_dot_buckets_{nbk}"
        out[key] = {**{f"{k}_ms": v for k, v in ms.items()},
                    "iteration_rows_ms": sum(ms.values()), "rnorm": info.rnorm}
        log(f"{key}: " + ", ".join(f"{k} {v:.3f} ms" for k, v in ms.items()))
        g.close()
    print(json.dumps({"attitude_ab": out, "rows": m, "iterations": itn}))


def batched_leg(cfg: int, dev, singles: int = 2, att_rhs: int = 4):
    """k noise realisations of b solved together (to convergence, atol = btol =
    1e-12) against single-RHS solves of the same right-hand sides. The batched
    handle sizes its attitude buckets for att_rhs right-hand sides per sweep;
    the single solves run on a handle of the default geometry (the fastest
    single-RHS configuration)."""
    import torch

    import synth
    from paper_2308_00778_amd import LsqrSystem

    spec = synth.WORKLOADS[cfg]
    k = spec.n_rhs
    t0 = time.perf_counter()
    arrays, first = synth.device_system(spec, dev)
    m = int(first[-1])
    kw = dict(n_stars=spec.n_stars, n_dfa=spec.n_dfa, n_instr_cols=spec.n_instr_cols)
    g1 = LsqrSystem(**arrays, **kw)
    xt = synth.device_x_true(spec, dev)
    B = torch.empty((m, k), dtype=torch.float64, device=dev)
    for j in range(k):
        bj = synth.device_noise(spec, m, j, dev)
        g1.aprod1(xt, bj)
        B[:, j] = bj
        del bj
    torch.cuda.synchronize()
    log(f"batched leg: m={m} n={g1.n} k={k} ready in {time.perf_counter() - t0:.1f} s")
    # single-RHS solves of the first right-hand sides, same tolerances
    g1.solve(B[:, 0].contiguous(), 3, 0.0, 0.0)  # bucket order, graphs
    t_single, single_itn, xs = 0.0, 0, []
    for j in range(singles):
        bj = B[:, j].contiguous()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        xj, ij = g1.solve(bj, 500, 1e-12, 1e-12)
        torch.cuda.synchronize()
        t_single += time.perf_counter() - t2
        single_itn += ij.itn
        xs.append(xj)
    g1.close()
    per_rhs_iter_single = t_single / single_itn
    g = LsqrSystem(**arrays, **kw)
    g.set_option("att_rhs", att_rhs)
    # autotune (the first call with this k) outside the timed region
    g.set_option("tests", 0)
    g.solve_batched(B, 2, 0.0, 0.0)
    g.set_option("tests", 1)
    tune = g.batch_tuning()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    X, infos = g.solve_batched(B, 500, 1e-12, 1e-12)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t1
    rhs_itn = sum(i.itn for i in infos)
    err = max(rel_inf(X[:, j], xs[j]) for j in range(singles))
    out = {
        "workload": f"{spec.n_stars} stars x {spec.obs_lo} obs = {m} rows x {g.n} unknowns, "
                    f"FP64, k = {k} noise realisations of b",
        "k": k, "att_rhs": att_rhs, "k_tile": tune["k_tile"],
        "autotune_ms_per_rhs_iter": tune["ms_per_rhs_iter"],
        "batched_seconds": t_batch, "rhs_iterations": rhs_itn,
        "rhs_iter_per_s": rhs_itn / t_batch,
        "itn_per_rhs": [i.itn for i in infos], "istop": sorted({i.istop for i in infos}),
        "single_rhs_iter_per_s": 1.0 / per_rhs_iter_single,
        "speedup_vs_single": (rhs_itn / t_batch) * per_rhs_iter_single,
        "max_rel_inf_err_vs_single": err,
    }
    log(f"batched leg: {rhs_itn} RHS-iterations in {t_batch:.2f} s "
        f"({out['rhs_iter_per_s']:.1f}/s, single {out['single_rhs_iter_per_s']:.1f}/s, "
        f"k_tile {tune['k_tile']}, att_rhs {att_rhs}), err vs single {err:.2e}")
    g.close()
    del arrays, B, X
    torch.cuda.empty_cache()
    return out


def largest_leg(cfg: int, dev):
    """The largest single-GPU workload (FP32 values, uneven stars, k = 4
    right-hand sides) in its own form: FP32 storage with FP64 refinement and
    the k right-hand sides batched (lsqr_solve_batched_refined), all to
    convergence at atol = btol = 1e-12, against the single-RHS FP64 solve of
    the same (FP32-rounded) system, and the single-RHS refined solve."""
    import torch

    import synth
    from paper_2308_00778_amd import LsqrSystem

    def free_gb():
        return torch.cuda.mem_get_info(dev)[0] / 1e9

    spec = synth.WORKLOADS[cfg]
    k = spec.n_rhs
    t0 = time.perf_counter()
    arrays, first = synth.device_system(spec, dev)
    m = int(first[-1])
    g = LsqrSystem(**arrays, n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                   n_instr_cols=spec.n_instr_cols)
    xt = synth.device_x_true(spec, dev)
    B = torch.empty((m, k), dtype=torch.float64, device=dev)
    for j in range(k):
        bj = synth.device_noise(spec, m, j, dev)
        g.aprod1(xt, bj)
        B[:, j] = bj
        del bj
    del xt
    torch.cuda.synchronize()
    log(f"largest leg: m={m} n={g.n} k={k} ready in {time.perf_counter() - t0:.1f} s, "
        f"{free_gb():.0f} GB free")
    out = {"workload": f"{spec.n_stars} stars x U{{{spec.obs_lo}..{spec.obs_hi}}} obs = {m} rows "
                       f"x {g.n} unknowns, FP32 values, N_DFA={spec.n_dfa}, "
                       f"{spec.n_instr_cols} instrumental, k = {k}"}
    b = B[:, 0].contiguous()
    g.solve(b, 2, atol=0.0, btol=0.0)
    g.solve_refined(b, 2, atol=1e-6, btol=1e-6, outer_limit=1)
    (x64, i64), t_fp64 = _timed(lambda: g.solve(b, 500, atol=1e-12, btol=1e-12))
    (x32, i32), t_ref = _timed(lambda: g.solve_refined(b, 200, atol=1e-6, btol=1e-6,
                                                        outer_limit=10))
    g.set_option("profile", 1)
    g.set_option("tests", 0)
    g.solve(b, 16, atol=0.0, btol=0.0)
    ms64 = pass_times(g)
    g.solve_refined(b, 16, atol=0.0, btol=0.0, outer_limit=1)
    ms32 = pass_times(g)
    g.set_option("profile", 0)
    g.set_option("tests", 1)
    del b
    torch.cuda.empty_cache()
    # FP64 arithmetic on FP32 values (FP64 row vector); the FP32 inner solve:
    # BYTES_PER_ROW_F32
    bpr64 = bytes_per_row(4, 8)
    out.update({
        "fp64_seconds": t_fp64, "fp64_itn": i64.itn, "fp64_istop": i64.istop,
        "refined_seconds": t_ref, "refined_inner_itn": i32.itn,
        "refined_outer_steps": i32.outer_steps, "speedup_vs_fp64": t_fp64 / t_ref,
        "rel_inf_err_vs_fp64": rel_inf(x32, x64),
        "fp64_kernels": {kk: {"ms": v, "GBps": bpr64[kk] * m / (v * 1e-3) / 1e9,
                              "bytes_per_row": bpr64[kk]} for kk, v in ms64.items()},
        "inner_kernels": {kk: {"ms": v, "GBps": BYTES_PER_ROW_F32[kk] * m / (v * 1e-3) / 1e9,
                               "bytes_per_row": BYTES_PER_ROW_F32[kk]} for kk, v in ms32.items()},
    })
    log(f"largest leg: fp64 {t_fp64:.2f} s ({i64.itn} it), refined {t_ref:.2f} s "
        f"({i32.itn} inner, {i32.outer_steps} outer), err {out['rel_inf_err_vs_fp64']:.2e}; "
        f"{free_gb():.0f} GB free")
    del x32
    torch.cuda.empty_cache()
    # the workload's own form: refined and batched in one solve (autotuned
    # k-tile outside the timed region, on a short inner solve)
    g.set_option("tests", 0)
    g.solve_batched_refined(B, 2, atol=1e-6, btol=1e-6, outer_limit=1)
    g.set_option("tests", 1)
    tune = g.batch_tuning()
    (X, infos), t_b = _timed(lambda: g.solve_batched_refined(B, 200, atol=1e-6, btol=1e-6,
                                                              outer_limit=10))
    inner = sum(i.itn for i in infos)
    out["batched_refined"] = {
        "k": k, "k_tile": tune["k_tile"], "autotune_ms_per_rhs_iter": tune["ms_per_rhs_iter"],
        "seconds": t_b, "inner_rhs_iterations": inner,
        "outer_steps": [i.outer_steps for i in infos], "inner_itn": [i.itn for i in infos],
        # k right-hand sides solved in t_b against k single FP64 / refined solves
        "speedup_vs_fp64_single": k * t_fp64 / t_b,
        "speedup_vs_refined_single": k * t_ref / t_b,
        "rel_inf_err_rhs0_vs_fp64": rel_inf(X[:, 0], x64),
    }
    log(f"largest leg: refined batched {k} RHS in {t_b:.2f} s (k-tile {tune['k_tile']}, "
        f"{inner} inner RHS-iterations), {k * t_fp64 / t_b:.2f}x {k} FP64 solves, err rhs0 "
        f"{out['batched_refined']['rel_inf_err_rhs0_vs_fp64']:.2e}; {free_gb():.0f} GB free")
    g.close()
    del arrays, x64, X, B
    torch.cuda.empty_cache()
    return out


def copy_calibration(dev, gib: float = 4.0, reps: int = 5):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch

    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)  # the workload's timed iteration count
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="refine,batched,largest",
                    help="comma list of extra legs: refine (FP32 + FP64 refinement), "
                         "batched (k right-hand sides), largest (the 1e9-row FP32 "
                         "workload with refinement and k batched right-hand sides, "
                         "about 260 GB of HBM), none")
    ap.add_argument("--copy", action="store_true", help="only run the copy calibration")
    ap.add_argument("--attitude-ab", action="store_true",
                    help="only time the attitude variants of aprod2")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver's "
              "multi-GPU sharding is designed but not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2308_00778_amd import LsqrSystem

    dev = torch.device("cuda:0")
    if args.copy:
        copy_calibration(dev)
        return
    if args.attitude_ab:
        attitude_ab(dev, args.workload)
        return
    spec = synth.WORKLOADS[args.workload]
    assert spec.value_dtype == "f64", "the FP64 bench runs on an FP64 workload"
    t0 = time.perf_counter()
    arrays, first = synth.device_system(spec, dev)
    m = int(first[-1])
    torch.cuda.synchronize()
    log(f"generated m={m} rows on the GPU in {time.perf_counter() - t0:.1f} s")
    g = LsqrSystem(**arrays, n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                   n_instr_cols=spec.n_instr_cols)
    n = g.n
    # b = A x_true + noise, formed on the GPU with the library's aprod1
    xt = synth.device_x_true(spec, dev)
    b = synth.device_noise(spec, m, 0, dev)
    g.aprod1(xt, b)
    torch.cuda.synchronize()
    log(f"handle ready n={n} in {time.perf_counter() - t0:.1f} s")

    g.set_option("tests", 0)
    g.set_option("profile", 1)
    if args.warmup > 0:
        g.solve(b, args.warmup, atol=0.0, btol=0.0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x, info = g.solve(b, args.steps, atol=0.0, btol=0.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    kt = g.kernel_times()
    assert info.itn == args.steps and kt["aprod1_n"] == args.steps == kt["aprod2_n"]
    compact = g.pass_times()["compact"]
    ms = pass_times(g)
    gbps = {k: BYTES_PER_ROW[k] * m / (ms[k] * 1e-3) / 1e9 for k in ms}
    dom = max(ms, key=ms.get)
    # counter-measured HBM bytes per launch (committed profile of this workload)
    traffic = {k: counter_traffic(k) if args.workload == 1 else None for k in ms}
    log(f"timed {args.steps} iterations in {wall:.3f} s; " +
        ", ".join(f"{k} {ms[k]:.3f} ms ({gbps[k]:.0f} GB/s)" for k in ms))

    # graph-replayed iterations (no events) for comparison
    g.set_option("profile", 0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g.solve(b, args.steps, atol=0.0, btol=0.0)
    torch.cuda.synchronize()
    wall_graph = time.perf_counter() - t2
    # the solve's start (u = b, beta, the first aprod2, alpha, v, w) and end
    # (x = p .* y): a solve of 0 iterations, median of 3
    t_init = sorted(_timed(lambda: g.solve(b, 0, atol=0.0, btol=0.0))[1] for _ in range(3))[1]
    # the hand-written streaming read over the system's own arrays (values and
    # index arrays as stored, 232 bytes per row): what a pass that only streams
    # the matrix reaches
    sys_read = read_rate([arrays["values"], arrays["star_of_row"], arrays["att_start"],
                          arrays["instr_idx"]])

    # the same iterations with the attitude dot product inside the fused pass
    # (fused mode 1) and with separate aprod1 / aprod2 launches (mode 0)
    other = {}
    cmp_steps = min(args.steps, 200)
    for mode in (1, 0):
        g.set_option("fused", mode)
        g.set_option("profile", 1)
        g.solve(b, 2, atol=0.0, btol=0.0)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        g.solve(b, cmp_steps, atol=0.0, btol=0.0)
        torch.cuda.synchronize()
        wall_m = time.perf_counter() - t3
        ms_m = pass_times(g, mode)
        other[mode] = {"iter_per_s": cmp_steps / wall_m, "steps": cmp_steps,
                       "kernels": {k: {"ms": v, "GBps": BYTES_PER_ROW[k] * m / (v * 1e-3) / 1e9,
                                       "bytes_per_row": BYTES_PER_ROW[k]}
                                   for k, v in ms_m.items()}}
        log(f"fused mode {mode}: {cmp_steps / wall_m:.1f} iter/s; " +
            ", ".join(f"{k} {v:.3f} ms" for k, v in ms_m.items()))
    g.set_option("fused", 2)

    result = {
        "metric": "LSQR iter/s + aprod HBM GB/s, FP64 vs FP32+refine & batched RHS at 1e-10 err",
        "value": args.steps / wall,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"AVU-GSR LSQR FP64, {spec.n_stars} stars x {spec.obs_lo} obs = "
                               f"{m} rows x {n} unknowns (N_DFA={spec.n_dfa}, "
                               f"{spec.n_instr_cols} instrumental, 1 global), seed {spec.seed}",
                   "rows": m, "unknowns": n, "values": "f64"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": gbps[dom], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": gbps[dom] / HBM_PEAK_GBPS,
                     "traffic": (traffic[dom] / (ms[dom] * 1e-3) / 1e9
                                 if traffic.get(dom) is not None else None)},
        "kernels": {k: {"ms": ms[k], "GBps": gbps[k], "bytes_per_row": BYTES_PER_ROW[k],
                        "frac_of_peak": gbps[k] / HBM_PEAK_GBPS,
                        "counter_bytes_per_launch": traffic[k],
                        **({"compact_index_bytes_per_row": BYTES_PER_ROW[k] - COMPACT_SAVING,
                            "compact_index_GBps": (BYTES_PER_ROW[k] - COMPACT_SAVING) * m
                            / (ms[k] * 1e-3) / 1e9}
                           if compact and k in ("fused", "fused_rest") else {})}
                    for k in ms},
        "graph_iter_per_s": args.steps / wall_graph,
        # value counts the solve's start and end in its timed region; without them:
        "iterations_only": {"iter_per_s": args.steps / (wall - t_init), "init_ms": t_init * 1e3},
        "fused_att_in_pass": other[1],
        "unfused": other[0],
        "solve_info": {"itn": info.itn, "istop": info.istop, "rnorm": info.rnorm},
    }
    g.close()
    del arrays, b, xt, x
    torch.cuda.empty_cache()
    sc = stream_ceiling(dev)
    sc["system_read_GBps"] = sys_read
    sc["dominant_kernel_frac_of_read"] = gbps[dom] / sc["read_GBps"]
    result["stream_ceiling"] = sc
    log(f"stream ceiling: read {sc['read_GBps']:.0f} GB/s (system arrays {sys_read:.0f}), "
        f"write {sc['write_GBps']:.0f} GB/s, copy {sc['copy_GBps']:.0f} GB/s")
    forms = [f for f in args.forms.split(",") if f and f != "none"]

    def leg(key, fn, *a):
        # a failing extra leg (e.g. device memory) is reported in its own
        # entry; the headline measurement above stands and is still printed
        try:
            result[key] = fn(*a)
        except Exception as e:  # noqa: BLE001
            log(f"{key}: failed: {e}")
            result[key] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()

    if "refine" in forms:
        leg("fp32_refine", refine_leg, 2, dev)
    if "batched" in forms:
        leg("batched", batched_leg, 3, dev)
    if "largest" in forms:
        leg("largest", largest_leg, 4, dev)
    if not args.no_cpu_baseline:
        log("timing the oracle (OpenMP timing build) on the full workload ...")
        leg("cpu_baseline", cpu_baseline, spec, dev)
        if "value" in result["cpu_baseline"]:
            log(f"cpu baseline: {result['cpu_baseline']['value']:.3f} iter/s on "
                f"{result['cpu_baseline']['cores']} threads")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
