"""GPU parity at the full workload sizes, in the configuration the benchmark
times (system generated on the GPU, default options: fused mode 2, graph
replay). Here the oracle checks sampled outputs it can compute on their own,
and the rest is checked through properties that hold at any size (the
equal-iteration comparison with the oracle at 1e8 rows, which needs its
OpenMP timing build and a minute per solve, is tests/test_gpu_fullsize_iterates.py):
  * aprod1 on sampled row ranges: the host generator produces just those rows
    and the oracle computes their products exactly;
  * aprod2 on sampled stars' astrometric columns, which only that star's rows
    touch; the adjoint identity <A x, y> = <x, A^T y> for the whole operator;
  * LSQR: the first iterate against its closed form
    y_1 = (||Abar^T b||^2 / ||Abar Abar^T b||^2) Abar^T b, and the converged
    solution against the normal equations;
  * the 4e8-row FP32 system: sampled rows, and the refined solution against
    the FP64 solution of the same system.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _handle(spec):
    from paper_2308_00778_amd import LsqrSystem

    arrays, first = synth.device_system(spec, "cuda:0")
    g = LsqrSystem(**arrays, n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                   n_instr_cols=spec.n_instr_cols)
    return g, first, arrays


@pytest.fixture(scope="module")
def c1(torch_cuda):
    torch = torch_cuda
    spec = synth.WORKLOADS[1]
    say(f"full size: generating the 1e8-row system on the GPU (seed {spec.seed})")
    g, first, arrays = _handle(spec)
    yield spec, g, first
    g.close()
    del arrays
    torch.cuda.empty_cache()


def _sample_ranges(first, rng, k=6, length=512):
    """Row ranges: the first and last rows, and random starts (star-aligned and
    not)."""
    m = int(first[-1])
    starts = {0, m - length}
    n_stars = first.shape[0] - 1
    for _ in range(k):
        starts.add(int(first[int(rng.integers(0, n_stars))]))
        starts.add(int(rng.integers(0, m - length)))
    return sorted((s, s + length) for s in starts)


def _rows_system(spec, first, r0, r1, absval=False):
    values, star, att, instr = synth.rows(spec, first, r0, r1)
    if absval:
        values = np.abs(values.astype(np.float64))
    return oracle.OracleSystem(values, star, att, instr, n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                               n_instr_cols=spec.n_instr_cols)


def _check_sampled_rows(torch, spec, g, first, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(g.n)
    y = torch.zeros(g.m, dtype=torch.float64, device="cuda")
    g.aprod1(torch.from_numpy(x).cuda(), y)
    torch.cuda.synchronize()
    worst = 0.0
    for r0, r1 in _sample_ranges(first, rng):
        want = _rows_system(spec, first, r0, r1).aprod1(x)
        bound = _rows_system(spec, first, r0, r1, absval=True).aprod1(np.abs(x))
        got = y[r0:r1].cpu().numpy()
        assert np.all(np.abs(got - want) <= 32 * EPS * bound), (r0, r1)
        worst = max(worst, float(np.max(np.abs(got - want) / bound)))
    return worst


def test_fullsize_aprod1_sampled_rows(torch_cuda, c1):
    spec, g, first = c1
    worst = _check_sampled_rows(torch_cuda, spec, g, first, 11)
    say(f"full size aprod1: worst |err| / sum|terms| = {worst:.2e}")


def test_fullsize_aprod2_sampled_stars_and_adjoint(torch_cuda, c1):
    torch = torch_cuda
    spec, g, first = c1
    rng = np.random.default_rng(12)
    y = torch.from_numpy(rng.standard_normal(g.m)).cuda()
    xg = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    g.aprod2(xg, y)
    torch.cuda.synchronize()
    x_all = xg.cpu().numpy()
    y_host = y.cpu().numpy()
    stars = sorted({0, spec.n_stars - 1, *rng.integers(0, spec.n_stars, 10).tolist()})
    for s in stars:
        r0, r1 = int(first[s]), int(first[s + 1])
        want = _rows_system(spec, first, r0, r1).aprod2(y_host[r0:r1])[5 * s:5 * s + 5]
        bound = _rows_system(spec, first, r0, r1, absval=True).aprod2(
            np.abs(y_host[r0:r1]))[5 * s:5 * s + 5]
        got = x_all[5 * s:5 * s + 5]
        assert np.all(np.abs(got - want) <= (2 * np.sqrt(r1 - r0) + 32) * EPS * bound), s
    # adjoint identity over the whole operator (any size): <A x0, y> = <x0, A^T y>
    x0 = torch.from_numpy(rng.standard_normal(g.n)).cuda()
    ax = torch.zeros(g.m, dtype=torch.float64, device="cuda")
    g.aprod1(x0, ax)
    lhs = float(torch.dot(ax, y))
    rhs = float(torch.dot(x0, xg))
    scale = float(torch.linalg.norm(ax)) * float(torch.linalg.norm(y))
    say(f"full size adjoint: |<Ax,y> - <x,A^T y>| / (||Ax|| ||y||) = {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-11 * scale


def _rhs(torch, spec, g):
    b = synth.device_noise(spec, g.m, 0, "cuda:0")
    g.aprod1(synth.device_x_true(spec, "cuda:0"), b)
    torch.cuda.synchronize()
    return b


def test_fullsize_first_iterate_closed_form(torch_cuda, c1):
    torch = torch_cuda
    spec, g, first = c1
    b = _rhs(torch, spec, g)
    p = g.precond()
    g.set_option("tests", 0)
    x1, info = g.solve(b, 1, atol=0.0, btol=0.0)
    g.set_option("tests", 1)
    atb = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    g.aprod2(atb, b)
    s = p * atb                                      # Abar^T b
    aas = torch.zeros(g.m, dtype=torch.float64, device="cuda")
    g.aprod1(p * s, aas)                             # Abar Abar^T b
    y1 = (torch.dot(s, s) / torch.dot(aas, aas)) * s
    want = p * y1
    err = float(torch.max(torch.abs(x1 - want)) / torch.max(torch.abs(want)))
    say(f"full size first iterate: rel inf err {err:.2e}")
    assert info.itn == 1 and err <= 1e-12


def test_fullsize_converged_normal_equations(torch_cuda, c1):
    torch = torch_cuda
    spec, g, first = c1
    b = _rhs(torch, spec, g)
    x, info = g.solve(b, 500, atol=1e-12, btol=1e-12)
    ax = torch.zeros(g.m, dtype=torch.float64, device="cuda")
    g.aprod1(x, ax)
    r = b - ax
    atr = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    g.aprod2(atr, r)
    ratio = float(torch.linalg.norm(g.precond() * atr)) / (info.anorm * float(torch.linalg.norm(r)))
    say(f"full size converged: itn {info.itn} istop {info.istop}, "
        f"||Abar^T r|| / (||Abar|| ||r||) = {ratio:.2e}")
    assert info.istop in (1, 2) and info.itn < 500
    # FP64 floor of forming r = b - A x explicitly (see the small-system test)
    assert ratio <= 1e-9


def test_fullsize_fp32_system_and_refinement(torch_cuda, c1):
    torch = torch_cuda
    spec = synth.WORKLOADS[2]
    say(f"full size: generating the 4e8-row FP32 system on the GPU (seed {spec.seed})")
    g, first, arrays = _handle(spec)
    try:
        worst = _check_sampled_rows(torch, spec, g, first, 13)
        say(f"FP32 system aprod1 (widened values): worst |err| / sum|terms| = {worst:.2e}")
        b = _rhs(torch, spec, g)
        x64, i64 = g.solve(b, 500, atol=1e-12, btol=1e-12)
        x32, i32 = g.solve_refined(b, 200, atol=1e-6, btol=1e-6, outer_limit=10)
        err = float(torch.max(torch.abs(x32 - x64)) / torch.max(torch.abs(x64)))
        say(f"refined vs FP64 at 4e8 rows: {err:.2e} ({i32.outer_steps} outer, "
            f"{i32.itn} inner; FP64 {i64.itn} iterations)")
        assert i64.istop in (1, 2) and err <= 1e-10
    finally:
        g.close()
        del arrays
        torch.cuda.empty_cache()
