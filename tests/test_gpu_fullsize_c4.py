"""GPU parity on the largest single-GPU workload: 10^7 stars x U{50..150}
observations (about 1e9 rows), FP32-stored values (96 GB), N_DFA = 10^6,
30,000 instrumental columns, k = 4 right-hand sides, generated on the GPU.

Neither the oracle nor the host can hold this system (about 136 GB of values
and indices), so, as for the other full-size workloads:
  * aprod1 on sampled row ranges against the oracle on just those rows (the
    host generator produces them);
  * the adjoint identity <A x, y> = <x, A^T y> over the whole operator;
  * the refined batched solve (FP32 inner solves of the four right-hand sides
    advancing together, FP64 refinement per right-hand side) against the FP64
    solve of the same FP32-rounded system on the GPU, which the smaller
    systems pin to the oracle, to 1e-10 for two of the right-hand sides.
This module runs on its own (about 250 GB of device memory at its peak).
"""
import numpy as np
import pytest

import synth
from test_gpu_fullsize import _check_sampled_rows

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def c4(torch_cuda):
    torch = torch_cuda
    from paper_2308_00778_amd import LsqrSystem

    spec = synth.WORKLOADS[4]
    say(f"full size: generating the 1e9-row FP32 system on the GPU (seed {spec.seed})")
    arrays, first = synth.device_system(spec, "cuda:0")
    g = LsqrSystem(**arrays, n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                   n_instr_cols=spec.n_instr_cols)
    say(f"  m={g.m} n={g.n}, {torch.cuda.mem_get_info()[0] / 1e9:.0f} GB free")
    yield spec, g, first
    g.close()
    del arrays
    torch.cuda.empty_cache()


def test_c4_sampled_rows_and_adjoint(torch_cuda, c4):
    torch = torch_cuda
    spec, g, first = c4
    worst = _check_sampled_rows(torch, spec, g, first, 17)
    say(f"c4 aprod1 (widened FP32 values): worst |err| / sum|terms| = {worst:.2e}")
    rng = np.random.default_rng(18)
    x0 = torch.from_numpy(rng.standard_normal(g.n)).cuda()
    y = torch.from_numpy(rng.standard_normal(g.m)).cuda()
    ax = torch.zeros(g.m, dtype=torch.float64, device="cuda")
    g.aprod1(x0, ax)
    aty = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    g.aprod2(aty, y)
    lhs = float(torch.dot(ax, y))
    rhs = float(torch.dot(x0, aty))
    scale = float(torch.linalg.norm(ax)) * float(torch.linalg.norm(y))
    del ax, y, aty, x0
    torch.cuda.empty_cache()
    say(f"c4 adjoint: |<Ax,y> - <x,A^T y>| / (||Ax|| ||y||) = {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-11 * scale


def test_c4_refined_batched_against_fp64(torch_cuda, c4):
    torch = torch_cuda
    spec, g, first = c4
    k = spec.n_rhs
    xt = synth.device_x_true(spec, "cuda:0")
    B = torch.empty((g.m, k), dtype=torch.float64, device="cuda")
    for j in range(k):
        bj = synth.device_noise(spec, g.m, j, "cuda:0")
        g.aprod1(xt, bj)
        B[:, j] = bj
        del bj
    torch.cuda.synchronize()
    # FP64 solves of the same (FP32-rounded) system for two right-hand sides,
    # before the batched buffers take their memory
    ref = {}
    for j in (0, 3):
        bj = B[:, j].contiguous()
        x64, i64 = g.solve(bj, 500, atol=1e-12, btol=1e-12)
        say(f"c4 FP64 rhs {j}: itn {i64.itn} istop {i64.istop}")
        assert i64.istop in (1, 2)
        ref[j] = x64
        del bj
    torch.cuda.empty_cache()
    say(f"  {torch.cuda.mem_get_info()[0] / 1e9:.0f} GB free before the batched solve")
    X, infos = g.solve_batched_refined(B, 200, atol=1e-6, btol=1e-6, outer_limit=10)
    torch.cuda.synchronize()
    say(f"c4 refined batched: k-tile {g.batch_tuning()['k_tile']}, outer "
        f"{[i.outer_steps for i in infos]}, inner {[i.itn for i in infos]}")
    for j, x64 in ref.items():
        err = float(torch.max(torch.abs(X[:, j] - x64)) / torch.max(torch.abs(x64)))
        say(f"  rhs {j}: refined batched vs FP64 {err:.2e}")
        assert err <= 1e-10, j
    assert all(1 <= i.outer_steps <= 10 for i in infos)
    del B, X
    torch.cuda.empty_cache()
