"""Equal-iteration parity at the full 1e8-row size: 50 LSQR iterations of the
GPU solve (single right-hand side, and two right-hand sides of a batched
k-tile) against 50 iterations of the oracle on the same system, relative
infinity-norm difference <= 1e-10.

The system is generated on the GPU (bit-identical to the host generator) and
copied to host memory; b_j = A x_true + noise_j is formed by the oracle. The
oracle runs as its OpenMP timing build (the same source as the pinned
single-thread oracle; tests/test_oracle_timing_build.py checks the two
builds against each other), about a minute per solve on the machine's cores.
This module holds about 30 GB of host memory and 30 GB of device memory.
"""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ITN = 50


def say(*a):
    print(*a, flush=True)


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def c1_pair():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_00778_amd import LsqrSystem

    spec = synth.WORKLOADS[1]
    say(f"full size iterates: the 1e8-row system (seed {spec.seed}), oracle timing build")
    if not os.path.exists(oracle.OMP_LIB_PATH):
        oracle.build(openmp=True)
    arrays, first = synth.device_system(spec, "cuda:0")
    m = int(first[-1])
    host = {k: v.cpu().numpy() for k, v in arrays.items()}
    g = LsqrSystem(**arrays, n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                   n_instr_cols=spec.n_instr_cols)
    oracle.use_library(oracle.OMP_LIB_PATH)
    try:
        o = oracle.OracleSystem(host["values"], host["star_of_row"], host["att_start"],
                                host["instr_idx"], n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                                n_instr_cols=spec.n_instr_cols)
        xt = synth.x_true(spec)
        bs = [o.aprod1(xt, synth.noise(spec, m, rhs=j)) for j in range(2)]
        refs = []
        for j, b in enumerate(bs):
            say(f"  oracle: {ITN} iterations of rhs {j} on {oracle.num_threads()} threads")
            refs.append(o.lsqr(b, ITN, atol=0.0, btol=0.0, conlim=0.0, tests=False))
    finally:
        oracle.use_library(None)
    del o, host
    yield torch, g, bs, refs
    g.close()
    del arrays
    torch.cuda.empty_cache()


def test_fullsize_50_iterations_match_oracle(c1_pair):
    torch, g, bs, refs = c1_pair
    x_ref, i_ref = refs[0]
    g.set_option("tests", 0)
    x, info = g.solve(torch.from_numpy(bs[0]).cuda(), ITN, atol=0.0, btol=0.0)
    torch.cuda.synchronize()
    err = rel_inf(x.cpu().numpy(), x_ref)
    say(f"1e8 rows, {ITN} iterations: GPU vs oracle {err:.2e}")
    assert info.itn == i_ref.itn == ITN and info.istop == 7
    assert err <= 1e-10
    for k in ("rnorm", "xnorm", "bnorm"):
        a, r = getattr(info, k), getattr(i_ref, k)
        assert abs(a - r) <= 1e-8 * abs(r), (k, a, r)


@pytest.mark.parametrize("ktile", [2, 4])
def test_fullsize_batched_50_iterations_match_oracle(c1_pair, ktile):
    torch, g, bs, refs = c1_pair
    # the two right-hand sides twice over, so that a 4-RHS tile is full
    B = np.stack([bs[0], bs[1], bs[0], bs[1]], axis=1)
    g.set_option("tests", 0)
    g.set_option("ktile", ktile)
    X, infos = g.solve_batched(torch.from_numpy(np.ascontiguousarray(B)).cuda(), ITN, 0.0, 0.0)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    g.set_option("ktile", 0)
    for j in range(4):
        x_ref, i_ref = refs[j % 2]
        err = rel_inf(Xh[:, j], x_ref)
        say(f"1e8 rows, batched k-tile {ktile}, rhs {j}: GPU vs oracle {err:.2e}")
        assert infos[j].itn == ITN and infos[j].istop == 7
        assert err <= 1e-10, j
