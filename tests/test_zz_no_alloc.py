"""The entry point that allocates nothing (lsqr_aprod1_noalloc) against the
allocating lsqr_aprod1 and the oracle, through the C ABI.

Two calls in a row share the library's per-GPU scratch: the second system is
smaller (fewer attitude columns) than the first, so stale scratch contents
from the first call would show up in the second. Each result must equal
lsqr_aprod1's on the same inputs within the aprod bound c * eps * sum |terms|
(the same kernels run, so they agree bit for bit in practice) and the oracle's
within the same bound.
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


def _abs_bound(S, x, y0):
    sp = S.spec
    oa = oracle.OracleSystem(np.abs(S.values.astype(np.float64)), S.star_of_row, S.att_start,
                             S.instr_idx, n_stars=sp.n_stars, n_dfa=sp.n_dfa,
                             n_instr_cols=sp.n_instr_cols)
    return oa.aprod1(np.abs(x), np.abs(y0))


# larger first, then smaller (fewer attitude columns, fewer rows), then FP32
# values smaller still
CALLS = [
    ("large", synth.tiny(seed=81, n_stars=400, obs=(20, 70), n_dfa=5000, n_instr_cols=300)),
    ("small", synth.tiny(seed=82, n_stars=60, obs=(10, 40), n_dfa=70, n_instr_cols=25)),
    ("small_f32", synth.tiny(seed=83, n_stars=30, obs=(10, 30), n_dfa=40, n_instr_cols=13,
                             value_dtype="f32")),
]


def test_noalloc_matches_aprod1_on_calls_in_a_row(torch_cuda):
    torch = torch_cuda
    from paper_2308_00778_amd import LsqrSystem

    for name, spec in CALLS:
        S = synth.make_system(spec)
        o = oracle.OracleSystem.from_synth(S)
        say(f"noalloc aprod1: {name} m={S.m} n={o.n} n_dfa={spec.n_dfa} seed={spec.seed}")
        rng = np.random.default_rng(spec.seed)
        x = rng.standard_normal(o.n)
        y0 = rng.standard_normal(o.m)
        want = o.aprod1(x, y0)
        bound = 32 * EPS * _abs_bound(S, x, y0) + 1e-300
        g = LsqrSystem.from_host(S, "cuda:0")
        xd = torch.from_numpy(x).cuda()
        y_ref = torch.from_numpy(y0).cuda()
        g.aprod1(xd, y_ref)
        y_na = torch.from_numpy(y0).cuda()
        g.aprod1_noalloc(xd, y_na)
        torch.cuda.synchronize()
        ref, got = y_ref.cpu().numpy(), y_na.cpu().numpy()
        g.close()
        assert np.all(np.abs(got - ref) <= bound), name
        assert np.all(np.abs(got - want) <= bound), name
        say(f"  max |noalloc - aprod1| = {np.max(np.abs(got - ref)):.3e}")


def test_noalloc_rejects_sizes_beyond_scratch(torch_cuda):
    torch = torch_cuda
    from paper_2308_00778_amd import LSQR_E_INVALID, LsqrError, LsqrSystem

    # 2^20 + 1 attitude columns per axis: 3 n_dfa exceeds the scratch
    spec = synth.tiny(seed=84, n_stars=4, obs=(10, 10), n_dfa=(1 << 20) + 1, n_instr_cols=8)
    S = synth.make_system(spec)
    say(f"noalloc size check: m={S.m} n_dfa={spec.n_dfa}")
    g = LsqrSystem.from_host(S, "cuda:0")
    x = torch.zeros(g.n, dtype=torch.float64, device="cuda:0")
    y = torch.zeros(g.m, dtype=torch.float64, device="cuda:0")
    with pytest.raises(LsqrError) as ei:
        g.aprod1_noalloc(x, y)
    assert ei.value.status == LSQR_E_INVALID
    assert "scratch" in str(ei.value)
    # the allocating entry point still serves it
    g.aprod1(x, y)
    torch.cuda.synchronize()
    g.close()
