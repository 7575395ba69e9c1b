"""Batched right-hand sides against the oracle's single-RHS solves."""
import numpy as np
import pytest

import oracle
import synth

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
def c0():
    S = synth.make_system(synth.WORKLOADS[0])
    o = oracle.OracleSystem.from_synth(S)
    xt = synth.x_true(S.spec)
    B = np.stack([o.aprod1(xt, synth.noise(S.spec, S.m, rhs=j)) for j in range(5)], axis=1)
    return S, o, B


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# (attitude mode, fused mode, compact indices): the fused pass serves
# attitude mode 1; fused mode 2 runs the attitude pre-pass in one-RHS tiles
@pytest.mark.parametrize("att_mode,fused,compact", [(1, 2, 1), (1, 2, 0), (1, 1, 1), (1, 0, 1),
                                                    (0, 1, 1)])
@pytest.mark.parametrize("ktile", [1, 2, 4, 8])
def test_batched_fixed_iterations(torch_cuda, c0, ktile, att_mode, fused, compact):
    torch = torch_cuda
    from paper_2308_00778_amd import LsqrSystem

    S, o, B = c0
    itn = 40
    say(f"batched parity: c0 k=5 ktile={ktile} att_mode={att_mode} fused={fused} itn={itn}")
    g = LsqrSystem.from_host(S, "cuda:0")
    g.set_option("att_mode", att_mode)
    g.set_option("fused", fused)
    g.set_option("compact_index", compact)
    g.set_option("att_buckets", 4)
    g.set_option("tests", 0)
    g.set_option("ktile", ktile)
    X, infos = g.solve_batched(torch.from_numpy(np.ascontiguousarray(B)).cuda(), itn, 0.0, 0.0)
    Xh = X.cpu().numpy()
    g.close()
    for j in range(B.shape[1]):
        x_ref, i_ref = o.lsqr(B[:, j], itn, atol=0.0, btol=0.0, conlim=0.0, tests=False)
        assert infos[j].itn == itn and infos[j].istop == 7
        assert rel_inf(Xh[:, j], x_ref) <= 1e-10, j
        assert abs(infos[j].rnorm - i_ref.rnorm) <= 1e-8 * i_ref.rnorm


# The 16-RHS tile (the fused pass and the first aprod2 with the right-hand
# sides of a row across 16 lanes) on 18 right-hand sides: one 16-tile and a
# ragged 2-tile; against the oracle at a fixed iteration count. Also the
# K-values-per-lane layout of the 2- to 8-RHS tiles (LSQR_OPT_RHS_LANES 0).
@pytest.fixture(scope="module")
def c0_18():
    S = synth.make_system(synth.WORKLOADS[0])
    o = oracle.OracleSystem.from_synth(S)
    xt = synth.x_true(S.spec)
    B = np.stack([o.aprod1(xt, synth.noise(S.spec, S.m, rhs=j)) for j in range(18)], axis=1)
    return S, o, B


@pytest.mark.parametrize("fused,compact,lanes,ktile", [(2, 1, 1, 16), (3, 0, 1, 16),
                                                       (2, 1, 0, 8), (2, 1, 0, 4),
                                                       (2, 0, 1, 8)])
def test_batched_wide_tiles(torch_cuda, c0_18, fused, compact, lanes, ktile):
    torch = torch_cuda
    from paper_2308_00778_amd import LsqrSystem

    S, o, B = c0_18
    itn = 30
    say(f"batched parity: c0 k=18 ktile={ktile} fused={fused} compact={compact} "
        f"rhs_lanes={lanes} itn={itn}")
    g = LsqrSystem.from_host(S, "cuda:0")
    g.set_option("fused", fused)
    g.set_option("compact_index", compact)
    g.set_option("rhs_lanes", lanes)
    g.set_option("att_buckets", 4)
    g.set_option("tests", 0)
    g.set_option("ktile", ktile)
    X, infos = g.solve_batched(torch.from_numpy(np.ascontiguousarray(B)).cuda(), itn, 0.0, 0.0)
    Xh = X.cpu().numpy()
    g.close()
    for j in range(B.shape[1]):
        x_ref, i_ref = o.lsqr(B[:, j], itn, atol=0.0, btol=0.0, conlim=0.0, tests=False)
        assert infos[j].itn == itn and infos[j].istop == 7
        assert rel_inf(Xh[:, j], x_ref) <= 1e-10, j
        assert abs(infos[j].rnorm - i_ref.rnorm) <= 1e-8 * i_ref.rnorm


def test_batched_16_tile_needs_the_lane_layout(torch_cuda, c0_18):
    torch = torch_cuda
    from paper_2308_00778_amd import LSQR_E_UNSUPPORTED, LsqrError, LsqrSystem

    S, o, B = c0_18
    say("batched 16-RHS tile in fused mode 1: LSQR_E_UNSUPPORTED")
    g = LsqrSystem.from_host(S, "cuda:0")
    g.set_option("fused", 1)
    g.set_option("ktile", 16)
    with pytest.raises(LsqrError) as ei:
        g.solve_batched(torch.from_numpy(np.ascontiguousarray(B[:, :16])).cuda(), 5, 0.0, 0.0)
    g.close()
    assert ei.value.status == LSQR_E_UNSUPPORTED


def test_batched_masks_freeze_converged_rhs(torch_cuda, c0):
    # RHS 0 is consistent (b = one column of A) and stops early by S1; the
    # others stop later by S2. Each must equal its own single solve.
    torch = torch_cuda
    from paper_2308_00778_amd import LsqrSystem

    S, o, B = c0
    B = B.copy()
    e = np.zeros(o.n)
    e[-1] = 1.0
    B[:, 0] = o.aprod1(e)
    B[:, 3] = 0.0  # b = 0: stops before the first iteration
    say("batched masks: c0 k=5, consistent + zero + noisy RHS")
    g = LsqrSystem.from_host(S, "cuda:0")
    g.set_option("ktile", 8)
    X, infos = g.solve_batched(torch.from_numpy(np.ascontiguousarray(B)).cuda(), 300,
                               1e-12, 1e-12)
    Xh = X.cpu().numpy()
    singles = []
    for j in range(B.shape[1]):
        xs, inf = g.solve(torch.from_numpy(np.ascontiguousarray(B[:, j])).cuda(), 300,
                          1e-12, 1e-12)
        singles.append((xs.cpu().numpy(), inf))
    g.close()
    assert infos[3].istop == 0 and infos[3].itn == 0 and not np.any(Xh[:, 3])
    assert infos[0].istop == 1 and infos[0].itn < infos[1].itn
    for j in (0, 1, 2, 4):
        x_ref, i_ref = o.lsqr(B[:, j], 300, atol=1e-12, btol=1e-12, conlim=1e8)
        xs, inf = singles[j]
        assert infos[j].istop == i_ref.istop and abs(infos[j].itn - i_ref.itn) <= 1, j
        assert (infos[j].istop, infos[j].itn) == (inf.istop, inf.itn), j
        assert rel_inf(Xh[:, j], x_ref) <= 1e-10, j
        assert rel_inf(Xh[:, j], xs) <= 1e-10, j


def test_batched_autotune_picks_a_tile(torch_cuda, c0):
    torch = torch_cuda
    from paper_2308_00778_amd import LsqrSystem

    S, o, B = c0
    say("batched autotune: c0 k=5")
    g = LsqrSystem.from_host(S, "cuda:0")
    g.set_option("tests", 0)
    X, infos = g.solve_batched(torch.from_numpy(np.ascontiguousarray(B)).cuda(), 30, 0.0, 0.0)
    t = g.batch_tuning()
    Xh = X.cpu().numpy()
    g.close()
    assert t["k_tile"] in (1, 2, 4)
    assert all(t["ms_per_rhs_iter"][k] > 0 for k in (1, 2, 4))
    x_ref, _ = o.lsqr(B[:, 2], 30, atol=0.0, btol=0.0, conlim=0.0, tests=False)
    assert rel_inf(Xh[:, 2], x_ref) <= 1e-10


# 9000 instrumental columns: a K = 2 tile keeps the instrumental slice of VP
# in LDS (144 KB) beside a 704-column histogram and leaves the other columns
# to one tail window; a K = 4 tile keeps a 4,864-column histogram, gathers
# the slice from memory and leaves the rest to the tail.
@pytest.mark.parametrize("ktile", [2, 4])
def test_batched_wide_instrumental(torch_cuda, ktile):
    torch = torch_cuda
    from paper_2308_00778_amd import LsqrSystem

    spec = synth.tiny(seed=24, n_stars=200, obs=(20, 60), n_dfa=300, n_instr_cols=9000)
    S = synth.make_system(spec)
    o = oracle.OracleSystem.from_synth(S)
    xt = synth.x_true(spec)
    B = np.stack([o.aprod1(xt, synth.noise(spec, S.m, rhs=j)) for j in range(3)], axis=1)
    itn = 30
    say(f"batched parity: wide_instr k=3 ktile={ktile} itn={itn}")
    g = LsqrSystem.from_host(S, "cuda:0")
    g.set_option("tests", 0)
    g.set_option("ktile", ktile)
    X, infos = g.solve_batched(torch.from_numpy(np.ascontiguousarray(B)).cuda(), itn, 0.0, 0.0)
    Xh = X.cpu().numpy()
    g.close()
    for j in range(B.shape[1]):
        x_ref, _ = o.lsqr(B[:, j], itn, atol=0.0, btol=0.0, conlim=0.0, tests=False)
        assert infos[j].itn == itn
        assert rel_inf(Xh[:, j], x_ref) <= 1e-10, j


# 7000 attitude starts: the bucket count sets how many right-hand sides one
# sweep of the bucket-order attitude passes holds (3 (W + 3) KS doubles in
# LDS): 2 buckets -> 1 per sweep, 3 -> 2, 6 -> 4. Five RHS in tiles of 2, 4
# and 8 (the last tile of each carries frozen slots). 35,815 rows for 24,041
# unknowns: with 300 stars x 20..60 rows the system is underdetermined and
# two FP64 LSQRs drift apart within 30 iterations (the oracle and SciPy's
# LSQR differ by 8e-8 there, by 4e-15 on this system).
@pytest.fixture(scope="module")
def wide_att():
    spec = synth.tiny(seed=25, n_stars=600, obs=(40, 80), n_dfa=7000, n_instr_cols=40)
    S = synth.make_system(spec)
    o = oracle.OracleSystem.from_synth(S)
    xt = synth.x_true(spec)
    B = np.stack([o.aprod1(xt, synth.noise(spec, S.m, rhs=j)) for j in range(5)], axis=1)
    return S, o, B


# ("att_rhs", r): the bucket geometry sized for r RHS per sweep (2 -> 3
# buckets, 4 -> 5, 8 -> 9 here).
@pytest.mark.parametrize("geometry", [("att_buckets", 2), ("att_buckets", 3),
                                      ("att_buckets", 6), ("att_rhs", 2), ("att_rhs", 4),
                                      ("att_rhs", 8)])
@pytest.mark.parametrize("ktile", [2, 4, 8])
def test_batched_attitude_sweeps(torch_cuda, wide_att, geometry, ktile):
    torch = torch_cuda
    from paper_2308_00778_amd import LsqrSystem

    S, o, B = wide_att
    itn = 30
    say(f"batched parity: wide_att k=5 ktile={ktile} {geometry[0]}={geometry[1]} itn={itn}")
    g = LsqrSystem.from_host(S, "cuda:0")
    g.set_option(*geometry)
    g.set_option("tests", 0)
    g.set_option("ktile", ktile)
    X, infos = g.solve_batched(torch.from_numpy(np.ascontiguousarray(B)).cuda(), itn, 0.0, 0.0)
    Xh = X.cpu().numpy()
    g.close()
    for j in range(B.shape[1]):
        x_ref, i_ref = o.lsqr(B[:, j], itn, atol=0.0, btol=0.0, conlim=0.0, tests=False)
        assert infos[j].itn == itn
        assert rel_inf(Xh[:, j], x_ref) <= 1e-10, j
        assert abs(infos[j].rnorm - i_ref.rnorm) <= 1e-8 * i_ref.rnorm


# The refined form of the batched solve (lsqr_solve_batched_refined) on a
# system with the features of the largest workload: FP32-stored values,
# uneven stars (50..150 observations), 30,000 instrumental columns (beyond
# one LDS histogram: tail windows), 150 attitude buckets, no compact index
# copies, k = 4. Among the right-hand sides: a consistent one (b = a column
# of A, stops refining early), a zero one (x = 0, frozen from the start) and
# noisy ones. Every x[:, j] must match the converged FP64 oracle to 1e-10
# (the FP32-rounded values define the system) and the single refined solve.
@pytest.fixture(scope="module")
def f32_c4like():
    spec = synth.tiny(seed=41, n_stars=500, obs=(50, 150), n_dfa=1200, n_instr_cols=30000,
                      value_dtype="f32", astro_scale=(-2.0, 2.0))
    S = synth.make_system(spec)
    o = oracle.OracleSystem.from_synth(S)
    xt = synth.x_true(spec)
    B = np.stack([o.aprod1(xt, synth.noise(spec, S.m, rhs=j)) for j in range(4)], axis=1)
    e = np.zeros(o.n)
    e[5 * 17 + 2] = 1.0
    B[:, 1] = o.aprod1(e)   # consistent: b = one column of A
    B[:, 2] = 0.0           # zero right-hand side
    refs = [o.lsqr(B[:, j], 600, atol=1e-14, btol=1e-14, conlim=0.0) for j in range(4)]
    return S, o, B, refs


@pytest.mark.parametrize("ktile", [4, 2, 1, 0])
def test_batched_refined_matches_fp64_oracle(torch_cuda, f32_c4like, ktile):
    torch = torch_cuda
    from paper_2308_00778_amd import LsqrSystem

    S, o, B, refs = f32_c4like
    say(f"batched refined: FP32 m={S.m} n={o.n} k=4 ktile={ktile}, 150 buckets, "
        f"30000 instrumental columns, no compact indices")
    g = LsqrSystem.from_host(S, "cuda:0")
    g.set_option("att_buckets", 150)
    g.set_option("compact_index", 0)
    g.set_option("ktile", ktile)
    Bd = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    X, infos = g.solve_batched_refined(Bd, 200, atol=1e-6, btol=1e-6, outer_limit=8)
    Xh = X.cpu().numpy()
    singles = [g.solve_refined(torch.from_numpy(np.ascontiguousarray(B[:, j])).cuda(), 200,
                               atol=1e-6, btol=1e-6, outer_limit=8) for j in range(4)]
    tuned = g.batch_tuning()["k_tile"]
    g.close()
    for j in range(4):
        x_ref, i_ref = refs[j]
        xs, inf = singles[j]
        xs = xs.cpu().numpy()
        say(f"  rhs {j}: outer {infos[j].outer_steps} inner {infos[j].itn} "
            f"(single {inf.outer_steps}/{inf.itn})")
        if j == 2:  # b = 0: x = 0, no iteration
            assert infos[j].itn == 0 and infos[j].istop == 0 and not np.any(Xh[:, j])
            continue
        assert rel_inf(Xh[:, j], x_ref) <= 1e-10, j
        assert rel_inf(Xh[:, j], xs) <= 1e-10, j
        assert infos[j].outer_steps == inf.outer_steps, j
        assert abs(infos[j].itn - inf.itn) <= infos[j].outer_steps, j
        # ||b|| of the first inner solve's FP32 start vector
        assert infos[j].bnorm == pytest.approx(inf.bnorm, rel=1e-12)
        assert infos[j].bnorm == pytest.approx(float(np.linalg.norm(B[:, j])), rel=1e-6)
    if ktile == 0:
        assert tuned in (1, 2, 4)


def test_batched_refined_needs_fp32_values(torch_cuda, c0):
    torch = torch_cuda
    from paper_2308_00778_amd import LSQR_E_STATE, LsqrError, LsqrSystem

    S, o, B = c0
    say("batched refined on an FP64 system: LSQR_E_STATE")
    g = LsqrSystem.from_host(S, "cuda:0")
    with pytest.raises(LsqrError) as ei:
        g.solve_batched_refined(torch.from_numpy(np.ascontiguousarray(B)).cuda(), 10)
    g.close()
    assert ei.value.status == LSQR_E_STATE
