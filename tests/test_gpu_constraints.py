"""GPU parity with constraint rows (Sect. 2: equations at the bottom of the
system, replicated on every process in the paper's code) appended to the
observation rows: operators, column norms, solves (fused and separate passes,
graph replay and single launches), the refined solve and the variance,
against the oracle given the same rows. Tolerances as in the full-layout
parity tests.
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


def _with_empty_row(con, at):
    rp = np.insert(con.rowptr, at + 1, con.rowptr[at])
    return synth.Constraints(rowptr=rp, col=con.col, val=con.val)


# Constraint rows weighted like observation rows (2-norm sqrt(24)): much
# heavier rows add a few large singular values that the bidiagonalisation
# resolves within a few iterations, after which it loses orthogonality and any
# two FP64 implementations drift apart at equal iteration count (measured with
# unscaled N(0,1) rows of 2,000 entries: the oracle and SciPy's LSQR differ by
# 2e-5 at 40 iterations).
RN = float(np.sqrt(24.0))


def _case(name):
    if name == "full":  # rows of 0..3000 entries (several workgroup strides), one empty
        sp = synth.tiny(seed=71, n_stars=300, obs=(10, 60), n_dfa=150, n_instr_cols=31)
        return sp, _with_empty_row(synth.constraints(sp, 9, nnz=(1, 3000), seed=1,
                                                     row_norm=RN), 4)
    if name == "rank_deficient":  # stars of 2..4 rows, astrometric columns fixed by constraints
        sp = synth.tiny(seed=72, n_stars=200, obs=(2, 4), n_axes=0, n_instr=0, n_glob=0)
        return sp, synth.constraints(sp, 700, nnz=(8, 24), seed=2, row_norm=RN)
    if name == "f32":
        sp = synth.tiny(seed=73, n_stars=300, obs=(20, 50), n_dfa=120, n_instr_cols=19,
                        value_dtype="f32")
        return sp, synth.constraints(sp, 12, nnz=(50, 800), seed=3, row_norm=RN)
    if name == "mixed_layout":
        sp = synth.tiny(seed=74, n_stars=250, obs=(10, 40), n_dfa=90, n_instr_cols=27,
                        n_astro=3, n_instr=2, n_glob=3)
        return sp, synth.constraints(sp, 6, nnz=(20, 400), seed=4, row_norm=RN)
    raise KeyError(name)


NAMES = ["full", "rank_deficient", "f32", "mixed_layout"]
_SYS = {}


def system(name):
    if name not in _SYS:
        sp, C = _case(name)
        S = synth.make_system(sp)
        _SYS[name] = (S, C, oracle.OracleSystem.from_synth(S, con=C))
    return _SYS[name]


def abs_system(S, C):
    sp = S.spec
    ac = synth.Constraints(rowptr=C.rowptr, col=C.col, val=np.abs(C.val))
    return oracle.OracleSystem(np.abs(S.values.astype(np.float64)), S.star_of_row, S.att_start,
                               S.instr_idx, n_stars=sp.n_stars, n_dfa=sp.n_dfa,
                               n_instr_cols=sp.n_instr_cols, n_astro=sp.n_astro,
                               n_axes=sp.n_axes, n_par_axis=sp.n_par_axis, n_instr=sp.n_instr,
                               n_glob=sp.n_glob, con=ac)


def gpu_system(S, C):
    from paper_2308_00778_amd import LsqrSystem

    return LsqrSystem.from_host(S, "cuda:0", con=C)


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _b(S, o):
    return o.aprod1(synth.x_true(S.spec), synth.noise(S.spec, o.m))


@pytest.mark.parametrize("name", NAMES)
def test_constraints_aprod1(torch_cuda, name):
    torch = torch_cuda
    S, C, o = system(name)
    say(f"aprod1 constraints: {name} m={o.m_obs}+{o.n_con} n={o.n} nnz={C.nnz}")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(o.n)
    y0 = rng.standard_normal(o.m)
    want = o.aprod1(x, y0)
    bound = abs_system(S, C).aprod1(np.abs(x), np.abs(y0))
    g = gpu_system(S, C)
    assert g.m == o.m
    yd = torch.from_numpy(y0).cuda()
    g.aprod1(torch.from_numpy(x).cuda(), yd)
    torch.cuda.synchronize()
    got = yd.cpu().numpy()
    g.close()
    # up to 3000 terms per constraint row
    c = 2.0 * np.sqrt(3000.0) + 32
    assert np.all(np.abs(got - want) <= c * EPS * bound + 1e-300)


@pytest.mark.parametrize("att_mode", [1, 0])
@pytest.mark.parametrize("name", NAMES)
def test_constraints_aprod2(torch_cuda, name, att_mode):
    torch = torch_cuda
    S, C, o = system(name)
    say(f"aprod2 constraints: {name} att_mode={att_mode}")
    rng = np.random.default_rng(6)
    y = rng.standard_normal(o.m)
    x0 = rng.standard_normal(o.n)
    want = o.aprod2(y, x0)
    bound = abs_system(S, C).aprod2(np.abs(y), np.abs(x0))
    g = gpu_system(S, C)
    g.set_option("att_mode", att_mode)
    xd = torch.from_numpy(x0).cuda()
    g.aprod2(xd, torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    got = xd.cpu().numpy()
    g.close()
    c = 2.0 * np.sqrt(o.m) + 32
    assert np.all(np.abs(got - want) <= c * EPS * bound + 1e-300)


@pytest.mark.parametrize("name", NAMES)
def test_constraints_column_norms(torch_cuda, name):
    S, C, o = system(name)
    say(f"column norms constraints: {name}")
    g = gpu_system(S, C)
    p = g.precond().cpu().numpy()
    g.close()
    assert np.max(np.abs(p - o.precond()) / o.precond()) < 1e-13


# (fused, graph) variants of the FP64 solve; fused needs the attitude section
@pytest.mark.parametrize("fused,graph", [(1, 1), (0, 1), (1, 0)])
@pytest.mark.parametrize("name", NAMES)
def test_constraints_solve_fixed_iterations(torch_cuda, name, fused, graph):
    torch = torch_cuda
    S, C, o = system(name)
    itn = 40
    b = _b(S, o)
    x_ref, i_ref = o.lsqr(b, itn, atol=0.0, btol=0.0, conlim=0.0, tests=False)
    say(f"solve constraints: {name} itn={itn} fused={fused} graph={graph}")
    g = gpu_system(S, C)
    g.set_option("fused", fused)
    g.set_option("graph", graph)
    g.set_option("att_buckets", 3)
    g.set_option("tests", 0)
    g.set_option("chunk", 7)
    x, info = g.solve(torch.from_numpy(b).cuda(), itn, atol=0.0, btol=0.0)
    xg = x.cpu().numpy()
    g.close()
    assert info.itn == i_ref.itn == itn
    assert rel_inf(xg, x_ref) <= 1e-10
    for k in ("rnorm", "xnorm", "bnorm"):
        a, r = getattr(info, k), getattr(i_ref, k)
        assert abs(a - r) <= 1e-8 * abs(r), (k, a, r)


@pytest.mark.parametrize("name", ["full", "rank_deficient"])
def test_constraints_converged_and_variance(torch_cuda, name):
    torch = torch_cuda
    S, C, o = system(name)
    b = _b(S, o)
    x_ref, i_ref = o.lsqr(b, 3000, atol=1e-12, btol=1e-12, conlim=0.0)
    x20, _, var_ref = o.lsqr(b, 15, atol=0.0, btol=0.0, conlim=0.0, tests=False,
                             want_var=True)
    say(f"converged + variance constraints: {name} oracle itn={i_ref.itn}")
    g = gpu_system(S, C)
    g.set_option("conlim", 0.0)
    x, info = g.solve(torch.from_numpy(b).cuda(), 3000, atol=1e-12, btol=1e-12)
    xg = x.cpu().numpy()
    g.set_option("tests", 0)
    g.set_option("variance", 1)
    xv, _ = g.solve(torch.from_numpy(b).cuda(), 15, atol=0.0, btol=0.0)
    var = g.variance().cpu().numpy()
    g.close()
    assert info.istop == i_ref.istop and abs(info.itn - i_ref.itn) <= 1
    assert rel_inf(xg, x_ref) <= 1e-10
    assert rel_inf(xv.cpu().numpy(), x20) <= 1e-10
    assert rel_inf(var, var_ref) <= 1e-10


def test_constraints_refined_matches_fp64_oracle(torch_cuda):
    torch = torch_cuda
    S, C, o = system("f32")
    b = _b(S, o)
    x_ref, i_ref = o.lsqr(b, 3000, atol=1e-14, btol=1e-14, conlim=0.0)
    say(f"refined constraints: f32 oracle itn={i_ref.itn}")
    g = gpu_system(S, C)
    x, info = g.solve_refined(torch.from_numpy(b).cuda(), 300, atol=1e-6, btol=1e-6,
                              outer_limit=10)
    xg = x.cpu().numpy()
    g.close()
    say(f"refined: outer={info.outer_steps} inner itn={info.itn} err={rel_inf(xg, x_ref):.3e}")
    assert rel_inf(xg, x_ref) <= 1e-10


def test_constraints_batched_unsupported_and_bad_rows(torch_cuda):
    torch = torch_cuda
    from paper_2308_00778_amd import LSQR_E_INVALID, LSQR_E_UNSUPPORTED, LsqrError

    S, C, o = system("full")
    say("constraints: batched rejected, invalid rows rejected")
    g = gpu_system(S, C)
    with pytest.raises(LsqrError) as ei:
        g.solve_batched(torch.zeros((o.m, 2), dtype=torch.float64, device="cuda"), 5)
    assert ei.value.status == LSQR_E_UNSUPPORTED
    g.close()
    # row pointers decreasing, then a column out of range: rejected at create
    rp = C.rowptr.copy()
    rp[3], rp[4] = rp[4], rp[3]
    bad_rows = synth.Constraints(rowptr=rp, col=C.col, val=C.val)
    col = C.col.copy()
    col[-1] = o.n
    bad_cols = synth.Constraints(rowptr=C.rowptr, col=col, val=C.val)
    for bad in (bad_rows, bad_cols):
        assert bad.rowptr[0] == 0 and bad.rowptr[-1] == C.nnz  # reads stay in the arrays
        with pytest.raises(LsqrError) as ei:
            gpu_system(S, bad)
        assert ei.value.status == LSQR_E_INVALID
