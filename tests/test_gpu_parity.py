"""GPU parity: the HIP path through the C ABI against the oracle, element by
element, on seeded synthetic systems.

Tolerances. aprod outputs are sums of products; the summation orders differ
(FMA, wave trees, atomics), so each element is compared against the bound
c * eps * sum |terms| computed with the oracle on |A| and |x| (|y|), with c
covering the term count of that element (24 per row for aprod1; up to m for
the global column of aprod2). LSQR solutions must agree to a relative
infinity-norm of 1e-10 at equal iteration count (the target of this solver).
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


# Systems used by the solves have at least 10 observations per star, so the
# 5 astrometric unknowns of each star are well determined and the scaled
# system is well conditioned (equal-iteration parity needs that). Stars with
# 1..6 observations (rank-deficient astrometric blocks) appear in the exact
# operator checks only.
SPECS = {
    "c0": synth.WORKLOADS[0],
    "ragged": synth.tiny(seed=21, n_stars=37, obs=(10, 140), n_dfa=50, n_instr_cols=17),
    "short_stars": synth.tiny(seed=25, n_stars=300, obs=(1, 6), n_dfa=40, n_instr_cols=11),
    "one_star": synth.tiny(seed=22, n_stars=1, obs=(70, 70), n_dfa=8, n_instr_cols=6),
    "few_rows": synth.tiny(seed=23, n_stars=3, obs=(10, 14), n_dfa=5, n_instr_cols=7),
    "wide_instr": synth.tiny(seed=24, n_stars=200, obs=(20, 60), n_dfa=300,
                             n_instr_cols=9000),  # instrumental histogram beyond the LDS budget
    # 25,000 instrumental columns: beyond one FP64 LDS histogram (19,456), the
    # rest in a tail window
    "huge_instr": synth.tiny(seed=27, n_stars=300, obs=(30, 60), n_dfa=200,
                             n_instr_cols=25000),
    # the same with 10,240 rows: every value and index column starts on a
    # 128-byte line, so the tail windows take their nontemporal-load form
    # (the other small systems take the plain-load one)
    "huge_instr_lined": synth.tiny(seed=32, n_stars=256, obs=(40, 40), n_dfa=200,
                                   n_instr_cols=25000),
    # 70,000 instrumental columns: beyond a uint16 index (no compact index
    # copies) and four LDS windows (one histogram, three tail windows)
    "instr_70k": synth.tiny(seed=28, n_stars=300, obs=(30, 60), n_dfa=150,
                            n_instr_cols=70000),
    # 12,000 instrumental columns: the FP64 histogram and the slice of vp do
    # not both fit in LDS, so the fused pass keeps the slice and a 7,424-column
    # histogram and leaves the rest to one tail window (FP32 values: FP64
    # arithmetic on them, the same plan)
    "instr_12k": synth.tiny(seed=29, n_stars=600, obs=(40, 80), n_dfa=150,
                            n_instr_cols=12000),
    "instr_12k_f32": synth.tiny(seed=30, n_stars=600, obs=(40, 80), n_dfa=150,
                                n_instr_cols=12000, value_dtype="f32"),
    # FP32 values, 8,997 attitude starts: the default layout has two buckets
    # of FP64 histograms (exact operators and fixed-iteration solves only:
    # more attitude columns than rows)
    "wide_att_f32": synth.tiny(seed=26, n_stars=300, obs=(30, 50), n_dfa=9000,
                               n_instr_cols=40, value_dtype="f32"),
}

# attitude buckets per system in the aprod2 and solve tests: several buckets
# even on small systems, except where the default layout is the case tested
BUCKETS = {"wide_att_f32": 0}

_SYS = {}


def system(name):
    if name not in _SYS:
        S = synth.make_system(SPECS[name])
        _SYS[name] = (S, oracle.OracleSystem.from_synth(S))
    return _SYS[name]


def gpu_system(torch, S, precondition=True):
    from paper_2308_00778_amd import LsqrSystem

    return LsqrSystem.from_host(S, "cuda:0", precondition=precondition)


def abs_system(S):
    sp = S.spec
    return oracle.OracleSystem(np.abs(S.values.astype(np.float64)), S.star_of_row, S.att_start,
                               S.instr_idx, n_stars=sp.n_stars, n_dfa=sp.n_dfa,
                               n_instr_cols=sp.n_instr_cols)


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("interleave", [1, 0])
@pytest.mark.parametrize("name", list(SPECS))
def test_aprod1_parity(torch_cuda, name, interleave):
    torch = torch_cuda
    S, o = system(name)
    say(f"aprod1 parity: {name} m={S.m} n={o.n} seed={S.spec.seed} interleave={interleave}")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(o.n)
    y0 = rng.standard_normal(o.m)
    want = o.aprod1(x, y0)
    bound = abs_system(S).aprod1(np.abs(x), np.abs(y0))
    g = gpu_system(torch, S)
    g.set_option("att_interleave", interleave)
    yd = torch.from_numpy(y0).cuda()
    g.aprod1(torch.from_numpy(x).cuda(), yd)
    torch.cuda.synchronize()
    got = yd.cpu().numpy()
    g.close()
    assert np.all(np.abs(got - want) <= 32 * EPS * bound + 1e-300)


VARIANTS = [(1, 0), (0, 1), (0, 0), (1, 1)]  # (att_mode, astro_scan); first = default


@pytest.mark.parametrize("variant", VARIANTS, ids=[f"att{a}_scan{b}" for a, b in VARIANTS])
@pytest.mark.parametrize("name", list(SPECS))
def test_aprod2_parity(torch_cuda, name, variant):
    torch = torch_cuda
    S, o = system(name)
    say(f"aprod2 parity: {name} m={S.m} n={o.n} seed={S.spec.seed} variant={variant}")
    rng = np.random.default_rng(6)
    y = rng.standard_normal(o.m)
    x0 = rng.standard_normal(o.n)
    want = o.aprod2(y, x0)
    bound = abs_system(S).aprod2(np.abs(y), np.abs(x0))
    g = gpu_system(torch, S)
    g.set_option("att_mode", variant[0])
    g.set_option("astro_scan", variant[1])
    g.set_option("att_buckets", BUCKETS.get(name, 5))
    xd = torch.from_numpy(x0).cuda()
    g.aprod2(xd, torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    got = xd.cpu().numpy()
    g.close()
    # per-column term count: at most m (global column)
    c = 2.0 * np.sqrt(S.m) + 32
    assert np.all(np.abs(got - want) <= c * EPS * bound + 1e-300)


EPS32 = float(np.finfo(np.float32).eps)


# FP32 operators (FP32-stored values, FP32 vectors and accumulation) against
# the oracle on the same float values widened: each element within
# c * eps32 * sum |terms| (c as for the FP64 operators).
@pytest.mark.parametrize("variant", [(1, 1), (0, 0)], ids=["bucket_pass", "atomics_plain"])
@pytest.mark.parametrize("name", ["instr_12k_f32", "wide_att_f32"])
def test_aprod_f32_parity(torch_cuda, name, variant):
    torch = torch_cuda
    S, o = system(name)
    say(f"FP32 operators: {name} m={S.m} n={o.n} att_mode={variant[0]} "
        f"interleave={variant[1]}")
    rng = np.random.default_rng(8)
    x = rng.standard_normal(o.n).astype(np.float32)
    y = rng.standard_normal(o.m).astype(np.float32)
    y0 = rng.standard_normal(o.m).astype(np.float32)
    x0 = rng.standard_normal(o.n).astype(np.float32)
    want1 = o.aprod1(x.astype(np.float64), y0.astype(np.float64))
    bound1 = abs_system(S).aprod1(np.abs(x.astype(np.float64)), np.abs(y0.astype(np.float64)))
    want2 = o.aprod2(y.astype(np.float64), x0.astype(np.float64))
    bound2 = abs_system(S).aprod2(np.abs(y.astype(np.float64)), np.abs(x0.astype(np.float64)))
    g = gpu_system(torch, S)
    g.set_option("att_mode", variant[0])
    g.set_option("att_interleave", variant[1])
    g.set_option("att_buckets", BUCKETS.get(name, 5))
    yd = torch.from_numpy(y0).cuda()
    g.aprod1_f32(torch.from_numpy(x).cuda(), yd)
    xd = torch.from_numpy(x0).cuda()
    g.aprod2_f32(xd, torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    got1, got2 = yd.cpu().numpy().astype(np.float64), xd.cpu().numpy().astype(np.float64)
    g.close()
    assert np.all(np.abs(got1 - want1) <= 32 * EPS32 * bound1 + 1e-30)
    c = 2.0 * np.sqrt(S.m) + 32
    assert np.all(np.abs(got2 - want2) <= c * EPS32 * bound2 + 1e-30)


def test_aprod_f32_needs_fp32_values(torch_cuda):
    torch = torch_cuda
    from paper_2308_00778_amd import LSQR_E_STATE, LsqrError

    S, o = system("few_rows")
    say("FP32 operators on an FP64 system: LSQR_E_STATE")
    g = gpu_system(torch, S)
    with pytest.raises(LsqrError) as ei:
        g.aprod1_f32(torch.zeros(o.n, dtype=torch.float32, device="cuda"),
                     torch.zeros(o.m, dtype=torch.float32, device="cuda"))
    g.close()
    assert ei.value.status == LSQR_E_STATE


@pytest.mark.parametrize("name", ["c0", "ragged", "wide_instr", "huge_instr"])
def test_precond_parity(torch_cuda, name):
    torch = torch_cuda
    S, o = system(name)
    say(f"column norms: {name}")
    g = gpu_system(torch, S)
    p = g.precond().cpu().numpy()
    g.close()
    assert rel_inf(p, o.precond()) < 1e-13


def _b(S, o, rhs=0):
    xt = synth.x_true(S.spec)
    return o.aprod1(xt, synth.noise(S.spec, S.m, rhs=rhs))


# Iteration counts stay well below the unknown count of the tiny systems: as k
# approaches n the finite-precision bidiagonalisation nears termination and
# any two FP64 LSQR implementations drift apart (the oracle and SciPy's LSQR
# differ by 2e-9 at k = 30 on the 36-unknown "one_star" system, 1e-15 at 15).
@pytest.mark.parametrize("name,itn", [("c0", 50), ("c0", 200), ("ragged", 120),
                                       ("one_star", 15), ("few_rows", 15), ("wide_instr", 60),
                                       ("huge_instr", 30), ("huge_instr_lined", 30),
                                       ("instr_70k", 30),
                                       ("instr_12k", 30), ("instr_12k_f32", 30),
                                       ("wide_att_f32", 30)])
@pytest.mark.parametrize("graph", [1, 0])
def test_solve_fixed_iterations(torch_cuda, name, itn, graph):
    _solve_fixed(torch_cuda, name, itn, graph, VARIANTS[0])


@pytest.mark.parametrize("variant", VARIANTS[1:], ids=[f"att{a}_scan{b}" for a, b in VARIANTS[1:]])
@pytest.mark.parametrize("name,itn", [("c0", 50), ("ragged", 60)])
def test_solve_variants(torch_cuda, name, itn, variant):
    _solve_fixed(torch_cuda, name, itn, 1, variant)


@pytest.mark.parametrize("name,itn", [("c0", 50), ("wide_instr", 40)])
def test_solve_without_interleaved_attitude(torch_cuda, name, itn):
    _solve_fixed(torch_cuda, name, itn, 1, VARIANTS[0], interleave=0)


# The default iteration (fused mode 2: attitude pre-pass in bucket order, then
# the fused pass) against fused mode 1 (attitude dot product inside the fused
# pass) and separate aprod1/aprod2 launches (0): all must match the oracle.
@pytest.mark.parametrize("fused", [3, 1, 0])
@pytest.mark.parametrize("name,itn", [("c0", 60), ("ragged", 60), ("one_star", 15),
                                       ("few_rows", 15), ("wide_instr", 40),
                                       ("instr_12k", 30), ("wide_att_f32", 30)])
def test_solve_other_fused_modes(torch_cuda, name, itn, fused):
    _solve_fixed(torch_cuda, name, itn, 1, VARIANTS[0], fused=fused)


# The fused passes read compact copies of the star and instrumental indices
# by default; the caller's int64/int32 arrays without them.
@pytest.mark.parametrize("fused", [2, 3, 1])
@pytest.mark.parametrize("name,itn", [("c0", 60), ("huge_instr", 30), ("wide_att_f32", 30)])
def test_solve_without_compact_index(torch_cuda, name, itn, fused):
    _solve_fixed(torch_cuda, name, itn, 1, VARIANTS[0], fused=fused, compact=0)


def test_compact_index_toggle(torch_cuda):
    # copies built on the first solve, freed (graphs dropped) when the option
    # is switched off, rebuilt when it is switched on again: same iterates
    torch = torch_cuda
    S, o = system("c0")
    b = torch.from_numpy(_b(S, o)).cuda()
    say("compact index copies toggled between solves: c0")
    g = gpu_system(torch, S)
    g.set_option("tests", 0)  # graph replay: the captured graphs must follow
    xs, flags = [], []
    for compact in (1, 0, 1):
        g.set_option("compact_index", compact)
        x, _ = g.solve(b, 30, atol=0.0, btol=0.0)
        xs.append(x.cpu().numpy())
        flags.append(g.pass_times()["compact"])
    g.close()
    assert flags == [1, 0, 1]
    x_ref, _ = o.lsqr(_b(S, o), 30, atol=0.0, btol=0.0, conlim=0.0, tests=False)
    for xg in xs:
        assert rel_inf(xg, x_ref) <= 1e-10
    assert rel_inf(xs[1], xs[0]) <= 1e-13 and rel_inf(xs[2], xs[0]) <= 1e-13


def _solve_fixed(torch_cuda, name, itn, graph, variant, interleave=1, fused=2, compact=1):
    torch = torch_cuda
    S, o = system(name)
    b = _b(S, o)
    x_ref, i_ref = o.lsqr(b, itn, atol=0.0, btol=0.0, conlim=0.0, tests=False)
    say(f"solve parity: {name} itn={itn} graph={graph} variant={variant} "
        f"interleave={interleave} fused={fused}")
    g = gpu_system(torch, S)
    g.set_option("att_mode", variant[0])
    g.set_option("astro_scan", variant[1])
    g.set_option("att_interleave", interleave)
    g.set_option("fused", fused)
    g.set_option("compact_index", compact)
    if graph:
        g.set_option("att_buckets", BUCKETS.get(name, 3))
    g.set_option("tests", 0)
    g.set_option("graph", graph)
    g.set_option("chunk", 7)
    x, info = g.solve(torch.from_numpy(b).cuda(), itn, atol=0.0, btol=0.0)
    torch.cuda.synchronize()
    xg = x.cpu().numpy()
    g.close()
    assert info.itn == i_ref.itn == itn and info.istop == 7
    assert rel_inf(xg, x_ref) <= 1e-10
    # rnorm, xnorm, bnorm describe the converged iterate; anorm and acond sum
    # the whole alpha/beta history, which after the loss of orthogonality of
    # the finite-precision bidiagonalisation (well past convergence) differs
    # between any two summation orders
    late = itn > 50
    for k in ("rnorm", "anorm", "acond", "xnorm", "bnorm"):
        a, r = getattr(info, k), getattr(i_ref, k)
        tol = 1e-2 if (late and k in ("anorm", "acond")) else 1e-8
        assert abs(a - r) <= tol * abs(r), (k, a, r)


# Buckets shorter than a wave, and empty ones. The bucket-order passes start
# each bucket's row blocks on the 64-row boundary at or below its first row:
# here most lanes' rows lie before their bucket (they load its first row and
# contribute nothing), many threads have no row of their own (19 and 149
# buckets of about 50 rows on "short_stars" and "wide_instr"), and in
# "sparse_rows" (39 rows over 197 attitude starts, 99 buckets) most buckets
# hold no row. aprod2 (the attitude pass), a fixed-iteration solve (the
# attitude pre-pass) and a 2-RHS k-tile against the oracle.
TINY_BUCKETS = {"short_stars": 36, "wide_instr": 290, "sparse_rows": 150}
_SPARSE = synth.tiny(seed=31, n_stars=20, obs=(1, 3), n_dfa=200, n_instr_cols=8)


@pytest.mark.parametrize("name", list(TINY_BUCKETS))
def test_tiny_buckets_parity(torch_cuda, name):
    torch = torch_cuda
    if name == "sparse_rows":
        if name not in _SYS:
            S = synth.make_system(_SPARSE)
            _SYS[name] = (S, oracle.OracleSystem.from_synth(S))
    S, o = system(name)
    nbk, itn = TINY_BUCKETS[name], 10
    say(f"tiny buckets: {name} m={S.m} n={o.n} att_buckets={nbk}")
    rng = np.random.default_rng(9)
    y = rng.standard_normal(o.m)
    x0 = rng.standard_normal(o.n)
    want = o.aprod2(y, x0)
    bound = abs_system(S).aprod2(np.abs(y), np.abs(x0))
    g = gpu_system(torch, S)
    g.set_option("att_buckets", nbk)
    g.set_option("tests", 0)
    xd = torch.from_numpy(x0).cuda()
    g.aprod2(xd, torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    got = xd.cpu().numpy()
    c = 2.0 * np.sqrt(S.m) + 32
    assert np.all(np.abs(got - want) <= c * EPS * bound + 1e-300)
    bs = [_b(S, o, rhs=j) for j in range(2)]
    refs = [o.lsqr(b, itn, atol=0.0, btol=0.0, conlim=0.0, tests=False)[0] for b in bs]
    x, info = g.solve(torch.from_numpy(bs[0]).cuda(), itn, atol=0.0, btol=0.0)
    torch.cuda.synchronize()
    assert info.itn == itn and rel_inf(x.cpu().numpy(), refs[0]) <= 1e-10
    g.set_option("ktile", 2)
    X, infos = g.solve_batched(torch.from_numpy(np.ascontiguousarray(np.stack(bs, axis=1))).cuda(),
                               itn, 0.0, 0.0)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    g.close()
    for j in range(2):
        assert infos[j].itn == itn and rel_inf(Xh[:, j], refs[j]) <= 1e-10, j


# 2-RHS k-tile on the line-aligned system: its K-wide tail windows in the
# nontemporal-load form, against the oracle.
def test_batched_line_aligned_tail(torch_cuda):
    torch = torch_cuda
    S, o = system("huge_instr_lined")
    itn = 20
    say(f"batched tail windows, line-aligned columns: m={S.m} n={o.n} itn={itn}")
    bs = [_b(S, o, rhs=j) for j in range(2)]
    refs = [o.lsqr(b, itn, atol=0.0, btol=0.0, conlim=0.0, tests=False)[0] for b in bs]
    g = gpu_system(torch, S)
    g.set_option("att_buckets", 5)
    g.set_option("tests", 0)
    g.set_option("ktile", 2)
    X, infos = g.solve_batched(torch.from_numpy(np.ascontiguousarray(np.stack(bs, axis=1))).cuda(),
                               itn, 0.0, 0.0)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    g.close()
    for j in range(2):
        assert infos[j].itn == itn and rel_inf(Xh[:, j], refs[j]) <= 1e-10, j


# Iteration counts before convergence: the variance sums (w/rho)^2 over all
# iterations, and past convergence those terms depend on rounding like the
# anorm/acond estimates. On "ragged" the oracle and SciPy's LSQR (calc_var)
# differ by 1.5e-13 at 20 iterations, 3.4e-11 at 30, 2.8e-9 at 40 and 3.6% at
# 60, while their iterates x still agree.
@pytest.mark.parametrize("name,itn", [("c0", 50), ("ragged", 25), ("huge_instr", 30)])
def test_variance_parity(torch_cuda, name, itn):
    # Algorithm 1's per-iteration variance term, re-multiplied by p^2
    torch = torch_cuda
    from paper_2308_00778_amd import LSQR_E_STATE, LsqrError

    S, o = system(name)
    b = _b(S, o)
    x_ref, _, var_ref = o.lsqr(b, itn, atol=0.0, btol=0.0, conlim=0.0, tests=False,
                               want_var=True)
    say(f"variance parity: {name} itn={itn}")
    g = gpu_system(torch, S)
    g.set_option("tests", 0)
    with pytest.raises(LsqrError) as ei:  # nothing computed yet
        g.variance()
    assert ei.value.status == LSQR_E_STATE
    g.set_option("variance", 1)
    x, info = g.solve(torch.from_numpy(b).cuda(), itn, atol=0.0, btol=0.0)
    var = g.variance().cpu().numpy()
    xg = x.cpu().numpy()
    g.set_option("variance", 0)
    g.solve(torch.from_numpy(b).cuda(), 5, atol=0.0, btol=0.0)
    with pytest.raises(LsqrError):  # the last solve did not compute it
        g.variance()
    g.close()
    assert rel_inf(xg, x_ref) <= 1e-10
    assert np.all(var >= 0.0)
    assert rel_inf(var, var_ref) <= 1e-10


def test_solve_stopping_rules(torch_cuda):
    torch = torch_cuda
    S, o = system("c0")
    b = _b(S, o)
    x_ref, i_ref = o.lsqr(b, 300, atol=1e-12, btol=1e-12, conlim=1e8)
    say("solve stopping rules: c0 atol=btol=1e-12")
    g = gpu_system(torch, S)
    x, info = g.solve(torch.from_numpy(b).cuda(), 300, atol=1e-12, btol=1e-12)
    xg = x.cpu().numpy()
    g.close()
    assert info.istop == i_ref.istop and abs(info.itn - i_ref.itn) <= 1, (info, i_ref)
    assert rel_inf(xg, x_ref) <= 1e-10
    # converged: normal-equation residual of the scaled problem, recomputed
    # explicitly. Forming r = b - A x in FP64 (||b|| ~ 1.5e3, ||r|| ~ 3e-4)
    # leaves a floor of about eps ||A|| ||x|| / ||r|| ~ 1e-9 on this ratio; an
    # unconverged iterate (10 iterations) sits near 1e-5.
    p = o.precond()
    r = b - o.aprod1(xg)
    assert np.linalg.norm(p * o.aprod2(r)) <= 1e-9 * info.anorm * np.linalg.norm(r)


def test_repeated_solves_reuse_graphs(torch_cuda):
    # One handle, three solves: the captured iteration graph and the workspaces
    # are reused across right-hand sides and iteration counts.
    torch = torch_cuda
    S, o = system("c0")
    b1 = _b(S, o, rhs=0)
    b2 = _b(S, o, rhs=1)
    say("repeated solves on one handle: c0")
    g = gpu_system(torch, S)
    g.set_option("tests", 0)
    g.set_option("chunk", 5)
    runs = [(b1, 40), (b2, 33), (b1, 40), (b2, 12)]
    xs = []
    for b, itn in runs:
        x, info = g.solve(torch.from_numpy(b).cuda(), itn, atol=0.0, btol=0.0)
        assert info.itn == itn
        xs.append(x.cpu().numpy())
    g.close()
    for (b, itn), xg in zip(runs, xs):
        x_ref, _ = o.lsqr(b, itn, atol=0.0, btol=0.0, conlim=0.0, tests=False)
        assert rel_inf(xg, x_ref) <= 1e-10
    assert rel_inf(xs[2], xs[0]) <= 1e-13  # same solve again: rounding order only


def test_option_errors(torch_cuda):
    torch = torch_cuda
    from paper_2308_00778_amd import LSQR_E_INVALID, LSQR_E_STATE, LsqrError

    S, o = system("few_rows")
    say("option validation: few_rows")
    g = gpu_system(torch, S)
    bad = [("att_mode", 2), ("ktile", 3), ("chunk", 0), ("att_buckets", -1), ("outer_tol", -1.0),
           ("fused", 4), ("att_rhs", 3), ("att_rhs", 0)]
    for name, value in bad:
        with pytest.raises(LsqrError) as ei:
            g.set_option(name, value)
        assert ei.value.status == LSQR_E_INVALID, name
    g.set_option("att_buckets", 2)
    g.set_option("tests", 0)
    b = _b(S, o)
    g.solve(torch.from_numpy(b).cuda(), 5, atol=0.0, btol=0.0)
    for name, value in (("att_buckets", 3), ("att_rhs", 2)):
        with pytest.raises(LsqrError) as ei:  # the bucket order exists now
            g.set_option(name, value)
        assert ei.value.status == LSQR_E_STATE, name
    with pytest.raises(LsqrError) as ei:  # refinement needs FP32-stored values
        g.solve_refined(torch.from_numpy(b).cuda(), 5, atol=1e-6, btol=1e-6, outer_limit=2)
    assert ei.value.status == LSQR_E_STATE
    g.close()


def test_zero_rhs_and_zero_iterations(torch_cuda):
    torch = torch_cuda
    S, o = system("ragged")
    say("edge: b = 0, itn_limit = 0")
    g = gpu_system(torch, S)
    x, info = g.solve(torch.zeros(S.m, dtype=torch.float64, device="cuda"), 50)
    assert info.istop == 0 and info.itn == 0 and not torch.any(x).item()
    b = _b(S, o)
    x, info = g.solve(torch.from_numpy(b).cuda(), 0)
    assert info.itn == 0 and not torch.any(x).item()
    g.close()


def test_no_preconditioning(torch_cuda):
    # Without column scaling the iterates of any two FP64 LSQR codes part early
    # on this system (oracle vs SciPy: 4.5e-3 apart at k = 20), so the check is
    # on the converged least-squares solution, which is unique (kappa = 45).
    torch = torch_cuda
    S, o = system("ragged")
    b = _b(S, o)
    x_ref, i_ref = o.lsqr(b, 3000, atol=1e-14, btol=1e-14, conlim=0.0, precondition=False)
    say(f"solve without preconditioning: ragged, to convergence (oracle itn={i_ref.itn})")
    g = gpu_system(torch, S, precondition=False)
    g.set_option("conlim", 0)
    x, info = g.solve(torch.from_numpy(b).cuda(), 3000, atol=1e-14, btol=1e-14)
    xg = x.cpu().numpy()
    g.close()
    assert info.istop in (1, 2, 4, 5) and info.itn < 3000
    assert rel_inf(xg, x_ref) <= 1e-10


def test_invalid_indices_are_rejected(torch_cuda):
    torch = torch_cuda
    from paper_2308_00778_amd import LSQR_E_INVALID, LsqrError, LsqrSystem

    S, _ = system("few_rows")
    sp = S.spec
    base = dict(values=torch.from_numpy(S.values).cuda(),
                star_of_row=torch.from_numpy(S.star_of_row).cuda(),
                att_start=torch.from_numpy(S.att_start).cuda(),
                instr_idx=torch.from_numpy(S.instr_idx).cuda())
    cases = {
        "star_out_of_range": ("star_of_row", lambda t: t.__setitem__(-1, sp.n_stars)),
        "star_unsorted": ("star_of_row", lambda t: t.__setitem__(0, 2)),
        "att_out_of_range": ("att_start", lambda t: t.__setitem__(3, sp.n_dfa - 3)),
        "instr_out_of_range": ("instr_idx", lambda t: t.__setitem__((5, 2), sp.n_instr_cols)),
        "instr_negative": ("instr_idx", lambda t: t.__setitem__((0, 0), -1)),
    }
    for case, (key, mutate) in cases.items():
        say(f"invalid descriptor: {case}")
        arrays = {k: v.clone() for k, v in base.items()}
        mutate(arrays[key])
        torch.cuda.synchronize()
        with pytest.raises(LsqrError) as ei:
            LsqrSystem(**arrays, n_stars=sp.n_stars, n_dfa=sp.n_dfa,
                       n_instr_cols=sp.n_instr_cols)
        assert ei.value.status == LSQR_E_INVALID, case


F32_SPEC = synth.tiny(seed=31, n_stars=400, obs=(100, 100), n_dfa=400, n_instr_cols=120,
                      value_dtype="f32", astro_scale=(-2.0, 2.0))


def test_fp64_solve_on_float_values(torch_cuda):
    torch = torch_cuda
    S = synth.make_system(F32_SPEC)
    o = oracle.OracleSystem.from_synth(S)  # widens the float values
    b = _b(S, o)
    x_ref, _ = o.lsqr(b, 60, atol=0.0, btol=0.0, conlim=0.0, tests=False)
    say("FP64 solve on float-stored values: itn=60")
    g = gpu_system(torch, S)
    g.set_option("tests", 0)
    x, info = g.solve(torch.from_numpy(b).cuda(), 60, atol=0.0, btol=0.0)
    xg = x.cpu().numpy()
    g.close()
    assert rel_inf(xg, x_ref) <= 1e-10


# F32_WIDE: 30,000 instrumental columns. The FP32 inner solve keeps the
# instrumental slice of vp (120 KB) and a 4,416-column histogram in LDS and
# leaves the other columns to two tail windows; the FP64 residual and the
# oracle see every column.
F32_WIDE = synth.tiny(seed=32, n_stars=700, obs=(60, 100), n_dfa=200, n_instr_cols=30000,
                      value_dtype="f32", astro_scale=(-2.0, 2.0))


@pytest.mark.parametrize("fused", [2, 3])
@pytest.mark.parametrize("spec", [F32_SPEC, F32_WIDE], ids=["f32", "f32_wide_instr"])
def test_refined_matches_fp64_oracle(torch_cuda, spec, fused):
    torch = torch_cuda
    S = synth.make_system(spec)
    o = oracle.OracleSystem.from_synth(S)
    b = _b(S, o)
    x_ref, i_ref = o.lsqr(b, 500, atol=1e-14, btol=1e-14, conlim=0.0)
    say(f"refined solve: FP32 values m={S.m} fused={fused}; oracle itn={i_ref.itn} "
        f"istop={i_ref.istop}")
    g = gpu_system(torch, S)
    g.set_option("fused", fused)
    x, info = g.solve_refined(torch.from_numpy(b).cuda(), 200, atol=1e-6, btol=1e-6,
                              outer_limit=8)
    xg = x.cpu().numpy()
    g.close()
    say(f"refined: outer={info.outer_steps} inner itn={info.itn} "
        f"err={rel_inf(xg, x_ref):.3e}")
    assert info.outer_steps <= 6
    assert rel_inf(xg, x_ref) <= 1e-10


# Harder conditioning: astrometric coefficients correlated with rho = 0.999
# (the generator's astro_corr knob) give a condition estimate of 2e4 after
# column scaling, against ~30 for the default systems, and 900 iterations to
# converge instead of 40. Equal-iteration parity is checked at 40 iterations:
# the oracle and SciPy's LSQR differ by 1.5e-14 there, 1e-12 at 60, 3e-10 at
# 80 and 4e-5 at 150 (loss of orthogonality), while their converged solutions
# agree to 2.7e-14.
HARD = synth.tiny(seed=81, n_stars=400, obs=(20, 60), n_dfa=150, n_instr_cols=23,
                  value_dtype="f32", astro_corr=0.999)


def test_harder_conditioning_fp64_and_refined(torch_cuda):
    torch = torch_cuda
    S = synth.make_system(HARD)
    o = oracle.OracleSystem.from_synth(S)
    b = _b(S, o)
    x_conv, i_conv = o.lsqr(b, 20000, atol=1e-14, btol=1e-14, conlim=0.0)
    x_fix, _ = o.lsqr(b, 40, atol=0.0, btol=0.0, conlim=0.0, tests=False)
    say(f"harder conditioning: oracle itn={i_conv.itn} acond={i_conv.acond:.2e}")
    g = gpu_system(torch, S)
    g.set_option("tests", 0)
    x, _ = g.solve(torch.from_numpy(b).cuda(), 40, atol=0.0, btol=0.0)
    e_fix = rel_inf(x.cpu().numpy(), x_fix)
    g.set_option("tests", 1)
    xr, info = g.solve_refined(torch.from_numpy(b).cuda(), 3000, atol=1e-6, btol=1e-6,
                               outer_limit=30)
    e_ref = rel_inf(xr.cpu().numpy(), x_conv)
    g.close()
    say(f"fixed 40 itn err={e_fix:.3e}; refined outer={info.outer_steps} "
        f"inner itn={info.itn} err={e_ref:.3e}")
    assert e_fix <= 1e-10
    assert e_ref <= 1e-10


def test_profile_pass_times(torch_cuda):
    torch = torch_cuda
    S, o = system("c0")
    b = _b(S, o)
    say("profile pass times: c0 itn=12, fused modes 2 and 1")
    g = gpu_system(torch, S)
    g.set_option("tests", 0)
    g.set_option("profile", 1)
    g.solve(torch.from_numpy(b).cuda(), 12, atol=0.0, btol=0.0)
    pt = g.pass_times()
    assert pt.pop("mode") == 2  # default: attitude pre-pass
    assert pt.pop("compact") == 1  # default: compact index copies (small system)
    assert all(n == 12 for _, n in pt.values()) and all(ms > 0 for ms, _ in pt.values())
    g.set_option("fused", 1)
    g.solve(torch.from_numpy(b).cuda(), 12, atol=0.0, btol=0.0)
    pt1 = g.pass_times()
    kt = g.kernel_times()
    g.close()
    # mode 1 has no pre-pass: the first window holds only the interleave copy
    assert pt1["mode"] == 1 and pt1["pre"][0] < pt1["fused"][0]
    assert abs(pt1["pre"][0] + pt1["fused"][0] - kt["aprod1_ms"]) <= 1e-6 * kt["aprod1_ms"]
    # many attitude buckets (84 windows of 12 starts): pre-pass windows at
    # every bucket boundary, same iterates
    g = gpu_system(torch, S)
    g.set_option("att_buckets", 90)
    g.set_option("tests", 0)
    g.set_option("profile", 1)
    x, _ = g.solve(torch.from_numpy(b).cuda(), 12, atol=0.0, btol=0.0)
    assert g.pass_times()["mode"] == 2
    g.close()
    x_ref, _ = o.lsqr(b, 12, atol=0.0, btol=0.0, conlim=0.0, tests=False)
    assert rel_inf(x.cpu().numpy(), x_ref) <= 1e-10


def test_profile_counts_launches(torch_cuda):
    torch = torch_cuda
    S, o = system("c0")
    b = _b(S, o)
    say("profile mode: c0 itn=20")
    g = gpu_system(torch, S)
    g.set_option("tests", 0)
    g.set_option("profile", 1)
    x, info = g.solve(torch.from_numpy(b).cuda(), 20, atol=0.0, btol=0.0)
    t = g.kernel_times()
    g.close()
    assert t["aprod1_n"] == t["aprod2_n"] == 20
    assert t["aprod1_ms"] > 0 and t["aprod2_ms"] > 0
    x_ref, _ = o.lsqr(b, 20, atol=0.0, btol=0.0, conlim=0.0, tests=False)
    assert rel_inf(x.cpu().numpy(), x_ref) <= 1e-10
