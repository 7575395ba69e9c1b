"""GPU parity on rows whose sections differ from the full layout (5 astrometric,
3 x 4 attitude, 6 instrumental, 1 global coefficients): absent sections,
fewer astrometric or instrumental coefficients, several global columns. These
layouts run the general-layout kernels; the oracle takes the same section
sizes. Tolerances as in the full-layout parity tests.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps

# Several workgroups and a ragged tail per system; at least 10 observations
# per star where a star has astrometric unknowns (well-determined blocks).
LAYOUTS = {
    "astro_only": dict(n_axes=0, n_instr=0, n_glob=0),
    "att_only": dict(n_astro=0, n_instr=0, n_glob=0),
    "mixed": dict(n_astro=3, n_instr=2, n_glob=3),
    "no_att_five_glob": dict(n_axes=0, n_glob=5),
    "no_glob": dict(n_glob=0),
    "instr_glob_only": dict(n_astro=0, n_axes=0, n_instr=4, n_glob=2),
    # instrumental columns beyond one FP64 LDS histogram: tail windows
    "mixed_huge_instr": dict(n_astro=2, n_instr=3, n_glob=2, n_instr_cols=25000),
    "mixed_f32": dict(n_astro=4, n_instr=5, n_glob=2, value_dtype="f32"),
}

# Fixed iteration counts: well below the unknown count (25 on
# instr_glob_only), and past the window in which mixed_f32's iterates are
# sensitive to rounding while LSQR converges (oracle vs SciPy's LSQR: 1.9e-11
# at 20 iterations, 8.6e-9 at 30, 1.1e-12 at 40, 1e-15 at 50).
ITN = {"instr_glob_only": 10, "mixed_huge_instr": 30, "mixed_f32": 60}

_SYS = {}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def system(name, seed=61):
    if name not in _SYS:
        kw = dict(LAYOUTS[name])
        cols = kw.pop("n_instr_cols", 23)
        dt = kw.pop("value_dtype", "f64")
        spec = synth.tiny(seed=seed + list(LAYOUTS).index(name), n_stars=260, obs=(10, 70),
                          n_dfa=120, n_instr_cols=cols, value_dtype=dt, **kw)
        S = synth.make_system(spec)
        _SYS[name] = (S, oracle.OracleSystem.from_synth(S))
    return _SYS[name]


def abs_system(S):
    sp = S.spec
    return oracle.OracleSystem(np.abs(S.values.astype(np.float64)), S.star_of_row, S.att_start,
                               S.instr_idx, n_stars=sp.n_stars, n_dfa=sp.n_dfa,
                               n_instr_cols=sp.n_instr_cols, n_astro=sp.n_astro,
                               n_axes=sp.n_axes, n_par_axis=sp.n_par_axis, n_instr=sp.n_instr,
                               n_glob=sp.n_glob)


def gpu_system(S):
    from paper_2308_00778_amd import LsqrSystem

    return LsqrSystem.from_host(S, "cuda:0")


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _b(S, o):
    return o.aprod1(synth.x_true(S.spec), synth.noise(S.spec, S.m))


@pytest.mark.parametrize("name", list(LAYOUTS))
def test_sections_aprod1(torch_cuda, name):
    torch = torch_cuda
    S, o = system(name)
    say(f"aprod1 sections: {name} m={S.m} n={o.n}")
    rng = np.random.default_rng(5)
    x = rng.standard_normal(o.n)
    y0 = rng.standard_normal(o.m)
    want = o.aprod1(x, y0)
    bound = abs_system(S).aprod1(np.abs(x), np.abs(y0))
    g = gpu_system(S)
    yd = torch.from_numpy(y0).cuda()
    g.aprod1(torch.from_numpy(x).cuda(), yd)
    torch.cuda.synchronize()
    got = yd.cpu().numpy()
    g.close()
    assert np.all(np.abs(got - want) <= 32 * EPS * bound + 1e-300)


@pytest.mark.parametrize("att_mode", [1, 0])
@pytest.mark.parametrize("name", list(LAYOUTS))
def test_sections_aprod2(torch_cuda, name, att_mode):
    torch = torch_cuda
    S, o = system(name)
    say(f"aprod2 sections: {name} m={S.m} n={o.n} att_mode={att_mode}")
    rng = np.random.default_rng(6)
    y = rng.standard_normal(o.m)
    x0 = rng.standard_normal(o.n)
    want = o.aprod2(y, x0)
    bound = abs_system(S).aprod2(np.abs(y), np.abs(x0))
    g = gpu_system(S)
    g.set_option("att_mode", att_mode)
    g.set_option("att_buckets", 4)
    xd = torch.from_numpy(x0).cuda()
    g.aprod2(xd, torch.from_numpy(y).cuda())
    torch.cuda.synchronize()
    got = xd.cpu().numpy()
    g.close()
    c = 2.0 * np.sqrt(S.m) + 32
    assert np.all(np.abs(got - want) <= c * EPS * bound + 1e-300)


@pytest.mark.parametrize("name", list(LAYOUTS))
def test_sections_column_norms(torch_cuda, name):
    S, o = system(name)
    say(f"column norms sections: {name}")
    g = gpu_system(S)
    p = g.precond().cpu().numpy()
    g.close()
    assert np.max(np.abs(p - o.precond()) / o.precond()) < 1e-13


@pytest.mark.parametrize("att_mode", [1, 0])
@pytest.mark.parametrize("name", list(LAYOUTS))
def test_sections_solve_fixed_iterations(torch_cuda, name, att_mode):
    torch = torch_cuda
    S, o = system(name)
    itn = ITN.get(name, 40)
    b = _b(S, o)
    x_ref, i_ref = o.lsqr(b, itn, atol=0.0, btol=0.0, conlim=0.0, tests=False)
    say(f"solve sections: {name} itn={itn} att_mode={att_mode}")
    g = gpu_system(S)
    g.set_option("att_mode", att_mode)
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


# Iteration counts where two FP64 LSQR implementations still agree on the
# variance sum: on "mixed" the oracle and SciPy's LSQR (calc_var) differ by
# 2.9e-12 at 15 iterations and 3.2e-10 at 20; on "att_only" by 1.8e-13 at 20.
@pytest.mark.parametrize("name,itn", [("mixed", 15), ("att_only", 20)])
def test_sections_variance(torch_cuda, name, itn):
    torch = torch_cuda
    S, o = system(name)
    b = _b(S, o)
    x_ref, _, var_ref = o.lsqr(b, itn, atol=0.0, btol=0.0, conlim=0.0, tests=False,
                               want_var=True)
    say(f"variance sections: {name} itn={itn}")
    g = gpu_system(S)
    g.set_option("tests", 0)
    g.set_option("variance", 1)
    x, _ = g.solve(torch.from_numpy(b).cuda(), itn, atol=0.0, btol=0.0)
    var = g.variance().cpu().numpy()
    xg = x.cpu().numpy()
    g.close()
    assert rel_inf(xg, x_ref) <= 1e-10
    assert rel_inf(var, var_ref) <= 1e-10


def test_sections_refined_matches_fp64_oracle(torch_cuda):
    torch = torch_cuda
    S, o = system("mixed_f32")
    b = _b(S, o)
    x_ref, i_ref = o.lsqr(b, 2000, atol=1e-14, btol=1e-14, conlim=0.0)
    say(f"refined sections: mixed_f32 m={S.m}; oracle itn={i_ref.itn} istop={i_ref.istop}")
    g = gpu_system(S)
    x, info = g.solve_refined(torch.from_numpy(b).cuda(), 300, atol=1e-6, btol=1e-6,
                              outer_limit=10)
    xg = x.cpu().numpy()
    g.close()
    say(f"refined: outer={info.outer_steps} inner itn={info.itn} err={rel_inf(xg, x_ref):.3e}")
    assert rel_inf(xg, x_ref) <= 1e-10


def test_sections_batched_is_unsupported(torch_cuda):
    torch = torch_cuda
    from paper_2308_00778_amd import LSQR_E_UNSUPPORTED, LsqrError

    S, o = system("mixed")
    say("batched on a general layout: rejected")
    g = gpu_system(S)
    B = torch.zeros((S.m, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(LsqrError) as ei:
        g.solve_batched(B, 5)
    assert ei.value.status == LSQR_E_UNSUPPORTED
    g.close()
