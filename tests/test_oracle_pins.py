"""Pins for the oracle: each check ties the oracle to something other than
itself (dense brute force, LAPACK least squares, SciPy's implementation of the
same published LSQR, CGLS, closed forms, invariants, special cases).

The mutation test at the bottom compiles modified copies of oracle.c with
plausible mistakes planted (dropped term, wrong sign, wrong index, transposed
operand) and requires that at least one check fails for each.
"""
import os
import shutil
import tempfile

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

import oracle
import synth
from dense_ref import cgls, dense_matrix, with_constraints

ORACLE_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle", "oracle.c")


def _tiny_systems():
    return [
        synth.make_system(synth.tiny(seed=5)),  # 20 stars x 30 obs, 173 columns
        synth.make_system(synth.tiny(seed=9, n_stars=13, obs=(9, 41), n_dfa=11,
                                     n_instr_cols=7)),  # ragged, narrow attitude
        synth.make_system(synth.tiny(seed=13, n_stars=8, obs=(40, 60), n_dfa=30,
                                     n_instr_cols=6, value_dtype="f32",
                                     astro_scale=(-1.0, 1.0))),
    ]


_CACHE = {}


def systems():
    if "tiny" not in _CACHE:
        _CACHE["tiny"] = [(S, dense_matrix(S)) for S in _tiny_systems()]
    return _CACHE["tiny"]


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _problem(S, A, noise=1e-3, seed=0):
    rng = np.random.default_rng(seed)
    xt = rng.standard_normal(A.shape[1])
    b = A @ xt + noise * rng.standard_normal(A.shape[0])
    return xt, b


# ---------------------------------------------------------------- operators
def check_aprod_dense():
    rng = np.random.default_rng(1)
    for S, A in systems():
        o = oracle.OracleSystem.from_synth(S)
        assert A.shape == (o.m, o.n)
        x = rng.standard_normal(o.n)
        y = rng.standard_normal(o.m)
        assert rel(o.aprod1(x), A @ x) < 1e-13
        assert rel(o.aprod1(x, y), y + A @ x) < 1e-13
        assert rel(o.aprod2(y), A.T @ y) < 1e-13
        assert rel(o.aprod2(y, x), x + A.T @ y) < 1e-13
        rows = np.array([0, o.m // 3, o.m - 1])
        assert rel(o.aprod1_rows(x, rows), (A @ x)[rows]) < 1e-13


def check_adjoint_identity():
    rng = np.random.default_rng(2)
    S = synth.make_system(synth.WORKLOADS[0])
    o = oracle.OracleSystem.from_synth(S)
    x = rng.standard_normal(o.n)
    y = rng.standard_normal(o.m)
    lhs = o.aprod1(x) @ y
    rhs = x @ o.aprod2(y)
    fro = np.sqrt(np.sum(S.values.astype(np.float64) ** 2))
    assert abs(lhs - rhs) <= 1e-14 * fro * np.linalg.norm(x) * np.linalg.norm(y)


def check_unit_columns():
    # closed form: A e_k is column k of A; the global column is the last
    # coefficient of every row, an astrometric column is one coefficient of
    # one star's rows.
    S, A = systems()[0]
    sp = S.spec
    o = oracle.OracleSystem.from_synth(S)
    e = np.zeros(o.n)
    e[-1] = 1.0
    assert np.array_equal(o.aprod1(e), S.values[-1].astype(np.float64))
    e[:] = 0.0
    star, j = 7, 2
    e[sp.n_astro * star + j] = 1.0
    expect = np.zeros(o.m)
    r0, r1 = S.first_row[star], S.first_row[star + 1]
    expect[r0:r1] = S.values[j, r0:r1]
    assert np.array_equal(o.aprod1(e), expect)
    # attitude axis 1, parameter 2, t = 3 -> column att_base + n_dfa + 5
    e[:] = 0.0
    col = sp.n_astro * sp.n_stars + sp.n_dfa + 5
    e[col] = 1.0
    got = o.aprod1(e)
    want = np.zeros(o.m)
    for q in range(sp.n_par_axis):
        hit = S.att_start + q == 5
        want[hit] += S.values[sp.n_astro + sp.n_par_axis + q][hit]
    assert np.array_equal(got, want)


# -------------------------------------------------------------------- norms
def check_norm_eq4():
    rng = np.random.default_rng(3)
    a = rng.standard_normal(1001)
    assert abs(oracle.norm(a) - np.linalg.norm(a)) <= 4e-16 * np.linalg.norm(a)
    assert oracle.norm(np.zeros(5)) == 0.0
    assert oracle.norm(np.array([3.0, -4.0])) == 5.0
    assert oracle.norm(np.array([-2.5])) == 2.5
    # the scaling keeps huge and tiny vectors representable
    assert abs(oracle.norm(np.full(4, 1e200)) / 2e200 - 1.0) < 1e-15
    assert abs(oracle.norm(np.full(4, 1e-200)) / 2e-200 - 1.0) < 1e-15


def check_precond_dense():
    for S, A in systems():
        o = oracle.OracleSystem.from_synth(S)
        cn = np.linalg.norm(A, axis=0)
        want = np.where(cn > 0, 1.0 / np.where(cn > 0, cn, 1.0), 1.0)
        assert rel(o.precond(), want) < 1e-14


# --------------------------------------------------------------------- LSQR
def check_lstsq():
    for k, (S, A) in enumerate(systems()):
        o = oracle.OracleSystem.from_synth(S)
        xt, b = _problem(S, A, seed=k)
        xls = np.linalg.lstsq(A, b, rcond=None)[0]
        x, info = o.lsqr(b, 2000, atol=0.0, btol=0.0, conlim=0.0)
        assert info.istop in (4, 5), info
        assert rel(x, xls) < 1e-10
        # normal equations: ||A^T r|| / (||A|| ||r||) small at convergence
        r = b - A @ x
        assert np.linalg.norm(A.T @ r) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(r)


def _scipy_lsqr(S, A, b, k, p):
    Ab = A * p[None, :]
    return scipy.sparse.linalg.lsqr(scipy.sparse.csr_matrix(Ab), b, damp=0.0, atol=0.0,
                                    btol=0.0, conlim=0.0, iter_lim=k, calc_var=True)


def check_scipy_iterates():
    for idx, (S, A) in enumerate(systems()):
        o = oracle.OracleSystem.from_synth(S)
        _, b = _problem(S, A, seed=10 + idx)
        p = o.precond()
        for k in (1, 2, 3, 5, 10, 20):
            x, info, var = o.lsqr(b, k, atol=0.0, btol=0.0, conlim=0.0, want_var=True)
            res = _scipy_lsqr(S, A, b, k, p)
            ys, istop, itn, r1, r2, anorm, acond, arnorm, xnorm, vs = res
            assert itn == info.itn == k
            assert rel(x, p * ys) < 1e-12, (k, rel(x, p * ys))
            assert abs(info.rnorm - r1) <= 1e-12 * abs(r1)
            assert abs(info.anorm - anorm) <= 1e-12 * anorm
            assert abs(info.acond - acond) <= 1e-11 * acond
            assert abs(info.arnorm - arnorm) <= 1e-8 * abs(arnorm) + 1e-14 * info.bnorm
            assert abs(info.xnorm - xnorm) <= 1e-10 * xnorm
            assert rel(var, p * p * vs) < 1e-12


def check_scipy_stopping():
    for idx, (S, A) in enumerate(systems()):
        o = oracle.OracleSystem.from_synth(S)
        _, b = _problem(S, A, seed=20 + idx)
        p = o.precond()
        for atol, conlim in ((1e-12, 1e8), (1e-6, 1e8), (1e-12, 3.0)):
            x, info = o.lsqr(b, 500, atol=atol, btol=atol, conlim=conlim)
            Ab = A * p[None, :]
            res = scipy.sparse.linalg.lsqr(Ab, b, atol=atol, btol=atol, conlim=conlim,
                                           iter_lim=500)
            if idx < 2:
                assert (info.istop, info.itn) == (res[1], res[2]), (atol, conlim, info, res[1:3])
                assert rel(x, p * res[0]) < 1e-9
            else:
                # this system loses orthogonality early (k ~ 30), after which any
                # two FP64 implementations drift at the 1e-11..1e-9 level, so a
                # threshold crossing may move by one iteration
                assert info.istop == res[1] and abs(info.itn - res[2]) <= 1, (info, res[1:3])


def check_cgls():
    for idx, (S, A) in enumerate(systems()):
        o = oracle.OracleSystem.from_synth(S)
        _, b = _problem(S, A, seed=30 + idx)
        p = o.precond()
        its = cgls(A * p[None, :], b, 10)
        for k in range(1, 11):
            x, _ = o.lsqr(b, k, atol=0.0, btol=0.0, conlim=0.0, tests=False)
            assert rel(x, p * its[k - 1]) < 1e-10, k


def check_first_iterate_closed_form():
    for idx, (S, A) in enumerate(systems()):
        o = oracle.OracleSystem.from_synth(S)
        _, b = _problem(S, A, seed=40 + idx)
        p = o.precond()
        Ab = A * p[None, :]
        g = Ab.T @ b
        y1 = (g @ g) / np.sum((Ab @ g) ** 2) * g
        x, info = o.lsqr(b, 1, atol=0.0, btol=0.0, conlim=0.0)
        assert rel(x, p * y1) < 1e-13


def check_recurrence_invariants():
    # phibar_{k+1} = ||b - A x_k||, arnorm = ||Abar^T (b - A x_k)||
    S, A = systems()[0]
    o = oracle.OracleSystem.from_synth(S)
    _, b = _problem(S, A, seed=50)
    p = o.precond()
    for k in (2, 6, 12):
        x, info = o.lsqr(b, k, atol=0.0, btol=0.0, conlim=0.0)
        r = b - A @ x
        assert abs(info.rnorm - np.linalg.norm(r)) <= 1e-10 * np.linalg.norm(r)
        arn = np.linalg.norm(p * (A.T @ r))
        assert abs(info.arnorm - arn) <= 1e-8 * arn
        assert abs(info.xnorm - np.linalg.norm(x / p)) <= 1e-12 * np.linalg.norm(x / p)


def check_noise_free_recovery():
    S = synth.make_system(synth.WORKLOADS[0])
    o = oracle.OracleSystem.from_synth(S)
    xt = synth.x_true(S.spec)
    b = o.aprod1(xt)
    x, info = o.lsqr(b, 200, atol=1e-14, btol=1e-14)
    assert info.istop in (1, 2, 4, 5) and info.itn < 200
    assert rel(x, xt) < 1e-10


def check_precondition_invariance():
    S, A = systems()[1]
    o = oracle.OracleSystem.from_synth(S)
    _, b = _problem(S, A, seed=60)
    x1, i1 = o.lsqr(b, 3000, atol=0.0, btol=0.0, conlim=0.0, precondition=True)
    x0, i0 = o.lsqr(b, 3000, atol=0.0, btol=0.0, conlim=0.0, precondition=False)
    assert rel(x1, x0) < 1e-9


def check_special_cases():
    S, A = systems()[0]
    o = oracle.OracleSystem.from_synth(S)
    x, info = o.lsqr(np.zeros(o.m), 50)
    assert info.istop == 0 and info.itn == 0 and not np.any(x)
    # a consistent system (b is one column of A): the residual test S1 stops it
    # and the solution is that unit vector
    e = np.zeros(o.n)
    e[-1] = 1.0
    b = A @ e
    x, info = o.lsqr(b, 500, atol=1e-12, btol=1e-12)
    assert rel(x, e) < 1e-10 and info.istop == 1 and info.rnorm < 1e-10 * info.bnorm


def check_variance_limit():
    # In exact arithmetic sum_k d_k d_k^T grows towards (Abar^T Abar)^{-1}
    # (reached after n steps), so the re-scaled diagonal estimate increases
    # with k and stays below diag((A^T A)^{-1}).
    S, A = systems()[1]
    o = oracle.OracleSystem.from_synth(S)
    _, b = _problem(S, A, seed=70)
    want = np.diag(np.linalg.inv(A.T @ A))
    prev = np.zeros(o.n)
    for k in (3, 8, 20):
        _, _, var = o.lsqr(b, k, atol=0.0, btol=0.0, conlim=0.0, tests=False, want_var=True)
        assert np.all(var >= prev) and np.all(var <= want * (1 + 1e-10))
        prev = var
    assert np.all(prev > 0)


# Row layouts with some sections absent or resized (the paper's subset
# systems: astrometric-only, attitude-only, several global columns).
SECTION_LAYOUTS = {
    "astro_only": dict(n_axes=0, n_instr=0, n_glob=0),
    "att_only": dict(n_astro=0, n_instr=0, n_glob=0),
    "mixed": dict(n_astro=3, n_instr=2, n_glob=3),
    "no_att_five_glob": dict(n_axes=0, n_glob=5),
}


def section_system(name, seed=41):
    spec = synth.tiny(seed=seed, n_stars=30, obs=(10, 30), n_dfa=40, n_instr_cols=15,
                      **SECTION_LAYOUTS[name])
    return synth.make_system(spec)


def check_section_layouts():
    for name in SECTION_LAYOUTS:
        S = section_system(name)
        o = oracle.OracleSystem.from_synth(S)
        A = dense_matrix(S)
        rng = np.random.default_rng(3)
        x = rng.standard_normal(o.n)
        y = rng.standard_normal(o.m)
        assert np.max(np.abs(o.aprod1(x) - A @ x)) <= 1e-12 * np.max(np.abs(A) @ np.abs(x)), name
        assert np.max(np.abs(o.aprod2(y) - A.T @ y)) <= 1e-12 * np.max(np.abs(A.T) @ np.abs(y)), name
        # converged solution against LAPACK (empty columns: p = 1, x = 0)
        b = o.aprod1(synth.x_true(S.spec), synth.noise(S.spec, S.m))
        x_orc, info = o.lsqr(b, 2000, atol=1e-14, btol=1e-14, conlim=0.0)
        x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
        assert np.max(np.abs(x_orc - x_ls)) <= 1e-9 * np.max(np.abs(x_ls)), (name, info)


def _with_empty_row(con, at):
    rp = np.insert(con.rowptr, at + 1, con.rowptr[at])
    return synth.Constraints(rowptr=rp, col=con.col, val=con.val)


def constraint_cases():
    """(system, constraints, name): a full-layout system with long sparse
    constraint rows (one empty), and an astrometric-only system whose stars
    have 2..4 observations (rank-deficient blocks) that the constraint rows
    over the astrometric columns make full rank."""
    if "con" not in _CACHE:
        S1 = synth.make_system(synth.tiny(seed=5))
        C1 = _with_empty_row(synth.constraints(S1.spec, 6, nnz=(1, 90), seed=1), 2)
        sp2 = synth.tiny(seed=17, n_stars=6, obs=(2, 4), n_axes=0, n_instr=0, n_glob=0)
        S2 = synth.make_system(sp2)
        C2 = synth.constraints(sp2, 24, nnz=(6, 14), seed=2)
        _CACHE["con"] = [(S1, C1, "full_layout"), (S2, C2, "rank_deficient")]
    return _CACHE["con"]


def check_constraints():
    rng = np.random.default_rng(8)
    for S, C, name in constraint_cases():
        o = oracle.OracleSystem.from_synth(S, con=C)
        A0 = dense_matrix(S)
        A = with_constraints(A0, C)
        assert A.shape == (o.m, o.n) and o.m == S.m + C.n_con
        x = rng.standard_normal(o.n)
        y = rng.standard_normal(o.m)
        assert rel(o.aprod1(x, y), y + A @ x) < 1e-13, name
        assert rel(o.aprod2(y, x), x + A.T @ y) < 1e-13, name
        cn = np.linalg.norm(A, axis=0)
        p = np.where(cn > 0, 1.0 / np.where(cn > 0, cn, 1.0), 1.0)
        assert rel(o.precond(), p) < 1e-13, name
        b = A @ rng.standard_normal(o.n) + 1e-3 * rng.standard_normal(o.m)
        for k in (2, 5, 12):  # iterates and estimates: SciPy's LSQR on the scaled matrix
            xo, info = o.lsqr(b, k, atol=0.0, btol=0.0, conlim=0.0, tests=False)
            res = scipy.sparse.linalg.lsqr(A * p[None, :], b, atol=0.0, btol=0.0, conlim=0.0,
                                           iter_lim=k)
            assert rel(xo, p * res[0]) < 1e-11, (name, k)
            assert abs(info.rnorm - res[3]) <= 1e-11 * res[3], (name, k)
        # the constraints complete the rank; converged solution = LAPACK's
        assert np.linalg.matrix_rank(A) == o.n, name
        if name == "rank_deficient":
            assert np.linalg.matrix_rank(A0) < o.n
        xo, info = o.lsqr(b, 5000, atol=1e-14, btol=1e-14, conlim=0.0)
        x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
        assert rel(xo, x_ls) < 1e-9, (name, info)


CHECKS = [check_aprod_dense, check_adjoint_identity, check_unit_columns, check_norm_eq4,
          check_precond_dense, check_lstsq, check_scipy_iterates, check_scipy_stopping,
          check_cgls, check_first_iterate_closed_form, check_recurrence_invariants,
          check_noise_free_recovery, check_precondition_invariance, check_special_cases,
          check_variance_limit, check_section_layouts, check_constraints]


@pytest.mark.parametrize("check", CHECKS, ids=[c.__name__ for c in CHECKS])
def test_pin(check):
    check()


# ------------------------------------------------------------- mutation test
MUTANTS = {
    "rhobar_sign": ("rhobar = -c * alpha;", "rhobar = c * alpha;"),
    "drop_alpha_u": ("u[i] = -alpha * u[i];", "u[i] = 0.0 * u[i];"),
    "drop_beta_v": ("v[j] = -beta * v[j];", "v[j] = 0.0 * v[j];"),
    "att_param_order": ("s->att[i] + q;", "s->att[i] + (s->n_par_axis - 1 - q);"),
    "instr_base": ("return instr_base + s->instr", "return att_base + s->instr"),
    "eq4_unscaled": ("return mx * sqrt(ssq);", "return sqrt(ssq);"),
    "no_remultiply": ("x[j] = p[j] * y[j];", "x[j] = y[j];"),
    "aprod2_wrong_coef": ("x[column(s, c, i)] += coef(s, c, i) * y[i];",
                          "x[column(s, c, i)] += coef(s, (c + 1) % np, i) * y[i];"),
    "phibar_cos": ("phibar = sn * phibar;", "phibar = c * phibar;"),
    "w_sign": ("w[j] = v[j] - (theta / rho) * w[j];", "w[j] = v[j] + (theta / rho) * w[j];"),
    "acond_no_sqrt": ("acond = anorm * sqrt(ddnorm);", "acond = anorm * ddnorm;"),
    "arnorm_no_c": ("arnorm = alpha * fabs(c) * phibar;", "arnorm = alpha * phibar;"),
    "precond_no_sqrt": ("1.0 / sqrt(ssq[j])", "1.0 / ssq[j]"),
    "anorm_drop_beta": ("anorm * anorm + alpha * alpha + beta * beta",
                        "anorm * anorm + alpha * alpha"),
    "con_aprod1_overwrite": ("y[s->m + r] += sum;", "y[s->m + r] = sum;"),
    "con_aprod2_row": ("x[s->con_col[e]] += s->con_val[e] * y[s->m + r];",
                       "x[s->con_col[e]] += s->con_val[e] * y[s->m];"),
    "con_norm_unsquared": ("ssq[s->con_col[e]] += s->con_val[e] * s->con_val[e];",
                           "ssq[s->con_col[e]] += fabs(s->con_val[e]);"),
    "con_unscaled": ("con_scaled[e] = s->con_val[e] * p[s->con_col[e]];",
                     "con_scaled[e] = s->con_val[e];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutants_are_caught(name):
    old, new = MUTANTS[name]
    src = open(ORACLE_SRC).read()
    assert src.count(old) == 1, name
    tmp = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        path = os.path.join(tmp, "oracle_mut.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        lib = oracle.build(src=path, out=os.path.join(tmp, "liboracle_mut.so"))
        oracle.use_library(lib)
        _CACHE.clear()
        failed = []
        for check in CHECKS:
            try:
                check()
            except AssertionError:
                failed.append(check.__name__)
        assert failed, f"mutant {name} passed every pin"
    finally:
        oracle.use_library(None)
        _CACHE.clear()
        shutil.rmtree(tmp, ignore_errors=True)
