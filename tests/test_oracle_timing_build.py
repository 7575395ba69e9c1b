"""The OpenMP timing build of the oracle (used only for the CPU baseline)
against the pinned single-thread reference build of the same source.

Rows of aprod1 are independent, so they agree bit for bit; aprod2, the column
norms and the norms of Eq. (4) add the same terms in another order (private
per-thread accumulators for the attitude, instrumental and global columns),
so they agree within c * eps * sum |terms|; LSQR iterates within 1e-10.
"""
import numpy as np
import pytest

import oracle
import synth

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def builds():
    import os

    if not os.path.exists(oracle.OMP_LIB_PATH):
        oracle.build(openmp=True)
    yield
    oracle.use_library(None)


def _run(path, fn):
    oracle.use_library(path)
    try:
        return fn()
    finally:
        oracle.use_library(None)


SPECS = [synth.WORKLOADS[0],
         synth.tiny(seed=61, n_stars=300, obs=(30, 140), n_dfa=400, n_instr_cols=900,
                    value_dtype="f32")]


@pytest.mark.parametrize("spec", SPECS, ids=["c0", "ragged_f32"])
def test_timing_build_matches_reference(builds, spec):
    S = synth.make_system(spec)
    o = oracle.OracleSystem.from_synth(S)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(o.n)
    y = rng.standard_normal(o.m)
    b = o.aprod1(synth.x_true(spec), synth.noise(spec, o.m))

    def compute():
        return (oracle.num_threads(), o.aprod1(x), o.aprod2(y), o.precond(),
                oracle.norm(y), o.lsqr(b, 50, atol=0.0, btol=0.0, conlim=0.0, tests=False)[0])

    ref = _run(None, compute)
    omp = _run(oracle.OMP_LIB_PATH, compute)
    assert ref[0] == 1 and omp[0] >= 1
    assert np.array_equal(omp[1], ref[1])
    absS = oracle.OracleSystem(np.abs(S.values.astype(np.float64)), S.star_of_row, S.att_start,
                               S.instr_idx, n_stars=spec.n_stars, n_dfa=spec.n_dfa,
                               n_instr_cols=spec.n_instr_cols)
    bound = absS.aprod2(np.abs(y))
    c = 2.0 * np.sqrt(o.m) + 32
    assert np.all(np.abs(omp[2] - ref[2]) <= c * EPS * bound + 1e-300)
    assert np.allclose(omp[3], ref[3], rtol=1e-13, atol=0.0)
    # sums of m squares in two orders: each within (m - 1) eps of the exact sum
    assert abs(omp[4] - ref[4]) <= o.m * EPS * ref[4]
    assert np.max(np.abs(omp[5] - ref[5])) <= 1e-10 * np.max(np.abs(ref[5]))
