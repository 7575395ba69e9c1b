"""Dense construction of the AVU-GSR coefficient matrix for tiny systems.

Built section by section from the block picture of the paper's Sect. 2 and
Fig. 1 (block-diagonal astrometric part, attitude blocks of 4 consecutive
columns per axis at stride N_DFA, scattered instrumental columns, global
column), independently of the oracle's per-coefficient column function, so
that a dense matrix product checks the oracle's sparse operators.
"""
import numpy as np
import scipy.linalg


def dense_matrix(S):
    sp = S.spec
    m = S.m
    vals = S.values.astype(np.float64)
    k = 0
    # astrometric: one (obs_s x n_astro) block per star on the diagonal
    blocks = []
    for s in range(sp.n_stars):
        r0, r1 = int(S.first_row[s]), int(S.first_row[s + 1])
        blocks.append(vals[k:k + sp.n_astro, r0:r1].T)
    astro = scipy.linalg.block_diag(*blocks) if sp.n_astro else np.zeros((m, 0))
    assert astro.shape == (m, sp.n_astro * sp.n_stars)
    k += sp.n_astro
    # attitude: per axis a band of n_par_axis columns starting at t_i
    att = np.zeros((m, sp.n_axes * sp.n_dfa))
    rows = np.arange(m)
    for a in range(sp.n_axes):
        for q in range(sp.n_par_axis):
            att[rows, a * sp.n_dfa + S.att_start + q] += vals[k + a * sp.n_par_axis + q]
    k += sp.n_axes * sp.n_par_axis
    instr = np.zeros((m, sp.n_instr_cols))
    for j in range(sp.n_instr):
        np.add.at(instr, (rows, S.instr_idx[j]), vals[k + j])
    k += sp.n_instr
    glob = vals[k:k + sp.n_glob].T.copy()
    return np.hstack([astro, att, instr, glob])


def with_constraints(A, con):
    """A with the constraint rows (CSR rowptr/col/val) appended below it."""
    extra = np.zeros((con.rowptr.shape[0] - 1, A.shape[1]))
    for r in range(extra.shape[0]):
        sl = slice(int(con.rowptr[r]), int(con.rowptr[r + 1]))
        np.add.at(extra[r], con.col[sl], con.val[sl])
    return np.vstack([A, extra])


def cgls(A, b, iters):
    """Conjugate gradients on the normal equations (Hestenes-Stiefel form of
    CGLS, Bjorck 1996, Alg. 7.4.1); iterates equal LSQR's in exact arithmetic."""
    x = np.zeros(A.shape[1])
    r = b.copy()
    s = A.T @ r
    p = s.copy()
    gamma = s @ s
    out = []
    for _ in range(iters):
        q = A @ p
        alpha = gamma / (q @ q)
        x = x + alpha * p
        r = r - alpha * q
        s = A.T @ r
        gamma_new = s @ s
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
        out.append(x.copy())
    return out
