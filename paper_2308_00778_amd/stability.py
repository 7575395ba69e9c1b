"""Consistency of two solutions of the same system (Sect. 6).

Two solvers of one system (different codes, precisions or hardware) agree
when, section by section, the differences of their solutions (d_x) and of
their errors (d_sigma) are small, and every unknown satisfies Eq. (5):
q = |x_a - x_b| / sqrt(sigma_a^2 + sigma_b^2) < 1, i.e. the two solutions lie
within one standard error of each other. Errors are reported in arcseconds
with Eq. (6).

Readings: the error of an unknown is its standard error, the square root of
its variance estimate (the diagonal accumulated by LSQR and re-multiplied by
p^2, as returned by LsqrSystem.variance) times the residual standard
deviation rnorm / sqrt(m - n); mean and standard deviation are the population
ones (ddof = 0). Host-side post-processing of finished solves.
"""
from dataclasses import dataclass

import numpy as np

RAD_PER_ARCSEC = 4.84814e-6  # Eq. (6)


def sections(n_stars, n_dfa, n_instr_cols, n_astro=5, n_axes=3, n_glob=1):
    """Column ranges of the unknowns, in the order astro | att | instr | glob
    (absent sections omitted)."""
    a = n_astro * n_stars
    t = a + n_axes * n_dfa
    i = t + (n_instr_cols if n_instr_cols else 0)
    g = i + n_glob
    out = {"astrometric": (0, a), "attitude": (a, t), "instrumental": (t, i), "global": (i, g)}
    return {k: v for k, v in out.items() if v[1] > v[0]}


def standard_errors(var, rnorm, m, n):
    """sigma_j = sqrt(var_j) * rnorm / sqrt(m - n); needs more rows m than unknowns n."""
    if m <= n:
        raise ValueError("standard errors need more rows than unknowns")
    return np.sqrt(np.asarray(var, np.float64)) * (float(rnorm) / np.sqrt(float(m - n)))


def sigma_arcsec(sigma_rad):
    """Eq. (6): an error in radians, in arcseconds."""
    return np.asarray(sigma_rad, dtype=np.float64) / RAD_PER_ARCSEC


@dataclass
class SectionReport:
    section: str
    count: int
    mean_dx: float
    std_dx: float
    mean_dsigma: float
    std_dsigma: float
    q_max: float  # largest Eq. (5) ratio in the section

    @property
    def consistent(self) -> bool:
        return self.q_max < 1.0


def compare(x_a, sigma_a, x_b, sigma_b, secs):
    """Per-section statistics of d_x = x_a - x_b and d_sigma = sigma_a - sigma_b
    and the largest q of Eq. (5). Inputs: host arrays (or anything
    numpy.asarray accepts) of the n unknowns and their errors."""
    x_a, x_b = np.asarray(x_a, np.float64), np.asarray(x_b, np.float64)
    s_a, s_b = np.asarray(sigma_a, np.float64), np.asarray(sigma_b, np.float64)
    if not (x_a.shape == x_b.shape == s_a.shape == s_b.shape and x_a.ndim == 1):
        raise ValueError("solutions and errors must be 1-D arrays of one length")
    if np.any(s_a < 0) or np.any(s_b < 0):
        raise ValueError("errors must be >= 0")
    rows = []
    for name, (lo, hi) in secs.items():
        dx = x_a[lo:hi] - x_b[lo:hi]
        ds = s_a[lo:hi] - s_b[lo:hi]
        den = np.sqrt(s_a[lo:hi] ** 2 + s_b[lo:hi] ** 2)
        with np.errstate(divide="ignore", invalid="ignore"):
            q = np.where(den > 0, np.abs(dx) / den, np.where(dx == 0, 0.0, np.inf))
        rows.append(SectionReport(name, hi - lo, float(dx.mean()), float(dx.std()),
                                  float(ds.mean()), float(ds.std()), float(q.max())))
    return rows


def format_table(rows):
    """Rows as a text table in the layout of the paper's comparison table."""
    out = [f"{'section':<13} {'mean(d_x) +- std(d_x)':>26} {'mean(d_s) +- std(d_s)':>26} "
           f"{'max q':>9}"]
    for r in rows:
        out.append(f"{r.section:<13} {r.mean_dx:>12.2e} +- {r.std_dx:<9.2e} "
                   f"{r.mean_dsigma:>12.2e} +- {r.std_dsigma:<9.2e} {r.q_max:>9.2e}")
    return "\n".join(out)
