"""Independent reference values used to pin the oracle.

Nothing here re-types the oracle's update loops: each helper computes what
the mathematics fixes for the simulated process by another route --
Chapman-Kolmogorov propagation of the survivor density, closed-form
first-passage results, Gaussian moment recursions -- so that a dropped term,
a wrong sign or a transposed operand in the oracle shows up as a
disagreement.
"""
import math

import numpy as np
from scipy import special, stats


def ddm_walk_density(a, b, theta, start=0.0, max_steps=3000, cells=1000, tol=1e-15):
    """First-passage probabilities of the discrete Gaussian walk
    x_n = x_{n-1} + a + b z_n (z ~ N(0,1)), stopped when x_n >= theta (upper)
    or x_n <= -theta (lower), by propagating the survivor mass on a grid of
    cells over (-theta, theta) with the exact Gaussian step kernel (midpoint
    rule in the source cell, exact CDF differences in the target cell).
    Returns (upper[n], lower[n]) for n = 1..max_steps (index n-1)."""
    h = 2.0 * theta / cells
    edges = -theta + h * np.arange(cells + 1)
    centres = 0.5 * (edges[:-1] + edges[1:])

    def step_from(points):
        z_edges = (edges[None, :] - points[:, None] - a) / b
        cdf = special.ndtr(z_edges)
        kern = np.diff(cdf, axis=1)
        up = special.ndtr(-(theta - points - a) / b)
        lo = special.ndtr((-theta - points - a) / b)
        return kern, up, lo

    upper = np.zeros(max_steps)
    lower = np.zeros(max_steps)
    k0, u0, l0 = step_from(np.array([start]))
    mass = k0[0]
    upper[0], lower[0] = u0[0], l0[0]
    K, up, lo = step_from(centres)
    for n in range(1, max_steps):
        upper[n] = mass @ up
        lower[n] = mass @ lo
        mass = mass @ K
        if mass.sum() < tol:
            break
    return upper, lower


def ddm_continuous(drift, noise, theta):
    """Continuous DDM from 0 with absorbing bounds +-theta: P(lower) and mean
    decision time (Bogacz et al. 2006, eqs. for the unbiased pure DDM)."""
    k = drift * theta / noise ** 2
    p_err = 1.0 / (1.0 + math.exp(2.0 * k))
    mean_dt = (theta / drift) * math.tanh(k)
    return p_err, mean_dt


def ddm_bgk(drift, noise, theta, dt):
    """Continuous formulas with the Broadie-Glasserman-Kou boundary shift
    (theta + 0.5826 sigma sqrt(dt)) for discretely monitored crossings."""
    return ddm_continuous(drift, noise, theta + 0.5826 * noise * math.sqrt(dt))


def binned(prob_by_step, n_bins, max_steps):
    """Sum per-step probabilities into bins floor((n-1) * B / N)."""
    n = np.arange(1, max_steps + 1)
    bins = ((n - 1) * n_bins) // max_steps
    out = np.zeros(n_bins)
    np.add.at(out, bins, prob_by_step)
    return out


def chisq_pvalue(observed, expected_prob, min_expected=5.0):
    """Pearson chi-square of integer counts against probabilities; cells with
    small expectation are pooled into one."""
    observed = np.asarray(observed, np.float64)
    total = observed.sum()
    e = np.asarray(expected_prob, np.float64) * total
    big = e >= min_expected
    obs = list(observed[big]) + [observed[~big].sum()]
    exp = list(e[big]) + [e[~big].sum()]
    obs, exp = np.array(obs), np.array(exp)
    keep = exp > 0
    obs, exp = obs[keep], exp[keep]
    # rescale so totals agree exactly (probabilities may miss a tail < 1e-12)
    exp = exp * obs.sum() / exp.sum()
    chi = ((obs - exp) ** 2 / exp).sum()
    return float(stats.chi2.sf(chi, len(obs) - 1))


def lca_linear_moments(inp, leak, comp, dt, b, n):
    """Mean and covariance of the linear two-unit LCA after n steps from 0:
    x_n = A x_{n-1} + dt I + b z with A = I + dt M, M = [[-leak, -comp],
    [-comp, -leak]]."""
    A = np.eye(2) + dt * np.array([[-leak, -comp], [-comp, -leak]])
    m = np.zeros(2)
    Cov = np.zeros((2, 2))
    for _ in range(n):
        m = A @ m + dt * np.asarray(inp)
        Cov = A @ Cov @ A.T + b * b * np.eye(2)
    return m, Cov


def ou_moments(dt, b, g, n):
    """Euler OU unit x_n = (1-dt) x_{n-1} + dt g u + b xi from 0: returns
    (slope of E[x_n | u] in u, residual variance)."""
    lam = 1.0 - dt
    slope = g * (1.0 - lam ** n)
    resid = b * b * (1.0 - lam ** (2 * n)) / (1.0 - lam * lam)
    return slope, resid
