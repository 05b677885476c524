"""The FP64 LCA state tolerance of the parity tests, on synthetic states:
the stable sum mode gets no amplification, the difference mode gets
1e-13 g^n capped at 1e-6 absolute."""
import numpy as np
import pytest

from paper_2110_15425_amd import workloads as W
from parity import AMP_CAP, lca_amp, lca_growth, lca_state_check


def _states(n, d_sum, d_diff):
    o = np.array([[0.5, 0.3]] * len(n))
    g = o + np.array([[(d_sum + d_diff) / 2, (d_sum - d_diff) / 2]])
    return g, o


def test_growth_is_the_difference_mode_eigenvalue():
    w = W.conflict(trials=1)
    dt, leak, comp = w["params"][:3]
    A = np.eye(2) + dt * np.array([[-leak, -comp], [-comp, -leak]])
    ev = np.sort(np.linalg.eigvals(A))
    assert np.isclose(ev[1], lca_growth(w)) and np.isclose(ev[0], 1 - dt * (leak + comp))
    assert lca_amp(w, 10_000) == AMP_CAP and np.isclose(lca_amp(w, 10), lca_growth(w) ** 10)


def test_sum_mode_has_no_amplification():
    w = W.conflict(trials=1)
    g, o = _states([400], 1e-8, 0.0)  # 1e-8 in the sum mode, even after 400 steps
    with pytest.raises(AssertionError, match="sum mode"):
        lca_state_check(w, g, o, [400])
    g, o = _states([400], 5e-10, 0.0)
    lca_state_check(w, g, o, [400])


def test_difference_mode_amplification_is_capped():
    w = W.conflict(trials=1)
    g, o = _states([10], 0.0, 1e-9)  # 1e-13 * 1.05^10 << 1e-9
    with pytest.raises(AssertionError, match="difference mode"):
        lca_state_check(w, g, o, [10])
    g, o = _states([400], 0.0, 9e-7)  # 1.05^400 > AMP_CAP: tolerance 1e-6
    lca_state_check(w, g, o, [400])
    g, o = _states([900], 0.0, 2e-6)  # beyond the cap at any length
    with pytest.raises(AssertionError, match="difference mode"):
        lca_state_check(w, g, o, [900])


def test_clipping_couples_the_modes():
    w = W.conflict(trials=1, nonneg=1.0)
    g, o = _states([400], 5e-7, 0.0)
    lca_state_check(w, g, o, [400])
