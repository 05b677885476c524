"""Comparison helpers for GPU-vs-oracle parity tests."""
import numpy as np

NSTAT = 9


def reduce_dumps(w, d, correct, exclude=None):
    """Histogram and statistics rebuilt from per-run dumps (optionally
    leaving out some runs), for comparisons when runs are flagged."""
    S, T, B, N = int(w["n_settings"]), int(w["trials"]), int(w["n_bins"]), int(w["max_steps"])
    hist = np.zeros((S, 2, B), np.uint64)
    stats = np.zeros((S, NSTAT), np.uint64)
    ch = d["run_choice"].astype(np.int64)
    n = d["run_step"].astype(np.uint64)
    keep = np.ones(ch.size, bool) if exclude is None else ~exclude
    idx = np.arange(ch.size)
    s = idx // T
    stim = (idx % T) % int(w["n_stimuli"])
    for c in (0, 1):
        m = keep & (ch == c)
        b = ((n[m] - 1) * B) // N
        np.add.at(hist, (s[m], c, b.astype(np.int64)), 1)
        np.add.at(stats[:, c], s[m], 1)
        np.add.at(stats[:, 4 + c], s[m], n[m])
        np.add.at(stats[:, 6 + c], s[m], n[m] * n[m])
    np.add.at(stats[:, 2], s[keep & (ch < 0)], 1)
    tgt = np.asarray(correct)[stim]
    np.add.at(stats[:, 3], s[keep & (ch >= 0) & (ch == tgt)], 1)
    np.add.at(stats[:, 8], s[keep & (d["run_flag"] != 0)], 1)
    return hist, stats


def lca_growth(w):
    """Per-step growth factor of the LCA's difference mode x0 - x1:
    1 + dt (comp - leak) (the mode is unstable when comp > leak)."""
    p = w["params"]
    dt, leak, comp = p[0], p[1], p[2]
    return 1.0 + dt * max(0.0, comp - leak)


# Largest amplification the difference-mode tolerance allows: 1e-13 * AMP_CAP
# = 1e-6 absolute, about 1e-6 of the threshold.
AMP_CAP = 1e7


def lca_amp(w, n):
    """Amplification of a per-step perturbation after n steps in the LCA's
    difference mode, capped at AMP_CAP."""
    return np.minimum(lca_growth(w) ** np.asarray(n, np.float64), AMP_CAP)


def lca_state_check(w, g_state, o_state, n, state_rtol=1e-9, state_atol=1e-12):
    """FP64 LCA final states, checked in the two modes of the linear update.

    The update is x' = A x + dt I + b z with A = I + dt M, M = -[[leak, comp],
    [comp, leak]].  A has the eigenvectors (1, 1) and (1, -1): the sum mode
    x0 + x1 is multiplied by 1 - dt (leak + comp) per step (stable), the
    difference mode x0 - x1 by g = 1 + dt (comp - leak) (g > 1 at the
    configured leak 0.5, comp 1.0).  The two sides differ per step by a few
    ulps of the noise increment (host and device libm round log/cos/sin
    differently, ~1e-16 absolute), so after n steps the difference mode may
    differ by up to ~1e-16 g^n / (g - 1): 1e-13 g^n leaves a margin of ~50.
    That term is capped at 1e-13 * AMP_CAP = 1e-6 absolute.  The sum mode
    gets the plain FP64 acceptance (1e-9 relative) with no amplification,
    except with clipping at 0 (NONNEG), where clipping couples the modes and
    both get the capped term.  Returns (max |difference|, max ratio of
    difference to tolerance) over both modes."""
    g_state = np.asarray(g_state, np.float64)
    o_state = np.asarray(o_state, np.float64)
    amp = 1e-13 * lca_amp(w, n)
    nonneg = float(w["params"][8]) != 0.0  # the NONNEG parameter of the LCA and the loop
    worst_d, worst_r = 0.0, 0.0
    for name, sign in (("sum", 1.0), ("difference", -1.0)):
        gv = g_state[:, 0] + sign * g_state[:, 1]
        ov = o_state[:, 0] + sign * o_state[:, 1]
        d = np.abs(gv - ov)
        tol = state_atol + state_rtol * np.abs(ov)
        if sign < 0 or nonneg:
            tol = tol + amp
        if d.size:
            worst_d = max(worst_d, float(d.max()))
            worst_r = max(worst_r, float((d / tol).max()))
        bad = np.flatnonzero(d > tol)
        assert bad.size == 0, (f"{name} mode: {bad.size} runs beyond tolerance; first {bad[:3]}: "
                               f"diff {d[bad[:3]]} tol {tol[bad[:3]]} steps {np.asarray(n)[bad[:3]]}")
    return worst_d, worst_r


def assert_parity(w, g, o, correct, state_rtol=1e-9, state_atol=1e-12, max_flag_frac=1e-4):
    """FP64 acceptance: per-run integers bit-exact on runs neither side
    flagged, final states within state_rtol (the LCA's in its two modes, see
    lca_state_check), aggregate integers exact when nothing is flagged (else
    exact after removing the flagged runs).  Prints the flagged fraction and
    the largest state difference."""
    flagged = (g["run_flag"] != 0) | (o["run_flag"] != 0)
    ok = ~flagged
    frac = flagged.mean()
    assert frac <= max_flag_frac, f"flagged fraction {frac}"
    bad = np.flatnonzero(ok & ((g["run_choice"] != o["run_choice"]) | (g["run_step"] != o["run_step"])))
    assert bad.size == 0, (f"{bad.size} unflagged runs differ; first {bad[:5]}: gpu "
                           f"{g['run_choice'][bad[:5]]}/{g['run_step'][bad[:5]]} oracle "
                           f"{o['run_choice'][bad[:5]]}/{o['run_step'][bad[:5]]}")
    if int(w["kind"]) in (1, 3):  # the conflict LCA, open or closed loop
        worst_d, worst_r = lca_state_check(w, g["run_state"][ok], o["run_state"][ok],
                                           o["run_step"][ok], state_rtol, state_atol)
    else:
        gs_, os2 = g["run_state"][ok], o["run_state"][ok]
        np.testing.assert_allclose(gs_, os2, rtol=state_rtol, atol=state_atol)
        d = np.abs(gs_ - os2)
        worst_d = float(d.max()) if d.size else 0.0
        worst_r = float((d / (state_atol + state_rtol * np.abs(os2))).max()) if d.size else 0.0
    print(f"parity: {flagged.size} runs, flagged fraction {frac:.2e}, largest state difference "
          f"{worst_d:.3e} ({worst_r:.3f} of its tolerance)", flush=True)
    # each side's aggregates are the reduction of its own per-run outcomes
    gh, gs = reduce_dumps(w, g, correct)
    assert np.array_equal(gh, g["hist"]) and np.array_equal(gs, g["stats"])
    if not flagged.any():
        assert np.array_equal(g["hist"], o["hist"])
        assert np.array_equal(g["stats"], o["stats"])
    else:
        gh, gs = reduce_dumps(w, g, correct, exclude=flagged)
        oh, os_ = reduce_dumps(w, o, correct, exclude=flagged)
        assert np.array_equal(gh, oh) and np.array_equal(gs[:, :8], os_[:, :8])
    return frac


def hist_l1(a, b, trials):
    """Per-setting L1 distance between outcome distributions (choice x bin,
    plus the undecided mass)."""
    pa = a["hist"].reshape(a["hist"].shape[0], -1) / trials
    pb = b["hist"].reshape(b["hist"].shape[0], -1) / trials
    ua = a["stats"][:, 2] / trials
    ub = b["stats"][:, 2] / trials
    return np.abs(pa - pb).sum(1) + np.abs(ua - ub)
