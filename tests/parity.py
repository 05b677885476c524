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


def assert_parity(w, g, o, correct, state_rtol=1e-9, state_atol=1e-12, max_flag_frac=1e-4):
    """FP64 acceptance: per-run integers bit-exact on runs neither side
    flagged, final states within state_rtol, aggregate integers exact when
    nothing is flagged (else exact after removing the flagged runs).

    The two sides' normals may differ in the last bit (different libm), and
    the LCA's difference mode amplifies such differences by lca_growth()
    per step, so for the LCA the state tolerance grows as 1e-13 * growth^n
    for a run of n steps (1e-13: a few hundred ulps at unit scale)."""
    flagged = (g["run_flag"] != 0) | (o["run_flag"] != 0)
    ok = ~flagged
    frac = flagged.mean()
    assert frac <= max_flag_frac, f"flagged fraction {frac}"
    bad = np.flatnonzero(ok & ((g["run_choice"] != o["run_choice"]) | (g["run_step"] != o["run_step"])))
    assert bad.size == 0, (f"{bad.size} unflagged runs differ; first {bad[:5]}: gpu "
                           f"{g['run_choice'][bad[:5]]}/{g['run_step'][bad[:5]]} oracle "
                           f"{o['run_choice'][bad[:5]]}/{o['run_step'][bad[:5]]}")
    if int(w["kind"]) in (1, 3):  # the conflict LCA, open or closed loop
        amp = lca_growth(w) ** o["run_step"][ok].astype(np.float64)
        tol = np.maximum(state_atol, 1e-13 * amp)[:, None] + state_rtol * np.abs(o["run_state"][ok])
        diff = np.abs(g["run_state"][ok] - o["run_state"][ok])
        assert np.all(diff <= tol), f"max state excess {np.max(diff - tol)}"
    else:
        np.testing.assert_allclose(g["run_state"][ok], o["run_state"][ok], rtol=state_rtol,
                                   atol=state_atol)
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
