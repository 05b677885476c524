"""GPU time course (cm_launch_timecourse) against the oracle's: counts of
contributing runs bit-exact and fixed-point sums within the FP64 state
tolerance; integer totals identical under any launch shape; the ordinary
outputs identical to cm_launch."""
import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import cm, workloads as W
from parity import lca_amp, lca_growth

pytestmark = pytest.mark.gpu

S32 = 2.0 ** 32

CASES = {
    "ddm_c0": (W.ddm(trials=4000), 30),
    "ddm_grid_ragged": (W.ddm(trials=501, drifts=np.linspace(0, 0.6, 7), max_steps=700, seed=4), 7),
    "ddm_every_step_direct": (W.ddm(trials=300, max_steps=1500, n_bins=10, seed=5), 1),
    "lca_c1": (W.conflict(trials=900, grid=W.control_grid(4)[::5], seed=2), 10),
    "lca_c2_small_T": (W.grid_search(trials=20, n=8, seed=3), 5),
    "lca_every_step_direct": (W.conflict(trials=450, grid=W.control_grid(4)[:3], max_steps=900,
                                         n_bins=9, seed=6), 1),
}


def _compare(w, g_tc, o_tc, g_out, fp32=False):
    S, K = o_tc.shape[:2]
    assert g_tc.shape == o_tc.shape
    flagged = g_out["stats"][:, 8].astype(np.int64)
    every = int(w["max_steps"]) // K if K else 1
    growth = lca_growth(w) if int(w["kind"]) == W.LCA else 1.0
    for s in range(S):
        gc, oc = g_tc[s, :, 0], o_tc[s, :, 0]
        if fp32:  # FP32 transcendentals differ between host and device: near-exact counts
            assert np.all(np.abs(gc - oc) <= max(2, 0.002 * int(w["trials"]))), s
        elif flagged[s] == 0:
            assert np.array_equal(gc, oc), (s, np.nonzero(gc != oc)[0][:5])
        else:
            assert np.all(np.abs(gc - oc) <= flagged[s]), s
        same = gc == oc
        n = (np.arange(K) + 1) * every
        if fp32:  # host and device FP32 transcendentals differ by ~1e-7, grown by the LCA mode
            delta = 1e-5 + 1e-6 * growth ** np.minimum(n, 600)
        else:
            # per-run state tolerance of the FP64 parity tests (difference-mode
            # amplification capped at 1e-6 absolute), for each of the squared and
            # product sums as well
            delta = 20 * (1e-12 + 1e-13 * (lca_amp(w, n) if int(w["kind"]) == W.LCA else 1.0))
        for c in range(1, 6):
            d = np.abs(g_tc[s, :, c].astype(np.float64) - o_tc[s, :, c].astype(np.float64))
            tol = gc * (S32 * delta + 1.0)
            bad = same & (d > tol)
            assert not bad.any(), (s, c, np.nonzero(bad)[0][:5], d[bad][:3], tol[bad][:3])


@pytest.mark.parametrize("name", list(CASES))
def test_timecourse_fp64_parity(name):
    w, every = CASES[name]
    print(f"case {name} S={w['n_settings']} T={w['trials']} N={w['max_steps']} every={every}",
          flush=True)
    h = cm.Handle(0)
    g_out, g_tc = cm.timecourse(w, every, handle=h)
    o_tc = oracle.timecourse(w, every)
    _compare(w, g_tc, o_tc, g_out)
    # the ordinary outputs are those of cm_launch
    plain = cm.run(w, handle=h)
    for k in ("hist", "stats"):
        assert np.array_equal(g_out[k], plain[k]), k


@pytest.mark.parametrize("kind", ["ddm", "lca"])
def test_timecourse_fp32_against_fp32_oracle(kind):
    if kind == "ddm":
        w, every = W.ddm(trials=3000, precision=W.FP32_STEP, max_steps=1200), 40
    else:
        w, every = W.conflict(trials=900, grid=W.control_grid(4)[::5], precision=W.FP32_STEP), 10
    g_out, g_tc = cm.timecourse(w, every)
    o_tc = oracle.timecourse(w, every)
    _compare(w, g_tc, o_tc, g_out, fp32=True)


def test_timecourse_large_states():
    """States far from the unit scale: squares beyond 2^19, where the kernel
    quantises with the general rounding instead of its short form (both give
    round-half-even of v 2^32), in waves that mix the two ranges."""
    w, every = W.ddm(trials=40, drift=0.0, noise=400.0, thresh=3000.0, max_steps=2000,
                     n_bins=10, seed=8), 7
    h = cm.Handle(0)
    g_out, g_tc = cm.timecourse(w, every, handle=h)
    o_tc = oracle.timecourse(w, every)
    assert g_tc.shape == o_tc.shape
    assert np.abs(o_tc[0, :, 3]).max() > 2 ** 19 * S32  # the general form is reached
    flagged = int(g_out["stats"][0, 8])
    gc, oc = g_tc[0, :, 0], o_tc[0, :, 0]
    assert np.all(np.abs(gc - oc) <= flagged)
    same = gc == oc
    # the walk's states agree to ~n ulps of |x| <= 3200: 1e-8 bounds the
    # state difference and 2 * 3200 * 1e-8 that of the square
    for c, dv in ((1, 1e-8), (3, 6.4e-5)):
        d = (g_tc[0, :, c].astype(np.uint64) - o_tc[0, :, c].astype(np.uint64)).view(np.int64)
        tol = gc * (S32 * dv + 1.0)
        bad = same & (np.abs(d) > tol)
        assert not bad.any(), (c, np.nonzero(bad)[0][:5], d[bad][:3])


@pytest.mark.parametrize("kind", ["ddm", "lca"])
def test_timecourse_independent_of_launch_shape(kind):
    """Integer sums: identical bits for every launch shape and for the
    LDS-window and direct-atomic paths."""
    if kind == "ddm":
        w, every, k = W.ddm(trials=5000, drifts=[0.1, 0.3], precision=W.FP32_STEP), 25, W.DDM
    else:
        w, every, k = W.conflict(trials=2000, grid=W.control_grid(4)[:6]), 4, W.LCA
    ref = None
    for rpl, sps in ((0, 0), (1, 1), (3, 7), (16, 32)):
        h = cm.Handle(0)
        h.set_tuning(k, int(w["precision"]), runs_per_lane=rpl, steps_per_sync=sps)
        out, tc = cm.timecourse(w, every, handle=h)
        if ref is None:
            ref = (out, tc)
            continue
        assert np.array_equal(tc, ref[1]), (rpl, sps)
        assert np.array_equal(out["hist"], ref[0]["hist"]), (rpl, sps)


def test_timecourse_rejects_bad_arguments():
    h = cm.Handle(0)
    ds = cm.DeviceSweep(h, W.ddm(trials=10, max_steps=50, n_bins=5))
    with pytest.raises(cm.CmError):
        ds.launch_timecourse(0)
    with pytest.raises(cm.CmError):
        ds.launch_timecourse(51)
    ds2 = cm.DeviceSweep(h, W.rnn(trials=16, n_units=64, max_steps=10, n_bins=5))
    with pytest.raises(cm.CmError):
        ds2.launch_timecourse(1)
