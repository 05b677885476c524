"""GPU parity for the recurrent rate network (matrix-core kernels).

FP64: per-run integers bit-exact on unflagged runs, final readout and unit
states within 1e-9 relative.  BF16 projection: paired with the FP64 oracle
(same random words), compared by decision agreement and histogram L1."""
import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import cm, workloads as W
from parity import assert_parity, hist_l1

pytestmark = pytest.mark.gpu


def _case(n_units, trials, seed=1, **kw):
    return W.rnn(trials=trials, seed=seed, n_units=n_units,
                 weights=W.rnn_weights(n_units, 7), **kw)


def _both(w):
    print(f"case rnn prec={w['precision']} n={w['n_units']} S={w['n_settings']} "
          f"T={w['trials']} N={w['max_steps']} seed={w['seed']}", flush=True)
    return cm.run(w, dumps=True), oracle.run(w, dumps=True, n_threads=0)


@pytest.mark.parametrize("n_units,trials", [(64, 600), (128, 300), (192, 200), (256, 250)])
def test_rnn_fp64_parity(n_units, trials):
    w = _case(n_units, trials)
    g, o = _both(w)
    assert_parity(w, g, o, [-1])
    # both choices occur and some runs hit the cap at the reference shape
    if n_units == 256:
        st = g["stats"][0]
        assert st[0] > 0 and st[1] > 0


def test_rnn_fp64_gain_grid_and_ragged():
    w = _case(128, 37, seed=3, gains=np.linspace(0.5, 1.5, 7))
    g, o = _both(w)
    assert_parity(w, g, o, [-1])


def test_rnn_fp64_short_cap_and_bins():
    w = _case(64, 500, seed=4, max_steps=17, n_bins=17)
    g, o = _both(w)
    assert_parity(w, g, o, [-1])


def test_rnn_uncoupled_noise_free():
    nu = 64
    wts = np.concatenate([np.zeros(nu * nu), W.rnn_weights(nu, 3)[nu * nu:] * 4.0])
    w = W.rnn(trials=100, seed=2, n_units=nu, noise=0.0, weights=wts, max_steps=120)
    g, o = _both(w)
    assert_parity(w, g, o, [-1])


@pytest.mark.parametrize("n_units,trials", [(64, 2000), (256, 400)])
def test_rnn_bf16_against_fp64(n_units, trials):
    w = _case(n_units, trials, seed=5)
    wb = W.with_(w, precision=W.BF16_PROJ)
    g = cm.run(wb, dumps=True)
    o64 = oracle.run(w, dumps=True)
    ob = oracle.run(wb, dumps=True)
    agree = (g["run_choice"] == o64["run_choice"]).mean()
    agree_b = (g["run_choice"] == ob["run_choice"]).mean()
    print(f"bf16 n={n_units}: choice agreement with fp64 oracle {agree:.4f}, "
          f"with bf16 oracle {agree_b:.4f}, L1 {hist_l1(g, o64, trials)[0]:.4f}")
    assert agree > 0.9 and agree_b > 0.9
    # aggregate outcome probabilities close to the fp64 oracle
    T = trials
    pg = np.array([g["stats"][0, k] for k in (0, 1, 2)]) / T
    po = np.array([o64["stats"][0, k] for k in (0, 1, 2)]) / T
    assert np.abs(pg - po).max() < 0.05


def test_rnn_full_size_sampled():
    """65,536 runs of the 256-unit network as the benchmark launches it; a
    sample of runs recomputed one by one by the oracle."""
    w = W.rnn()
    g = cm.run(w, dumps=True)
    st = g["stats"][0]
    assert st[0] + st[1] + st[2] == 65536
    rng = np.random.default_rng(0)
    for t in rng.choice(65536, 6, replace=False):
        traj, ch, fl = oracle.trajectory(w, 0, int(t))
        if fl or g["run_flag"][t]:
            continue
        assert g["run_choice"][t] == ch and g["run_step"][t] == traj.shape[0], t
        np.testing.assert_allclose(g["run_state"][t], traj[-1], rtol=1e-9, atol=1e-12)
    # the reduction agrees with the per-run dumps
    from parity import reduce_dumps
    h, s = reduce_dumps(w, g, [-1])
    assert np.array_equal(h, g["hist"]) and np.array_equal(s, g["stats"])


def test_rnn_invariant_to_dumps():
    w = _case(256, 3000, seed=9, precision=W.BF16_PROJ)
    a, b = cm.run(w), cm.run(w, dumps=True)
    assert np.array_equal(a["hist"], b["hist"]) and np.array_equal(a["stats"], b["stats"])


@pytest.mark.parametrize("prec", [W.FP64, W.BF16_PROJ])
def test_rnn_coupled_fixed_point(prec):
    """Two groups of 32 units, coupled within and across groups with
    different strengths each way, no noise, no input: every run settles at
    the fixed point of the continuous dynamics, found by root finding
    (bf16 weights move it by their rounding)."""
    from scipy.optimize import fsolve
    a, b, c_ab, c_ba = 1.0, -0.5, 0.8, -0.6
    nu, h = 64, 32
    Wm = np.zeros((nu, nu))
    Wm[:h, :h] = a / (h - 1)
    Wm[:h, h:] = c_ab / h
    Wm[h:, :h] = c_ba / h
    Wm[h:, h:] = b / (h - 1)
    np.fill_diagonal(Wm, 0.0)
    wts = np.concatenate([Wm.ravel(), np.zeros(2 * nu)])
    w = W.rnn(trials=40, seed=5, n_units=nu, dt=0.05, noise=0.0, thresh=1e300, input_gain=0.0,
              max_steps=1500, n_bins=10, weights=wts, precision=prec)
    g = cm.run(w, dumps=True)

    def s(x):
        return 1.0 / (1.0 + np.exp(-x))

    xa, xb = fsolve(lambda v: [v[0] - a * s(v[0]) - c_ab * s(v[1]),
                               v[1] - c_ba * s(v[0]) - b * s(v[1])], [0.5, -0.5], xtol=1e-14)
    tol = 1e-9 if prec == W.FP64 else 2e-2
    x = g["run_state"][:, 2:]
    assert np.abs(x[:, :h] - xa).max() < tol and np.abs(x[:, h:] - xb).max() < tol
    assert int(g["stats"][0, 2]) == 40  # undecided at the cap
