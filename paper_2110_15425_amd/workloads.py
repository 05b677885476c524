"""Seeded synthetic workloads: the inputs of a sweep and nothing else.

This module builds the arrays a sweep is made of -- parameter vectors,
weight matrices drawn from numpy's PCG64, control grids -- as plain dicts.
It holds none of the simulation's arithmetic, imports neither the HIP
library nor the oracle, and is the one module both of them are fed from.

The paper's models (PsyNeuLink scripts, trained weights) are not available;
these synthetic models stand in for them with the shapes of its workloads:
a single drift-diffusion decision (the DDM nodes of the extended Stroop
models), a two-pathway conflict network feeding a leaky competing
accumulator (Stroop/multitasking), a control grid search over two signals
(the Control node's allocation search), the same network under closed-loop
control re-optimised before every step (the control loop of the
predator-prey model), and a recurrent logistic rate network (a scaled
analogue of the Necker-cube networks).
"""
import numpy as np

DDM, LCA, RNN, LOOP = 0, 1, 2, 3
FP64, FP32_STEP, BF16_PROJ = 0, 1, 2

# parameter slots, one enum per kind (string keys become fixed offsets)
DDM_P = dict(dt=0, drift=1, noise=2, thresh=3, start=4, t0=5)
LCA_P = dict(dt=0, leak=1, comp=2, noise=3, thresh=4, offset=5, hid_gain=6, hid_bias=7,
             nonneg=8, t0=9)
RNN_P = dict(dt=0, noise=1, thresh=2, input_gain=3, t0=4)
LOOP_P = dict(LCA_P, levels=10, amax=11, samples=12, cost=13)

KIND_NAMES = {DDM: "ddm", LCA: "conflict_lca", RNN: "rate_rnn", LOOP: "conflict_loop"}
PREC_NAMES = {FP64: "fp64", FP32_STEP: "fp32_step", BF16_PROJ: "bf16_proj"}


def _params(table, **values):
    p = np.zeros(len(table), np.float64)
    for k, v in values.items():
        p[table[k]] = v
    return p


def _base(kind, precision, params, weights, n_units, n_stimuli, grid, trials, seed,
          max_steps, n_bins, reward=0.0, cost=0.0, flag_eps=1e-10):
    grid = None if grid is None else np.ascontiguousarray(grid, np.float64)
    n_signals = 0 if grid is None else grid.shape[1]
    n_settings = 1 if grid is None else grid.shape[0]
    return dict(kind=kind, precision=precision, params=params, weights=weights,
                n_units=n_units, n_stimuli=n_stimuli, n_signals=n_signals, grid=grid,
                n_settings=n_settings, trials=int(trials), seed=int(seed),
                max_steps=int(max_steps), n_bins=int(n_bins), reward=float(reward),
                cost=float(cost), flag_eps=float(flag_eps))


def ddm(trials=10_000, seed=1, drift=0.3, noise=1.0, thresh=1.0, start=0.0, dt=0.01, t0=0.2,
        max_steps=3000, n_bins=100, drifts=None, precision=FP64, **kw):
    """Single drift-diffusion model.  ``drifts`` (optional) gives one
    setting per drift value."""
    p = _params(DDM_P, dt=dt, drift=drift, noise=noise, thresh=thresh, start=start, t0=t0)
    grid = None if drifts is None else np.asarray(drifts, np.float64).reshape(-1, 1)
    return _base(DDM, precision, p, None, 1, 1, grid, trials, seed, max_steps, n_bins, **kw)


def conflict_weights(weights_seed=11):
    """W_A, W_B [4x3] and O_A, O_B [2x4], all U(-2, 2), drawn in that order."""
    g = np.random.Generator(np.random.PCG64(weights_seed))
    WA = g.uniform(-2.0, 2.0, (4, 3))
    WB = g.uniform(-2.0, 2.0, (4, 3))
    OA = g.uniform(-2.0, 2.0, (2, 4))
    OB = g.uniform(-2.0, 2.0, (2, 4))
    return np.concatenate([WA.ravel(), WB.ravel(), OA.ravel(), OB.ravel()])


def control_levels(n=64, hi=5.0):
    """n evenly spaced control levels over [0, hi], end points included."""
    return np.array([hi * i / (n - 1) for i in range(n)], np.float64)


def conflict(trials=10_000, seed=1, weights_seed=11, grid=None, leak=0.5, comp=1.0, noise=0.1,
             thresh=0.8, dt=0.1, max_steps=1000, n_bins=100, hid_gain=1.0, hid_bias=-4.0,
             offset=0.0, nonneg=0.0, t0=0.0, precision=FP64, weights=None, **kw):
    """Two-pathway conflict network driving a 2-unit LCA.  ``grid`` is
    [settings x 2] control signals (c_A, c_B); default: 64 levels of c_A
    with c_B = 1."""
    p = _params(LCA_P, dt=dt, leak=leak, comp=comp, noise=noise, thresh=thresh, offset=offset,
                hid_gain=hid_gain, hid_bias=hid_bias, nonneg=nonneg, t0=t0)
    if grid is None:
        lv = control_levels()
        grid = np.stack([lv, np.ones_like(lv)], 1)
    w = conflict_weights(weights_seed) if weights is None else np.asarray(weights, np.float64)
    return _base(LCA, precision, p, w, 2, 9, grid, trials, seed, max_steps, n_bins, **kw)


def control_grid(n=64, hi=5.0):
    """Exhaustive allocation grid over two signals: setting 64*i + j is
    (level_i, level_j)."""
    lv = control_levels(n, hi)
    a, b = np.meshgrid(lv, lv, indexing="ij")
    return np.stack([a.ravel(), b.ravel()], 1)


def grid_search(trials=100, seed=1, weights_seed=11, n=64, reward=1.0, cost=0.1, **kw):
    return conflict(trials=trials, seed=seed, weights_seed=weights_seed, grid=control_grid(n),
                    reward=reward, cost=cost, **kw)


def rnn_weights(n_units=256, weights_seed=7):
    """Recurrent W [n x n] ~ N(0, 1/n) and readout R [2 x n] ~ N(0, 1/n)."""
    g = np.random.Generator(np.random.PCG64(weights_seed))
    sd = 1.0 / np.sqrt(n_units)
    W = g.normal(0.0, sd, (n_units, n_units))
    R = g.normal(0.0, sd, (2, n_units))
    return np.concatenate([W.ravel(), R.ravel()])


def rnn(trials=65_536, seed=1, weights_seed=7, n_units=256, dt=0.05, noise=0.05, thresh=1.0,
        input_gain=1.0, max_steps=200, n_bins=100, gains=None, precision=FP64, weights=None,
        t0=0.0, **kw):
    p = _params(RNN_P, dt=dt, noise=noise, thresh=thresh, input_gain=input_gain, t0=t0)
    w = rnn_weights(n_units, weights_seed) if weights is None else np.asarray(weights, np.float64)
    grid = None if gains is None else np.asarray(gains, np.float64).reshape(-1, 1)
    return _base(RNN, precision, p, w, n_units, 1, grid, trials, seed, max_steps, n_bins, **kw)


def control_loop(trials=1000, seed=1, weights_seed=11, levels=8, amax=5.0, samples=4, cost=0.01,
                 costs=None, leak=0.5, comp=1.0, noise=0.1, thresh=0.8, dt=0.1, max_steps=1000,
                 n_bins=100, hid_gain=1.0, hid_bias=-4.0, offset=0.0, nonneg=0.0, t0=0.0,
                 precision=FP64, weights=None, **kw):
    """Closed-loop control of the conflict network: before every step each run
    searches the levels x levels grid of control allocations (c_A, c_B) in
    [0, amax]^2 with ``samples`` look-ahead draws per allocation.  ``costs``
    (optional) gives one setting per control-cost weight."""
    p = _params(LOOP_P, dt=dt, leak=leak, comp=comp, noise=noise, thresh=thresh, offset=offset,
                hid_gain=hid_gain, hid_bias=hid_bias, nonneg=nonneg, t0=t0, levels=levels,
                amax=amax, samples=samples, cost=cost)
    w = conflict_weights(weights_seed) if weights is None else np.asarray(weights, np.float64)
    grid = None if costs is None else np.asarray(costs, np.float64).reshape(-1, 1)
    return _base(LOOP, precision, p, w, 2, 9, grid, trials, seed, max_steps, n_bins, **kw)


def with_(w, **changes):
    """Copy of a workload with some fields replaced."""
    out = dict(w)
    out.update(changes)
    if "grid" in changes:
        g = out["grid"]
        out["n_signals"] = 0 if g is None else g.shape[1]
        out["n_settings"] = 1 if g is None else g.shape[0]
    return out
