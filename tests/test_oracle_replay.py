"""High-precision replay: a few runs recomputed at 50 significant digits
from the same Philox words.  This checks the oracle's FP64 rounding (state
within 1e-12 relative, same decision step unless flagged); the dynamics are
pinned by the distributional tests."""
import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_2110_15425_amd import workloads as W

mp.mp.dps = 50


def _normals(words):
    ma = ((int(words[1]) << 32) | int(words[0])) >> 11
    mb = ((int(words[3]) << 32) | int(words[2])) >> 11
    ua = mp.mpf(ma + 1) / mp.mpf(2) ** 53
    ub = mp.mpf(mb + 1) / mp.mpf(2) ** 53
    rho = mp.sqrt(-2 * mp.log(ua))
    phi = mp.mpf(6.283185307179586) * ub
    return rho * mp.cos(phi), rho * mp.sin(phi)


def _key(w):
    return [w["seed"] & 0xFFFFFFFF, w["seed"] >> 32]


@pytest.mark.parametrize("trial", range(6))
def test_ddm_replay(trial):
    w = W.ddm(trials=6, seed=17)
    traj, ch, fl = oracle.trajectory(w, 0, trial)
    a = mp.mpf(0.3 * 0.01)
    b = mp.mpf(1.0) * mp.sqrt(mp.mpf(0.01))
    x = mp.mpf(0)
    for n in range(1, traj.shape[0] + 1):
        z = _normals(oracle.philox([(n - 1) >> 1, trial, 0, 0], _key(w)))[(n - 1) & 1]
        x = x + a + b * z
        assert abs(float(x) - traj[n - 1, 0]) <= 1e-12 * max(1.0, abs(float(x)))
    if not fl:
        assert (x >= 1) if ch == 1 else (x <= -1)


@pytest.mark.parametrize("trial", range(9))
def test_lca_replay(trial):
    w = W.conflict(trials=9, seed=19, grid=np.array([[0.7, 1.0]]))
    traj, ch, fl = oracle.trajectory(w, 0, trial)
    drive = oracle.conflict_drive(w["weights"], 1.0, -4.0, 0.0, 0.7, 1.0)[trial % 9]
    I = [mp.mpf(drive[0]), mp.mpf(drive[1])]
    dt, leak, comp = mp.mpf(0.1), mp.mpf(0.5), mp.mpf(1.0)
    b = mp.mpf(0.1) * mp.sqrt(dt)
    x = [mp.mpf(0), mp.mpf(0)]
    for n in range(1, traj.shape[0] + 1):
        z = _normals(oracle.philox([n - 1, trial, 0, 0], _key(w)))
        x = [x[0] + (I[0] - leak * x[0] - comp * x[1]) * dt + b * z[0],
             x[1] + (I[1] - leak * x[1] - comp * x[0]) * dt + b * z[1]]
        for i in range(2):
            assert abs(float(x[i]) - traj[n - 1, i]) <= 1e-12 * max(1.0, abs(float(x[i])))
    if not fl and ch >= 0:
        assert max(x) >= mp.mpf(0.8) and (x[1] > x[0]) == (ch == 1)
