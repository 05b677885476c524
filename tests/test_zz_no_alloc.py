"""cm_launch_scratch, the entry point that allocates nothing: the same kernels
as cm_launch with the library's static per-device scratch array as the
workspace.  Each case makes two calls in a row, the second on a smaller
sweep (the array then still holds the first call's tables), and compares
every output, per-run dumps included, with cm_launch on the same inputs."""
import numpy as np
import pytest

from paper_2110_15425_amd import cm, workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("hist", "stats", "score", "best", "run_choice", "run_step", "run_flag", "run_state")


def _pair(h, w):
    ref = cm.DeviceSweep(h, w, dumps=True)
    ref.launch()
    want = ref.results()
    scr = cm.DeviceSweep(h, w, dumps=True)
    scr.launch_scratch()
    got = scr.results()
    return want, got


def _same(want, got, what):
    for k in KEYS:
        if want.get(k) is None:
            assert got.get(k) is None, (what, k)
            continue
        assert want[k].shape == got[k].shape, (what, k)
        assert np.array_equal(want[k], got[k]), (what, k)


CASES = {
    # conflict network on a control grid, scored: the drive table lives in scratch
    "grid_search_fp64": (W.grid_search(n=32, trials=150, seed=3),
                         W.grid_search(n=6, trials=40, seed=4)),
    "grid_search_fp32": (W.grid_search(n=24, trials=100, seed=5, precision=W.FP32_STEP),
                         W.grid_search(n=5, trials=33, seed=6, precision=W.FP32_STEP)),
    # rate network: W's matrix-core fragments live in scratch
    "rnn_bf16": (W.rnn(trials=300, n_units=256, precision=W.BF16_PROJ, max_steps=120, seed=7),
                 W.rnn(trials=70, n_units=64, precision=W.BF16_PROJ, max_steps=90, n_bins=45, seed=8)),
    "rnn_fp64": (W.rnn(trials=200, n_units=256, max_steps=100, seed=9),
                 W.rnn(trials=50, n_units=128, max_steps=80, n_bins=40, seed=10)),
    # closed loop: the allocation drive and norm tables live in scratch
    "loop_fp64": (W.control_loop(trials=120, levels=8, samples=2, max_steps=300, seed=11),
                  W.control_loop(trials=40, levels=3, samples=1, max_steps=200, seed=12)),
    # drift-diffusion: only the correct-response table
    "ddm_fp64": (W.ddm(trials=3000, drifts=np.linspace(0.0, 0.6, 4), seed=13),
                 W.ddm(trials=500, seed=14, max_steps=700, n_bins=70)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_scratch_launch_equals_launch(name):
    h = cm.Handle(0)
    big, small = CASES[name]
    assert cm.workspace_bytes(big) >= cm.workspace_bytes(small)
    for i, w in enumerate((big, small)):
        print(f"{name}: call {i + 1}, {w['n_settings']} settings x {w['trials']} trials", flush=True)
        want, got = _pair(h, w)
        _same(want, got, (name, i))


def test_scratch_launch_rejects_oversize_sweep():
    """A sweep whose tables exceed the array is refused before any launch."""
    h = cm.Handle(0)
    w = W.grid_search(n=171, trials=1)  # 29,241 settings: 4.2 MB of drive table
    assert cm.workspace_bytes(w) > 4 << 20
    d = cm.DeviceSweep(h, w)
    with pytest.raises(cm.CmError) as e:
        d.launch_scratch()
    assert e.value.status == cm.E_BUDGET
    assert "scratch" in str(e.value)
    # the largest grid that fits still runs and matches cm_launch
    w = W.conflict(trials=3, grid=np.tile(W.control_grid(8), (456, 1))[:29_125])
    assert cm.workspace_bytes(w) <= 4 << 20
    want, got = _pair(h, w)
    _same(want, got, "largest grid")
