"""The library's per-kernel timing (avl_timing / avl_kernel_time) on the GPU.

The count, scatter and reconstruction phases carry their HIP event pair on
their own dispatch; the scan and field phases, and the whole step, record
events around their launches.  Checked: every phase is timed once per step,
the single-kernel phases report the kernel's own (positive) duration, their
sum stays below the step's, and a step with no markers reports zero-length
kernel phases without leaving events behind for a later launch.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1804_03901_amd import avl, inputs

pytestmark = pytest.mark.gpu

PHASES = ["push_count", "scan", "scatter", "reconstruct", "field"]


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _times(sim):
    out = {}
    for k, name in enumerate(avl.KERNEL_NAMES):
        ms, cnt = avl.avl_kernel_time(sim.h, k)
        out[name] = (ms, cnt)
    return out


@pytest.mark.parametrize("precision", [avl.AVL_FP32, avl.AVL_FP64])
def test_phase_times_once_per_step(precision):
    _need_gpu()
    w = inputs.bump_on_tail(nx=256, nv=256, ppc=8, seed=21)
    x, v, f = inputs.markers(w)
    sim = avl.Simulation(w, x, v.reshape(-1), f, precision=precision)
    sim.step(2, graph=False, diag=False)
    torch.cuda.synchronize()
    steps = 6
    avl.avl_timing(sim.h, True)
    sim.step(steps, graph=False, diag=False)
    torch.cuda.synchronize()
    t = _times(sim)
    avl.avl_timing(sim.h, False)
    sim.check()
    sim.close()
    print({k: (round(ms / max(c, 1), 4), c) for k, (ms, c) in t.items()}, flush=True)
    for name in PHASES + ["step"]:
        assert t[name][1] == steps, (name, t[name])
    for name in ["push_count", "scatter", "reconstruct"]:
        assert t[name][0] > 0.0, (name, t[name])
    phase_sum = sum(t[name][0] for name in PHASES)
    assert phase_sum <= t["step"][0] * 1.02, (phase_sum, t["step"][0])


def test_empty_step_times_and_later_launches():
    _need_gpu()
    w = inputs.landau_small().replace(name="empty_timing")
    e = np.zeros(0)
    sim = avl.Simulation(w, e, e, e)
    avl.avl_timing(sim.h, True)
    sim.step(3, graph=False, diag=False)
    torch.cuda.synchronize()
    t = _times(sim)
    avl.avl_timing(sim.h, False)
    sim.check()
    sim.close()
    # no marker kernels ran: the phases that hand their events to a launch
    # record them back to back instead
    for name in ["push_count", "scatter", "reconstruct"]:
        assert t[name][1] == 3
        assert 0.0 <= t[name][0] < 0.05 * 3, (name, t[name])
    # a launch after timing is off carries no leftover events: a normal
    # simulation still steps and reports nothing timed
    w2 = inputs.landau_small()
    x, v, f = inputs.markers(w2)
    sim2 = avl.Simulation(w2, x, v.reshape(-1), f)
    sim2.step(2, graph=False, diag=False)
    torch.cuda.synchronize()
    sim2.check()
    assert all(c == 0 for _, c in _times(sim2).values())
    sim2.close()
