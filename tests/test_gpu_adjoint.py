"""The hand-written adjoint against finite differences.

J = sum_{n=1..N} sum_i (E_i^n)^2 dx dt for a small bump-on-tail run; the
gradient with respect to all 16 initial mode amplitudes and the beam drift
(through f_l = f0(x_l, v_l; theta), written in torch) is compared with
central differences of J computed by the GPU FP64 path, and two components
with those of the CPU oracle, within 1e-4 relative.  The gradient is the same
bit for bit for any checkpoint interval.  Each reverse stage is checked on
its own by the dot-product tests of test_gpu_adjoint_stages.py."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1804_03901_amd import adjoint, avl, inputs

pytestmark = pytest.mark.gpu

W = inputs.bump_on_tail(nx=64, nv=64, ppc=4, seed=21, steps=30)
NSTEPS = 30


def setup_case(precision=avl.AVL_FP64, w=None):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = w or W
    x, v, f = inputs.markers_threaded(w)
    dev = torch.device("cuda:0")
    xt = torch.tensor(x, device=dev)
    vt = torch.tensor(v.reshape(-1), device=dev)
    sim = avl.Simulation(w, x, v.reshape(-1), f, precision=precision)
    print(f"[case] adjoint {w.name} prec={precision}", flush=True)
    return sim, xt, vt, f


def theta0(dev):
    amps = torch.full((len(W.mode_numbers),), W.mode_amplitude, dtype=torch.float64, device=dev)
    drift = torch.tensor(W.populations[1].drift[0], dtype=torch.float64, device=dev)
    return amps, drift


def J_gpu(sim, xt, vt, amps, drift, nsteps=NSTEPS):
    with torch.no_grad():
        f = adjoint.f0_torch(sim.w, xt, vt, amps, drift)
        J, _ = adjoint.energy_and_gradient(sim, xt, vt, f, nsteps, want_grad=False)
    return float(J)


def J_oracle(x, v, amps, drift):
    f = adjoint.f0_torch(W, torch.tensor(x), torch.tensor(v), amps.cpu(), drift.cpu()).numpy()
    r = oracle.run(oracle.Grid.from_workload(W), x, v.reshape(1, -1), f, NSTEPS)
    return 2.0 * W.c_p * W.dt * float(r["diag"][:, 0].sum())


def adjoint_grad(sim, xt, vt, every=10, nsteps=NSTEPS):
    amps, drift = theta0(xt.device)
    amps.requires_grad_(True)
    drift.requires_grad_(True)
    f = adjoint.f0_torch(sim.w, xt, vt, amps, drift)
    J = adjoint.field_energy(f, sim, xt, vt, nsteps, every)
    J.backward()
    return float(J.detach()), amps.grad.detach().clone(), float(drift.grad)


def test_f0_torch_matches_the_generator():
    x, v, f = inputs.markers(W)
    ft = adjoint.f0_torch(W, torch.tensor(x), torch.tensor(v)).numpy()
    assert np.max(np.abs(ft - f)) <= 1e-15 * np.max(np.abs(f))


def test_adjoint_J_matches_a_plain_run():
    sim, xt, vt, f = setup_case()
    J, g = adjoint.energy_and_gradient(sim, xt, vt, torch.tensor(f, device=xt.device), NSTEPS, every=10)
    J0, _ = adjoint.energy_and_gradient(sim, xt, vt, torch.tensor(f, device=xt.device), NSTEPS, want_grad=False)
    assert abs(float(J) - float(J0)) <= 1e-10 * abs(float(J0))
    assert bool(torch.isfinite(g).all())


def test_all_sixteen_amplitude_gradients_match_gpu_finite_differences():
    """dJ/dA_k for every one of the 16 mode amplitudes and dJ/du_b against
    central differences of the GPU FP64 path."""
    sim, xt, vt, _ = setup_case()
    J, gA, gd = adjoint_grad(sim, xt, vt)
    amps, drift = theta0(xt.device)
    assert gA.numel() == 16
    worst = 0.0
    for k in range(16):
        h = 1e-7
        e = torch.zeros_like(amps)
        e[k] = h
        fd = (J_gpu(sim, xt, vt, amps + e, drift) - J_gpu(sim, xt, vt, amps - e, drift)) / (2 * h)
        ad = float(gA[k])
        rel = abs(ad - fd) / abs(fd)
        worst = max(worst, rel)
        print(f"A{k + 1}: adjoint {ad:.10e} fd {fd:.10e} rel {rel:.1e}", flush=True)
        assert rel <= 1e-4, (k + 1, ad, fd)
    # the beam is 1e-6 of the density, so dJ/du_b is small: a wider step
    # keeps J's rounding out of the difference (J is smooth in u_b on the
    # beam's thermal scale 0.5)
    h = 1e-3
    fd = (J_gpu(sim, xt, vt, amps, drift + h) - J_gpu(sim, xt, vt, amps, drift - h)) / (2 * h)
    print(f"drift: adjoint {gd:.10e} fd {fd:.10e}", flush=True)
    assert abs(gd - fd) <= 1e-4 * abs(fd)
    print(f"[result] worst amplitude rel {worst:.1e}", flush=True)


@pytest.mark.parametrize("which", ["A1", "drift"])
def test_gradient_matches_oracle_finite_differences(which):
    sim, xt, vt, _ = setup_case()
    J, gA, gd = adjoint_grad(sim, xt, vt)
    x, v, _ = inputs.markers(W)
    amps, drift = theta0("cpu")
    if which == "drift":
        h = 1e-3
        fd = (J_oracle(x, v, amps, drift + h) - J_oracle(x, v, amps, drift - h)) / (2 * h)
        ad = gd
    else:
        h = 1e-7
        e = torch.zeros_like(amps)
        e[0] = h
        fd = (J_oracle(x, v, amps + e, drift) - J_oracle(x, v, amps - e, drift)) / (2 * h)
        ad = float(gA[0])
    print(f"{which}: adjoint {ad:.10e} oracle fd {fd:.10e}")
    assert abs(ad - fd) <= 1e-4 * abs(fd)


def test_checkpoint_interval_does_not_change_the_gradient():
    """The forward steps are bit-reproducible and every reverse sum is order
    free, so the gradient is the same bit for bit whatever the checkpoint
    interval, and from one run to the next."""
    sim, xt, vt, f = setup_case()
    ft = torch.tensor(f, device=xt.device)
    grads = [adjoint.energy_and_gradient(sim, xt, vt, ft, NSTEPS, every=e)[1] for e in (1, 7, 30, 7)]
    for g in grads[1:]:
        assert torch.equal(g, grads[0])


def test_fp32_form_gradient_bit_reproducible():
    sim, xt, vt, f = setup_case(avl.AVL_FP32)
    ft = torch.tensor(f, device=xt.device)
    a = adjoint.energy_and_gradient(sim, xt, vt, ft, NSTEPS, every=10)
    b = adjoint.energy_and_gradient(sim, xt, vt, ft, NSTEPS, every=3)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_weight_gradient_directional_derivative():
    sim, xt, vt, f = setup_case()
    ft = torch.tensor(f, device=xt.device)
    _, g = adjoint.energy_and_gradient(sim, xt, vt, ft, NSTEPS, every=10)
    rng = np.random.default_rng(3)
    d = torch.tensor(rng.normal(size=f.size) * f, device=xt.device)
    h = 1e-6
    Jp, _ = adjoint.energy_and_gradient(sim, xt, vt, ft + h * d, NSTEPS, want_grad=False)
    Jm, _ = adjoint.energy_and_gradient(sim, xt, vt, ft - h * d, NSTEPS, want_grad=False)
    fd = (float(Jp) - float(Jm)) / (2 * h)
    ad = float((g * d).sum())
    print(f"directional: adjoint {ad:.10e} fd {fd:.10e}")
    assert abs(ad - fd) <= 1e-4 * abs(fd)


def test_fp32_form_gradient_matches_fp64_finite_differences():
    """The adjoint of the FP32-form run against central differences of the
    FP64 path (the two runs agree to the FP32 form's accuracy)."""
    sim32, xt, vt, f = setup_case(avl.AVL_FP32)
    _, gA, gd = adjoint_grad(sim32, xt, vt)
    sim64, _, _, _ = setup_case(avl.AVL_FP64)
    amps, drift = theta0(xt.device)
    e = torch.zeros_like(amps)
    e[0] = 1e-7
    fdA = (J_gpu(sim64, xt, vt, amps + e, drift) - J_gpu(sim64, xt, vt, amps - e, drift)) / 2e-7
    fdd = (J_gpu(sim64, xt, vt, amps, drift + 1e-3) - J_gpu(sim64, xt, vt, amps, drift - 1e-3)) / 2e-3
    print(f"fp32 adjoint A1 {float(gA[0]):.10e} fd64 {fdA:.10e}; drift {gd:.10e} fd64 {fdd:.10e}")
    assert abs(float(gA[0]) - fdA) <= 1e-4 * abs(fdA)
    assert abs(gd - fdd) <= 1e-4 * abs(fdd)


@pytest.mark.slow
def test_adjoint_at_full_size():
    """The adjoint configuration at full size: bump-on-tail nx = 1024, nv = 512,
    8 markers per cell (4,194,304 markers), 500 steps, FP32 forward with a
    checkpoint every 50 steps; two gradient components against central
    differences of the FP64 path."""
    w = inputs.adjoint_case()
    sim32, xt, vt, f = setup_case(avl.AVL_FP32, w)
    _, gA, gd = adjoint_grad(sim32, xt, vt, every=50, nsteps=w.steps)
    sim32.close()
    sim64 = avl.Simulation(w, xt, vt, torch.tensor(f, device=xt.device), precision=avl.AVL_FP64)
    amps, drift = theta0(xt.device)
    e = torch.zeros_like(amps)
    e[0] = 1e-7
    fdA = (J_gpu(sim64, xt, vt, amps + e, drift, w.steps) - J_gpu(sim64, xt, vt, amps - e, drift, w.steps)) / 2e-7
    fdd = (J_gpu(sim64, xt, vt, amps, drift + 1e-3, w.steps) - J_gpu(sim64, xt, vt, amps, drift - 1e-3, w.steps)) / 2e-3
    print(f"full size: A1 adjoint {float(gA[0]):.10e} fd64 {fdA:.10e}; drift {gd:.10e} fd64 {fdd:.10e}")
    assert abs(float(gA[0]) - fdA) <= 1e-4 * abs(fdA)
    assert abs(gd - fdd) <= 1e-4 * abs(fdd)


@pytest.mark.parametrize("precision", [avl.AVL_FP64, avl.AVL_FP32])
def test_gradient_with_markers_outside_the_velocity_grid(precision):
    """A fifth of the markers beyond the velocity grid (the overflow run; in
    the FP32 form the recorded states keep their stored cell indices): the
    weight gradient's directional derivative against central differences of
    the FP64 path.  Those markers reach no grid cell, so their gradient is
    zero, and the others' is unchanged in kind."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    x, v, f = inputs.markers_threaded(W)
    v = v.copy()
    dv = W.dv(0)
    rng = np.random.default_rng(17)
    out = rng.random(x.size) < 0.2
    up = rng.random(x.size) < 0.5
    spread = 2.0 + 6.0 * rng.random(x.size)
    v[0] = np.where(out & up, W.vmax[0] + spread * dv, np.where(out, W.vmin[0] - spread * dv, v[0]))
    dev = torch.device("cuda:0")
    xt = torch.tensor(x, device=dev)
    vt = torch.tensor(v.reshape(-1), device=dev)
    ft = torch.tensor(f, device=dev)
    print(f"[case] adjoint outside-grid prec={precision} n={x.size} out={int(out.sum())}", flush=True)
    sim = avl.Simulation(W, x, v.reshape(-1), f, precision=precision)
    _, g = adjoint.energy_and_gradient(sim, xt, vt, ft, NSTEPS, every=10)
    sim64 = sim if precision == avl.AVL_FP64 else avl.Simulation(W, x, v.reshape(-1), f, precision=avl.AVL_FP64)
    d = torch.tensor(rng.normal(size=f.size) * f, device=dev)
    h = 1e-6
    Jp, _ = adjoint.energy_and_gradient(sim64, xt, vt, ft + h * d, NSTEPS, want_grad=False)
    Jm, _ = adjoint.energy_and_gradient(sim64, xt, vt, ft - h * d, NSTEPS, want_grad=False)
    fd = (float(Jp) - float(Jm)) / (2 * h)
    ad = float((g * d).sum())
    print(f"[result] outside-grid prec={precision}: adjoint {ad:.10e} fd64 {fd:.10e}", flush=True)
    assert abs(ad - fd) <= 1e-4 * abs(fd)
    assert float(g[torch.tensor(out, device=dev)].abs().max()) == 0.0
    sim.check()
