"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/avl.h, and rejects bad configurations on the host before
any device work."""
import ctypes
import math
import os
import re

import pytest

from paper_1804_03901_amd import avl, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "avl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(avl_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = avl.load()
    syms = declared_symbols()
    assert "avl_init" in syms and "avl_step" in syms and "avl_reconstruct" in syms
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(avl.EXPORTS)


def _cfg(**kw):
    w = inputs.landau_small()
    c = avl.make_config(w)
    for k, v in kw.items():
        if k in ("nv", "vmin", "vmax", "tune"):
            arr = getattr(c, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(c, k, v)
    return c


def test_workspace_bytes_valid_config():
    c = _cfg()
    n = avl.avl_workspace_bytes(c)
    # two marker buffers of 3 doubles per marker at least
    assert n >= 2 * 24 * c.n_markers


@pytest.mark.parametrize("bad", [
    dict(nx=48), dict(nx=4), dict(nx=8192), dict(vdim=2), dict(precision=7), dict(first_kick=2),
    dict(options=2), dict(options=1), dict(L=0.0), dict(L=float("nan")), dict(dt=-0.1), dict(c_p=0.0), dict(m=0.0),
    dict(nv=(1, 1, 1)), dict(vmin=(6.0, 0, 0)), dict(n_markers=-1), dict(n_markers=2 ** 31),
    dict(tune=(-1, 0, 0, 0)), dict(tune=(300, 0, 0, 0)), dict(tune=(0, 3, 0, 0)), dict(tune=(0, -1, 0, 0)),
    dict(tune=(0, 0, 65, 0)), dict(tune=(0, 0, -1, 0)), dict(tune=(0, 0, 0, 1)),
])
def test_invalid_configs_rejected_on_host(bad):
    assert avl.avl_workspace_bytes(_cfg(**bad)) == 0
    lib = avl.load()
    h = ctypes.c_void_p()
    c = _cfg(**bad)
    rc = lib.avl_init(ctypes.byref(c), ctypes.c_void_p(256), 1 << 30, None, None, None, None, ctypes.byref(h))
    assert rc in (-1, -2, -6)
    assert not h.value


def test_workspace_checks_before_device_work():
    lib = avl.load()
    c = _cfg()
    need = avl.avl_workspace_bytes(c)
    h = ctypes.c_void_p()
    assert lib.avl_init(ctypes.byref(c), None, need, None, None, None, None, ctypes.byref(h)) == -1
    assert lib.avl_init(ctypes.byref(c), ctypes.c_void_p(4096 + 8), need, None, None, None, None, ctypes.byref(h)) == -3
    assert lib.avl_init(ctypes.byref(c), ctypes.c_void_p(4096), need - 1, None, None, None, None, ctypes.byref(h)) == -2
    assert lib.avl_init(ctypes.byref(c), ctypes.c_void_p(4096), need, None, None, None, None, None) == -1


def test_null_handle_and_strerror():
    lib = avl.load()
    for name in ("avl_push", "avl_sort", "avl_check", "avl_status", "avl_destroy"):
        fn = getattr(lib, name)
        args = [None] * len(fn.argtypes)
        assert fn(*args) == -1
    assert lib.avl_step(None, 1, None) == -1
    assert avl.strerror(-4) == "call not valid in the current state"
    assert lib.avl_step_count(None) == -1


def test_three_v_config_sizes():
    """1D-3V sizes for the two-stream workload at full size stay within int32 indexing."""
    w = inputs.two_stream_3v()
    c = avl.make_config(w, precision=avl.AVL_FP32)
    n = avl.avl_workspace_bytes(c)
    assert n == 0 or n > 2 * 24 * w.n_markers


def test_three_v_rejects_kahan_option():
    """The 1D-3V reconstruction sums in FP64 only; the compensated FP32 option is refused."""
    w = inputs.two_stream_3v(nx=16, nv=8, ppc=2)
    c = avl.make_config(w, precision=avl.AVL_FP32, options=avl.AVL_OPT_KAHAN32)
    assert avl.avl_workspace_bytes(c) == 0
    lib = avl.load()
    h = ctypes.c_void_p()
    rc = lib.avl_init(ctypes.byref(c), ctypes.c_void_p(256), 1 << 30, None, None, None, None, ctypes.byref(h))
    assert rc == -6 and not h.value


def test_tuning_knobs_accepted():
    for t in [(0, 0, 0, 0), (4, 0, 0, 0), (256, 0, 0, 0), (0, 1, 0, 0), (0, 2, 0, 0), (0, 0, 1, 0), (0, 0, 64, 0),
              (8, 2, 3, 0)]:
        assert avl.avl_workspace_bytes(_cfg(tune=t)) > 0


def test_batch_workspace_and_rejections():
    ws = inputs.batched_scan(count=3, seed=5, ppc=2, nx_choices=(16, 32), nv_choices=(8, 16))
    cfgs = [avl.make_config(w, precision=avl.AVL_FP32) for w in ws]
    total = avl.avl_batch_workspace_bytes(cfgs)
    assert total >= sum(avl.avl_workspace_bytes(c) for c in cfgs)
    # precisions must agree, 1D-3V is not batched, the count must be positive
    mixed = cfgs[:2] + [avl.make_config(ws[2], precision=avl.AVL_FP64)]
    assert avl.avl_batch_workspace_bytes(mixed) == 0
    three_v = cfgs[:2] + [avl.make_config(inputs.two_stream_3v(nx=16, nv=4, ppc=1), precision=avl.AVL_FP32)]
    assert avl.avl_batch_workspace_bytes(three_v) == 0
    lib = avl.load()
    assert lib.avl_batch_workspace_bytes(None, 0) == 0
    b = ctypes.c_void_p()
    arr = avl._cfg_array(three_v)
    rc = lib.avl_batch_init(arr, 3, ctypes.c_void_p(256), 1 << 30, None, None, None, None, ctypes.byref(b))
    assert rc == -6 and not b.value
    assert lib.avl_batch_step(None, 1, None) == -1
    assert lib.avl_batch_count(None) == -1
    assert lib.avl_batch_destroy(None) == -1


def test_batched_scan_recipe():
    ws = inputs.batched_scan()
    assert len(ws) == 64
    assert {w.nx for w in ws} <= {128, 256, 512, 1024} and {w.nv[0] for w in ws} <= {128, 256, 512}
    for w in ws:
        drift, dens = w.populations[1].drift[0], w.populations[1].density
        assert 3.0 <= drift <= 6.0 and 1e-6 <= dens <= 1e-2
        assert w.ppc == 8 and w.vmin[0] == -8.0 and w.vmax[0] == 8.0
    assert 5e7 < sum(w.n_markers for w in ws) < 1.2e8


def test_adjoint_workspace_rules():
    w = inputs.bump_on_tail(nx=64, nv=64, ppc=2)
    c64 = avl.make_config(w, precision=avl.AVL_FP64)
    n1 = avl.avl_adjoint_workspace_bytes(c64, 30, 10)
    n2 = avl.avl_adjoint_workspace_bytes(c64, 30, 30)
    assert n1 > 0 and n2 > n1          # a longer segment keeps more states
    assert avl.avl_adjoint_workspace_bytes(c64, 0, 10) == 0
    assert avl.avl_adjoint_workspace_bytes(c64, 10, 0) == 0
    assert avl.avl_adjoint_workspace_bytes(avl.make_config(w, precision=avl.AVL_FP32), 30, 10) > 0
    assert avl.avl_adjoint_workspace_bytes(avl.make_config(inputs.two_stream_3v(nx=16, nv=4, ppc=1)), 30, 10) == 0
    lib = avl.load()
    assert lib.avl_adjoint(None, None, None, None, 1, 1, None, 0, None, None) == -1


def test_magnetic_field_rules():
    """A background B is accepted for 1D-3V FP64 only, with at least 2 pi steps
    per gyration (|q/m| |B| dt <= 1)."""
    w3 = inputs.two_stream_3v(nx=16, nv=4, ppc=1).replace(B=(0.0, 0.0, 0.5))
    assert avl.avl_workspace_bytes(avl.make_config(w3)) > 0
    assert avl.avl_workspace_bytes(avl.make_config(w3, precision=avl.AVL_FP32)) == 0
    assert avl.avl_workspace_bytes(avl.make_config(w3.replace(B=(0.0, 11.0, 0.0)))) == 0      # 1.1 rad a step
    assert avl.avl_workspace_bytes(avl.make_config(w3.replace(B=(0.0, float("nan"), 0.0)))) == 0
    w1 = inputs.landau_small().replace(B=(0.0, 0.0, 0.5))
    assert avl.avl_workspace_bytes(avl.make_config(w1)) == 0


def test_multi_species_workspace_rules():
    assert avl.avl_multi_workspace_bytes(2, 64) > 0
    assert avl.avl_multi_workspace_bytes(0, 64) == 0
    assert avl.avl_multi_workspace_bytes(65, 64) == 0
    assert avl.avl_multi_workspace_bytes(2, 4) == 0
    lib = avl.load()
    assert lib.avl_multi_step(None, 1, None) == -1
    assert lib.avl_multi_destroy(None) == -1
    assert lib.avl_multi_init(None, 0, None, 0, None) == -1


def test_config_fuzz_host_validation():
    """Seeded draws of every config field, extremes included (sizes up to
    2^31 - 1, zero, negative, non-finite and huge floats): the host
    validation either rejects the config or returns a workspace that holds at
    least the two marker buffers, and never reads or computes out of range
    (the sanitizer build runs this same test)."""
    import numpy as np
    rng = np.random.default_rng(2024)
    ints = [-(2 ** 31), -1, 0, 1, 2, 3, 7, 8, 16, 64, 4096, 8192, 2 ** 20, 2 ** 20 + 1, 2 ** 30, 2 ** 31 - 1]
    floats = [0.0, -1.0, 1e-300, 1e-3, 0.5, 1.0, 12.566, 1e300, float("inf"), float("-inf"), float("nan")]
    big = [-1, 0, 1, 63, 64, 2 ** 20, 2 ** 31 - 2, 2 ** 31 - 1, 2 ** 31, 2 ** 40, 2 ** 62]
    lib = avl.load()
    accepted = 0
    # the largest velocity grids the validation admits per axis, all at once
    for vd, nv, nx in [(3, 2 ** 20, 4096), (3, 2 ** 20 + 1, 4096), (3, 2 ** 20, 8), (1, 2 ** 20, 4096)]:
        for prec in (avl.AVL_FP64, avl.AVL_FP32):
            c = _cfg(vdim=vd, nv=(nv, nv, nv), nx=nx, precision=prec, n_markers=2 ** 31 - 2,
                     vmin=(-1.0, -1.0, -1.0), vmax=(1.0, 1.0, 1.0))
            assert avl.avl_workspace_bytes(c) == 0
    for i in range(3000):
        c = _cfg()
        pick = lambda xs: xs[int(rng.integers(len(xs)))]
        if rng.random() < 0.5: c.vdim = pick([-1, 0, 1, 2, 3, 3, 1])
        if rng.random() < 0.5: c.nx = pick(ints + [2 ** int(rng.integers(0, 31))])
        for d in range(3):
            if rng.random() < 0.4: c.nv[d] = pick(ints + [int(rng.integers(2, 300))])
            if rng.random() < 0.2: c.vmin[d] = pick(floats) * pick([-1, 1])
            if rng.random() < 0.2: c.vmax[d] = pick(floats)
            if rng.random() < 0.1: c.B[d] = pick(floats)
        if rng.random() < 0.3: c.precision = pick([-1, 0, 1, 2])
        if rng.random() < 0.2: c.first_kick = pick([-1, 0, 1, 2])
        if rng.random() < 0.2: c.options = pick([-1, 0, 1, 2, 3])
        if rng.random() < 0.4: c.n_markers = pick(big + [int(rng.integers(0, 2 ** 24))])
        for k in ("L", "dt", "q", "m", "c_p"):
            if rng.random() < 0.15: setattr(c, k, pick(floats) * pick([-1, 1]))
        if rng.random() < 0.2: c.tune[0] = pick([-1, 0, 1, 255, 256, 257, 2 ** 31 - 1])
        if rng.random() < 0.1: c.tune[1] = pick([-1, 0, 1, 2, 3])
        if rng.random() < 0.1: c.tune[2] = pick([-1, 0, 1, 64, 65, 2 ** 31 - 1])
        n = avl.avl_workspace_bytes(c)
        if n:
            accepted += 1
            per = (8 if c.precision == avl.AVL_FP64 else 4) * (2 + c.vdim)
            assert n >= 2 * per * max(c.n_markers, 0), (i, n)
            assert 1 <= c.vdim <= 3 and c.nx >= 8 and 0 <= c.n_markers < 2 ** 31 - 1
        h = ctypes.c_void_p()
        rc = lib.avl_init(ctypes.byref(c), ctypes.c_void_p(4096 + 8), 1 << 40, None, None, None, None,
                          ctypes.byref(h))
        assert rc < 0 and not h.value
    assert accepted > 50


def test_load_shares_torchs_hip_runtime():
    """Loading the library before anything imports torch still leaves one HIP
    runtime in the process (the one torch ships), checked in a fresh
    interpreter from its memory map."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1804_03901_amd import avl\n"
            "avl.load()\n"
            "import torch\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, check=True)
    assert out.stdout.strip().splitlines()[-1] == "1"
