"""Python binding of libavl: argument marshalling only.

Every entry point of ``include/avl.h`` is exposed under the same name and takes
torch tensors (device memory) or plain numbers; the work runs in the HIP
kernels of ``libavl.so``.  PyTorch provides device memory and the stream.  If
the library has not been built, loading fails loudly: there is no fallback.

``Simulation`` bundles one handle with its torch-owned workspace.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

from . import inputs

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libavl.so")

AVL_FP64 = 0
AVL_FP32 = 1
AVL_OPT_KAHAN32 = 1
K_PUSH_COUNT, K_SCAN, K_SCATTER, K_RECONSTRUCT, K_FIELD, K_STEP = range(6)
KERNEL_NAMES = ["push_count", "scan", "scatter", "reconstruct", "field", "step"]

STATUS = {0: "AVL_OK", -1: "AVL_EINVAL", -2: "AVL_ESIZE", -3: "AVL_EALIGN", -4: "AVL_ESTATE",
          -5: "AVL_EDEVICE", -6: "AVL_ENOTSUP", -7: "AVL_ENONFINITE", -8: "AVL_EINTERNAL"}


class AvlError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({strerror(status)})")


class AvlConfig(ctypes.Structure):
    _fields_ = [
        ("vdim", ctypes.c_int32), ("nx", ctypes.c_int32), ("nv", ctypes.c_int32 * 3),
        ("precision", ctypes.c_int32), ("first_kick", ctypes.c_int32), ("options", ctypes.c_int32),
        ("n_markers", ctypes.c_int64), ("L", ctypes.c_double),
        ("vmin", ctypes.c_double * 3), ("vmax", ctypes.c_double * 3),
        ("dt", ctypes.c_double), ("q", ctypes.c_double), ("m", ctypes.c_double), ("c_p", ctypes.c_double),
        ("tune", ctypes.c_int32 * 4),
        ("B", ctypes.c_double * 3),
    ]


# avl_config.tune slots (0 leaves the library's choice)
TUNE_RECON_ROWS = 0       # target velocity rows per 1D-1V reconstruction task, 1..256
TUNE_RECON_FORM = 1       # FP32 1D-1V reconstruction rows: 1 dense, 2 sparse
TUNE_SORT_BLOCKS = 2      # resident blocks per compute unit of the FP32 1D-1V tiled sort passes, 1..64


_lib = None

EXPORTS = ["avl_workspace_bytes", "avl_init", "avl_push", "avl_sort", "avl_reconstruct", "avl_moments",
           "avl_poisson", "avl_step", "avl_step_graph", "avl_get_markers", "avl_set_markers", "avl_get_field",
           "avl_step_count", "avl_check", "avl_status", "avl_set_stream", "avl_timing", "avl_kernel_time", "avl_kernel_bytes",
           "avl_copy_probe", "avl_strerror", "avl_destroy", "avl_batch_workspace_bytes", "avl_batch_init",
           "avl_batch_step", "avl_batch_instance", "avl_batch_count", "avl_batch_check", "avl_batch_destroy",
           "avl_adjoint_workspace_bytes", "avl_adjoint", "avl_diagnostics", "avl_multi_workspace_bytes",
           "avl_multi_init", "avl_multi_step", "avl_multi_destroy", "avl_reconstruct_noalloc",
           "avl_adjoint_deposit", "avl_adjoint_push", "avl_adjoint_field"]

# size of the static scratch array avl_reconstruct_noalloc uses per GPU
NOALLOC_SCRATCH_BYTES = 64 << 20

# avl_diagnostics output slots
DIAG_NAMES = ("Ee", "Ekin", "Etot", "N", "S", "P")


def load(path: str = LIB_PATH):
    """Load libavl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libavl is not built ({path} missing): run paper_1804_03901_amd/build.py")
    # torch first: the library then binds to the HIP runtime torch has loaded.
    # Opened first, it would load the system runtime beside torch's, and
    # pointers and streams from one runtime are invalid in the other.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, c = ctypes.c_void_p, ctypes
    P = ctypes.POINTER
    lib.avl_workspace_bytes.argtypes = [P(AvlConfig)]
    lib.avl_workspace_bytes.restype = c.c_size_t
    lib.avl_init.argtypes = [P(AvlConfig), vp, c.c_size_t, vp, vp, vp, vp, P(vp)]
    lib.avl_push.argtypes = [vp, vp]
    lib.avl_sort.argtypes = [vp]
    lib.avl_reconstruct.argtypes = [vp, vp, vp]
    lib.avl_moments.argtypes = [vp, vp]
    lib.avl_poisson.argtypes = [vp, vp, vp, vp]
    lib.avl_step.argtypes = [vp, c.c_int32, vp]
    lib.avl_step_graph.argtypes = [vp, c.c_int32, vp]
    lib.avl_get_markers.argtypes = [vp, vp, vp, vp]
    lib.avl_set_markers.argtypes = [vp, vp, vp, vp]
    lib.avl_get_field.argtypes = [vp, vp, vp]
    lib.avl_diagnostics.argtypes = [vp, vp, vp, vp]
    lib.avl_multi_workspace_bytes.argtypes = [c.c_int32, c.c_int32]
    lib.avl_multi_workspace_bytes.restype = c.c_size_t
    lib.avl_multi_init.argtypes = [P(vp), c.c_int32, vp, c.c_size_t, P(vp)]
    lib.avl_multi_step.argtypes = [vp, c.c_int32, vp]
    lib.avl_multi_destroy.argtypes = [vp]
    lib.avl_step_count.argtypes = [vp]
    lib.avl_step_count.restype = c.c_int64
    lib.avl_check.argtypes = [vp]
    lib.avl_status.argtypes = [vp]
    lib.avl_set_stream.argtypes = [vp, vp]
    lib.avl_timing.argtypes = [vp, c.c_int]
    lib.avl_kernel_time.argtypes = [vp, c.c_int, P(c.c_double), P(c.c_int64)]
    lib.avl_kernel_bytes.argtypes = [vp, c.c_int]
    lib.avl_kernel_bytes.restype = c.c_double
    lib.avl_copy_probe.argtypes = [vp, vp, c.c_size_t, vp]
    lib.avl_strerror.argtypes = [c.c_int]
    lib.avl_strerror.restype = c.c_char_p
    lib.avl_destroy.argtypes = [vp]
    lib.avl_batch_workspace_bytes.argtypes = [P(AvlConfig), c.c_int32]
    lib.avl_batch_workspace_bytes.restype = c.c_size_t
    lib.avl_batch_init.argtypes = [P(AvlConfig), c.c_int32, vp, c.c_size_t, vp, vp, vp, vp, P(vp)]
    lib.avl_batch_step.argtypes = [vp, c.c_int32, vp]
    lib.avl_batch_instance.argtypes = [vp, c.c_int32]
    lib.avl_batch_instance.restype = vp
    lib.avl_batch_count.argtypes = [vp]
    lib.avl_batch_check.argtypes = [vp]
    lib.avl_batch_destroy.argtypes = [vp]
    lib.avl_adjoint_workspace_bytes.argtypes = [P(AvlConfig), c.c_int32, c.c_int32]
    lib.avl_adjoint_workspace_bytes.restype = c.c_size_t
    lib.avl_adjoint.argtypes = [vp, vp, vp, vp, c.c_int32, c.c_int32, vp, c.c_size_t, vp, vp]
    lib.avl_adjoint_deposit.argtypes = [vp] * 10
    lib.avl_adjoint_push.argtypes = [vp, vp, vp, c.c_double, vp, vp, vp, vp, vp]
    lib.avl_adjoint_field.argtypes = [vp, vp, vp]
    lib.avl_reconstruct_noalloc.argtypes = [P(AvlConfig), vp, vp, vp, vp, vp, vp]
    for name in EXPORTS:
        if name not in ("avl_workspace_bytes", "avl_step_count", "avl_kernel_bytes", "avl_strerror",
                        "avl_batch_workspace_bytes", "avl_batch_instance", "avl_adjoint_workspace_bytes",
                        "avl_multi_workspace_bytes"):
            getattr(lib, name).restype = c.c_int
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().avl_strerror(int(status)).decode()


def _ck(rc: int, where: str) -> int:
    if rc != 0:
        raise AvlError(rc, where)
    return rc


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def make_config(w: "inputs.Workload", precision: int = AVL_FP64, n_markers: Optional[int] = None,
                options: int = 0, tune: Optional[dict] = None) -> AvlConfig:
    c = AvlConfig()
    c.vdim = w.vdim
    c.nx = w.nx
    for d in range(3):
        c.nv[d] = w.nv[d] if d < w.vdim else 1
        c.vmin[d] = w.vmin[d] if d < w.vdim else 0.0
        c.vmax[d] = w.vmax[d] if d < w.vdim else 1.0
    c.precision = precision
    c.first_kick = w.first_kick
    c.options = options
    c.n_markers = w.n_markers if n_markers is None else n_markers
    c.L = w.L
    c.dt, c.q, c.m, c.c_p = w.dt, w.q, w.m, w.c_p
    for d in range(3):
        c.B[d] = w.B[d]
    for slot, value in (tune or {}).items():
        c.tune[slot] = int(value)
    return c


# ---------------------------------------------------------------------------
# Entry points under their C names (tensors in, status checked).
# ---------------------------------------------------------------------------

def avl_workspace_bytes(cfg: AvlConfig) -> int:
    return int(load().avl_workspace_bytes(ctypes.byref(cfg)))


def avl_init(cfg: AvlConfig, workspace, stream, x, v, f) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _ck(load().avl_init(ctypes.byref(cfg), _ptr(workspace), workspace.numel() * workspace.element_size(),
                        _stream_ptr(stream), _ptr(x), _ptr(v), _ptr(f), ctypes.byref(h)), "avl_init")
    return h


def avl_push(h, E=None):
    return _ck(load().avl_push(h, _ptr(E)), "avl_push")


def avl_sort(h):
    return _ck(load().avl_sort(h), "avl_sort")


def avl_reconstruct(h, f_out=None, D_out=None):
    return _ck(load().avl_reconstruct(h, _ptr(f_out), _ptr(D_out)), "avl_reconstruct")


def avl_reconstruct_noalloc(cfg: AvlConfig, stream, x, v, f, f_out, D_out=None):
    return _ck(load().avl_reconstruct_noalloc(ctypes.byref(cfg), _stream_ptr(stream), _ptr(x), _ptr(v), _ptr(f),
                                              _ptr(f_out), _ptr(D_out)), "avl_reconstruct_noalloc")


def avl_moments(h, rho_out=None):
    return _ck(load().avl_moments(h, _ptr(rho_out)), "avl_moments")


def avl_poisson(h, rho=None, E_out=None, W_out=None):
    return _ck(load().avl_poisson(h, _ptr(rho), _ptr(E_out), _ptr(W_out)), "avl_poisson")


def avl_step(h, nsteps: int, diag_out=None):
    return _ck(load().avl_step(h, int(nsteps), _ptr(diag_out)), "avl_step")


def avl_step_graph(h, nsteps: int, diag_out=None):
    return _ck(load().avl_step_graph(h, int(nsteps), _ptr(diag_out)), "avl_step_graph")


def avl_get_markers(h, x, v, f):
    return _ck(load().avl_get_markers(h, _ptr(x), _ptr(v), _ptr(f)), "avl_get_markers")


def avl_set_markers(h, x, v, f):
    return _ck(load().avl_set_markers(h, _ptr(x), _ptr(v), _ptr(f)), "avl_set_markers")


def avl_get_field(h, E_out=None, rho_out=None):
    return _ck(load().avl_get_field(h, _ptr(E_out), _ptr(rho_out)), "avl_get_field")


def avl_diagnostics(h, out, j_out=None, drho_out=None):
    return _ck(load().avl_diagnostics(h, _ptr(out), _ptr(j_out), _ptr(drho_out)), "avl_diagnostics")


def avl_multi_workspace_bytes(nspecies: int, nx: int) -> int:
    return int(load().avl_multi_workspace_bytes(int(nspecies), int(nx)))


def avl_multi_init(handles, workspace) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])
    m = ctypes.c_void_p()
    _ck(load().avl_multi_init(arr, len(handles), _ptr(workspace), workspace.numel() * workspace.element_size(),
                              ctypes.byref(m)), "avl_multi_init")
    return m


def avl_multi_step(m, nsteps: int, diag_out=None):
    return _ck(load().avl_multi_step(m, int(nsteps), _ptr(diag_out)), "avl_multi_step")


def avl_multi_destroy(m):
    return _ck(load().avl_multi_destroy(m), "avl_multi_destroy")


def avl_step_count(h) -> int:
    return int(load().avl_step_count(h))


def avl_check(h) -> int:
    return int(load().avl_check(h))


def avl_status(h) -> int:
    return int(load().avl_status(h))


def avl_set_stream(h, stream):
    return _ck(load().avl_set_stream(h, _stream_ptr(stream)), "avl_set_stream")


def avl_timing(h, enable: bool):
    return _ck(load().avl_timing(h, int(bool(enable))), "avl_timing")


def avl_kernel_time(h, kernel: int):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _ck(load().avl_kernel_time(h, int(kernel), ctypes.byref(ms), ctypes.byref(cnt)), "avl_kernel_time")
    return ms.value, cnt.value


def avl_kernel_bytes(h, kernel: int) -> float:
    return float(load().avl_kernel_bytes(h, int(kernel)))


def avl_copy_probe(dst, src, nbytes: int, stream=None):
    return _ck(load().avl_copy_probe(_ptr(dst), _ptr(src), int(nbytes), _stream_ptr(stream)), "avl_copy_probe")


def avl_destroy(h):
    return _ck(load().avl_destroy(h), "avl_destroy")


def avl_adjoint_workspace_bytes(cfg: AvlConfig, nsteps: int, every: int) -> int:
    return int(load().avl_adjoint_workspace_bytes(ctypes.byref(cfg), int(nsteps), int(every)))


def avl_adjoint(h, x, v, f, nsteps: int, every: int, rec, J_out, grad_f):
    return _ck(load().avl_adjoint(h, _ptr(x), _ptr(v), _ptr(f), int(nsteps), int(every), _ptr(rec),
                                  rec.numel() * rec.element_size(), _ptr(J_out), _ptr(grad_f)), "avl_adjoint")


def avl_adjoint_deposit(h, x, v, f, f_grid, D_grid, rho_bar, f_bar, lam_x=None, lam_v=None):
    return _ck(load().avl_adjoint_deposit(h, _ptr(x), _ptr(v), _ptr(f), _ptr(f_grid), _ptr(D_grid), _ptr(rho_bar),
                                          _ptr(f_bar), _ptr(lam_x), _ptr(lam_v)), "avl_adjoint_deposit")


def avl_adjoint_push(h, x, E, kick: float, lam_x_in, lam_v_in, lam_x, lam_v, E_bar):
    return _ck(load().avl_adjoint_push(h, _ptr(x), _ptr(E), float(kick), _ptr(lam_x_in), _ptr(lam_v_in), _ptr(lam_x),
                                       _ptr(lam_v), _ptr(E_bar)), "avl_adjoint_push")


def avl_adjoint_field(h, mu, rho_bar):
    return _ck(load().avl_adjoint_field(h, _ptr(mu), _ptr(rho_bar)), "avl_adjoint_field")


def _cfg_array(cfgs):
    arr = (AvlConfig * len(cfgs))()
    for i, c in enumerate(cfgs):
        arr[i] = c
    return arr


def avl_batch_workspace_bytes(cfgs) -> int:
    return int(load().avl_batch_workspace_bytes(_cfg_array(cfgs), len(cfgs)))


def avl_batch_init(cfgs, workspace, stream, x, v, f) -> ctypes.c_void_p:
    b = ctypes.c_void_p()
    _ck(load().avl_batch_init(_cfg_array(cfgs), len(cfgs), _ptr(workspace),
                              workspace.numel() * workspace.element_size(), _stream_ptr(stream), _ptr(x), _ptr(v),
                              _ptr(f), ctypes.byref(b)), "avl_batch_init")
    return b


def avl_batch_step(b, nsteps: int, diag_out=None):
    return _ck(load().avl_batch_step(b, int(nsteps), _ptr(diag_out)), "avl_batch_step")


def avl_batch_instance(b, i: int):
    h = load().avl_batch_instance(b, int(i))
    if not h:
        raise AvlError(-1, "avl_batch_instance")
    return ctypes.c_void_p(h)


def avl_batch_count(b) -> int:
    return int(load().avl_batch_count(b))


def avl_batch_check(b):
    return load().avl_batch_check(b)


def avl_batch_destroy(b):
    return _ck(load().avl_batch_destroy(b), "avl_batch_destroy")


# ---------------------------------------------------------------------------
# Convenience wrappers
# ---------------------------------------------------------------------------

class Simulation:
    """One VHS species on one GPU: owns a torch workspace and a libavl handle."""

    def __init__(self, w: "inputs.Workload", x, v, f, precision: int = AVL_FP64, device: str = "cuda:0",
                 stream=None, options: int = 0, tune: Optional[dict] = None):
        import torch
        self.w = w
        self.device = torch.device(device)
        self.precision = precision
        x = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        v = torch.as_tensor(v, dtype=torch.float64, device=self.device).reshape(-1).contiguous()
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous()
        self.n = x.numel()
        self.cfg = make_config(w, precision, self.n, options, tune)
        nbytes = avl_workspace_bytes(self.cfg)
        if nbytes == 0:
            raise AvlError(-1, "avl_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.workspace = self.workspace[off:off + nbytes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = avl_init(self.cfg, self.workspace, self.stream, x, v, f)
        self._grid_dtype = torch.float64 if precision == AVL_FP64 else torch.float32

    # shapes ---------------------------------------------------------------
    @property
    def grid_shape(self):
        w = self.w
        return tuple(w.nv[d] for d in reversed(range(w.vdim))) + (w.nx,)

    def _empty(self, n, dtype=None):
        import torch
        return torch.empty(n, dtype=dtype or torch.float64, device=self.device)

    # stages ---------------------------------------------------------------
    def push(self, E=None):
        avl_push(self.h, E)

    def sort(self):
        avl_sort(self.h)

    def reconstruct(self, want_D: bool = False):
        import math
        G = math.prod(self.grid_shape)
        fo = self._empty(G, self._grid_dtype)
        Do = self._empty(G, self._grid_dtype) if want_D else None
        avl_reconstruct(self.h, fo, Do)
        fo = fo.reshape(self.grid_shape)
        return (fo, Do.reshape(self.grid_shape)) if want_D else fo

    def moments(self):
        rho = self._empty(self.w.nx)
        avl_moments(self.h, rho)
        return rho

    def poisson(self, rho=None):
        E = self._empty(self.w.nx)
        W = self._empty(1)
        avl_poisson(self.h, rho, E, W)
        return E, W

    def step(self, nsteps: int, graph: bool = False, diag: bool = True):
        d = self._empty(2 * max(nsteps, 1)) if diag else None
        (avl_step_graph if graph else avl_step)(self.h, nsteps, d)
        return d[: 2 * nsteps].reshape(nsteps, 2) if diag else None

    def markers(self):
        x = self._empty(self.n)
        v = self._empty(self.n * self.w.vdim)
        f = self._empty(self.n)
        avl_get_markers(self.h, x, v, f)
        return x, v.reshape(self.w.vdim, self.n), f

    def set_markers(self, x, v, f):
        import torch
        x = torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()
        v = torch.as_tensor(v, dtype=torch.float64, device=self.device).reshape(-1).contiguous()
        f = torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous()
        avl_set_markers(self.h, x, v, f)

    def field(self):
        E = self._empty(self.w.nx)
        rho = self._empty(self.w.nx)
        avl_get_field(self.h, E, rho)
        return E, rho

    def diagnostics(self, spatial: bool = False):
        """{Ee, Ekin, Etot, N, S, P} of the current state as floats; with
        spatial=True also the current density j(x) and the solver's residual
        charge (device tensors of nx doubles)."""
        out = self._empty(len(DIAG_NAMES))
        j = self._empty(self.w.nx) if spatial else None
        dr = self._empty(self.w.nx) if spatial else None
        avl_diagnostics(self.h, out, j, dr)
        vals = dict(zip(DIAG_NAMES, out.cpu().tolist()))
        return (vals, j, dr) if spatial else vals

    def check(self):
        _ck(avl_check(self.h), "avl_check")

    @property
    def steps(self) -> int:
        return avl_step_count(self.h)

    def close(self):
        if getattr(self, "h", None):
            avl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Instance(Simulation):
    """A batch instance seen as a Simulation (the handle belongs to the batch)."""

    def __init__(self, batch: "Batch", i: int):  # noqa: D401 - no Simulation.__init__
        self.w = batch.workloads[i]
        self.device = batch.device
        self.precision = batch.precision
        self.n = self.w.n_markers
        self.h = avl_batch_instance(batch.b, i)
        self.stream = batch.stream
        import torch
        self._grid_dtype = torch.float64 if self.precision == AVL_FP64 else torch.float32
        self._batch = batch

    def close(self):
        self.h = None


class Batch:
    """Independent 1D-1V instances stepped together (one set of batched launches per step)."""

    def __init__(self, workloads, markers, precision: int = AVL_FP32, device: str = "cuda:0", stream=None,
                 options: int = 0, tunes=None):
        """``markers``: per-instance (x, v, f) arrays (FP64), concatenated here in instance order."""
        import torch
        self.workloads = list(workloads)
        self.device = torch.device(device)
        self.precision = precision
        xs, vs, fs = zip(*markers)
        to = lambda a: torch.as_tensor(a, dtype=torch.float64, device=self.device).reshape(-1)
        x = torch.cat([to(a) for a in xs]).contiguous()
        v = torch.cat([to(a) for a in vs]).contiguous()
        f = torch.cat([to(a) for a in fs]).contiguous()
        tunes = tunes or [None] * len(self.workloads)
        self.cfgs = [make_config(w, precision, None, options, t) for w, t in zip(self.workloads, tunes)]
        nbytes = avl_batch_workspace_bytes(self.cfgs)
        if nbytes == 0:
            raise AvlError(-6, "avl_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.workspace = self.workspace[off:off + nbytes]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.b = avl_batch_init(self.cfgs, self.workspace, self.stream, x, v, f)
        self.n_markers = sum(w.n_markers for w in self.workloads)

    def __len__(self):
        return len(self.workloads)

    def instance(self, i: int) -> Simulation:
        return _Instance(self, i)

    def step(self, nsteps: int, diag: bool = True):
        import torch
        d = torch.empty(len(self) * 2 * max(nsteps, 1), dtype=torch.float64, device=self.device) if diag else None
        avl_batch_step(self.b, nsteps, d)
        return d[: len(self) * 2 * nsteps].reshape(len(self), nsteps, 2) if diag else None

    def check(self):
        _ck(avl_batch_check(self.b), "avl_batch_check")

    def close(self):
        if getattr(self, "b", None):
            avl_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass



class MultiSpecies:
    """Several Simulations (species) stepped in one self-consistent field.

    The Simulations share nx, L, c_p, dt and their stream; each keeps its own
    markers, velocity grid, charge and mass.  ``step`` advances all of them;
    each Simulation's ``field()`` then returns the common field and its own
    species' charge density."""

    def __init__(self, sims):
        import torch
        self.sims = list(sims)
        nbytes = avl_multi_workspace_bytes(len(self.sims), self.sims[0].w.nx)
        if nbytes == 0:
            raise AvlError(-1, "avl_multi_workspace_bytes")
        dev = self.sims[0].device
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        self.workspace = ws[off:off + nbytes]
        self.m = avl_multi_init([s.h for s in self.sims], self.workspace)

    def step(self, nsteps: int, diag: bool = True):
        d = self.sims[0]._empty(2 * max(nsteps, 1)) if diag else None
        avl_multi_step(self.m, nsteps, d)
        return d[: 2 * nsteps].reshape(nsteps, 2) if diag else None

    def close(self):
        if getattr(self, "m", None):
            avl_multi_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
