"""Throughput of the VHS time step on one MI355X.

Workload: 1D-1V bump-on-tail, nx = nv = 1024 cells on v in [-8, 8), 16 markers
per cell (16,777,216 markers), synthetic seeded markers (no dataset).  A step is
the whole hot path: gather+push, counting sort, weight-normalised
reconstruction of f with the fused rho partials, spectral field solve.

Prints ONE JSON line.  ``value`` is marker-steps/s of the FP32 form (the
form the metric names) replayed as a HIP graph; the plain FP64 path and the
Kahan-accumulation variant are measured on the same markers and reported
beside it.  ``roofline`` is for the reconstruction kernel, timed with HIP
events on the library's stream around every launch in a second timed region
of direct launches.
``cpu_baseline`` times the CPU oracle on a bounded sample of the same workload.

``batched`` reports the parameter scan (64 uneven 1D-1V instances, FP32 form)
stepped as batched launches, and its throughput over the plain FP64 path.

``--workload two_stream_3v`` measures the 1D-3V two-stream case instead (512 x
64^3 cells, 4 markers per cell, 536,870,912 markers; FP32 form by default, no
CPU baseline).
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PAPER_RATE_PER_CORE = 1.0e7      # marker updates per second on one CPU core, as the paper states it


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


FORMS = {"fp32": ("AVL_FP32", 0), "fp32_kahan": ("AVL_FP32", "AVL_OPT_KAHAN32"), "fp64": ("AVL_FP64", 0)}


def copy_probe(avl, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth of a plain streaming copy (read + write bytes / time)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    avl.avl_copy_probe(dst, src, nbytes)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        avl.avl_copy_probe(dst, src, nbytes)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    ok = bool(torch.equal(dst[:1024], src[:1024]))
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9, ms, ok


def run_form(avl, inputs, w, x, v, f, form, steps, warmup):
    import torch
    prec_name, opt = FORMS[form]
    precision = getattr(avl, prec_name)
    options = getattr(avl, opt) if isinstance(opt, str) else opt
    sim = avl.Simulation(w, x, v, f, precision=precision, options=options)
    torch.cuda.synchronize()
    sim.step(warmup, graph=True, diag=False)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    # timed region 1: the step as a replayed HIP graph (the production path)
    torch.cuda.synchronize()
    t0.record(sim.stream)
    sim.step(steps, graph=True, diag=False)
    t1.record(sim.stream)
    torch.cuda.synchronize()
    ms_graph = t0.elapsed_time(t1)
    # timed region 2: the same steps as direct launches with HIP events on the
    # library's stream around every kernel (per-kernel times for the roofline)
    avl.avl_timing(sim.h, True)
    torch.cuda.synchronize()
    t0.record(sim.stream)
    sim.step(steps, graph=False, diag=False)
    t1.record(sim.stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    kt = {}
    for k, name in enumerate(avl.KERNEL_NAMES):
        tot, cnt = avl.avl_kernel_time(sim.h, k)
        nbytes = avl.avl_kernel_bytes(sim.h, k)
        ms_avg = tot / cnt if cnt else None
        # algorithmic bytes per launch over the launch's mean duration, against the HBM peak
        frac = nbytes / (ms_avg * 1e-3) / 1e9 / HBM_PEAK_GBS if ms_avg else None
        kt[name] = {"ms_avg": ms_avg, "launches": cnt, "bytes_per_launch": nbytes, "hbm_frac": frac}
    # the step entry counts the method's own bytes (push and reconstruction,
    # sorting excluded); the sort's bytes are listed beside it
    sort_bytes = sum(kt[k]["bytes_per_launch"] for k in ("push_count", "scan", "scatter"))
    kt["step"]["bytes_kind"] = "method (push + reconstruction, sort excluded)"
    kt["step"]["sort_bytes_per_step"] = sort_bytes
    if kt["step"]["ms_avg"]:
        both = kt["step"]["bytes_per_launch"] + sort_bytes
        kt["step"]["hbm_frac_with_sort_bytes"] = both / (kt["step"]["ms_avg"] * 1e-3) / 1e9 / HBM_PEAK_GBS
    avl.avl_timing(sim.h, False)
    sim.check()
    sim.close()
    return ms / steps, ms_graph / steps, kt


# per workload: the PMC traffic summary and the sources of the reconstruction
# kernel its counters belong to
TRAFFIC = {
    "bump_on_tail": ("profiles/hbm_traffic_bump_on_tail_16M.txt",
                     ("paper_1804_03901_amd/csrc/avl_recon.hip", "paper_1804_03901_amd/csrc/avl_device.h")),
    "two_stream_3v": ("profiles/hbm_traffic_two_stream_3v_537M.txt",
                      ("paper_1804_03901_amd/csrc/avl_recon3.hip", "paper_1804_03901_amd/csrc/avl_device.h")),
}


def source_digest(paths):
    """sha256 over the sources that define the reconstruction kernel."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel_tag):
    """HBM bytes per launch of the reconstruction from the committed PMC
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel
    calibration), or None when the kernel sources changed since the counters
    were taken or no summary exists."""
    if workload not in TRAFFIC:
        return None
    rel, sources = TRAFFIC[workload]
    path = os.path.join(ROOT, rel)
    if not os.path.exists(path):
        return None
    digest = None
    rows = {}
    for line in open(path):
        if line.startswith("# source_sha256"):
            digest = line.split()[-1]
        elif line.startswith("traffic "):
            _, tag, fetch, write = line.split()[:4]
            rows[tag] = (float(fetch), float(write))
    if digest != source_digest(sources) or kernel_tag not in rows:
        return None
    return rows[kernel_tag][0] + rows[kernel_tag][1]


def run_batched(avl, inputs, steps, warmup, count, one_by_one=True):
    """The parameter-scan batch (uneven 1D-1V bump-on-tail instances, FP32
    form), stepped as batched launches replayed as a HIP graph, and beside it
    the same instances stepped one after another, each as its own handle with
    its own graph (the library's defaults), so that the batch's gain is
    measured rather than assumed."""
    import torch
    from paper_1804_03901_amd import tune
    ws = inputs.batched_scan(count=count)
    mk = [inputs.markers_threaded(w) for w in ws]
    # reconstruction rows per task and row form for the batch, chosen by timing candidates
    tunes, tables = tune.tune_batch(ws, mk, precision=avl.AVL_FP32, candidates=(0, 6, 12, 24), forms=(1, 2),
                                    steps=5, warmup=2, cache_path=None)
    b = avl.Batch(ws, mk, precision=avl.AVL_FP32, tunes=tunes)
    torch.cuda.synchronize()
    b.step(warmup, diag=False)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(b.stream)
    b.step(steps, diag=False)
    t1.record(b.stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    b.check()
    n_markers = b.n_markers
    b.close()
    # one instance at a time: the sum of the instances' own graph-replayed steps
    one_ms = 0.0
    for w, (x, v, f) in zip(ws, mk) if one_by_one else ():
        sim = avl.Simulation(w, x, v.reshape(-1), f, precision=avl.AVL_FP32)
        sim.step(warmup, graph=True, diag=False)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(sim.stream)
        sim.step(steps, graph=True, diag=False)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        one_ms += e0.elapsed_time(e1) / steps
        sim.check()
        sim.close()
    del mk
    names = {avl.TUNE_RECON_ROWS: "recon_rows", avl.TUNE_RECON_FORM: "recon_form"}
    obo = None
    if one_by_one:
        obo = {"ms_per_step": one_ms, "marker_steps_per_s": n_markers / (one_ms * 1e-3),
               "batched_speedup": one_ms / ms,
               "timing": "each instance alone, its own graph replay, library defaults; "
                         "sum over the instances of their ms per step"}
    return {"instances": len(ws), "markers": n_markers, "ms_per_step": ms,
            "marker_steps_per_s": n_markers / (ms * 1e-3), "steps": steps, "form": "fp32",
            "nx": sorted({w.nx for w in ws}), "nv": sorted({w.nv[0] for w in ws}),
            "tuned": {names[k]: v for k, v in tunes[0].items()},
            "tuning_ms_per_step": {names[k]: {str(c): t for c, t in tab.items()} for k, tab in tables.items()},
            "one_by_one": obo}


def run_adjoint(avl, inputs, every=50):
    """The adjoint configuration: bump-on-tail at nx = 1024, nv = 512, 8
    markers per cell (4,194,304 markers), 500 steps, FP32 forward with a
    checkpoint every 50 steps; the time of one whole gradient (forward with
    checkpoints, segment recomputation, reverse sweep) against the time of the
    plain 500-step forward run."""
    import torch
    from paper_1804_03901_amd import adjoint
    w = inputs.adjoint_case()
    x, v, f = inputs.markers_threaded(w)
    dev = torch.device("cuda:0")
    xt = torch.tensor(x, device=dev)
    vt = torch.tensor(v.reshape(-1), device=dev)
    ft = torch.tensor(f, device=dev)
    sim = avl.Simulation(w, xt, vt, ft, precision=avl.AVL_FP32)
    adjoint.energy_and_gradient(sim, xt, vt, ft, w.steps, every=every)      # warm-up (workspace, code)
    torch.cuda.synchronize()
    t = time.perf_counter()
    J, grad = adjoint.energy_and_gradient(sim, xt, vt, ft, w.steps, every=every)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t
    t = time.perf_counter()
    adjoint.energy_and_gradient(sim, xt, vt, ft, w.steps, want_grad=False)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    sim.check()
    sim.close()
    return {"workload": w.name, "markers": w.n_markers, "steps": w.steps, "checkpoint_every": every, "form": "fp32",
            "seconds_gradient": t_grad, "seconds_forward": t_fwd, "gradient_over_forward": t_grad / t_fwd,
            "J": float(J), "grad_l2": float(torch.linalg.vector_norm(grad)),
            "timing": "host clock around one call, device synchronised on both sides"}


def cpu_baseline(inputs, w, x, v, f, steps):
    import oracle
    g = oracle.Grid.from_workload(w)
    r0 = oracle.run(g, x, v, f, 0)
    t = time.perf_counter()
    oracle.run(g, x, v, f, steps, E=r0["E"])
    dt = time.perf_counter() - t
    return x.size * steps / dt, dt


def cpu_child(args):
    """One copy of the all-core CPU baseline: generate the workload's markers,
    solve once, report ready, wait for the go line on stdin, time
    ``--cpu-steps`` oracle steps and print the rate.  Imports no GPU module."""
    import oracle
    from paper_1804_03901_amd import inputs
    w = inputs.bump_on_tail(nx=args.nx, nv=args.nv, ppc=args.ppc)
    x, v, f = inputs.markers(w)
    g = oracle.Grid.from_workload(w)
    r0 = oracle.run(g, x, v, f, 0)
    print("ready", flush=True)
    sys.stdin.readline()
    t = time.perf_counter()
    oracle.run(g, x, v, f, args.cpu_steps, E=r0["E"])
    dt = time.perf_counter() - t
    print(json.dumps({"rate": x.size * args.cpu_steps / dt, "seconds": dt}), flush=True)


def cpu_baseline_all_cores(args, procs):
    """The oracle on every core at once: ``procs`` independent copies of the
    workload (child processes of their own, started together), each timing
    ``--cpu-steps`` steps; the aggregate is the sum of their rates."""
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", "--nx", str(args.nx), "--nv", str(args.nv),
           "--ppc", str(args.ppc), "--cpu-steps", str(args.cpu_steps)]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    kids = [subprocess.Popen(cmd, stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True, env=env)
            for _ in range(procs)]
    try:
        for k in kids:
            if k.stdout.readline().strip() != "ready":
                raise RuntimeError("a CPU baseline child did not start")
        for k in kids:
            k.stdin.write("go\n")
            k.stdin.flush()
        res = [json.loads(k.stdout.readline()) for k in kids]
    finally:
        for k in kids:
            k.wait(timeout=300)
    return sum(r["rate"] for r in res), max(r["seconds"] for r in res)


def cpu_model():
    """The host CPU as lscpu reports it: model name, then family, model and
    stepping numbers, sockets, cores per socket and threads per core."""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        f = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                f[k.strip()] = v.strip()
        name = f.get("Model name", platform.processor() or "unknown")
        extra = [f"{k.lower()} {f[k]}" for k in ("CPU family", "Model", "Stepping", "Socket(s)", "Core(s) per socket",
                                                  "Thread(s) per core", "CPU max MHz") if k in f]
        return f"{name} ({', '.join(extra)})" if extra else name
    except Exception:
        return platform.processor() or "unknown"


def cpu_count():
    """Logical CPUs the process may use (nproc)."""
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nx", type=int, default=1024)
    ap.add_argument("--nv", type=int, default=1024)
    ap.add_argument("--ppc", type=int, default=16)
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default=None, help="default: fp32,fp32_kahan,fp64 (1D-1V); fp32 (1D-3V)")
    ap.add_argument("--workload", default="bump_on_tail", choices=["bump_on_tail", "two_stream_3v"],
                    help="two_stream_3v: the 1D-3V two-stream case, 512 x 64^3 cells, 4 markers per cell")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--adjoint", default=True, action=argparse.BooleanOptionalAction,
                    help="time one gradient of the adjoint configuration (default on)")
    ap.add_argument("--batch", type=int, default=64, help="instances of the batched parameter scan (0: skip)")
    ap.add_argument("--one-by-one", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the batch's instances one after another (default on)")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--cpu-cores", type=int, default=16,
                    help="most processes of the all-core CPU baseline (nproc of the host, capped here: a GPU "
                         "box grants one GPU's share of 16 CPUs; 0: skip)")
    ap.add_argument("--cpu-child", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_child:
        cpu_child(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        sys.exit(2)

    import torch
    from paper_1804_03901_amd import avl, inputs

    three_v = args.workload == "two_stream_3v"
    if three_v:
        w = inputs.two_stream_3v()
        args.no_cpu = True
    else:
        w = inputs.bump_on_tail(nx=args.nx, nv=args.nv, ppc=args.ppc)
    forms = (args.forms or ("fp32" if three_v else "fp32,fp32_kahan,fp64")).split(",")
    log(f"generating {w.n_markers} markers ({w.name})")
    x, v, f = inputs.markers_threaded(w)
    v = v.reshape(-1)
    results = {}
    probe = None
    if not args.no_probe:
        probe = copy_probe(avl)
        log(f"copy probe: {probe[0]:.0f} GB/s")
    for form in forms:
        log(f"form {form}: warmup {args.warmup}, timed {args.steps}")
        results[form] = run_form(avl, inputs, w, x, v, f, form, args.steps, args.warmup)
        log(f"form {form}: {results[form][1]:.4f} ms/step graph, {results[form][0]:.4f} direct with events")
    main_form = "fp32" if "fp32" in results else next(iter(results))
    ms_direct, ms, kt = results[main_form]
    value = w.n_markers / (ms * 1e-3)
    rk = kt["reconstruct"]
    recon_kernel = "k_recon_3v" if three_v else "k_recon_1v"
    achieved = rk["bytes_per_launch"] / (rk["ms_avg"] * 1e-3) / 1e9
    out = {
        "metric": ("marker-steps/s, 1D-3V two-stream 537M markers, FP32 form; % HBM peak" if three_v else
                   "marker-steps/s, 1D-1V 16.8M markers, FP32+batched vs FP64 plain; % HBM peak"),
        "value": value,
        "unit": "marker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_form == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "markers": w.n_markers, "nx": w.nx, "nv": list(w.nv[: w.vdim]), "ppc": w.ppc,
                   "form": main_form, "weights": w.weights, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, f"{'recon3' if three_v else 'recon'}_{main_form}"),
                     "traffic_unit": "bytes per launch (PMC, calibrated)", "kernel": recon_kernel,
                     "bytes_per_launch": rk["bytes_per_launch"], "ms_per_launch": rk["ms_avg"]},
        "timing": "value: HIP-graph replay of the step, events around the whole timed region; kernels: a "
                  "second timed region of direct launches; count, scatter and reconstruction carry HIP events "
                  "attached to their own dispatch (the kernel's start and end), scan and field have events "
                  "recorded around their launches",
        "forms": {k: {"ms_per_step": r[1], "marker_steps_per_s": w.n_markers / (r[1] * 1e-3),
                      "ms_per_step_direct": r[0], "marker_steps_per_s_direct": w.n_markers / (r[0] * 1e-3),
                      "kernels": r[2]} for k, r in results.items()},
    }
    for k in results:
        t = measured_traffic(args.workload, f"{'recon3' if three_v else 'recon'}_{k}")
        rk_k = out["forms"][k]["kernels"]["reconstruct"]
        rk_k["traffic"] = t
        # the reconstruction's target: at least 60% of the HBM peak on its own bytes
        rk_k["meets_60pct_gate"] = bool(rk_k["hbm_frac"] is not None and rk_k["hbm_frac"] >= 0.6)
    out["roofline"]["gate"] = 0.6
    out["roofline"]["meets_gate"] = bool(out["roofline"]["frac"] >= 0.6)
    # the paper's own throughput figure (Sec. Performance and Parallelization), quoted with its
    # hardware: context next to the measured rate, not a target (its workload is not stated)
    out["paper_figure"] = {"value": PAPER_RATE_PER_CORE, "unit": "marker-steps/s per core",
                           "hardware": "Intel Xeon E5-2650 @ 2.6 GHz, one core", "precision": "FP64 (inferred)",
                           "source": "Sec. Performance and Parallelization", "workload": "not stated"}
    if "fp32" in results and "fp64" in results:
        out["fp32_speedup_over_fp64"] = results["fp64"][1] / results["fp32"][1]
    if args.adjoint and not three_v:
        log("adjoint: 4.2M markers, 500 steps, FP32 forward, checkpoint every 50")
        out["adjoint"] = run_adjoint(avl, inputs)
        log(f"adjoint: {out['adjoint']['seconds_gradient']:.3f} s a gradient, "
            f"{out['adjoint']['gradient_over_forward']:.2f}x the forward run")
    if args.batch and not three_v:
        log(f"batched scan: {args.batch} instances, warmup {args.warmup}, timed {args.batch_steps}")
        out["batched"] = run_batched(avl, inputs, args.batch_steps, args.warmup, args.batch, args.one_by_one)
        obo = out["batched"]["one_by_one"]
        log(f"batched scan: {out['batched']['ms_per_step']:.4f} ms/step, "
            f"{out['batched']['marker_steps_per_s']:.3e} marker-steps/s"
            + (f"; one by one {obo['ms_per_step']:.4f} ms/step" if obo else ""))
        if "fp64" in results:
            fp64_rate = w.n_markers / (results["fp64"][1] * 1e-3)
            out["batched"]["fp32_batched_over_fp64_plain"] = out["batched"]["marker_steps_per_s"] / fp64_rate
    if probe is not None:
        out["roofline"]["copy_probe_GBs"] = probe[0]
        out["roofline"]["frac_of_copy"] = achieved / probe[0]
        out["copy_probe"] = {"GB_per_s": probe[0], "ms": probe[1], "bytes_moved": 2 * (1 << 30), "checked": probe[2]}
    if not args.no_cpu:
        log(f"cpu baseline: oracle, {args.cpu_steps} steps on the full marker set, 1 thread")
        rate, secs = cpu_baseline(inputs, w, x, v.reshape(1, -1), f, args.cpu_steps)
        nproc = cpu_count()
        out["cpu_baseline"] = {"value": rate, "unit": "marker-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{args.cpu_steps} steps of the full {w.n_markers}-marker workload "
                                         f"after the initial solve ({secs:.1f} s), FP64, single thread",
                               "cpu": cpu_model(), "nproc": nproc}
        procs = min(args.cpu_cores, nproc)
        if procs > 1:
            steps_all = max(1, args.cpu_steps // 8)
            log(f"cpu baseline, all cores: {procs} oracle processes, {steps_all} steps each")
            a = argparse.Namespace(**vars(args))
            a.cpu_steps = steps_all
            rate_all, secs_all = cpu_baseline_all_cores(a, procs)
            out["cpu_baseline_all_cores"] = {
                "value": rate_all, "unit": "marker-steps/s", "cores": procs, "kind": "oracle", "nproc": nproc,
                "cpu": cpu_model(),
                "sample": f"{procs} independent copies of the full {w.n_markers}-marker workload, "
                          f"{steps_all} steps each after the initial solve ({secs_all:.1f} s), FP64, one thread each "
                          f"(nproc {nproc}; at most {args.cpu_cores} processes, the CPU share a GPU box grants)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
