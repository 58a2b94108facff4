"""Benchmark of the AT finite-difference step on one MI355X.

Workload: 3-D advection-diffusion on a periodic 256^3 grid split into 8x8x8
PEs of 32^3, fourth-order AT scheme (T = 3 levels), L = 4 uniform delays per
PE face and step, AB2, 500 steps, u0 = four plane waves with random phases.
A "step" is one AT time step of the whole grid (delay draw, AT halo
combination, interior sweep, right-hand side, AB2 update, halo publish).

Prints one JSON line: grid-point updates/s of the FP32-bulk AT run (FP64 AT
combination), its HBM roofline fraction, the FP64 and synchronous-scheme arms
with their errors against the exact solution, and the FP64 CPU oracle timed on
a bounded sample on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, AMD published figure

p = argparse.ArgumentParser()
p.add_argument("--gpus", type=int, default=1)
p.add_argument("--steps", type=int, default=500)
p.add_argument("--warmup", type=int, default=20)
p.add_argument("--graph", type=int, default=50, help="steps per captured HIP graph (0: plain launches)")
p.add_argument("--n", type=int, default=256)
p.add_argument("--b", type=int, default=32)
p.add_argument("--no-cpu-baseline", action="store_true")
p.add_argument("--arms", default="f32,f64,sync32", help="comma list of arms to time")
p.add_argument("--cpu-steps", type=int, default=10)
p.add_argument("--no-autotune", action="store_true")
p.add_argument("--variant", type=int, default=0, help="fixed schedule variant of the 3-D sweep (skips autotuning)")
p.add_argument("--others", default="burgers,ensemble,adjoint,space,study,nonuniform,matched,generic3d,c1",
               help="other workloads timed after the headline (comma list; empty: none)")
args = p.parse_args()

if args.gpus != 1:
    print(json.dumps({"error": "this benchmark runs on one GPU only: the simulated PEs all live "
                      "on one device; run with --gpus 1"}))
    sys.exit(2)

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
import workloads as W  # noqa: E402
from paper_1702_00496_amd import Solver  # noqa: E402

cfg = W.config_3d_advdiff(n=args.n, b=args.b)
N = cfg["n"][0]
npts = N ** 3
u0_host = torch.from_numpy(W.eval_modes(cfg["modes"], cfg["n"], 3))
dev = torch.device("cuda:0")
u0 = u0_host.to(dev)


def make(precision, mode):
    return Solver(ndim=3, n=cfg["n"], pe=cfg["pe"], dt=cfg["dt"], order=4, equation="advdiff",
                  c=cfg["c"], alpha=cfg["alpha"], integrator="ab2", precision=precision,
                  L=cfg["L"], T=cfg["T"], mode=mode, seed=cfg["seed"])


def bytes_per_update(precision, mode):
    """Algorithmic HBM bytes per grid-point update of the AB2 AT step.

    Bulk: u^n read, u^{n+1} written, f^{n-1} read, f^n written (4 values).
    Faces: h = 2 * dim * s / b halo values per point and level; a face with
    delay k reads T levels when k > 0 and one level when k = 0 (zero weights
    are skipped), so E[levels] = p0 + (1 - p0) T with p0 = 1/L; the new edge
    values are published once (h values written)."""
    w = 8 if precision == "f64" else 4
    if mode == "sync":
        return 4 * w
    h = 2 * 3 * 2 / args.b
    p0 = 1.0 / cfg["L"]
    levels = p0 + (1 - p0) * cfg["T"]
    return (4 + h * (levels + 1)) * w


def graph_chunk():
    """Steps per captured HIP graph: the largest divisor of the timed step count
    not above --graph, so that every timed step runs from a graph replay."""
    if args.graph <= 0:
        return 0
    return max(d for d in range(1, min(args.graph, args.steps) + 1) if args.steps % d == 0)


GRAPH = graph_chunk()


def time_arm(precision, mode):
    s = make(precision, mode)
    s.set_state(u0)
    tuned = None
    if args.variant:
        s.set_tuning(args.variant)
    elif not args.no_autotune:
        s.step(3)
        tuned = s.autotune(nsteps=20)       # schedule choice, state restored
    if GRAPH:
        s.set_graph(GRAPH)
    s.set_state(u0)
    if GRAPH:
        s.step(GRAPH)                       # capture and instantiate the graph outside the timing
    s.step(args.warmup)
    s.set_state(u0)                     # the timed run is steps 0..K-1 of the workload
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nrm = s.norms(modes=cfg["modes"])
    # five more timed runs of the same K steps (after the reported one), for
    # the spread between runs
    repeats = []
    for _ in range(5):
        s.set_state(u0)
        torch.cuda.synchronize()
        e0.record()
        s.step(args.steps)
        e1.record()
        torch.cuda.synchronize()
        repeats.append(e0.elapsed_time(e1) / args.steps)
    ups = npts * args.steps / (ms / 1e3)
    bpu = bytes_per_update(precision, mode)
    gbs = ups * bpu / 1e9
    return dict(precision=precision, mode=mode, depth=s.tuning(), autotune_ms=tuned[1] if tuned else None,
                ms=ms, ms_per_step=ms / args.steps, repeat_ms_per_step=repeats,
                median_ms_per_step=float(np.median([ms / args.steps] + repeats)),
                updates_per_s=ups, bytes_per_update=bpu, achieved_gbs=gbs,
                frac=gbs / HBM_PEAK_GBS, l2_error=nrm["l2"], linf_error=nrm["linf"])


def copy_bandwidth():
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * a.numel() * 4 * 10 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    return gbs


KERNEL_SOURCES = ("step3d_fast.hpp", "atfd_internal.hpp", "fast3d_f32_s2.hip", "fast3d_f64_s2.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "at_step3d_fast_256cube_traffic.md")


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, per schedule variant and arm; empty where the kernel sources
    changed since it was taken or the workload differs."""
    import hashlib
    if args.n != 256 or args.b != 32 or not os.path.exists(TRAFFIC_FILE):
        return {}
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1702_00496_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    with open(TRAFFIC_FILE) as fh:
        line = next((ln for ln in fh if ln.startswith("bench-traffic: ")), None)
    if line is None:
        return {}
    meta = json.loads(line[len("bench-traffic: "):])
    if meta.get("kernel_sources_sha256_16") != h.hexdigest()[:16]:
        return {}
    return {int(v): arms for v, arms in meta["variants"].items()}


def cpu_baseline():
    """The FP64 oracle on the host cores: the first cpu_steps steps of the same
    workload (a bounded sample of the run)."""
    from oracle.solver import DelayModel, Oracle, Problem
    torch.set_num_threads(os.cpu_count() or 1)
    prob = Problem(ndim=3, n=cfg["n"], pe=cfg["pe"], dt=cfg["dt"], order=4, equation="advdiff",
                   c=cfg["c"], alpha=cfg["alpha"], integrator="ab2")
    o = Oracle(prob, DelayModel(L=cfg["L"], T=cfg["T"], mode="rng", seed=cfg["seed"]), u0_host)
    t0 = time.perf_counter()
    o.run(args.cpu_steps)
    dt_ = time.perf_counter() - t0
    cores = torch.get_num_threads()
    # one thread: the next step of the same run
    torch.set_num_threads(1)
    t0 = time.perf_counter()
    o.run(1)
    dt1 = time.perf_counter() - t0
    torch.set_num_threads(cores)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), None)
    except OSError:
        pass
    return dict(value=npts * args.cpu_steps / dt_, unit="grid-pt updates/s",
                cores=cores, cpu_model=model, kind="oracle",
                sample=f"first {args.cpu_steps} of {cfg['steps']} steps of the {N}^3 workload, FP64, "
                       f"{dt_:.1f} s",
                single_thread=dict(value=npts / dt1, cores=1,
                                   sample=f"step {args.cpu_steps + 1} of the same run on one thread, "
                                          f"{dt1:.1f} s"))


arms = {}
for arm in args.arms.split(","):
    precision = "f64" if "64" in arm else "f32"
    mode = "sync" if arm.startswith("sync") else "rng"
    arms[arm] = time_arm(precision, mode)
    print(f"[bench] {arm}: {arms[arm]['ms_per_step']:.4f} ms/step "
          f"{arms[arm]['updates_per_s']:.3e} upd/s {arms[arm]['achieved_gbs']:.0f} GB/s "
          f"l2={arms[arm]['l2_error']:.3e}", file=sys.stderr, flush=True)

def time_burgers():
    """3-D viscous Burgers, 512^3, 16^3 PEs of 32^3, sixth order (T = 4), L = 8,
    Heun RK2, 200 steps: FP32 bulk with FP64 AT combination, full FP64, and
    the synchronous FP32 arm; the relative L2 and Linf difference of the FP32
    field from the FP64 one after 200 steps; the adjoint of the final energy
    J = 1/2 sum u_T^2 dx^3 with respect to u0 (checkpoints every 40 steps),
    FP32. Bytes per update (two launches per step): u^n and u* read or written
    5 times, plus per stage the halo reads h E[levels] and the publish h,
    h = 2 * 3 * 3 / 32, E[levels] = p0 + (1 - p0) T, p0 = 1/8."""
    c5 = W.config_3d_burgers()
    n5 = c5["n"]
    u5 = torch.from_numpy(W.burgers_spectrum_field(n5[0], 3, seed=c5["seed"])).to(dev)
    res = {}
    fields = {}

    def make(precision, mode):
        return Solver(ndim=3, n=n5, pe=c5["pe"], dt=c5["dt"], order=6, equation="burgers", alpha=c5["alpha"],
                      integrator="rk2", precision=precision, L=c5["L"], T=c5["T"], mode=mode, seed=c5["seed"])

    for arm, precision, mode in (("at32", "f32", "rng"), ("at64", "f64", "rng"), ("sync32", "f32", "sync")):
        s = make(precision, mode)
        s.set_state(u5)
        s.step(2)
        best = s.autotune(nsteps=5)[0]
        s.set_graph(20)
        s.set_state(u5)
        s.step(20)
        s.set_state(u5)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(c5["steps"])
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = s.state()
        finite = bool(torch.isfinite(st).all())
        if mode == "rng":
            fields[precision] = st.to(torch.float64)
        w = 8 if precision == "f64" else 4
        h = 2 * 3 * 3 / 32
        p0 = 1.0 / c5["L"]
        bpu = w * (5 + (2 * h * (p0 + (1 - p0) * c5["T"] + 1) if mode == "rng" else 0.0))
        ups = n5[0] ** 3 * c5["steps"] / (ms / 1e3)
        res[arm] = dict(ms_per_step=ms / c5["steps"], updates_per_s=ups, bytes_per_update=bpu,
                        achieved_gbs=ups * bpu / 1e9, frac=ups * bpu / 1e9 / HBM_PEAK_GBS, variant=best,
                        finite=finite)
        print(f"[bench] burgers {arm}: {ms / c5['steps']:.3f} ms/step {ups:.3e} upd/s", file=sys.stderr, flush=True)
        del s, st
        torch.cuda.empty_cache()
    d = fields["f32"] - fields["f64"]
    f32_vs_f64 = dict(rel_l2=float(torch.linalg.norm(d) / torch.linalg.norm(fields["f64"])),
                      rel_linf=float(d.abs().max() / fields["f64"].abs().max()))
    del d, fields
    torch.cuda.empty_cache()
    # adjoint: J = 1/2 sum u_T^2 dV, seed dJ/du_T = u_T dV
    dV = (2 * math.pi / n5[0]) ** 3
    s = make("f32", "rng")
    s.set_state(u5)
    s.step(c5["steps"])
    seed = s.state().to(torch.float64) * dV
    s = make("f32", "rng")
    s.set_state(u5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.adjoint(c5["steps"], seed, 40)
    torch.cuda.synchronize()
    adj_ms = (time.perf_counter() - t0) * 1e3
    print(f"[bench] burgers adjoint: {adj_ms:.1f} ms", file=sys.stderr, flush=True)
    del s, seed
    torch.cuda.empty_cache()
    return dict(workload="3-D viscous Burgers 512^3, 16^3 PEs of 32^3, 6th-order AT (T=4), L=8, RK2, "
                         "200 steps: FP32 bulk / FP64 AT combination, full FP64, synchronous FP32; adjoint of "
                         "the final energy w.r.t. u0 (FP32, checkpoints every 40)",
                arms=res, f32_vs_f64=f32_vs_f64, adjoint_ms=adj_ms,
                adjoint_ratio_to_forward=adj_ms / (res["at32"]["ms_per_step"] * c5["steps"]))


def time_space():
    """The space-expanded single-level schemes against the time-expanded one on
    a 3-D grid: 256^3, 8^3 PEs of 32^3, second-order CD, advection-diffusion,
    Euler, L = 3 with p = {0.5, 0.3, 0.2} (the delay law of Sec. 5.1 Cases
    2 and 3), FP32 bulk, 100 steps. Bytes per update (solution in place): u
    read and written, halo reads h (p0 + (1 - p0) D) and the publish h D, with
    h = 2 * 3 / 32 face columns per point and D buffer points per column: 3
    for (1,2,2)a + (2,2,2)a, 2 for (1,2,2)a + (2,1,2); the time-expanded
    (1,2,2)b + (2,2,2)b reads h (p0 + 2 (1 - p0)) values of its two levels and
    publishes h."""
    cfg3 = W.config_3d_advdiff(n=256, b=32)
    n3 = cfg3["n"]
    alpha = 0.1
    dx = 2 * math.pi / n3[0]
    dt = 0.05 * dx * dx / alpha
    steps = 100
    u3 = torch.from_numpy(W.eval_modes(cfg3["modes"], n3, 3))
    p0 = 0.5
    h = 2 * 3 / 32
    res = {}
    for scheme, depth in (("space222", 3), ("space212", 2), ("time", None)):
        s = Solver(ndim=3, n=n3, pe=cfg3["pe"], dt=dt, order=2, c=(1.0, 1.0, 1.0), alpha=alpha,
                   integrator="euler", precision="f32", L=3, weights=[5, 3, 2], seed=cfg3["seed"], scheme=scheme)
        s.set_state(u3)
        s.step(5)
        s.set_graph(20)
        s.set_state(u3)
        s.step(20)
        s.set_state(u3)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        nrm = s.norms(modes=cfg3["modes"])
        if depth is None:
            bpu = 4 * (2 + h * (p0 + (1 - p0) * 2) + h)
        else:
            bpu = 4 * (2 + h * (p0 + (1 - p0) * depth) + h * depth)
        ups = n3[0] ** 3 * steps / (ms / 1e3)
        res[scheme] = dict(ms_per_step=ms / steps, updates_per_s=ups, bytes_per_update=bpu,
                           achieved_gbs=ups * bpu / 1e9, frac=ups * bpu / 1e9 / HBM_PEAK_GBS,
                           l2_error=nrm["l2"], l2_error_boundary=nrm["l2_b"], l2_error_interior=nrm["l2_i"])
        print(f"[bench] space-expanded {scheme}: {ms / steps:.4f} ms/step {ups:.3e} upd/s l2={nrm['l2']:.3e}",
              file=sys.stderr, flush=True)
        del s
        torch.cuda.empty_cache()
    return dict(workload="3-D advection-diffusion 256^3, 8^3 PEs of 32^3, 2nd-order CD, Euler, L=3 with "
                         "p={0.5,0.3,0.2}, 100 FP32 steps: space-expanded (1,2,2)a+(2,2,2)a and (1,2,2)a+(2,1,2) "
                         "against time-expanded (1,2,2)b+(2,2,2)b", arms=res)


def time_nonuniform():
    """The non-uniform-delay scheme (Sec. 3.4 Example 1: own delays at the two
    buffer points next to a face) against the uniform-delay (1,2,2)a/(2,1,2)
    pair and the time-expanded (1,2,2)b/(2,2,2)b (T = 2) on one kernel, the
    generic sweep: 2-D 4096^2, 64 x 64 PEs of 64^2, second-order CD,
    advection-diffusion, Euler, L = 4 with uniform delays, FP32 bulk, 100
    steps. Bytes per update (solution in place): u read and written, plus per
    face column (h = 4 / 64 per point) the halo values the sweep loads and the
    strip it publishes: 2 + 2 for the single-level pair and the non-uniform
    scheme (2-deep strips, one level each), T + 1 for the time-expanded one."""
    n2 = (4096, 4096)
    pe = (64, 64)
    alpha = 0.1
    dx = 2 * math.pi / n2[0]
    dt = 0.05 * dx * dx / alpha
    steps = 100
    modes = W.make_modes([(1, 2, 0), (3, 1, 0), (2, 5, 0)], [1.0, 0.5, 0.25], seed=5)
    u2 = torch.from_numpy(W.eval_modes(modes, n2 + (1,), 2))
    h = 4 / 64
    res = {}
    for scheme, per_col in (("nonuniform212", 4), ("space212", 4), ("time", 3)):
        s = Solver(ndim=2, n=n2, pe=pe, dt=dt, order=2, c=(1.0, 0.5), alpha=alpha, integrator="euler",
                   precision="f32", L=4, seed=17, scheme=scheme)
        s.set_state(u2)
        s.step(5)
        s.set_graph(20)
        s.set_state(u2)
        s.step(20)
        s.set_state(u2)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        nrm = s.norms(modes=modes)
        bpu = 4 * (2 + h * per_col)
        ups = n2[0] * n2[1] * steps / (ms / 1e3)
        res[scheme] = dict(ms_per_step=ms / steps, updates_per_s=ups, bytes_per_update=bpu,
                           achieved_gbs=ups * bpu / 1e9, frac=ups * bpu / 1e9 / HBM_PEAK_GBS,
                           l2_error=nrm["l2"], l2_error_boundary=nrm["l2_b"])
    res["config"] = {"n": list(n2), "pe": list(pe), "order": 2, "integrator": "euler", "L": 4,
                     "weights": "uniform", "precision": "f32", "steps": steps, "kernel": "generic sweep"}
    return res


def time_c1():
    """The 1-D workload (N = 256, 8 PEs of 32, order 2, Euler, L = 3, 1000
    steps, FP64) is a few KB: per-step launches (even replayed from HIP
    graphs) cost far more than its arithmetic. Timed two ways: the context's
    per-step sweep, and the same problem as a one-member ensemble, whose
    persistent launch runs all steps in one workgroup; the two final fields
    agree to rounding."""
    from paper_1702_00496_amd import Ensemble
    cfg = W.config_1d_advdiff()
    steps = cfg["steps"]
    u = torch.from_numpy(W.eval_modes(cfg["modes"], cfg["n"], 1))
    ms, _ = _run_family_point(cfg, "rng", steps)
    s = Solver(ndim=1, n=cfg["n"][:1], pe=cfg["pe"][:1], dt=cfg["dt"], order=2, c=cfg["c"][:1], alpha=cfg["alpha"],
               integrator="euler", precision="f64", L=cfg["L"], seed=cfg["seed"])
    s.set_state(u)
    s.step(steps)
    ref = s.state().double().reshape(-1).cpu()
    m = dict(n=cfg["n"][0], pe=cfg["pe"][0], order=2, integrator="euler", L=cfg["L"], T=0, mode="rng",
             c=cfg["c"][0], alpha=cfg["alpha"], dt=cfg["dt"], seed=cfg["seed"])
    ens = Ensemble([m], precision="f64")
    u1 = u.reshape(-1)
    ens.set_state(u1)
    ens.run(steps)                          # capture + warm-up
    ens.set_state(u1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    ens.run(steps)
    e1.record()
    torch.cuda.synchronize()
    ems = e0.elapsed_time(e1)
    got = ens.state().double().reshape(-1).cpu()
    return dict(workload=f"1-D N = {cfg['n'][0]}, {cfg['pe'][0]} PEs, order 2, Euler, L = {cfg['L']}, "
                         f"{steps} steps, FP64",
                per_step_launch_ms=ms, persistent_ms=ems, speedup=ms / ems,
                rel_l2_between=float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref)))


def time_generic3d():
    """The generic 3-D sweep (PE edges other than 32: 192^3 in 4^3 PEs of 48^3,
    fourth order, AB2, L = 4, FP32 bulk, 100 steps), AT and synchronous arms.
    Its 64 PEs are split into z-chunks of several workgroups. Bytes per update
    (two solution buffers): u read and written, f^{n-1} read and f^n written,
    plus per face column (h = 2 * 3 * 2 / 48 per point) the T = 3 delayed halo
    levels read and the strip published: 4 * (4 + 4 h) = 20 B (synchronous:
    16 B)."""
    cfg = W.config_3d_advdiff(n=192, b=48)
    u = torch.from_numpy(W.eval_modes(cfg["modes"], cfg["n"], 3))
    steps = 100
    res = {}
    for mode, bpu in (("rng", 20.0), ("sync", 16.0)):
        s = Solver(ndim=3, n=cfg["n"], pe=cfg["pe"], dt=cfg["dt"], order=4, c=cfg["c"], alpha=cfg["alpha"],
                   integrator="ab2", precision="f32", L=cfg["L"], seed=cfg["seed"], mode=mode)
        s.set_state(u)
        s.step(3)
        variant, tune_ms = s.autotune(nsteps=10)      # z-chunk count, state restored
        s.set_graph(20)
        s.set_state(u)
        s.step(20)
        s.set_state(u)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        ups = 192 ** 3 * steps / (ms / 1e3)
        res["at" if mode == "rng" else "sync"] = dict(
            ms_per_step=ms / steps, updates_per_s=ups, bytes_per_update=bpu, achieved_gbs=ups * bpu / 1e9,
            frac=ups * bpu / 1e9 / HBM_PEAK_GBS, l2_error=s.norms(modes=cfg["modes"])["l2"],
            chunk_variant=variant, autotune_ms_per_step={str(k): v for k, v in tune_ms.items()})
    res["config"] = {"n": 192, "pe_edge": 48, "order": 4, "integrator": "ab2", "L": cfg["L"], "precision": "f32",
                     "steps": steps, "kernel": "generic sweep, z-chunks autotuned"}
    return res


def _run_family_point(cfg, mode, steps, precision="f64", graph=50):
    nd = cfg["ndim"]
    s = Solver(ndim=nd, n=cfg["n"][:nd], pe=cfg["pe"][:nd], dt=cfg["dt"], order=cfg["order"], c=cfg["c"][:nd],
               alpha=cfg["alpha"], integrator=cfg["integrator"], precision=precision, L=cfg["L"],
               seed=cfg["seed"], mode=mode)
    u = torch.from_numpy(W.eval_modes(cfg["modes"], cfg["n"], nd))
    s.set_graph(graph)
    s.set_state(u)
    s.step(graph)                       # capture outside the timing
    s.set_state(u)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return ms, s.norms(modes=cfg["modes"])["l2"]


def time_matched():
    """Standard scheme against AT at matched error (FP64): for the 1-D
    (N = 256, 8 PEs, order 2, Euler, L = 3, 1000 steps) and the 3-D (256^3,
    PEs of 32^3, order 4, AB2, L = 4, 500 steps) workloads, N is swept at
    fixed diffusive CFL and final time (steps scale with N^2). log E against
    log N and log time against log N are fitted by least squares for the AT
    arm; N* is where the AT error equals the synchronous error at the
    reference N, and the reported ratio is AT's time at N* over the
    synchronous time at the reference N (the intrinsic cost of AT on one GPU,
    where the synchronous scheme waits for nothing)."""
    fams = {
        "1d_order2": (W.config_1d_advdiff, 256, 1000, (128, 256, 512, 1024), lambda n: dict(n=n, pe=8)),
        "3d_order4": (W.config_3d_advdiff, 256, 500, (128, 192, 256, 320), lambda n: dict(n=n, b=32)),
    }
    res = {}
    for name, (make_cfg, n_ref, steps_ref, ns, kw) in fams.items():
        t_final = make_cfg(**kw(n_ref))["dt"] * steps_ref
        rows = []
        for n in ns:
            cfg = make_cfg(**kw(n))
            steps = int(round(steps_ref * (n / n_ref) ** 2))
            cfg["dt"] = t_final / steps
            at_ms, at_e = _run_family_point(cfg, "rng", steps)
            sy_ms, sy_e = _run_family_point(cfg, "sync", steps)
            rows.append(dict(n=n, steps=steps, at_ms=at_ms, sync_ms=sy_ms, at_l2=at_e, sync_l2=sy_e))
        ln = np.log([r["n"] for r in rows])
        fit_e = np.polyfit(ln, np.log([r["at_l2"] for r in rows]), 1)
        fit_t = np.polyfit(ln, np.log([r["at_ms"] for r in rows]), 1)
        ref = next(r for r in rows if r["n"] == n_ref)
        n_star = float(np.exp((np.log(ref["sync_l2"]) - fit_e[1]) / fit_e[0]))
        t_star = float(np.exp(np.polyval(fit_t, np.log(n_star))))
        res[name] = dict(rows=rows, t_final=t_final, at_error_slope=float(fit_e[0]),
                         sync_error_slope=float(np.polyfit(ln, np.log([r["sync_l2"] for r in rows]), 1)[0]),
                         at_time_slope=float(fit_t[0]), n_ref=n_ref, sync_l2_at_n_ref=ref["sync_l2"],
                         n_star=n_star, at_ms_at_n_star=t_star, sync_ms_at_n_ref=ref["sync_ms"],
                         time_to_solution_ratio=t_star / ref["sync_ms"])
    return res


def time_study():
    """The moment-law study of Sec. 5.2 on the ensemble kernel: the Case 1
    scheme (order 2, T = 2, Euler), N = 1024 with 16 PEs, p_k = 1/L for
    L = 2..6, 256 delay histories per L plus a synchronous member (1281
    members in one launch), r_alpha = 0.1, t = 0.1 (2653 steps), FP64."""
    from paper_1702_00496_amd import studies
    kw = dict(order=2, Ls=(2, 3, 4, 5, 6), realizations=256, n=1024, pe=16, r_alpha=0.1, t_final=0.1,
              precision="f64")
    studies.moment_study(**dict(kw, realizations=4, t_final=0.01))     # build and warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = studies.moment_study(**kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    npts = 1024 * len(res["members"])
    ratios = [r["ratio"] for r in res["per_L"].values()]
    print(f"[bench] moment study: {ms:.1f} ms for {len(res['members'])} members x {res['steps']} steps, "
          f"async/law {min(ratios):.3e}..{max(ratios):.3e}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    conv = studies.convergence_study(case="case6", Ns=(32, 64, 128, 256), precision="f64")
    torch.cuda.synchronize()
    ms6 = (time.perf_counter() - t0) * 1e3
    print(f"[bench] Case 6 convergence study: {ms6:.1f} ms, slopes "
          f"{[round(r['slopes'][-1], 2) for r in conv['per_law'].values()]}", file=sys.stderr, flush=True)
    return dict(workload="moment-law study (Sec. 5.2): order 2, T=2, Euler, N=1024 / 16 PEs, L=2..6 uniform, "
                         "256 histories per L + 1 synchronous member, FP64, set-up + run + norms",
                ms=ms, members=len(res["members"]), steps=res["steps"],
                updates_per_s=npts * res["steps"] / (ms / 1e3),
                per_L={str(L): dict(E=r["E"], E_sync=r["E_sync"], asynchronous=r["asynchronous"], law=r["law"],
                                    ratio=r["ratio"], perturbation=r["perturbation"],
                                    perturbation_ratio=r["perturbation_ratio"]) for L, r in res["per_L"].items()},
                case6_convergence=dict(ms=ms6, Ns=conv["Ns"],
                                       per_law={str(w): dict(E=r["E"], slopes=r["slopes"])
                                                for w, r in conv["per_law"].items()}))


def time_ensemble():
    """512 independent 1-D members (N log-uniform in [1024, 65536], PE 64,
    orders 2/4, L in {2, 4, 8}), 2000 steps in one persistent launch, FP32;
    schedule from the ensemble autotuner (timed outside the run). Reports the
    ensemble mean and unbiased variance of the members' RMS error against the
    exact solution, per order and per log-spaced dx bin."""
    from paper_1702_00496_amd import Ensemble
    inst = W.ensemble_instances()
    members = [dict(n=m["n"], pe=m["pe"], order=m["order"], integrator=m["integrator"], L=m["L"], T=m["T"],
                    mode="rng", c=m["c"], alpha=m["alpha"], dt=m["dt"], seed=m["seed"]) for m in inst]
    u3 = torch.from_numpy(np.concatenate([W.eval_modes(m["modes"], (m["n"],), 1).reshape(-1) for m in inst]))
    ens = Ensemble(members, precision="f32")
    ens.set_state(u3)
    default = ens.tuning()
    tuned, tune_ms = ens.autotune(nsteps=100)
    ens.run(2000)                           # capture + warm-up
    ens.set_state(u3)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    ens.run(2000)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ph = np.array([[mo[2] for mo in m["modes"]] for m in inst])
    err = ens.norms([3, 4, 5], [2.0, 0.5, 1.5], ph)
    dx = np.array([2 * math.pi / m["n"] for m in members])
    nb = 8
    edges = np.exp(np.linspace(np.log(dx.min()), np.log(dx.max() * (1 + 1e-9)), nb + 1))
    stats = ens.error_stats(edges, [3, 4, 5], [2.0, 0.5, 1.5], ph)
    table = {}
    for g, order in ((0, 2), (1, 4)):
        table[f"order{order}"] = [dict(dx_lo=float(edges[j]), dx_hi=float(edges[j + 1]), count=int(stats[g, j, 0]),
                                       mean_dx=float(stats[g, j, 1]), mean_rms_error=float(stats[g, j, 2]),
                                       var_rms_error=float(stats[g, j, 3]))
                                  for j in range(nb) if stats[g, j, 0] > 0]
    ups = u3.numel() * 2000 / (ms / 1e3)
    print(f"[bench] ensemble: {ms:.1f} ms for 2000 steps, {ups:.3e} upd/s, schedule {tuned} "
          f"(default {default})", file=sys.stderr, flush=True)
    return dict(workload="512-member 1-D delay ensemble, 7.5M points, 2000 steps, one persistent launch, FP32",
                ms=ms, updates_per_s=ups, schedule=dict(groups_per_cu=tuned[0], threads=tuned[1]),
                autotune_ms_per_step={f"{a}x{b}": v for (a, b), v in tune_ms.items()},
                max_rms_error=float(err[:, 1].max()), median_rms_error=float(np.median(err[:, 1])),
                error_vs_dx=table)


def time_adjoint():
    """Gradient of J = 1/2 sum (u_T - target)^2 dx^2 on the 1024^2 2-D
    workload (16^2 PEs of 64^2, order 4, L = 4, AB2, 2000 FP32 steps,
    checkpoints every 64): forward with checkpoints, segment recomputation
    and the reverse sweep."""
    c4 = W.config_2d_advdiff()
    n4 = c4["n"]
    u4 = torch.from_numpy(W.eval_modes(c4["modes"], n4, 2)).to(dev)
    seed = torch.from_numpy(W.eval_modes(c4["target_modes"], n4, 2)).to(dev)

    def make():
        return Solver(ndim=2, n=n4, pe=c4["pe"], dt=c4["dt"], order=4, c=c4["c"], alpha=c4["alpha"],
                      integrator="ab2", precision="f32", L=c4["L"], seed=c4["seed"])
    s = make()
    s.set_state(u4)
    s.adjoint(64, seed, 64)                 # warm-up
    s = make()
    s.set_state(u4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.adjoint(c4["steps"], seed, 64)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    f = make()
    f.set_state(u4)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    f.step(c4["steps"])
    e1.record()
    torch.cuda.synchronize()
    fms = e0.elapsed_time(e1)
    print(f"[bench] adjoint: {ms:.1f} ms (forward alone {fms:.1f} ms)", file=sys.stderr, flush=True)
    return dict(workload="gradient of a final-time misfit, 2-D 1024^2, 16^2 PEs of 64^2, order 4, L=4, AB2, "
                         "2000 FP32 steps, checkpoints every 64", ms=ms, forward_ms=fms,
                ratio_to_forward=ms / fms)


traffic = measured_traffic()
for arm, r in arms.items():
    r["traffic_bytes"] = traffic.get(r["depth"], {}).get(arm)
head_arm = "f32" if "f32" in arms else next(iter(arms))
head = arms[head_arm]
copy_gbs = copy_bandwidth()
out = {
    "metric": "AT stencil grid-pt updates/s, % HBM roofline, vs standard at matched error",
    "value": head["updates_per_s"],
    "unit": "grid-pt updates/s",
    "n_gpus": 1,
    "steps": args.steps,
    "warmup": args.warmup,
    "ms_per_step": head["ms_per_step"],
    "higher_is_better": True,
    "scaling": "weak",
    "vs_baseline": None,
    "dtype": "f32" if head["precision"] == "f32" else "f64",
    "data": "synthetic",
    "config": {"workload": f"3-D advection-diffusion {N}^3, {cfg['pe'][0]}^3 PEs of {args.b}^3, "
                           f"4th-order AT (T=3), L={cfg['L']} uniform delays, AB2, {cfg['steps']} steps",
               "grid": N, "pe_edge": args.b, "order": 4, "L": cfg["L"], "integrator": "ab2",
               "dt": cfg["dt"], "graph_chunk": GRAPH},
    "roofline": {"bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS,
                 "unit": "GB/s", "frac": head["frac"], "traffic": head["traffic_bytes"],
                 "traffic_unit": "bytes per launch between L2 and the fabric (rocprofv3 FETCH_SIZE x 2 + "
                                 "WRITE_SIZE, scaled by a copy kernel; includes Infinity Cache hits)",
                 "frac_of_measured_copy": head["achieved_gbs"] / copy_gbs,
                 "kernel": f"at_step3d_fast_kernel<{'float' if head['precision'] == 'f32' else 'double'}, s=2, variant={head['depth']}, AB2, advection-diffusion>",
                 "bytes_per_update": head["bytes_per_update"],
                 "measured_copy_gbs": copy_gbs},
    "arms": arms,
}
if "f32" in arms and "sync32" in arms:
    # the standard synchronous scheme on the same GPU, same grid and steps:
    # matched error when the L2 errors agree
    a, b = arms["f32"], arms["sync32"]
    out["vs_standard"] = {"at_ms_per_step": a["ms_per_step"], "sync_ms_per_step": b["ms_per_step"],
                          "time_ratio": a["ms_per_step"] / b["ms_per_step"],
                          "at_l2_error": a["l2_error"], "sync_l2_error": b["l2_error"],
                          "error_ratio": a["l2_error"] / b["l2_error"]}
others = {}
for w in [x for x in args.others.split(",") if x]:
    others[w] = {"burgers": time_burgers, "ensemble": time_ensemble, "adjoint": time_adjoint,
                 "space": time_space, "study": time_study, "nonuniform": time_nonuniform,
                 "matched": time_matched, "generic3d": time_generic3d, "c1": time_c1}[w]()
if others:
    out["other_workloads"] = others
if not args.no_cpu_baseline:
    out["cpu_baseline"] = cpu_baseline()
print(json.dumps(out))
