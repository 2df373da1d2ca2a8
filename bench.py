"""Throughput of the PonD time step on one MI355X.

Workload: the four-quadrant 2-D Riemann problem (D2Q16, zero-gradient edges,
tau = 0.55, seed 3) on a 1024^2 grid, run from its initial state for K steps.
A "step" is one pond_step call: propagation with the adaptive predictor-
corrector gauge iteration, then BGK.  MLUPS = nodes * steps / seconds / 1e6
with the state resident in HBM, timed with HIP events on the launch stream.

Prints one JSON line.  The FP64 path gives `value`; the FP32-mixed path, its
error against FP64, the adjoint/forward time ratios and the oracle timed on
host cores (`cpu_baseline`) are reported beside it.

Other modes (used for profiling, each prints its own line):
  --kernel-only   FP64 steps only (FP32-mixed with --kernel-precision f32), then
                  one replay with step statistics for the pass count and the
                  roofline fraction (for rocprofv3)
  --copy-probe    a plain device copy of known size (HBM counter calibration)
  --adjoint-only  FP64 adjoint of one step at the state after 50 steps, twice
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1806_05089_amd import autograd, pond, workloads  # noqa: E402

# Algorithmic flop count per node and predictor-corrector pass, the floor the
# method needs whatever the kernel: 16 populations x 16 collocation points x
# 42 flops (row-Kronecker contraction of a transformed point, 2(q^2 + q), and
# its weighted accumulate, 2), 8 departure coordinates x 16 flops for the
# Lagrange weights, 7 x 16 flops for the four moments.  Transfer-row
# construction is not counted (it depends on how rows are shared).  Per node
# and step, 560 flops for the regauge and BGK.
FLOPS_PER_NODE_PASS = 16 * 16 * 42 + 8 * 16 + 7 * 16
FLOPS_PER_NODE_STEP = 560
PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64: 256 CU x 2.4 GHz x 64 lanes x 2
PEAK_FP32_TFLOPS = 157.3  # MI355X published FP32 peak
PEAK_HBM_GBPS = 8000.0    # MI355X HBM3E
# the step kernel, its device helpers and the launch settings (bulk cap)
STEP_SOURCES = [os.path.join(ROOT, "paper_1806_05089_amd", "csrc", n)
                for n in ("pond_step.hip", "pond_device.hpp", "pond_api.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_riemann2d_1024_fp64_hbm_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def code_text(src: str) -> str:
    """C++ source without its comments and with runs of whitespace collapsed:
    what the compiler sees, so that editing a comment keeps a digest."""
    out, i, n = [], 0, len(src)
    while i < n:
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif src[i] == '"':  # string literal, copied as it is
            j = i + 1
            while j < n and src[j] != '"':
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(src[i])
            i += 1
    return " ".join("".join(out).split())


def source_digest(paths=None):
    """sha256[:16] of the step kernel's sources (comments and layout ignored)."""
    h = hashlib.sha256()
    for path in (STEP_SOURCES if paths is None else paths):
        h.update(code_text(open(path, encoding="utf-8").read()).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def make_cfg(w, precision, q1d=4):
    ny, nx = w.shape
    cfg = pond.PondConfig(nx=nx, ny=ny, q1d=q1d, precision=precision, isothermal=w.isothermal,
                          bc_x=w.bc_x, bc_y=w.bc_y, tau=w.tau, max_iter=20)
    if precision == pond.POND_F32_MIXED:
        cfg = cfg.replace(eps_abs=1e-6, eps_rel=1e-5)
    return cfg


def timed_steps(cfg, w, steps, warmup, runs=1):
    """Warm up on a throwaway run, then time `steps` steps from the initial
    state `runs` times (each from the initial state).  Returns the median run
    time in ms, the final state and the one before it, and every run's time."""
    a = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    b = pond.empty_state(cfg)
    for _ in range(warmup):
        pond.step(cfg, a, b)
        a, b = b, a
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(runs):
        a = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            pond.step(cfg, a, b)
            a, b = b, a
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times)), a, b, times


def count_passes(cfg, w, steps):
    """Replay the run with per-step statistics (predictor-corrector passes)."""
    a = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    b = pond.empty_state(cfg)
    total = 0.0
    nonconv = 0
    hist = np.zeros(64, dtype=np.int64)
    for _ in range(steps):
        _, st = pond.step(cfg, a, b, stats=True)
        total += st["mean_iters"]
        nonconv += st["nonconverged"]
        hist += np.array(st["iter_hist"], dtype=np.int64)
        a, b = b, a
    return {"mean_passes": total / steps, "nonconverged_node_steps": nonconv,
            "iter_hist": trim_hist(hist)}


def trim_hist(hist):
    """Histogram of node-steps per pass count as {passes: count}, empty bins left out."""
    return {str(k): int(v) for k, v in enumerate(hist) if v}


def alu_roofline(mean_passes, nodes, ms_per_step, peak):
    flops = FLOPS_PER_NODE_PASS * mean_passes * nodes + FLOPS_PER_NODE_STEP * nodes
    achieved = flops / (ms_per_step * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "flops_per_launch": flops}


def full_run(w, steps=2000, check_steps=(10, 100, 2000)):
    """The benchmark run in full, whatever --steps is: `steps` steps from the
    initial state in both precisions, timed once each (HIP events), then
    replayed in lockstep with step statistics for the pass counts, the pass
    histogram and the cap hits, and the FP32-mixed vs FP64 per-field error at
    `check_steps`."""
    nodes = w.rho.size
    out = {"steps": steps}
    cfgs = {"f64": make_cfg(w, pond.POND_F64), "f32_mixed": make_cfg(w, pond.POND_F32_MIXED)}
    for name, cfg in cfgs.items():
        ms, _, _, _ = timed_steps(cfg, w, steps, 0)
        out[name] = {"value": nodes * steps / (ms * 1e-3) / 1e6, "unit": "MLUPS",
                     "ms_per_step": ms / steps}
    st = {k: pond.init(c, w.rho, w.ux, w.uy, w.T) for k, c in cfgs.items()}
    nxt = {k: pond.empty_state(c) for k, c in cfgs.items()}
    acc = {k: {"passes": 0.0, "nonconv": 0, "bad": 0, "hist": np.zeros(64, dtype=np.int64)}
           for k in cfgs}
    errors = {}
    for n in range(1, steps + 1):
        for k, c in cfgs.items():
            _, s_ = pond.step(c, st[k], nxt[k], stats=True)
            st[k], nxt[k] = nxt[k], st[k]
            acc[k]["passes"] += s_["mean_iters"]
            acc[k]["nonconv"] += s_["nonconverged"]
            acc[k]["bad"] = s_["bad_state"]
            acc[k]["hist"] += np.array(s_["iter_hist"], dtype=np.int64)
        if n in check_steps:
            errors[f"step_{n}"] = field_errors(cfgs["f64"], st["f64"], cfgs["f32_mixed"],
                                               st["f32_mixed"])
    peaks = {"f64": PEAK_FP64_TFLOPS, "f32_mixed": PEAK_FP64_TFLOPS}
    for k in cfgs:
        mp = acc[k]["passes"] / steps
        out[k]["mean_pc_passes"] = mp
        out[k]["cap_hit_fraction"] = acc[k]["nonconv"] / (nodes * steps)
        out[k]["bad_nodes_at_end"] = acc[k]["bad"]
        out[k]["iter_hist_node_steps"] = trim_hist(acc[k]["hist"])
        out[k]["roofline"] = alu_roofline(mp, nodes, out[k]["ms_per_step"], peaks[k])
    out["f32_mixed"]["roofline"]["peak_note"] = (
        "78.6 TFLOP/s: the rate of the unpacked FP32 vector FMAs the library issues "
        "(packed FP32 is compiled out); against the 157.3 TFLOP/s packed peak the fraction "
        "is half")
    out["speedup_fp32_vs_fp64"] = out["f32_mixed"]["value"] / out["f64"]["value"]
    out["speedup_fp32_vs_fp64_per_node_pass"] = (
        out["f32_mixed"]["value"] * out["f32_mixed"]["mean_pc_passes"]
        / (out["f64"]["value"] * out["f64"]["mean_pc_passes"]))
    out["fp32_error_vs_fp64"] = errors
    out["workload"] = (f"riemann2d {w.rho.shape[1]}x{w.rho.shape[0]}, {steps} steps from the "
                       "initial state, adaptive passes (FP64 tolerances 1e-12/1e-10, FP32-mixed "
                       "1e-6/1e-5), cap 20")
    return out


def fixed_pass_speedup(w, steps=50, npass=2):
    """FP32-mixed vs FP64 at equal work: both precisions with exactly `npass`
    passes per node (fixed-iteration mode), so the ratio is the precision's
    alone, not that of the looser FP32 convergence test."""
    nodes = w.rho.size
    res = {}
    for name, prec in (("f64", pond.POND_F64), ("f32_mixed", pond.POND_F32_MIXED)):
        cfg = make_cfg(w, prec).replace(fixed_iter=npass)
        ms, _, _, _ = timed_steps(cfg, w, steps, 2)
        res[name] = {"value": nodes * steps / (ms * 1e-3) / 1e6, "unit": "MLUPS",
                     "ms_per_step": ms / steps}
    res["speedup"] = res["f32_mixed"]["value"] / res["f64"]["value"]
    res["passes_per_node"] = npass
    res["steps"] = steps
    return res


def adjoint_ratio_1024(cfg, state, reps=3):
    """Time of one pond_step_adjoint vs one pond_step about the same state."""
    out, _ = pond.step(cfg, state)
    g = torch.Generator(device="cuda").manual_seed(0)
    wf = torch.randn(out.f.shape, dtype=torch.float64, device="cuda", generator=g)
    wg = torch.randn(out.g.shape, dtype=torch.float64, device="cuda", generator=g)
    atau = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(pond.workspace_bytes(cfg), dtype=torch.uint8, device="cuda")
    pond.step_adjoint(cfg, state, out, wf, wg, atau, workspace=ws)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    for _ in range(reps):
        pond.step(cfg, state, out)
    e[1].record()
    e[2].record()
    for _ in range(reps):
        pond.step_adjoint(cfg, state, out, wf, wg, atau, workspace=ws)
    e[3].record()
    torch.cuda.synchronize()
    fwd = e[0].elapsed_time(e[1]) / reps
    adj = e[2].elapsed_time(e[3]) / reps
    # recorded form: the forward step writes its pass history
    # (pond_step_record), the adjoint reads it (pond_step_adjoint_recorded)
    rec, tape = pond.step_record(cfg, state)
    pond.step_adjoint_recorded(cfg, state, rec, tape, wf, wg, atau)
    torch.cuda.synchronize()
    e[0].record()
    for _ in range(reps):
        pond.step_record(cfg, state, rec, tape)
    e[1].record()
    e[2].record()
    for _ in range(reps):
        pond.step_adjoint_recorded(cfg, state, rec, tape, wf, wg, atau)
    e[3].record()
    torch.cuda.synchronize()
    fwd_r = e[0].elapsed_time(e[1]) / reps
    adj_r = e[2].elapsed_time(e[3]) / reps
    return {"forward_ms": fwd, "adjoint_ms": adj, "ratio": adj / fwd,
            "workspace_bytes": int(ws.numel()),
            "note": "pond_step_adjoint runs the step again to record its pass history",
            "recorded": {"forward_record_ms": fwd_r, "adjoint_recorded_ms": adj_r,
                         "ratio_to_plain_forward": adj_r / fwd,
                         "ratio_to_recording_forward": adj_r / fwd_r}}


def adjoint_ratio_tgv128():
    """Compressible Taylor-Green 128^2 (Mach 0.5, FP32-mixed), 200 steps,
    checkpoints every 20: forward rollout time vs backward time."""
    w = workloads.compressible_taylor_green(128, seed=1)
    cfg = pond.PondConfig(nx=128, ny=128, precision=pond.POND_F32_MIXED, tau=0.6,
                          eps_abs=1e-6, eps_rel=1e-5, max_iter=20)
    dev = torch.device("cuda")
    rho = torch.tensor(w.rho, dtype=torch.float64, device=dev)
    ux = torch.tensor(w.ux, dtype=torch.float64, device=dev, requires_grad=True)
    uy = torch.tensor(w.uy, dtype=torch.float64, device=dev, requires_grad=True)
    T = torch.tensor(w.T, dtype=torch.float64, device=dev)
    tau = torch.tensor(0.6, dtype=torch.float64, device=dev, requires_grad=True)
    # warm-up rollout (library load, allocator, first launches)
    f0, g0 = autograd.equilibrium_state(cfg, rho, ux, uy, T)
    autograd.kinetic_energy(*autograd.rollout(f0, g0, tau, cfg, 20, checkpoint_every=20)).backward()
    ux.grad = None
    uy.grad = None
    tau.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f0, g0 = autograd.equilibrium_state(cfg, rho, ux, uy, T)
    fT, gT = autograd.rollout(f0, g0, tau, cfg, 200, checkpoint_every=20)
    J = autograd.kinetic_energy(fT, gT)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    T_ref = float(w.meta.get("T0", 1.0))
    return {"forward_s": t1 - t0, "backward_s": t2 - t1, "ratio": (t2 - t1) / (t1 - t0),
            "dJ_dtau": float(tau.grad.item()), "dJ_dnu": float(tau.grad.item()) / T_ref,
            "T_ref": T_ref,
            "note": "backward includes the checkpoint replays (one extra forward per step); "
                    "nu = T_ref (tau - 1/2), so dJ/dnu = (dJ/dtau) / T_ref"}


def host_cpu():
    """The host the oracle ran on: CPU model and the threads this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)),
            "logical_cpus": os.cpu_count()}


def cpu_baseline(cfg, state, sample_nodes, seed=0):
    import oracle
    f = state.f.double().cpu().numpy()
    g = state.g.cpu().numpy()
    rng = np.random.default_rng(seed)
    nodes = rng.choice(cfg.nx * cfg.ny, size=sample_nodes, replace=False)
    oc = oracle.OracleConfig(q=4, isothermal=cfg.isothermal, bc_x=cfg.bc_x, bc_y=cfg.bc_y,
                             max_iter=cfg.max_iter, tau=cfg.tau, eps_abs=cfg.eps_abs,
                             eps_rel=cfg.eps_rel)
    t = time.perf_counter()
    _, _, it, _ = oracle.step_nodes(f, g, oc, nodes)
    dt = time.perf_counter() - t
    return {"value": sample_nodes / dt / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one step at {sample_nodes} random nodes of the FP64 state after the timed "
                      f"run ({it.mean():.2f} passes/node), {dt:.1f} s"}


def field_errors(cfg64, s64, cfg32, s32):
    m64 = [t.cpu().numpy() for t in pond.moments(cfg64, s64)]
    m32 = [t.cpu().numpy() for t in pond.moments(cfg32, s32)]
    out = {}
    for name, a, b, sc in zip(("rho", "ux", "uy", "T"), m32, m64, (None, 1.0, 1.0, None)):
        scale = float(np.max(np.abs(b))) if sc is None else max(sc, float(np.max(np.abs(b))))
        out[name] = {"max_rel": float(np.max(np.abs(a - b)) / scale),
                     "mean_rel": float(np.mean(np.abs(a - b)) / scale)}
    return out


def fp32_error_other_configs():
    """FP32-mixed vs FP64 per-field error at the end of the shock tube (1024 x 4,
    400 steps) and the Mach 5 flow (256^2, 1000 steps)."""
    res = {}
    for name, w, n in (("sod_1024x4_400_steps", workloads.sod(1024, 4), 400),
                       ("mach5_256_1000_steps", workloads.mach5(256, seed=0), 1000)):
        c64, c32 = make_cfg(w, pond.POND_F64), make_cfg(w, pond.POND_F32_MIXED)
        o64, _ = pond.step(c64, pond.init(c64, w.rho, w.ux, w.uy, w.T), nsteps=n)
        o32, _ = pond.step(c32, pond.init(c32, w.rho, w.ux, w.uy, w.T), nsteps=n)
        res[name] = field_errors(c64, o64, c32, o32)
    return res


def riemann_2048(steps=200, warmup=2):
    """FP64 and FP32-mixed throughput on the 2048^2 Riemann problem (first steps)."""
    w = workloads.riemann2d(2048, seed=3)
    nodes = 2048 * 2048
    out = {}
    for name, prec in (("f64", pond.POND_F64), ("f32_mixed", pond.POND_F32_MIXED)):
        ms, _, _, _ = timed_steps(make_cfg(w, prec), w, steps, warmup)
        out[name] = {"value": nodes * steps / (ms * 1e-3) / 1e6, "unit": "MLUPS",
                     "ms_per_step": ms / steps}
    out["speedup_fp32_vs_fp64"] = out["f32_mixed"]["value"] / out["f64"]["value"]
    out["steps"] = steps
    return out


def riemann_d2q9(size=1024, steps=200, warmup=2):
    """The paper's own lattice: the same Riemann flow on D2Q9 (temperatures
    scaled to T_L = 1/3, same Mach numbers), both precisions, first steps."""
    w = workloads.riemann2d(size, seed=3, T_scale=workloads.TL_D2Q9)
    nodes = size * size
    out, ends = {}, {}
    for name, prec in (("f64", pond.POND_F64), ("f32_mixed", pond.POND_F32_MIXED)):
        cfg = make_cfg(w, prec, q1d=3)
        ms, a, _, _ = timed_steps(cfg, w, steps, warmup)
        nxt, st = pond.step(cfg, a.clone(), stats=True)
        ends[name] = (cfg, a)
        out[name] = {"value": nodes * steps / (ms * 1e-3) / 1e6, "unit": "MLUPS",
                     "ms_per_step": ms / steps, "mean_pc_passes_at_end": st["mean_iters"]}
    out["speedup_fp32_vs_fp64"] = out["f32_mixed"]["value"] / out["f64"]["value"]
    out["fp32_error_vs_fp64_at_end"] = field_errors(ends["f64"][0], ends["f64"][1],
                                                    ends["f32_mixed"][0], ends["f32_mixed"][1])
    out["steps"] = steps
    out["workload"] = (f"riemann2d on D2Q9, {size}x{size}, temperatures x 1/3 (T_L = 1/3), "
                       "tau 0.55, zero-gradient edges, seed 3, adaptive")
    return out


def cpu_single_thread(cfg, state, sample_nodes=40000, seed=1):
    import oracle
    prev = oracle.set_num_threads(1)
    try:
        r = cpu_baseline(cfg, state, sample_nodes, seed)
    finally:
        oracle.set_num_threads(prev)
    return r


def cpu_small_configs():
    """The oracle on the Taylor-Green run (32^2, all 200 steps) and on the
    shock tube (1024 x 4, all 400 steps; the oracle parallelises over rows, so
    this tube keeps only 4 threads busy), all host threads."""
    import oracle
    out = {}
    for name, w, n in (("taylor_green_32_200_steps", workloads.taylor_green(32), 200),
                       ("sod_1024x4_400_steps", workloads.sod(1024, 4), 400)):
        oc = oracle.OracleConfig(q=4, isothermal=w.isothermal, bc_x=w.bc_x, bc_y=w.bc_y,
                                 max_iter=20, tau=w.tau)
        f, g = oracle.init(w.rho, w.ux, w.uy, w.T, q=4)
        t = time.perf_counter()
        for _ in range(n):
            f, g, _, _ = oracle.step(f, g, oc)
        dt = time.perf_counter() - t
        out[name] = {"value": w.rho.size * n / dt / 1e6, "unit": "MLUPS", "seconds": dt}
    out["cores"] = oracle.num_threads()
    return out


def traffic_per_launch(n_launch_nodes):
    """HBM bytes per step launch from the committed counter summary, if it was
    taken on the current step kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    if rec.get("source_sha256_16") != source_digest():
        return None
    return rec.get("bytes_per_launch")


def adjoint_only(size, reps=2):
    """pond_step_adjoint about one step of the Riemann problem after 50 steps."""
    w = workloads.riemann2d(size, seed=3)
    cfg = make_cfg(w, pond.POND_F64)
    a = pond.init(cfg, w.rho, w.ux, w.uy, w.T)
    a, _ = pond.step(cfg, a, nsteps=50)
    out, _ = pond.step(cfg, a)
    g = torch.Generator(device="cuda").manual_seed(0)
    wf = torch.randn(out.f.shape, dtype=torch.float64, device="cuda", generator=g)
    wg = torch.randn(out.g.shape, dtype=torch.float64, device="cuda", generator=g)
    atau = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.empty(pond.workspace_bytes(cfg), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pond.step_adjoint(cfg, a, out, wf, wg, atau, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    print(json.dumps({"adjoint_only": True, "ms_per_call": e0.elapsed_time(e1) / reps}), flush=True)


def copy_probe():
    n = 1 << 27  # 1 GiB of float64
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8,
                      "launches": 3}), flush=True)


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2000)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--size", type=int, default=1024)
    p.add_argument("--no-fp32", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-adjoint", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=1000000)
    p.add_argument("--no-pass-count", action="store_true")
    p.add_argument("--kernel-only", action="store_true")
    p.add_argument("--kernel-precision", choices=("f64", "f32"), default="f64",
                   help="precision of the --kernel-only steps")
    p.add_argument("--copy-probe", action="store_true")
    p.add_argument("--adjoint-only", action="store_true")
    p.add_argument("--runs", type=int, default=5, help="timed runs of K steps; value = median")
    p.add_argument("--full-steps", type=int, default=2000,
                   help="length of the full benchmark run reported beside value (0: skip)")
    args = p.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the PonD step here has no multi-GPU path "
              "(the halo exchange is a design note, not built); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.adjoint_only:
        adjoint_only(args.size)
        return

    w = workloads.riemann2d(args.size, seed=3)
    nodes = args.size * args.size
    if args.kernel_only and args.kernel_precision == "f32":
        cfg32 = make_cfg(w, pond.POND_F32_MIXED)
        log(f"[bench] FP32-mixed {args.size}^2, warmup {args.warmup}, steps {args.steps}")
        ms32, _, _, _ = timed_steps(cfg32, w, args.steps, args.warmup, 1)
        passes = count_passes(cfg32, w, args.steps)
        # rate of the unpacked FP32 FMAs the kernels issue (packed FP32 is compiled out)
        roof = alu_roofline(passes["mean_passes"], nodes, ms32 / args.steps, PEAK_FP64_TFLOPS)
        print(json.dumps({"kernel_only": True, "precision": "f32_mixed",
                          "ms_per_step": ms32 / args.steps,
                          "value": nodes * args.steps / (ms32 * 1e-3) / 1e6, "unit": "MLUPS",
                          "mean_pc_passes": passes["mean_passes"],
                          "flops_per_launch": roof["flops_per_launch"],
                          "achieved_tflops": roof["achieved"], "frac": roof["frac"],
                          "peak_tflops": PEAK_FP64_TFLOPS,
                          "replayed_steps_with_statistics": args.steps}), flush=True)
        return
    cfg64 = make_cfg(w, pond.POND_F64)
    runs = 1 if args.kernel_only else args.runs
    log(f"[bench] FP64 {args.size}^2, warmup {args.warmup}, steps {args.steps}, runs {runs}")
    ms64, s64, s64_prev, times64 = timed_steps(cfg64, w, args.steps, args.warmup, runs)
    mlups64 = nodes * args.steps / (ms64 * 1e-3) / 1e6
    log(f"[bench] FP64 {ms64 / args.steps:.3f} ms/step (median of {runs}), {mlups64:.1f} MLUPS")
    if args.kernel_only:
        # the timed window's pass count comes from a replay with step
        # statistics (the same steps again: a kernel trace holds both)
        passes = count_passes(cfg64, w, args.steps)
        roof = alu_roofline(passes["mean_passes"], nodes, ms64 / args.steps, PEAK_FP64_TFLOPS)
        print(json.dumps({"kernel_only": True, "ms_per_step": ms64 / args.steps,
                          "value": mlups64, "unit": "MLUPS",
                          "mean_pc_passes": passes["mean_passes"],
                          "flops_per_launch": roof["flops_per_launch"],
                          "achieved_tflops": roof["achieved"], "frac": roof["frac"],
                          "replayed_steps_with_statistics": args.steps}), flush=True)
        return

    result = {
        "metric": "PonD MLUPS (D2Q16, 1024^2) FP32 vs FP64 at stated error; adjoint/forward ratio",
        "value": mlups64,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"riemann2d: four-quadrant 2-D Riemann problem, D2Q16, "
                               f"{args.size}x{args.size}, zero-gradient edges, tau 0.55, seed 3, "
                               f"adaptive predictor-corrector (App. E tolerances 1e-12/1e-10, "
                               f"cap 20), {args.steps} steps from the initial state, median of "
                               f"{runs} timed runs",
                   "nx": args.size, "ny": args.size, "parallelism": "single GPU"},
        "run_ms": times64,
    }
    if not args.no_pass_count:
        passes64 = count_passes(cfg64, w, args.steps)
        result["mean_pc_passes"] = passes64["mean_passes"]
        result["nonconverged_node_steps"] = passes64["nonconverged_node_steps"]
        result["cap_hit_fraction"] = passes64["nonconverged_node_steps"] / (nodes * args.steps)
        result["iter_hist_node_steps"] = passes64["iter_hist"]
        traffic = traffic_per_launch(nodes)
        roof = alu_roofline(passes64["mean_passes"], nodes, ms64 / args.steps, PEAK_FP64_TFLOPS)
        roof.update({"traffic": traffic, "kernel": "k_step<4,double,32,16,5>",
                     "flops_per_node_pass": FLOPS_PER_NODE_PASS})
        result["roofline"] = roof
        if traffic:
            gbps = traffic / (ms64 / args.steps * 1e-3) / 1e9
            result["roofline"]["hbm_GBps"] = gbps
            result["roofline"]["hbm_frac"] = gbps / PEAK_HBM_GBPS

    if not args.no_fp32:
        cfg32 = make_cfg(w, pond.POND_F32_MIXED)
        log("[bench] FP32-mixed")
        ms32, s32, _, times32 = timed_steps(cfg32, w, args.steps, args.warmup, runs)
        mlups32 = nodes * args.steps / (ms32 * 1e-3) / 1e6
        log(f"[bench] FP32 {ms32 / args.steps:.3f} ms/step, {mlups32:.1f} MLUPS")
        fp32 = {"value": mlups32, "unit": "MLUPS", "ms_per_step": ms32 / args.steps,
                "run_ms": times32,
                "speedup_vs_fp64": mlups32 / mlups64,
                "error_vs_fp64_at_last_step": field_errors(cfg64, s64, cfg32, s32),
                "tolerances": {"eps_abs": cfg32.eps_abs, "eps_rel": cfg32.eps_rel,
                               "note": "FP32-mixed converges to 1e-6/1e-5 (FP32 resolution), "
                                       "FP64 to 1e-12/1e-10, so FP32 takes fewer passes; "
                                       "speedup_vs_fp64_per_node_pass and "
                                       "speedup_at_equal_passes separate the two effects"}}
        if not args.no_pass_count:
            passes32 = count_passes(cfg32, w, args.steps)
            fp32["mean_pc_passes"] = passes32["mean_passes"]
            fp32["speedup_vs_fp64_per_node_pass"] = (
                mlups32 * passes32["mean_passes"] / (mlups64 * result["mean_pc_passes"]))
            fp32["roofline"] = alu_roofline(passes32["mean_passes"], nodes, ms32 / args.steps,
                                            PEAK_FP64_TFLOPS)
            fp32["roofline"]["frac_vs_packed_fp32_peak"] = (
                fp32["roofline"]["achieved"] / PEAK_FP32_TFLOPS)
            fp32["roofline"]["peak_note"] = (
                "peak = 78.6 TFLOP/s, the unpacked FP32 vector FMA rate the library issues "
                "(packed FP32 is compiled out); frac_vs_packed_fp32_peak uses 157.3")
        log("[bench] FP32 vs FP64 at equal passes; other configs; 2048^2")
        fp32["speedup_at_equal_passes"] = fixed_pass_speedup(w)
        fp32["error_vs_fp64_other_configs"] = fp32_error_other_configs()
        result["fp32_mixed"] = fp32
        if args.full_steps > 0:
            log(f"[bench] full run: {args.full_steps} steps, both precisions")
            result["full_run"] = full_run(w, args.full_steps)
        result["riemann2d_2048"] = riemann_2048()
        log("[bench] D2Q9 Riemann 1024^2")
        result["d2q9_riemann2d_1024"] = riemann_d2q9()

    if not args.no_adjoint:
        log("[bench] adjoint / forward")
        result["adjoint_forward_ratio"] = {
            "riemann2d_1024_fp64_one_step": adjoint_ratio_1024(cfg64, s64_prev),
            "compressible_tgv_128_fp32_200_steps_K20": adjoint_ratio_tgv128(),
        }

    if not args.no_cpu_baseline:
        log("[bench] oracle on host cores")
        result["cpu_baseline"] = cpu_baseline(cfg64, s64, args.cpu_sample)
        result["cpu_baseline"]["single_thread"] = cpu_single_thread(cfg64, s64)
        result["cpu_baseline"]["whole_runs"] = cpu_small_configs()
        result["cpu_baseline"]["host"] = host_cpu()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
