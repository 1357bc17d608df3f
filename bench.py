#!/usr/bin/env python3
"""Benchmark of the LKS + Brinkman forward + adjoint hot path on one MI355X.

Workload: D3Q15, 128^3 analysis grid, 64^3 design grid (+4 margin), 5000 time
steps, body rotating about z (one revolution) with a small translation,
FP32 state with FP64 objective / sensitivity sums, checkpoint every 100 steps.
One benchmark "step" is a whole optimisation-iteration pass: lks_forward
(5000 steps) followed by lks_adjoint (segment recomputation + 5000 reverse
steps + sensitivities), on synthetic seeded inputs resident in HBM.

value = forward+adjoint MLUPS = N * nt / (time per pass) / 1e6.

Also reported: forward-only MLUPS, the roofline object of the dominant kernel
(per-kernel HIP event timing of one extra pass), the FP64 "plain form" run of
the same workload (speedup and the FP32 path's errors against it), and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("forward+adjoint MLUPS & HBM GB/s fraction, D3Q15 128^3, "
          "FP32 vs FP64 at stated grad err")
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_per_node(kind: str, d: int, s: int) -> float:
    """Bytes per node one launch of the kernel must move (body fields and
    target-box reads excluded; they touch a fraction of the nodes).
    fwd_step: read (p, u) + write (p, u) = 2 (d+1) s.
    adj_step: read lambda + write lambda + read u^(n-1) = (2 (d+1) + d) s."""
    if kind == "fwd_step":
        return 2 * (d + 1) * s
    if kind == "adj_step":
        return (2 * (d + 1) + d) * s
    raise ValueError(kind)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernels_d3q15_128_traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2608_01071_amd", "csrc", "lks_kernels.hip")
KERNEL_NAMES = {"fwd_step": "k_fwd3d<float>", "adj_step": "k_adj3d<float>"}


def kernel_source_digest() -> str:
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(kind: str):
    """HBM bytes per launch of the kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy kernel's readings), or
    None when the summary is missing or the kernel source changed since."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        parts = ln.split()
        if len(parts) >= 3 and parts[0] == "traffic":
            kv[parts[1]] = float(parts[2])
        elif len(parts) == 2 and parts[0] == "kernel_source_sha256":
            kv["sha"] = parts[1]
    if kv.get("sha") != kernel_source_digest():
        return None
    return kv.get(KERNEL_NAMES[kind])


def counters_drive():
    """Short workload for hardware-counter passes: 20 steps of the D3Q15 128^3
    forward + adjoint launched eagerly, then a plain 256 MiB device copy whose
    FETCH_SIZE / WRITE_SIZE readings calibrate the counters to bytes."""
    import torch
    from paper_2608_01071_amd import lks, workloads as W
    p, gamma, chi, psi = W.c4(precision=0, nt=20, ckpt_k=10)
    plan = lks.Plan(p)
    plan.set_graphs(False)
    dev = torch.device("cuda")
    g = torch.tensor(gamma, dtype=torch.float64, device=dev)
    c = torch.tensor(chi, dtype=torch.float64, device=dev)
    s = torch.tensor(psi, dtype=torch.float64, device=dev)
    plan.forward(g, c, s)
    plan.adjoint(g, c, s)
    torch.cuda.synchronize()
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[bench] counters drive done: copy of {src.numel() * 4} bytes x3", flush=True)


def c5_batch(nt: int = 4000):
    """The batched parameter study: 16 independent D2Q9 instances (sides
    128..384, Re and filter radius round-robin), FP32, forward + adjoint,
    run as one lks_batch_run call (one captured graph, one launch per kernel
    per step for all instances) and, for comparison, one instance after the
    other."""
    import torch
    from paper_2608_01071_amd import lks, workloads as W
    inst = W.c5_instances(nt=nt)
    ns = sum(p.N for p, *_ in inst) * nt
    G = [x[1] for x in inst]
    C = [x[2] for x in inst]
    S = [x[3] for x in inst]
    b = lks.Batch([lks.Plan(p) for p, *_ in inst])
    b.run(G, C, S)                      # capture + first replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(G, C, S)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    solo = [lks.Plan(p) for p, *_ in inst]
    for pl, (p, g, c, s) in zip(solo, inst):
        pl.forward(g, c, s)
        pl.adjoint(g, c, s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, (p, g, c, s) in zip(solo, inst):
        pl.forward(g, c, s)
        pl.adjoint(g, c, s)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    return {"instances": len(inst), "sides": [p.n[0] for p, *_ in inst], "nt": nt,
            "node_steps": ns, "batch_s": round(tb, 3), "batch_mlups": round(ns / tb / 1e6, 1),
            "sequential_s": round(ts, 3), "sequential_mlups": round(ns / ts / 1e6, 1)}


def fwd_step_out_of_cache(nside: int = 256, nt: int = 12):
    """The forward step on a D3Q15 grid whose state (nside^3 x 4 x 4 B, 268 MB
    at 256^3) exceeds the 256 MB last-level cache: an HBM-resident point for
    the same kernel (event-timed launches of one short forward march)."""
    import torch
    from paper_2608_01071_amd import lks, workloads as W
    p, gamma, chi, psi = W.make_3d(nside, nside // 2, nt, 500, nu=0.04, seed=5, precision=0,
                                   ckpt_k=nt)
    plan = lks.Plan(p)
    plan.forward(gamma, chi, psi)
    torch.cuda.synchronize()
    lks.profile_enable(True)
    plan.forward(gamma, chi, psi)
    torch.cuda.synchronize()
    prof = lks.profile_read()
    lks.profile_enable(False)
    tot_ms, cnt = prof["fwd_step"]
    avg_s = tot_ms / 1e3 / cnt
    bpn = algorithmic_bytes_per_node("fwd_step", 3, 4)
    achieved = p.N * bpn / avg_s / 1e9
    del plan
    torch.cuda.empty_cache()
    return {"workload": f"D3Q15 {nside}^3, {nside // 2}^3 design, FP32, {nt} forward steps",
            "kernel": "fwd_step", "avg_launch_us": round(avg_s * 1e6, 2),
            "algorithmic_bytes": round(p.N * bpn), "achieved": round(achieved, 1),
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "mlups": round(p.N / avg_s / 1e6, 1)}


def oar_j2(nt: int = 4000):
    """The 2D oar workload (objective J2, D2Q9 512^2, 256^2 design, FP32,
    4000 steps, K = 100): forward + adjoint rate with J2 and with J1 on the
    same shape and motion, and the J2 kernels' cost per step (event-timed
    launches of one eager pass)."""
    import torch
    from paper_2608_01071_amd import lks, workloads as W
    p, g, c, s = W.oar(nt=nt)
    seed = torch.ones(1, dtype=torch.float64, device="cuda")
    out = {"workload": "2D oar: D2Q9 512^2 channel, 256^2 design, J2 (w_D 0.01, w_T 0.15), "
                       f"FP32, {nt} steps, K 100"}
    for key, q in (("j2", p), ("j1_same_shape", p.replace(objective=0))):
        plan = lks.Plan(q)
        run_pass(plan, g, c, s, seed)  # warm-up (graph capture)
        J3, grads, tf, ta = run_pass(plan, g, c, s, seed)
        out[key] = {"mlups": round(p.N * nt / (tf + ta) / 1e6, 1),
                    "ms_per_pass": round((tf + ta) * 1e3, 2)}
        if key == "j2":
            out[key]["J_FL_FD"] = [float(v) for v in J3.cpu().numpy()]
            J32 = J3.cpu().numpy().copy()
            g32 = {k: grads[k].cpu().numpy().copy() for k in ("dgamma", "dchi", "dpsi")}
            lks.profile_enable(True)
            run_pass(plan, g, c, s, seed)
            torch.cuda.synchronize()
            prof = lks.profile_read()
            lks.profile_enable(False)
            out["us_per_step"] = {k: round(v[0] * 1e3 / nt, 2) for k, v in prof.items()}
        del plan
        torch.cuda.empty_cache()
    # FP32 state against the FP64 plain form over the whole horizon (J2 is a
    # difference of forces about a thousand times its size; the library's
    # single-precision J2 plans take the 2D transfer's sums in FP64 for it)
    import numpy as np
    plan = lks.Plan(p.replace(precision=1))
    J64, g64, _, _ = run_pass(plan, g, c, s, seed)
    J64 = J64.cpu().numpy()
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    out["fp32_err"] = {"J2": float(abs(J32[0] - J64[0]) / abs(J64[0])),
                       "F_L": float(abs(J32[1] - J64[1]) / abs(J64[1])),
                       "F_D": float(abs(J32[2] - J64[2]) / abs(J64[2])),
                       **{k: rel(g32[k], g64[k].cpu().numpy()) for k in ("dgamma", "dchi", "dpsi")}}
    del plan
    torch.cuda.empty_cache()
    return out


def design_side(plan, g, c, s, reps: int = 20):
    """The optimiser-side calls once per design iteration on the workload's
    design grid: filter + projection (radius 4.8, beta 8, eta 0.5), their
    chain rule, and the three constraints with gradients; event-timed on the
    stream they run on, averaged over `reps` calls."""
    import torch
    ev = lambda: torch.cuda.Event(enable_timing=True)
    gb = torch.ones_like(g)
    out = {"design_points": int(g.numel()), "radius": 4.8, "beta": 8.0, "eta": 0.5}
    calls = {
        "filter_us": lambda: plan.design_filter(g, 4.8, 8.0, 0.5),
        "chain_rule_us": lambda: plan.design_filter_adjoint(g, 4.8, 8.0, 0.5, gb),
        "constraints_us": lambda: plan.constraints(g, c, s, 0.8, 1e-3, 16.0),
    }
    for k, fn in calls.items():
        fn()
        a, b = ev(), ev()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[k] = round(a.elapsed_time(b) * 1e3 / reps, 2)
    return out


def run_pass(plan, g, c, s, seed):
    import torch
    t0 = time.perf_counter()
    J3, _ = plan.forward(g, c, s)          # synchronises at its end (instability check)
    t1 = time.perf_counter()
    grads = plan.adjoint(g, c, s, dJ=seed)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return J3, grads, t1 - t0, t2 - t1


def pass_rate(p, g, c, s, seed, reps: int = 1):
    """Forward and forward + adjoint MLUPS of a plan for problem p (graph
    capture on a first untimed pass)."""
    import torch
    from paper_2608_01071_amd import lks
    plan = lks.Plan(p)
    out = {"workspace_gib": round(plan.workspace_bytes / 2**30, 2)}
    run_pass(plan, g, c, s, seed)
    tf = ta = 0.0
    for _ in range(reps):
        J3, grads, a, b = run_pass(plan, g, c, s, seed)
        tf += a
        ta += b
    tf /= reps
    ta /= reps
    out.update({"forward_mlups": round(p.N * p.nt / tf / 1e6, 1),
                "mlups": round(p.N * p.nt / (tf + ta) / 1e6, 1),
                "ms_per_pass": round((tf + ta) * 1e3, 2)})
    res = (J3.cpu().numpy().copy(), {k: v.cpu().numpy().copy() for k, v in grads.items()
                                     if v is not None})
    del plan
    torch.cuda.empty_cache()
    return out, res


def d2q9_workload(name: str):
    """The D2Q9 workloads at full size: 512^2 x 20000 steps (K = 200) and
    1024^2 x 10000 steps (K = 100), FP32 state with FP64 sums: forward and
    forward + adjoint rates, the dominant kernel's roofline from one
    event-timed pass, and the FP32 errors against the FP64 plain form."""
    import numpy as np
    import torch
    from paper_2608_01071_amd import lks, workloads as W
    p, gamma, chi, psi = (W.c2 if name == "c2" else W.c3)(precision=0)
    dev = torch.device("cuda")
    g = torch.tensor(gamma, dtype=torch.float64, device=dev)
    c = torch.tensor(chi, dtype=torch.float64, device=dev)
    s = torch.tensor(psi, dtype=torch.float64, device=dev)
    seed = torch.ones(1, dtype=torch.float64, device=dev)
    out, (J32, g32) = pass_rate(p, g, c, s, seed)
    out["workload"] = (f"D2Q9 {p.n[0]}^2, {p.m[0]}^2 design, {p.nt} steps, K = {p.ckpt_k}, "
                       "FP32 state / FP64 sums")
    # one segment (K = nt): every state kept in HBM, no recompute
    o1, _ = pass_rate(p.replace(ckpt_k=p.nt), g, c, s, seed)
    out["one_segment"] = {k: o1[k] for k in ("workspace_gib", "forward_mlups", "mlups",
                                              "ms_per_pass")}
    # dominant kernel of one event-timed pass
    plan = lks.Plan(p)
    run_pass(plan, g, c, s, seed)
    lks.profile_enable(True)
    run_pass(plan, g, c, s, seed)
    torch.cuda.synchronize()
    prof = lks.profile_read()
    lks.profile_enable(False)
    del plan
    torch.cuda.empty_cache()
    dom = max(("fwd_step", "adj_step"), key=lambda k: prof.get(k, (0, 0))[0])
    tot_ms, cnt = prof[dom]
    avg_s = tot_ms / 1e3 / cnt
    bpn = algorithmic_bytes_per_node(dom, 2, 4)
    achieved = p.N * bpn / avg_s / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": dom, "avg_launch_us": round(avg_s * 1e6, 2),
                       "achieved": round(achieved, 1), "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4)}
    pass_bytes = 84 * p.N * p.nt  # 84 B per node-step, forward + checkpointed adjoint
    out["pass_roofline"] = {"bytes_per_node_step": 84,
                            "achieved": round(pass_bytes / (out["ms_per_pass"] / 1e3) / 1e9, 1),
                            "frac": round(pass_bytes / (out["ms_per_pass"] / 1e3) / 1e9
                                          / HBM_PEAK_GBS, 4)}
    o64, (J64, g64) = pass_rate(p.replace(precision=1), g, c, s, seed)
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    rms = float(np.sqrt(J64[2] + J64[1] ** 2))
    out["fp64_plain"] = {"mlups": o64["mlups"], "forward_mlups": o64["forward_mlups"],
                         "speedup_fp32": round(o64["ms_per_pass"] / out["ms_per_pass"], 3)}
    out["fp32_err"] = {"J": float(abs(J32[0] - J64[0]) / abs(J64[0])),
                       "J_rel_rms_flux": float(abs(J32[0] - J64[0]) / rms),
                       **{k: rel(g32[k], g64[k]) for k in ("dgamma", "dchi", "dpsi")}}
    return out


def cpu_sample_worker(nt_sample: int, q):
    from oracle import oracle as O
    from paper_2608_01071_amd import workloads as W
    p, gamma, chi, psi = W.c4(nt=nt_sample)
    O.lib()
    t0 = time.perf_counter()
    O.adjoint(p, gamma, chi, psi)
    q.put(time.perf_counter() - t0)


def cpu_all_cores(nt_sample: int, procs: int):
    """The oracle as it stands, one copy per host core (up to `procs`), each
    on the same bounded sample: the host's aggregate oracle throughput."""
    import multiprocessing as mp
    from paper_2608_01071_amd import workloads as W
    p, *_ = W.c4(nt=nt_sample)
    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    ps = [ctx.Process(target=cpu_sample_worker, args=(nt_sample, q)) for _ in range(procs)]
    t0 = time.perf_counter()
    for pr in ps:
        pr.start()
    times = [q.get() for _ in ps]
    for pr in ps:
        pr.join()
    wall = time.perf_counter() - t0
    return {"value": round(procs * p.N * nt_sample / max(times) / 1e6, 3), "unit": "MLUPS",
            "cores": procs, "kind": "oracle",
            "sample": f"{procs} concurrent copies of the single-thread sample "
                      f"(slowest {max(times):.1f} s, wall {wall:.1f} s)"}


def cpu_baseline(nt_sample: int):
    import numpy as np
    from oracle import oracle as O
    from paper_2608_01071_amd import workloads as W
    p, gamma, chi, psi = W.c4(nt=nt_sample)
    O.lib()
    t0 = time.perf_counter()
    O.adjoint(p, gamma, chi, psi)           # includes its own forward march
    dt = time.perf_counter() - t0
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                         model)
    except OSError:
        pass
    return {"value": p.N * nt_sample / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "host": f"{model}, {os.cpu_count()} logical CPUs visible",
            "sample": f"D3Q15 128^3, 64^3 design, first {nt_sample} of 5000 steps, "
                      f"forward + discrete adjoint + sensitivities, FP64, single thread "
                      f"({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=5000, help="time steps (the workload uses 5000)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain-form run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the batched 16-instance study")
    ap.add_argument("--no-alks", action="store_true", help="skip the ALKS reverse-sweep run")
    ap.add_argument("--no-oar", action="store_true", help="skip the 2D oar (J2) run")
    ap.add_argument("--no-design", action="store_true",
                    help="skip timing the design prelude and constraints")
    ap.add_argument("--no-big", action="store_true",
                    help="skip the 256^3 forward-step point (state larger than the LLC)")
    ap.add_argument("--no-store-all", action="store_true",
                    help="skip the one-segment run that keeps every state in HBM")
    ap.add_argument("--no-seg-tape", action="store_true",
                    help="skip the run with the per-segment body tape")
    ap.add_argument("--no-d2q9", action="store_true", help="skip the 512^2 and 1024^2 D2Q9 runs")
    ap.add_argument("--cpu-procs", type=int, default=min(os.cpu_count() or 1, 16),
                    help="concurrent oracle copies for the all-cores baseline (1: none)")
    ap.add_argument("--counters", action="store_true",
                    help="run only the short drive used for hardware-counter passes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; multi-GPU sharding is not "
              "implemented (see the sharding design notes).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2608_01071_amd import lks, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.counters:
        counters_drive()
        return
    p, gamma, chi, psi = W.c4(precision=0, nt=args.nt)
    dev = torch.device("cuda")
    g = torch.tensor(gamma, dtype=torch.float64, device=dev).contiguous()
    c = torch.tensor(chi, dtype=torch.float64, device=dev).contiguous()
    s = torch.tensor(psi, dtype=torch.float64, device=dev).contiguous()
    seed = torch.ones(1, dtype=torch.float64, device=dev)
    # one segment (K = nt), run first while the device is empty: the march
    # keeps every state and body field in HBM (about 230 GB at this size) and
    # the reverse sweep recomputes nothing
    store_all = None
    if not args.no_store_all:
        try:
            o, _ = pass_rate(p.replace(ckpt_k=0), g, c, s, seed)
            store_all = dict(o, bytes_per_node_step=78,
                             note="K = nt: states and body fields of every step kept")
        except Exception as e:  # the device may not hold it
            store_all = {"skipped": str(e)[:200]}
        torch.cuda.empty_cache()
        print(f"[bench] one-segment run: {store_all}", file=sys.stderr, flush=True)
    plan = lks.Plan(p)
    print(f"[bench] workload D3Q15 {p.n} design {p.m} nt={p.nt} K={p.ckpt_k} "
          f"workspace {plan.workspace_bytes / 2**30:.2f} GiB", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        _, _, tf, ta = run_pass(plan, g, c, s, seed)
        print(f"[bench] warmup {w}: fwd {tf:.3f}s adj {ta:.3f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tf_sum = ta_sum = 0.0
    t0 = time.perf_counter()
    for k in range(args.steps):
        J3, grads, tf, ta = run_pass(plan, g, c, s, seed)
        tf_sum += tf
        ta_sum += ta
        print(f"[bench] step {k}: fwd {tf:.3f}s adj {ta:.3f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    N, nt = p.N, p.nt
    value = N * nt / (elapsed / args.steps) / 1e6
    fwd_mlups = N * nt / (tf_sum / args.steps) / 1e6
    J32 = J3.cpu().numpy().copy()
    g32 = {k: v.cpu().numpy().copy() for k, v in grads.items() if v is not None}

    # per-kernel event timing of one more pass (the dominant kernel's roofline)
    roofline = None
    kernels = {}
    if not args.no_profile:
        lks.profile_enable(True)
        run_pass(plan, g, c, s, seed)
        torch.cuda.synchronize()
        prof = lks.profile_read()
        lks.profile_enable(False)
        kernels = {k: {"total_ms": v[0], "launches": v[1], "avg_us": 1e3 * v[0] / max(v[1], 1)}
                   for k, v in prof.items()}
        dom = max(("fwd_step", "adj_step"), key=lambda k: prof.get(k, (0, 0))[0])
        tot_ms, cnt = prof[dom]
        avg_s = tot_ms / 1e3 / cnt
        bpn = algorithmic_bytes_per_node(dom, p.d, 4)
        achieved = N * bpn / avg_s / 1e9
        tr = measured_traffic(dom)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None if tr is None else round(tr),
                    "algorithmic_bytes": round(N * bpn), "bytes_per_node": bpn,
                    "avg_launch_us": round(avg_s * 1e6, 2)}

    fp64 = None
    if not args.no_fp64:
        p64 = p.replace(precision=1)
        plan64 = lks.Plan(p64)
        run_pass(plan64, g, c, s, seed)  # warm-up
        J3d, gd, tf64, ta64 = run_pass(plan64, g, c, s, seed)
        J64 = J3d.cpu().numpy()
        rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        fp64 = {"ms_per_step": round((tf64 + ta64) * 1e3, 2),
                "value": round(N * nt / (tf64 + ta64) / 1e6, 2),
                "speedup_fp32": round((tf64 + ta64) / (elapsed / args.steps), 3),
                "fp32_err": {"J": float(abs(J32[0] - J64[0]) / max(abs(J64[0]), 1e-300)),
                             "dgamma": rel(g32["dgamma"], gd["dgamma"].cpu().numpy()),
                             "dchi": rel(g32["dchi"], gd["dchi"].cpu().numpy()),
                             "dpsi": rel(g32["dpsi"], gd["dpsi"].cpu().numpy())}}
        del plan64
        torch.cuda.empty_cache()

    alks = None
    if not args.no_alks:
        # the paper's ALKS reverse sweep on the same workload: its rate, and
        # how far its gradient lies from the exact one
        plan_a = lks.Plan(p.replace(scheme=1))
        run_pass(plan_a, g, c, s, seed)  # warm-up (graph capture)
        _, ga, tfa, taa = run_pass(plan_a, g, c, s, seed)
        rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        alks = {"value": round(N * nt / (tfa + taa) / 1e6, 2), "unit": "MLUPS",
                "ms_per_pass": round((tfa + taa) * 1e3, 2),
                "adjoint_ms": round(taa * 1e3, 2),
                "rel_to_exact_gradient": {k: rel(ga[k].cpu().numpy(), g32[k])
                                          for k in ("dgamma", "dchi", "dpsi")}}
        del plan_a
        torch.cuda.empty_cache()

    design = None if args.no_design else design_side(plan, g, c, s)

    del plan
    torch.cuda.empty_cache()
    seg_tape = None
    if not args.no_seg_tape:
        o, _ = pass_rate(p.replace(body_tape=-1), g, c, s, seed)
        seg_tape = dict(o, note="body fields of one segment kept; the recompute maps again")
    big = None if args.no_big else fwd_step_out_of_cache()
    c5 = None if args.no_c5 else c5_batch()
    oar = None if args.no_oar else oar_j2()
    d2 = {} if args.no_d2q9 else {k: d2q9_workload(k) for k in ("c2", "c3")}
    cpu = None if args.no_cpu else cpu_baseline(args.cpu_steps)
    cpu_all = None if (args.no_cpu or args.cpu_procs <= 1) else cpu_all_cores(args.cpu_steps,
                                                                              args.cpu_procs)
    pass_bytes = 110 * N * nt  # 110 B per node-step, forward + checkpointed adjoint
    pass_roofline = {"bytes_per_node_step": 110,
                     "achieved": round(pass_bytes / (ms_per_step / 1e3) / 1e9, 1),
                     "unit": "GB/s", "peak": HBM_PEAK_GBS,
                     "frac": round(pass_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "D3Q15 LKS 128^3, 64^3 design, 5000 steps, z-rotation, "
                               "FP32 state / FP64 sums, forward+adjoint, checkpoint K=100",
                   "nt": nt, "nodes": N, "ckpt_k": p.ckpt_k},
        "forward_mlups": round(fwd_mlups, 2),
        "J": float(J32[0]),
        "roofline": roofline,
        "pass_roofline": pass_roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "store_all": store_all,
        "segment_body_tape": seg_tape,
        "d2q9_512": d2.get("c2"),
        "d2q9_1024": d2.get("c3"),
        "fp64_plain": fp64,
        "alks": alks,
        "design_side": design,
        "c5_batch": c5,
        "oar_j2": oar,
        "fwd_step_256": big,
        "kernels": kernels,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
