#!/usr/bin/env python3
"""Benchmark of the direct-sum n-body hot path on one MI355X.

Workload (the throughput headline): two colliding Plummer spheres,
N = 2^20 = 1,048,576 bodies, mass ratio 1:3, centres (+-2, 0, 0), relative
speed 0.3, eps = 0.005, FP32 pair arithmetic with FP64 sums across source
tiles (NBODY_F32_F64ACC), leapfrog KDK with dt = 5e-4.  Synthetic inputs,
seeded, resident in HBM before the timed region.

One step = one force + potential evaluation over all N^2 pairs (nbody_accel)
plus the elementwise kick/drift pass (nbody_kick_drift), i.e. one KDK step.
value = N^2 / (seconds per step) / 1e9 = G-interactions/s.

Also reported on the same JSON line:
* roofline: the force kernel (VALU-bound, 20 flop per pair) against the
  MI355X FP32 vector peak, from HIP events around every force launch of the
  timed region;
* cpu_baseline: the FP64 oracle on a bounded sample of targets of the same
  workload, on the host cores, and the GPU's error against it;
* adjoint: forward+adjoint time / plain forward time for the differentiation
  workload (Plummer N = 16384, 200 steps, checkpoints every 20), and the same
  ratio for the bit-reversible fixed-point leapfrog (no checkpoints);
* batched: aggregate G-interactions/s for 512 ragged Plummer systems, 50
  steps captured in one HIP graph;
* tree: the tree code on the ORB cells of the same colliding pair with the
  four cell models (monopole, pseudo-particle, quadrupole, group local
  expansions) at theta 0.5, 0.7, 1.0: time, work and error against the exact
  sum;
* shard: one GPU's share of an 8-way target split (131072 x 1048576).
* modes: pure FP32 and Kahan-compensated FP32 sums on the same workload at
  step 0, each with its time and its error against the oracle sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (AMD), packed FP32 counted
FLOP_PER_PAIR = 20
VARIANTS = {0: "scalar-load sources", 1: "LDS sources"}
VARIANT_KERNELS = {0: "k_accel_f32", 1: "k_accel_lds_f32"}
FLOP_PER_QUAD_CELL = 54   # one quadrupole cell against one target, counted like the pair's 20
FLOP_PER_M2L = 313        # one cell folded into a group's third-order local expansion (m2l_f32)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extras", action="store_true", help="skip adjoint, batched and CPU legs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tree-counters", action="store_true",
                    help="two tree evaluations (theta 0.7, leaf 8) of the workload for counter runs")
    ap.add_argument("--tree-cells", action="store_true",
                    help="two tree evaluations (theta 0.7, leaf 4) per cell model for trace and counter runs")
    ap.add_argument("--fmm", action="store_true",
                    help="two multi-level FMM evaluations (theta 0.5, leaf 8) of the workload for trace runs")
    ap.add_argument("--adjoint", action="store_true",
                    help="the adjoint leg alone (plain, checkpointed and fixed-point), for trace runs")
    ap.add_argument("--counters", action="store_true",
                    help="counter-collection mode: two force launches of the headline workload "
                         "and one 1 GiB device copy (the copy calibrates byte counters); no JSON")
    ap.add_argument("--counters-variant", type=int, default=0, choices=(0, 1),
                    help="with --counters: 0 = the default kernel shape, 1 = sources staged in LDS "
                         "(2 targets per lane, 8 source splits, tiles of 512)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU target sharding is designed, not built)"}))
        sys.exit(2)

    import torch
    import ics
    import paper_1211_2292_amd as nb

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    nb.lib()
    dev = torch.device("cuda:0")
    w = ics.WORKLOADS["collide1m"]
    n, eps, dt = w["n"], w["eps"], w["dt"]
    prec = nb.F32_F64ACC
    log(f"[bench] generating colliding pair N={n}")
    pm_np, v_np = ics.colliding_pair(n, w["seed"])
    pm = torch.as_tensor(pm_np, dtype=torch.float32).to(dev).contiguous()
    vel = torch.as_tensor(v_np, dtype=torch.float32).to(dev).contiguous()
    acc = torch.empty_like(pm)
    pm0_host = pm.cpu().double().numpy()

    if args.counters:
        if args.counters_variant == 1:
            nb.set_tuning(0, prec, 2, 8, 512, 1)
        for _ in range(2):
            nb.accel(pm, eps, prec=prec, out=acc)
        nb.set_tuning(0, prec)
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] counters mode: 2 force launches (variant {args.counters_variant}), "
            "1 GiB copy (1073741824 B read + written)")
        return

    if args.tree_counters:
        q = nb.permute(pm, nb.orb_order(pm, 8))
        out = torch.empty_like(q)
        for _ in range(2):
            nb.tree_accel(q, eps, 0.7, 8, prec=prec, out=out)
        torch.cuda.synchronize()
        log("[bench] tree counters mode: 2 tree evaluations, theta 0.7, leaf 8, F32_F64ACC")
        return

    if args.adjoint:
        print(json.dumps(adjoint_leg(torch, nb, ics, dev)))
        return

    if args.fmm:
        q = nb.permute(pm, nb.orb_order(pm, 8))
        out = torch.empty_like(q)
        for _ in range(2):
            nb.fmm_accel(q, eps, 0.5, 8, prec=prec, out=out)
        torch.cuda.synchronize()
        log("[bench] fmm mode: 2 evaluations, theta 0.5, leaf 8, F32_F64ACC")
        return

    if args.tree_cells:
        q = nb.permute(pm, nb.orb_order(pm, 4))
        out = torch.empty_like(q)
        for cells in (nb.CELLS_MONOPOLE, nb.CELLS_PSEUDO, nb.CELLS_QUADRUPOLE, nb.CELLS_LOCAL):
            for _ in range(2):
                nb.tree_accel(q, eps, 0.7, 4, prec=prec, out=out, cells=cells)
        torch.cuda.synchronize()
        log("[bench] tree cells mode: 2 evaluations per cell model (0, 2, 3, 4), theta 0.7, leaf 4, F32_F64ACC")
        return

    # ORB body order (the paper's recursive bisection, used as an ordering):
    # the first call also allocates the library's ORB buffers and stages its
    # tables; a second call of the same shape is timed as well, then the
    # state is gathered into that order
    e_a, e_b, e_c, e_d = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    torch.cuda.synchronize()
    e_d.record()
    nb.orb_order(pm, 256)
    e_a.record()
    perm = nb.orb_order(pm, 256)
    e_b.record()
    pm = nb.permute(pm, perm)
    vel = nb.permute(vel, perm)
    e_c.record()
    torch.cuda.synchronize()
    orb_first_ms = e_d.elapsed_time(e_a)
    orb_ms, gather_ms = e_a.elapsed_time(e_b), e_b.elapsed_time(e_c)
    perm_host = perm.cpu().numpy()
    log(f"[bench] ORB order {orb_ms:.2f} ms (first call {orb_first_ms:.2f} ms), gather {gather_ms:.3f} ms")

    # first evaluation (step 0 forces, kept for the accuracy check, returned
    # to the input order)
    nb.accel(pm, eps, prec=prec, out=acc)
    torch.cuda.synchronize()
    acc0 = np.empty((n, 4))
    acc0[perm_host] = acc.cpu().double().numpy()
    modes = {} if args.no_extras else modes_leg(torch, nb, pm, eps, perm_host)
    energy0 = nb.energy(pm, vel, acc, prec=prec).cpu().numpy()
    h = 0.5 * dt
    nb.kick_drift(pm, vel, acc, h, dt, close=False, open=True, prec=prec)

    def step(e0=None, e1=None):
        if e0 is not None:
            e0.record()
        nb.accel(pm, eps, prec=prec, out=acc)
        if e1 is not None:
            e1.record()
        nb.kick_drift(pm, vel, acc, h, dt, close=True, open=True, prec=prec)

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record()
    for k in range(args.steps):
        step(*ev[k])
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)
    # FP64 energy at the final synchronised state: the loop leaves
    # (x_{m+1}, v_{m+1/2}); one more force and a closing half kick give v_{m+1}
    nb.accel(pm, eps, prec=prec, out=acc)
    nb.kick_drift(pm, vel, acc, h, dt, close=True, open=False, prec=prec)
    energy1 = nb.energy(pm, vel, acc, prec=prec).cpu().numpy()
    torch.cuda.synchronize()
    ms_per_step = total_ms / args.steps
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    kern_avg = float(np.mean(kern_ms))
    pairs = float(n) * float(n)
    value = pairs / (ms_per_step * 1e-3) / 1e9
    achieved = FLOP_PER_PAIR * pairs / (kern_avg * 1e-3) / 1e12
    tune = nb.get_tuning(0, prec, n)
    log(f"[bench] {ms_per_step:.2f} ms/step, force kernel {kern_avg:.2f} ms, {value:.1f} Gint/s, "
        f"{achieved:.2f} TFLOP/s ({100 * achieved / PEAK_FP32_TFLOPS:.1f}% of FP32 peak), tune {tune}")

    result = {
        "metric": "G-interactions/s and % FP32 peak at N=1M; fwd+adjoint step time vs plain fwd",
        "value": round(value, 2),
        "unit": "G-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair arithmetic, f64 cross-tile sums",
        "data": "synthetic (seeded colliding Plummer spheres)",
        "config": {"workload": "colliding Plummer pair, N=1048576, mass ratio 1:3, eps=0.005, "
                               "dt=5e-4, leapfrog KDK, NBODY_F32_F64ACC",
                   "n": n, "eps": eps, "dt": dt, "precision": "F32_F64ACC",
                   "kernel_shape": {"tpl": tune[0], "jsplit": tune[1], "jtile": tune[2],
                                    "variant": VARIANTS.get(tune[3], str(tune[3]))}},
        "pct_fp32_peak": round(100 * achieved / PEAK_FP32_TFLOPS, 2),
        "wall_s_timed": round(wall, 3),
        "orb": {"leaf": 256, "order_ms": round(orb_ms, 3), "first_call_ms": round(orb_first_ms, 3),
                "gather_ms": round(gather_ms, 3)},
        "energy_fp64": {"E0": float(energy0.sum()), "E_end": float(energy1.sum()),
                        "rel_change": float(energy1.sum() / energy0.sum() - 1.0),
                        "steps": args.steps + args.warmup + 1},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": measured_traffic(tune, n),
                     "kernel": VARIANT_KERNELS.get(tune[3], "k_accel_f32") + f"<{tune[0]}, F64ACC>",
                     "flop_per_pair": FLOP_PER_PAIR,
                     "avg_launch_ms": round(kern_avg, 4),
                     "launch_ms_std": round(float(np.std(kern_ms)), 4),
                     "launch_ms_min_max": [round(float(np.min(kern_ms)), 4), round(float(np.max(kern_ms)), 4)]},
    }

    if not args.no_extras:
        result["fp64"] = fp64_leg(torch, nb, ics, dev)
        result["adjoint"] = adjoint_leg(torch, nb, ics, dev)
        result["batched"] = batched_leg(torch, nb, ics, dev)
        result["tree"] = tree_leg(torch, nb, pm_np, eps, kern_avg, v_np=v_np, dt=dt)
        result["fmm"] = fmm_leg(torch, nb, pm_np, eps, kern_avg)
        result["shard"] = shard_leg(torch, nb, pm, eps, prec)
        result["cpu_baseline"] = cpu_leg(ics, pm0_host, acc0, eps, args.cpu_seconds, modes)
        result["modes"] = modes
    print(json.dumps(result), flush=True)


def force_source_sha1():
    """SHA-1 of the sources the force kernel is compiled from."""
    import hashlib
    h = hashlib.sha1()
    for f in ("accel.hip", "pair.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_1211_2292_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(tune, n):
    """HBM bytes per force launch from the committed rocprofv3 counter
    summary, if it was taken on the kernel shape in use now and on the same
    kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "k_accel_f32_collide1m_pmc.md")
    try:
        sha = force_source_sha1()
        for line in open(path):
            if line.startswith("traffic_record:"):
                rec = json.loads(line.split(":", 1)[1])
                if rec["shape"] == list(tune) and rec["n"] == n and rec.get("src_sha1") == sha:
                    return rec["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def fp64_leg(torch, nb, ics, dev):
    """FP64 force evaluation (FP64 pair arithmetic and sums) on a Plummer
    sphere of 2^17 bodies."""
    n = 1 << 17
    pm_np, _ = ics.plummer(n, 1006)
    p = torch.as_tensor(pm_np, dtype=torch.float64, device=dev).contiguous()
    out = torch.empty_like(p)
    nb.accel(p, 0.01, out=out)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        nb.accel(p, 0.01, out=out)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ms = float(np.median(ts))
    g = float(n) * n / (ms * 1e-3) / 1e9
    log(f"[bench] fp64: {ms:.2f} ms per evaluation at N={n}, {g:.1f} Gint/s")
    return {"workload": "Plummer N=131072, NBODY_F64, eps=0.01", "ms": round(ms, 3),
            "g_interactions_per_s": round(g, 2), "shape": list(nb.get_tuning(0, nb.F64, n))}


def adjoint_leg(torch, nb, ics, dev):
    """Plummer N = 16384, FP32 + Kahan, 200 steps, dt = 1e-3, checkpoints
    every 20: [forward with checkpoints + adjoint] / [plain forward]."""
    w = ics.WORKLOADS["adjoint16384"]
    n, eps, dt, steps, C = w["n"], w["eps"], w["dt"], w["steps"], w["ckpt"]
    log(f"[bench] adjoint leg N={n}, {steps} steps")
    pm_np, v_np = ics.plummer(n, w["seed"])
    y = torch.as_tensor(ics.perturbed_snapshot(pm_np, w["seed"] + 2), dtype=torch.float32, device=dev)
    p0 = torch.as_tensor(pm_np, dtype=torch.float32, device=dev).contiguous()
    v0 = torch.as_tensor(v_np, dtype=torch.float32, device=dev).contiguous()
    prec = nb.F32_KAHAN

    def plain():
        p, v = p0.clone(), v0.clone()
        a = torch.empty_like(p)
        nb.leapfrog_kdk(p, v, a, eps, dt, steps, prec=prec)
        return p

    def fwd_adj(scheme):
        def run():
            p, v = p0.clone(), v0.clone()
            ck = nb.trajectory_forward(p, v, eps, dt, steps, C, prec=prec)
            xb = torch.zeros_like(p)
            xb[:, :3] = 2 * (p[:, :3] - y)
            vb = torch.zeros_like(p)
            return nb.trajectory_adjoint(ck, eps, dt, steps, C, xb, vb, prec=prec, scheme=scheme)
        return run

    def fwd_adj_energy():
        # loss = final energy 1/2 sum m |v_T|^2 + 1/2 sum m phi(x_T): the
        # cotangents are m v_T on the velocities and m / 2 on the final potential
        p, v = p0.clone(), v0.clone()
        ck = nb.trajectory_forward(p, v, eps, dt, steps, C, prec=prec)
        m = p[:, 3]
        vb = torch.zeros_like(p)
        vb[:, :3] = m[:, None] * v[:, :3]
        return nb.trajectory_adjoint(ck, eps, dt, steps, C, torch.zeros_like(p), vb, prec=prec,
                                     scheme=nb.ADJ_REVERSE, phibar_T=0.5 * m)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    # the fixed-point, bit-reversible leapfrog sums in FP32 + FP64 partials:
    # its ratio is taken against the plain leapfrog in that mode
    def plain64():
        p, v = p0.clone(), v0.clone()
        a = torch.empty_like(p)
        nb.leapfrog_kdk(p, v, a, eps, dt, steps, prec=nb.F32_F64ACC)
        return p

    def janus_fwd():
        return nb.janus_forward(p0, v0, eps, dt, steps)

    def janus_fwd_adj():
        st, pT, _ = nb.janus_forward(p0, v0, eps, dt, steps)
        xb = torch.zeros_like(pT)
        xb[:, :3] = 2 * (pT[:, :3] - y)
        return nb.janus_adjoint(st, p0, eps, dt, steps, xb, torch.zeros_like(pT))

    t_plain = timed(plain)
    t_rev = timed(fwd_adj(nb.ADJ_REVERSE))
    t_rec = timed(fwd_adj(nb.ADJ_RECOMPUTE))
    t_plain64 = timed(plain64)
    t_jf = timed(janus_fwd)
    t_ja = timed(janus_fwd_adj)
    t_en = timed(fwd_adj_energy)
    log(f"[bench] adjoint: plain {t_plain:.1f} ms, fwd+adj reversal {t_rev:.1f} ms "
        f"(ratio {t_rev / t_plain:.2f}), recompute {t_rec:.1f} ms (ratio {t_rec / t_plain:.2f})")
    log(f"[bench] fixed-point: plain F32_F64ACC {t_plain64:.1f} ms, forward {t_jf:.1f} ms, "
        f"fwd+adj {t_ja:.1f} ms (ratio {t_ja / t_plain64:.2f})")
    return {"workload": "Plummer N=16384, F32_KAHAN, 200 steps dt=1e-3, checkpoints every 20",
            "plain_forward_ms": round(t_plain, 3),
            "fwd_plus_adjoint_ms": round(t_rev, 3), "ratio": round(t_rev / t_plain, 3),
            "scheme": "time reversal re-anchored at checkpoints (fused force+VJP)",
            "recompute_scheme_ms": round(t_rec, 3), "recompute_scheme_ratio": round(t_rec / t_plain, 3),
            "energy_loss": {"loss": "final energy 1/2 sum m v^2 + 1/2 sum m phi (cotangent on the final potential)",
                            "fwd_plus_adjoint_ms": round(t_en, 3), "ratio": round(t_en / t_plain, 3)},
            "fixed_point": {"prec": "F32_F64ACC", "plain_forward_ms": round(t_plain64, 3),
                            "forward_ms": round(t_jf, 3), "fwd_plus_adjoint_ms": round(t_ja, 3),
                            "ratio": round(t_ja / t_plain64, 3), "checkpoints": 0}}


def batched_leg(torch, nb, ics, dev):
    """512 Plummer systems, N_s log-uniform in [256, 32768], FP32 + Kahan,
    50 KDK steps dt = 1e-3 captured in one HIP graph, with the batched
    kernel's tile shape chosen by the library's autotuner (the default shape
    is timed beside it)."""
    w = ics.WORKLOADS["batch512"]
    log("[bench] batched leg: generating 512 systems")
    pm_np, v_np, off = ics.ragged_batch(w["nsys"], w["seed"])
    p0 = torch.as_tensor(pm_np, dtype=torch.float32, device=dev).contiguous()
    v0 = torch.as_tensor(v_np, dtype=torch.float32, device=dev).contiguous()
    p, v = p0.clone(), v0.clone()
    a = torch.empty_like(p)
    steps = w["steps"]
    ntot = int(off[-1])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def graph_steps():
        # same initial state for every timing; the warm-up call captures the
        # graph with the flags of the timed call, so the timed call replays
        for timed in (False, True):
            p.copy_(p0)
            v.copy_(v0)
            nb.leapfrog_kdk(p, v, a, w["eps"], w["dt"], 0, offsets=off)
            torch.cuda.synchronize()
            if timed:
                e0.record()
            nb.leapfrog_kdk(p, v, a, w["eps"], w["dt"], steps, offsets=off, graph=True, acc_valid=True)
            if timed:
                e1.record()
            torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    default_shape = nb.get_tuning(1, nb.F32_KAHAN, ntot)
    ms_default = graph_steps()
    nb.autotune(1, nb.F32_KAHAN, ntot, offsets=off)
    tuned_shape = nb.get_tuning(1, nb.F32_KAHAN, ntot)
    ms = graph_steps()
    sizes = np.diff(off).astype(np.float64)
    pairs = float((sizes ** 2).sum()) * steps
    gint = pairs / (ms * 1e-3) / 1e9
    # (ii) the same 50 steps launched eagerly, without the graph
    e0.record()
    nb.leapfrog_kdk(p, v, a, w["eps"], w["dt"], steps, offsets=off, graph=False, acc_valid=True)
    e1.record()
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1)
    # (i) one force evaluation as a loop of one launch per system (forces only,
    # the batched launch timed the same way for the comparison)
    sl = [(int(off[k]), int(off[k + 1])) for k in range(len(off) - 1)]
    views = [(p[b:e], a[b:e]) for b, e in sl]
    for pv, av in views[:4]:
        nb.accel(pv, w["eps"], prec=nb.F32_KAHAN, out=av)
    torch.cuda.synchronize()
    e0.record()
    for pv, av in views:
        nb.accel(pv, w["eps"], prec=nb.F32_KAHAN, out=av)
    e1.record()
    torch.cuda.synchronize()
    ms_loop = e0.elapsed_time(e1)
    nb.batched_accel(p, off, w["eps"], prec=nb.F32_KAHAN, out=a)
    torch.cuda.synchronize()
    e0.record()
    nb.batched_accel(p, off, w["eps"], prec=nb.F32_KAHAN, out=a)
    e1.record()
    torch.cuda.synchronize()
    ms_one = e0.elapsed_time(e1)
    log(f"[bench] batched: {ms:.1f} ms for {steps} steps in one graph ({gint:.1f} Gint/s) with the tuned shape "
        f"{tuned_shape[:3]}, {ms_default:.1f} ms with the default {default_shape[:3]}, eager {ms_eager:.1f} ms; "
        f"one evaluation: batched launch {ms_one:.2f} ms, loop of {len(sl)} launches {ms_loop:.2f} ms")
    shape = lambda t: {"tpl": t[0], "jtile": t[2]}
    return {"workload": "512 Plummer systems, N_s log-uniform [256, 32768], F32_KAHAN, 50 steps in one graph",
            "bodies": int(off[-1]), "ms": round(ms, 3), "g_interactions_per_s": round(gint, 2),
            "tuned_shape": shape(tuned_shape), "default_shape": shape(default_shape),
            "default_ms": round(ms_default, 3),
            "eager_50_steps_ms": round(ms_eager, 3),
            "one_evaluation_batched_ms": round(ms_one, 3),
            "one_evaluation_loop_of_launches_ms": round(ms_loop, 3)}


def shard_leg(torch, nb, pm, eps, prec):
    """One GPU's share of an 8-way target split of the same workload: 131072
    targets (the middle eighth of the ORB order) against all 2^20 sources,
    the call a multi-GPU run would make on each rank."""
    n = pm.shape[0]
    cnt = n // 8
    beg = 3 * cnt
    out = torch.empty((cnt, 4), dtype=pm.dtype, device=pm.device)
    nb.accel(pm, eps, prec=prec, out=out, target_begin=beg, target_count=cnt)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        nb.accel(pm, eps, prec=prec, out=out, target_begin=beg, target_count=cnt)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    t = float(np.mean(ts))
    gint = float(cnt) * n / (t * 1e-3) / 1e9
    log(f"[bench] shard: {cnt} x {n} in {t:.2f} ms, {gint:.1f} Gint/s")
    return {"workload": f"{cnt} targets x {n} sources (one of 8 target shards), F32_F64ACC",
            "ms": round(t, 3), "g_interactions_per_s": round(gint, 2),
            "tune_jsplit_rule": "source splits sized by the target count (32 here)"}


def _tree_groups(nodes, group):
    """(begin, end) of the groups: the maximal nodes of at most `group`
    bodies, in ORB order (node table rows: begin, end, left, right)."""
    out, stack = [], [0]
    while stack:
        k = stack.pop()
        b, e, l, r = nodes[k]
        if e - b <= group or l < 0:
            out.append((b, e))
        else:
            stack.extend((r, l))
    return out


def fmm_leg(torch, nb, pm_np, eps, direct_ms, fmm_args=None):
    """Multi-level FMM on the ORB nodes for the same colliding pair at step 0
    (F32_F64ACC): time per evaluation (ORB order excluded, as in the tree
    leg), list sizes, flop rate and the error against the exact direct sum on
    the same ordered input, per leaf size and theta."""
    dev = torch.device("cuda:0")
    n = pm_np.shape[0]
    p = torch.as_tensor(pm_np, dtype=torch.float32, device=dev).contiguous()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {"workload": "colliding Plummer pair, N=1048576, eps=0.005, step 0, F32_F64ACC; quadrupole cells, "
                       "third-order local expansions, L2L, M2P cells and leaf-leaf P2P at the leaves", "runs": {}}
    for leaf, thetas in (fmm_args or ((8, (0.4, 0.5, 0.6, 0.7, 0.8)), (16, (0.4, 0.5)))):
        q = nb.permute(p, nb.orb_order(p, leaf))
        direct = nb.accel(q, eps, prec=nb.F32_F64ACC).cpu().double().numpy()
        _, _, nodes = nb.tree_shape(n, leaf, nodes=True)
        size = (nodes[:, 1] - nodes[:, 0]).astype(np.float64)
        out = torch.empty_like(q)
        for theta in thetas:
            nb.fmm_accel(q, eps, theta, leaf, out=out)  # sizes the list buffers
            torch.cuda.synchronize()
            ts = []
            for _ in range(5):
                e0.record()
                nb.fmm_accel(q, eps, theta, leaf, out=out)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            t = float(np.mean(ts))
            got = out.cpu().double().numpy()
            rel = np.linalg.norm(got[:, :3] - direct[:, :3], axis=1) / np.linalg.norm(direct[:, :3], axis=1)
            mc, cc, pc, _, m2p, p2p = (x.cpu().numpy().astype(np.int64) for x in nb.fmm_lists(q, theta, leaf))
            tgt = np.repeat(np.arange(nodes.shape[0]), pc)
            pairs = float((size[tgt] * size[p2p]).sum())
            cells = float((size * cc).sum())  # M2P: one quadrupole cell per body of the target leaf
            flops = FLOP_PER_PAIR * pairs + FLOP_PER_M2L * float(mc.sum()) + FLOP_PER_QUAD_CELL * cells
            r = {"ms": round(t, 4), "ms_std": round(float(np.std(ts)), 4),
                 "m2l_per_node": round(float(mc.sum()) / nodes.shape[0], 1),
                 "m2p_cells_per_body": round(cells / n, 1),
                 "p2p_interactions_per_body": round(pairs / n, 1),
                 "gflop": round(flops / 1e9, 2), "tflops": round(flops / (t * 1e-3) / 1e12, 2),
                 "speedup_vs_direct_kernel": round(direct_ms / t, 1),
                 "rms_rel_err_vs_direct": float(np.sqrt(np.mean(rel ** 2))), "max_rel_err_vs_direct": float(rel.max())}
            res["runs"][f"leaf{leaf}_theta{theta}"] = r
            log(f"[bench] fmm leaf {leaf} theta {theta}: {t:.3f} ms, {r['m2l_per_node']} M2L/node, "
                f"{r['p2p_interactions_per_body']:.0f} P2P/body, {r['tflops']} TFLOP/s, rms err {r['rms_rel_err_vs_direct']:.2e}")
    return res


def tree_leg(torch, nb, pm_np, eps, direct_ms, leaf=4, v_np=None, dt=5e-4):
    """Tree code on the ORB cells (leaf 4, groups of 64) for the same
    colliding pair at step 0, FP32 pairs with FP64 batch sums: time per
    evaluation, interactions per body, and the error against the exact direct
    sum computed by the direct kernel on the same ordered input; then the
    tree leapfrog (10 steps, re-ordered by ORB every 10) per cell model."""
    import ctypes
    dev = torch.device("cuda:0")
    n = pm_np.shape[0]
    p = torch.as_tensor(pm_np, dtype=torch.float32, device=dev).contiguous()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    perm = nb.orb_order(p, leaf)
    q = nb.permute(p, perm)
    e1.record()
    torch.cuda.synchronize()
    orb_ms = e0.elapsed_time(e1)
    direct = nb.accel(q, eps, prec=nb.F32_F64ACC)
    torch.cuda.synchronize()
    d_host = direct.cpu().double().numpy()
    _, _, nodes = nb.tree_shape(n, leaf, nodes=True)
    nodes = nodes.astype(np.int64)
    groups = _tree_groups(nodes, nb.TREE_GROUP)
    gsz = np.array([e - b for b, e in groups], dtype=np.float64)
    L = nb.lib()
    out = torch.empty_like(q)
    res = {"workload": f"colliding Plummer pair, N=1048576, eps=0.005, step 0, ORB leaf {leaf}, groups of 64, "
                       "F32_F64ACC", "leaf": leaf, "orb_plus_gather_ms": round(orb_ms, 3), "theta": {}}
    reps = 10
    nn = nodes.shape[0]
    pseudo = torch.empty((nn, nb.TREE_PSEUDO, 4), dtype=torch.float32, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    quad = torch.empty((nn, 3, 4), dtype=torch.float32, device=dev)
    res["pseudo_cells"], res["quadrupole_cells"], res["local_cells"] = {}, {}, {}

    def moments_only(cells):
        # monopole moments; for the other models also the second moments and
        # the cells' records (plus their export copy, <= 0.02 ms at 2^20)
        if cells == nb.CELLS_MONOPOLE:
            return L.nbody_tree_moments(ctypes.c_void_p(q.data_ptr()), n, leaf, None, None, stream)
        if cells == nb.CELLS_PSEUDO:
            return L.nbody_tree_pseudo(ctypes.c_void_p(q.data_ptr()), n, leaf,
                                       ctypes.c_void_p(pseudo.data_ptr()), stream)
        # quadrupole records serve both the quadrupole and the local-expansion cells
        return L.nbody_tree_quad(ctypes.c_void_p(q.data_ptr()), n, leaf, ctypes.c_void_p(quad.data_ptr()), stream)

    for theta in (0.5, 0.7, 1.0):
        fc, ncnt, _, _ = nb.tree_lists(q, theta, leaf)
        mn = int(ncnt.max().item())
        fc, ncnt, _, ni = nb.tree_lists(q, theta, leaf, None, max(mn, 1))
        torch.cuda.synchronize()
        fc, ncnt, ni = fc.cpu().numpy(), ncnt.cpu().numpy(), ni.cpu().numpy()
        sizes = nodes[:, 1] - nodes[:, 0]
        near_bodies = np.array([sizes[ni[g, :ncnt[g]]].sum() for g in range(len(groups))], dtype=np.float64)
        for order in (nb.CELLS_MONOPOLE, nb.CELLS_PSEUDO, nb.CELLS_QUADRUPOLE, nb.CELLS_LOCAL):
            per_cell = nb.TREE_PSEUDO if order == nb.CELLS_PSEUDO else 1
            extra = {}
            if order == nb.CELLS_LOCAL:
                # the local walk's own lists (counts only; near leaves taken as full)
                lc, fc4, nc4 = (t.cpu().numpy().astype(np.float64) for t in nb.tree_local_counts(q, theta, leaf))
                pairs = float((gsz * (fc4 + nc4 * leaf) + gsz * (gsz - 1)).sum())
                flops = (FLOP_PER_PAIR * float((gsz * (nc4 * leaf) + gsz * (gsz - 1)).sum())
                         + FLOP_PER_QUAD_CELL * float((gsz * fc4).sum()) + FLOP_PER_M2L * float(lc.sum()))
                extra = {"local_cells_per_group": round(float(lc.mean()), 1),
                         "per_target_cells_per_group": round(float(fc4.mean()), 1),
                         "near_leaves_per_group": round(float(nc4.mean()), 1)}
            else:
                pairs = float((gsz * (per_cell * fc + near_bodies) + gsz * (gsz - 1)).sum())
                # walk flops: 20 per body or pseudo-body pair, 54 per quadrupole cell
                flops = FLOP_PER_PAIR * pairs
                if order == nb.CELLS_QUADRUPOLE:
                    flops += (FLOP_PER_QUAD_CELL - FLOP_PER_PAIR) * float((gsz * fc).sum())
            nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, out=out, cells=order)
            torch.cuda.synchronize()
            ts, tm = [], []
            for _ in range(reps):
                e0.record()
                nb.tree_accel(q, eps, theta, leaf, prec=nb.F32_F64ACC, out=out, cells=order)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
                e0.record()
                rc = moments_only(order)
                e1.record()
                torch.cuda.synchronize()
                if rc != 0:
                    raise RuntimeError("tree moments failed")
                tm.append(e0.elapsed_time(e1))
            t, t_mom = float(np.mean(ts)), float(np.mean(tm))
            t_walk = t - t_mom
            got = out.cpu().double().numpy()
            rel = np.linalg.norm(got[:, :3] - d_host[:, :3], axis=1) / np.linalg.norm(d_host[:, :3], axis=1)
            walk_tflops = flops / (t_walk * 1e-3) / 1e12
            kern = {0: "k_tree_walk<F64ACC>", 2: "k_tree_walk<F64ACC, pseudo-particle cells>",
                    3: "k_tree_walk<F64ACC, quadrupole cells>", 4: "k_tree_walk<F64ACC, local expansions>"}[order]
            r = {"ms": round(t, 4), "ms_std": round(float(np.std(ts)), 4), "moments_ms": round(t_mom, 4),
                 "walk_force_ms": round(t_walk, 4), "interactions_per_body": round(pairs / n, 1),
                 "far_cells_per_group": round(float(fc.mean()), 1),
                 "pairs_per_s": round(pairs / (t_walk * 1e-3), 1),
                 "direct_equivalent_g_interactions_per_s": round(float(n) * n / (t * 1e-3) / 1e9, 1),
                 "speedup_vs_direct_kernel": round(direct_ms / t, 2),
                 "rms_rel_err_vs_direct": float(np.sqrt(np.mean(rel ** 2))),
                 "max_rel_err_vs_direct": float(rel.max()),
                 "walk_roofline": {"bound": "alu", "achieved": round(walk_tflops, 3), "peak": PEAK_FP32_TFLOPS,
                                   "unit": "TFLOP/s", "frac": round(walk_tflops / PEAK_FP32_TFLOPS, 4),
                                   "kernel": kern, "flop_per_pair": FLOP_PER_PAIR,
                                   "flop_per_quadrupole_cell": FLOP_PER_QUAD_CELL, "flop_per_m2l": FLOP_PER_M2L}}
            r.update(extra)
            {0: res["theta"], 2: res["pseudo_cells"], 3: res["quadrupole_cells"],
             4: res["local_cells"]}[order][str(theta)] = r
            log(f"[bench] tree cells {order} theta {theta}: {t:.3f} ms ({t_mom:.3f} moments), "
                f"{pairs / n:.0f} interactions/body, {walk_tflops:.1f} TFLOP/s in the walk, "
                f"x{direct_ms / t:.1f} vs direct, rms err {r['rms_rel_err_vs_direct']:.2e}")
    if v_np is not None:
        # whole simulation steps: force, kick/drift, and the ORB re-ordering
        # (at entry and before the 10th force: 2 passes in the 10 timed steps)
        vel = torch.as_tensor(v_np, dtype=torch.float32, device=dev).contiguous()
        res["leapfrog"] = {}
        for cells, theta in ((nb.CELLS_MONOPOLE, 0.7), (nb.CELLS_QUADRUPOLE, 0.7), (nb.CELLS_LOCAL, 0.7)):
            qq, vq = p.clone(), vel.clone()
            acc_t = torch.empty_like(qq)
            nb.tree_leapfrog(qq, vq, acc_t, eps, theta, dt, 1, leaf, reorder_every=1, cells=cells, prec=nb.F32_F64ACC)
            torch.cuda.synchronize()
            steps = 10
            e0.record()
            nb.tree_leapfrog(qq, vq, acc_t, eps, theta, dt, steps, leaf, reorder_every=10, acc_valid=True,
                             cells=cells, prec=nb.F32_F64ACC)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            key = {0: "monopole", 3: "quadrupole", 4: "local"}[cells]
            res["leapfrog"][key] = {"theta": theta, "ms_per_step": round(ms, 3), "steps": steps, "orb_passes": 2,
                                    "speedup_vs_direct_step": round(direct_ms / ms, 1)}
            log(f"[bench] tree leapfrog ({key} cells, theta {theta}): {ms:.3f} ms per step, 2 ORB passes in 10 steps")
    return res


def modes_leg(torch, nb, pm, eps, perm_host):
    """Pure FP32 and Kahan-compensated FP32 sums on the headline workload at
    its step-0 positions: the time of one force evaluation, and the result in
    input order, whose error the CPU leg takes against the oracle sample."""
    n = pm.shape[0]
    out = torch.empty_like(pm)
    res = {}
    for name in ("F32", "F32_KAHAN"):
        prec = getattr(nb, name)
        nb.accel(pm, eps, prec=prec, out=out)
        torch.cuda.synchronize()
        ts = []
        for _ in range(2):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            nb.accel(pm, eps, prec=prec, out=out)
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        host = np.empty((n, 4))
        host[perm_host] = out.cpu().double().numpy()
        ms = min(ts)
        res[name] = {"ms": round(ms, 3), "g_interactions_per_s": round(float(n) * n / ms / 1e6, 2), "_out": host}
        log(f"[bench] mode {name}: {ms:.2f} ms")
    return res


def cpu_leg(ics, pm0_host, acc0, eps, seconds, modes=None):
    """FP64 oracle on a bounded sample of targets of the headline workload;
    also the error of each other mode's result (`modes`) on the same sample."""
    import oracle
    n = pm0_host.shape[0]
    threads = oracle.num_threads()
    # chunks of sampled targets until about `seconds` of CPU work
    order = ics.sample_targets(n, min(n, 65536), 1003)
    ics.rng(1004).shuffle(order)
    log(f"[bench] cpu oracle on {threads} threads for ~{seconds:.0f} s")
    done, parts_a, parts_p = 0, [], []
    t0 = time.perf_counter()
    while done < order.shape[0] and time.perf_counter() - t0 < seconds:
        chunk = order[done:done + 4096]
        a, p = oracle.accel(pm0_host, eps, targets=chunk)
        parts_a.append(a)
        parts_p.append(p)
        done += chunk.shape[0]
    secs = time.perf_counter() - t0
    tg = order[:done]
    ref_a, ref_p = np.concatenate(parts_a), np.concatenate(parts_p)
    k = done
    gint = k * n / secs / 1e9
    da = np.linalg.norm(acc0[tg, :3] - ref_a, axis=1) / np.linalg.norm(ref_a, axis=1)
    dp = np.abs(acc0[tg, 3] - ref_p) / np.abs(ref_p)
    for m in (modes or {}).values():
        out = m.pop("_out")
        ma = np.linalg.norm(out[tg, :3] - ref_a, axis=1) / np.linalg.norm(ref_a, axis=1)
        mp = np.abs(out[tg, 3] - ref_p) / np.abs(ref_p)
        m["error_vs_oracle"] = {"force_rms_rel": float(np.sqrt(np.mean(ma ** 2))), "force_max_rel": float(ma.max()),
                                "pot_rms_rel": float(np.sqrt(np.mean(mp ** 2))), "targets": int(k)}
    # one full evaluation of the Plummer sphere of 65536 bodies (4.29e9 pairs)
    pm65, _ = ics.plummer(65536, 1001)
    t65 = time.perf_counter()
    oracle.accel(pm65.astype(np.float32).astype(np.float64), 0.01)
    t65 = time.perf_counter() - t65
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(gint, 5), "unit": "G-interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} sampled targets x {n} sources of the colliding pair, FP64 Neumaier sums",
            "seconds": round(secs, 2), "cpu_model": cpu_model,
            "full_evaluation_s_extrapolated": round(float(n) * n / (gint * 1e9), 1),
            "plummer65536_full_evaluation": {"seconds": round(t65, 2),
                                             "g_interactions_per_s": round(65536.0 ** 2 / t65 / 1e9, 4)},
            "gpu_error_vs_oracle": {"force_rms_rel": float(np.sqrt(np.mean(da ** 2))),
                                    "force_max_rel": float(da.max()),
                                    "pot_rms_rel": float(np.sqrt(np.mean(dp ** 2)))}}


if __name__ == "__main__":
    main()
