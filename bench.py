#!/usr/bin/env python
"""Benchmark of the gfx950 modal FMM on one MI355X.

Workload (default): 50,000 ring sources and 50,000 distinct field points,
uniform in r in [0.1, 1], z in [-1, 1], modes n = 0..16, complex N(0, 1)
strengths, at most 64 points per leaf.  A step is one whole pass of the hot
path for a new geometry: plan creation (tree sort, occupancy, Taylor tables)
plus FMM evaluation (moments, upward pass, S2L/L2L downward pass, local
expansion + near field), inputs already in HBM.

Metric: modal ring-pair interactions per second = ns * nf * n_modes * nrhs /
(seconds per step), at the expansion order whose max-over-modes relative
error (eq. results:error) against the FP64 oracle on sampled field points is
<= 1e-10.  Also reported: evaluation-only rate, the same at the order M = 12,
the GPU direct-sum rate and the FMM-vs-direct speed-up, the roofline of the
dominant kernel (FP64 vector ALU) and the oracle's CPU rate.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--order M] [--depth d]
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

PEAK_FP64_VALU_TFLOPS = 78.6     # MI355X: 256 CUs x 2.4 GHz x 64 lanes x 2 (FMA)
HEADLINE_ORDER = 24              # smallest M with max-over-modes error <= 1e-10 here (M = 22: 1.6e-10)
CONFIG_ORDER = 12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--order", type=int, default=HEADLINE_ORDER)
    ap.add_argument("--depth", type=int, default=0, help="0 = autotuned (with the tile width)")
    ap.add_argument("--tile", type=int, default=-1,
                    help="S2L kernel: 0 = matrix cores (tiles of up to 16 boxes), 2, 4 or 8 = vector units "
                         "with that tile width; -1 = autotuned")
    ap.add_argument("--max-leaf", type=int, default=64)
    ap.add_argument("--ns", type=int, default=50000)
    ap.add_argument("--nf", type=int, default=50000)
    ap.add_argument("--modes", type=int, default=17)
    ap.add_argument("--sample", type=int, default=5000,
                    help="field points checked against the oracle and timed on it (about 12 s on 16 cores)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batch measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 200k-ring adjoint measurement")
    ap.add_argument("--no-curve", action="store_true", help="skip the 1M-ring generator-curve measurement")
    ap.add_argument("--no-leaf-rule", action="store_true", help="skip the <= max_leaf depth's measurement")
    ap.add_argument("--no-standalone", action="store_true",
                    help="skip the kernels' standalone timing (near field after the downward pass)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    return ap.parse_args()


def copy_probe(torch, mib):
    """A plain copy kernel of known size, for scaling the HBM byte counters."""
    n = mib * (1 << 20) // 8
    x = torch.randn(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 5}))


def read_traffic(phase, kernel_file="axf_fmm.hip"):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary profiles/<phase>_traffic.txt, if it was taken on the current
    kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{phase}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2301_01179_amd", "csrc", kernel_file)
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("source_sha256") != sha:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def autotune_depth(torch, axf, coords, S, nmodes, order, candidates, tiles=(0,)):
    """Pick the (depth, S2L kernel) with the shortest plan + evaluate time
    (the second of two trials each); tile 0 is the matrix-core S2L, 2, 4 and
    8 the vector-unit one with that tile width."""
    rs, zs, rf, zf = coords
    best = None
    for d in candidates:
        for tb in tiles:
            try:
                for rep in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    plan = axf.Plan(rs, zs, rf, zf, nmodes, order, depth=d, tile=tb)
                    plan.evaluate(S)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    plan.close()
            except axf.AxfError:
                continue
            if best is None or dt < best[2]:
                best = (d, tb, dt)
    return best[0], best[1]


def measure(torch, axf, coords, S, nmodes, order, depth, steps, warmup, tile=0):
    rs, zs, rf, zf = coords
    ns, nf = rs.numel(), rf.numel()
    for _ in range(warmup):
        p = axf.Plan(rs, zs, rf, zf, nmodes, order, depth=depth, tile=tile)
        p.evaluate(S)
        p.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        p = axf.Plan(rs, zs, rf, zf, nmodes, order, depth=depth, tile=tile)
        phi = p.evaluate(S)
        p.close()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps

    # evaluation only, with per-phase HIP events on the launch stream
    plan = axf.Plan(rs, zs, rf, zf, nmodes, order, depth=depth, tile=tile)
    plan.evaluate(S)
    torch.cuda.synchronize()
    plan.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        phi = plan.evaluate(S)
    torch.cuda.synchronize()
    t_eval = (time.perf_counter() - t0) / steps
    timing = plan.read_timing()
    plan.set_timing(False)
    return plan, phi, t_step, t_eval, timing


def _median_time(torch, fn, reps):
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def leaf_occupancy(info, coords_np):
    """Largest number of sources and of field points in one leaf of the
    plan's tree (box index floor(((v - lo) / L) 2^d), clamped)."""
    rlo, zlo, L, invL = info["square"]
    d = info["depth"]
    nb = 1 << d
    out = []
    for r, z in (coords_np[:2], coords_np[2:]):
        ir = np.clip(np.floor(((r - rlo) * invL) * nb).astype(np.int64), 0, nb - 1)
        iz = np.clip(np.floor(((z - zlo) * invL) * nb).astype(np.int64), 0, nb - 1)
        out.append(int(np.bincount(ir * nb + iz).max()))
    return {"sources": out[0], "field_points": out[1]}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_single_thread(args, npts=250):
    """The oracle's direct sum on one host thread (OMP_NUM_THREADS=1, in a
    child process that touches no GPU), at npts sampled field points of the
    same workload."""
    import subprocess
    code = (
        "import sys, time, json, numpy as np; sys.path.insert(0, %r)\n"
        "from oracle import oracle as O; from paper_2301_01179_amd import inputs\n"
        "rs, zs, rf, zf, S = inputs.annulus(%d, %d, %d, 1, seed=%d)\n"
        "idx = np.sort(np.random.default_rng(7).choice(rf.size, %d, replace=False))\n"
        "t0 = time.perf_counter(); O.direct(rs, zs, rf[idx], zf[idx], S); t = time.perf_counter() - t0\n"
        "print(json.dumps({'seconds': t}))\n"
    ) % (ROOT, args.ns, args.nf, args.modes, args.seed, npts)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return None
    t = json.loads(r.stdout.strip().splitlines()[-1])["seconds"]
    return {"value": float(npts) * args.ns * args.modes / t, "cores": 1,
            "sample": f"{npts} sampled field points x {args.ns} sources x {args.modes} modes ({t:.1f} s)"}


def phase_roofline(timing, flops, reps):
    """Model FP64 rate of each timed phase and the fraction of the FP64
    vector peak; the dominant phase first."""
    out = {}
    for p, (ms, n) in timing.items():
        if ms <= 0 or flops.get(p, 0.0) <= 0:
            continue
        tf = flops[p] / (ms / 1e3 / reps) / 1e12
        out[p] = {"ms": round(ms / reps, 4), "model_tflops": round(tf, 3),
                  "frac": round(tf / PEAK_FP64_VALU_TFLOPS, 4)}
    return dict(sorted(out.items(), key=lambda kv: -kv[1]["ms"]))


def measure_curve(torch, axf, inputs, dev):
    """Generator-curve workload: 1,000,000 rings = field points on r = 1 +
    0.3 cos t, z = 0.3 sin t + 0.05 N(0, 1), modes 0..32.  Error against the
    GPU direct sum at 1,000 sampled field points (the direct sum is itself
    checked against the oracle in the tests) at M = 16 and at increasing M up
    to 24, stopping at the first M whose max-over-modes error is <= 1e-10;
    plan + evaluate time of each, at the depth (7, 8 or 9) timed fastest at
    M = 16."""
    n, nm = 1_000_000, 33
    r, z, S = inputs.generator_curve(n, nm, 1, seed=3)
    rt, zt = torch.from_numpy(r).to(dev), torch.from_numpy(z).to(dev)
    St = torch.from_numpy(S).to(dev)
    samp = np.sort(np.random.default_rng(21).choice(n, 1000, replace=False))
    dplan = axf.Plan(rt, zt, rt[samp], zt[samp], nm, 0, depth=2)
    ref = dplan.evaluate_direct(St).cpu().numpy()
    dplan.close()
    units = float(n) * n * nm
    depth, _ = autotune_depth(torch, axf, (rt, zt, rt, zt), St, nm, 16, [7, 8, 9])
    results = []
    for M in (16, 20, 22, 24):
        state = {}

        def step():
            p = axf.Plan(rt, zt, rt, zt, nm, M, depth=depth)
            state["phi"] = p.evaluate(St)
            state["info"] = p.info()
            p.close()

        step()
        t = _median_time(torch, step, 3)
        phi = state["phi"][..., samp].cpu().numpy()
        eps = float((np.abs(phi - ref).max(axis=-1) / np.abs(ref).max(axis=-1)).max())
        results.append({"order": M, "ms_per_step": t * 1e3, "value": units / t, "max_rel_err": eps})
        if eps <= 1e-10:
            break
    occ = leaf_occupancy(state["info"], (r, z, r, z))
    return {"workload": f"{n} rings = field points on the jittered generator curve, modes 0..{nm - 1}",
            "depth": depth, "max_points_per_leaf": occ, "orders": results,
            "meets_1e-10": any(x["max_rel_err"] <= 1e-10 for x in results),
            "error_reference": "GPU direct sum at 1000 sampled field points",
            "unit": "modal ring-pair interactions/s"}


def measure_adjoint(torch, axf, inputs, dev):
    """Adjoint workload: 200,000 rings (sources = field points, ring-box
    geometry), modes 0..16, M = 12; loss sum |phi - phi_target|^2.  Times the
    forward evaluation and the adjoint (strength and coordinate gradients)."""
    n, nm, M = 200_000, 17, 12
    r, z, S = inputs.ring_box(n, nm, 1, seed=5)
    _, _, St = inputs.ring_box(n, nm, 1, seed=6)
    rt, zt = torch.from_numpy(r).to(dev), torch.from_numpy(z).to(dev)
    S, St = torch.from_numpy(S).to(dev), torch.from_numpy(St).to(dev)
    plan = axf.Plan(rt, zt, rt, zt, nm, M, depth=0, max_leaf=32)
    phi_t = plan.evaluate(St)
    state = {}

    def fwd():
        state["phi"] = plan.evaluate(S)

    def adj():
        g = 2 * (state["phi"] - phi_t)
        state["grads"] = plan.adjoint(g, S)

    fwd(); adj()
    t_f = _median_time(torch, fwd, 5)
    t_a = _median_time(torch, adj, 5)
    # per-phase model FP64 rates (HIP events on the launch stream); sources
    # and field points are one set here, so the swapped FMM of the adjoint
    # has the forward's work model (its leaf also forms the coordinate
    # gradients, which the model leaves out)
    flops = plan.work()["flops"]
    reps = 5
    plan.set_timing(True)
    for _ in range(reps):
        fwd()
    roof_f = phase_roofline(plan.read_timing(), flops, reps)
    for _ in range(reps):
        adj()
    roof_a = phase_roofline(plan.read_timing(), flops, reps)
    plan.set_timing(False)
    total = sum(flops[p] for p in ("p2m", "m2m", "s2l", "l2l", "leaf", "l2p"))
    units = float(n) * n * nm
    out = {"workload": f"{n} rings = field points, ring box [0.5,1.5]x[-0.5,0.5], modes 0..{nm - 1}, M = {M}",
           "depth": plan.info()["depth"], "ms_forward": t_f * 1e3, "ms_adjoint": t_a * 1e3,
           "adjoint_value": units / t_a, "unit": "modal ring-pair interactions/s",
           "forward_roofline": {"model_tflops": round(total / t_f / 1e12, 3),
                                "frac": round(total / t_f / 1e12 / PEAK_FP64_VALU_TFLOPS, 4),
                                "phases": roof_f},
           "adjoint_roofline": {"model_tflops": round(total / t_a / 1e12, 3),
                                "frac": round(total / t_a / 1e12 / PEAK_FP64_VALU_TFLOPS, 4),
                                "phases": roof_a,
                                "note": "forward work model (potential part of the leaf only)"}}
    d_rule = plan.info()["depth"]
    out["depth_choice"] = "the workload's <= 32 points-per-leaf rule"
    plan.close()
    # the same workload at the fastest of the depths around the rule's
    best = None
    for d in (d_rule - 2, d_rule - 1, d_rule):
        p = axf.Plan(rt, zt, rt, zt, nm, M, depth=d)
        phi = p.evaluate(S)
        g = 2 * (phi - p.evaluate(St))
        p.adjoint(g, S)
        tf = _median_time(torch, lambda: p.evaluate(S), 3)
        ta = _median_time(torch, lambda: p.adjoint(g, S), 3)
        if best is None or tf + ta < best[1] + best[2]:
            best = (d, tf, ta)
        p.close()
    out["fastest_depth"] = {"depth": best[0], "ms_forward": best[1] * 1e3, "ms_adjoint": best[2] * 1e3,
                            "adjoint_value": units / best[2],
                            "choice": "fastest forward + adjoint of depths rule-2 .. rule"}
    return out


def measure_batch(torch, axf, inputs, dev):
    """Batched workload: 64 problems, sizes log-uniform in 1e3..2e5 rings of
    the ring-box geometry (sources = field points), 1..8 right-hand sides,
    modes 0..16, M = 12, depths from the autotuner.  Times the captured graph
    replay against per-problem plain launches."""
    nm, M = 17, 12
    sizes, nrhs = inputs.batched_sizes(64, 1e3, 2e5, seed=4)
    probs = []
    units = 0.0
    for i, (n, q) in enumerate(zip(sizes, nrhs)):
        r, z, S = inputs.ring_box(int(n), nm, nrhs=int(q), seed=1000 + i)
        probs.append((r, z, r, z, S))
        units += float(n) * n * nm * q
    t0 = time.perf_counter()
    b = axf.Batch(probs, nm, M)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    b.launch()
    b.launch_plain()
    t_graph = _median_time(torch, b.launch, 7)
    t_plain = _median_time(torch, b.launch_plain, 7)
    out = {"workload": "64 problems, 1e3..2e5 rings log-uniform, nrhs 1..8, modes 0..16, M = 12",
           "total_rings": int(sizes.sum()), "ms_graph": t_graph * 1e3, "ms_plain": t_plain * 1e3,
           "graph_value": units / t_graph, "plain_value": units / t_plain,
           "unit": "modal ring-pair interactions/s", "s_create": t_create,
           "depths": b.depths()}
    b.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); a run over "
              "several GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_probe:
        copy_probe(torch, args.copy_probe)
        return

    from paper_2301_01179_amd import axf, inputs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    # a step creates a new plan: let released plan memory be reused (the
    # library's arena cache is off by default)
    axf.set_cache_limit(16 << 30)
    nm = args.modes
    rs_np, zs_np, rf_np, zf_np, S_np = inputs.annulus(args.ns, args.nf, nm, 1, seed=args.seed)
    rs, zs = torch.from_numpy(rs_np).to(dev), torch.from_numpy(zs_np).to(dev)
    rf, zf = torch.from_numpy(rf_np).to(dev), torch.from_numpy(zf_np).to(dev)
    S = torch.from_numpy(S_np).to(dev)
    coords = (rs, zs, rf, zf)
    coords_np = (rs_np, zs_np, rf_np, zf_np)
    ns, nf = args.ns, args.nf
    units = float(ns) * nf * nm

    rng = np.random.default_rng(args.seed + 1000)
    sample = np.sort(rng.choice(nf, size=min(args.sample, nf), replace=False))

    depth, tile = args.depth, args.tile
    if depth == 0:
        depth, tile = autotune_depth(torch, axf, coords, S, nm, args.order, [3, 4, 5, 6, 7],
                                     (0, 2, 4, 8) if tile < 0 else (tile,))
    tile = max(tile, 0)

    plan, phi, t_step, t_eval, timing = measure(torch, axf, coords, S, nm, args.order, depth,
                                                args.steps, args.warmup, tile)
    info = plan.info()
    work = plan.work()
    census = plan.census()["near"]

    # GPU direct sum (same points) for the speed-up
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    plan.evaluate_direct(S)
    ev0.record()
    ref_gpu = plan.evaluate_direct(S)
    ev1.record()
    torch.cuda.synchronize()
    t_direct = ev0.elapsed_time(ev1) / 1e3

    phi_s = phi[..., sample].cpu().numpy()
    ref_gpu_s = ref_gpu[..., sample].cpu().numpy()

    # oracle: accuracy reference on the sampled field points and CPU baseline
    cpu = None
    eps_oracle = None
    if not args.no_cpu:
        from oracle import oracle as O
        t0 = time.perf_counter()
        ref_cpu = O.direct(rs_np, zs_np, rf_np[sample], zf_np[sample], S_np)
        t_cpu = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
        cpu = {"value": float(len(sample)) * ns * nm / t_cpu, "unit": "modal ring-pair interactions/s",
               "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"direct modal sum of the oracle at {len(sample)} sampled field points "
                         f"x {ns} sources x {nm} modes ({t_cpu:.1f} s)",
               "single_thread": oracle_single_thread(args)}
        num = np.abs(phi_s - ref_cpu).max(axis=-1)
        den = np.abs(ref_cpu).max(axis=-1)
        eps_oracle = (num / den).ravel()
        gd = np.abs(ref_gpu_s - ref_cpu).max(axis=-1) / den
        direct_parity = float(gd.max())
    num = np.abs(phi_s - ref_gpu_s).max(axis=-1)
    den = np.abs(ref_gpu_s).max(axis=-1)
    eps_gpu = (num / den).ravel()
    eps = eps_oracle if eps_oracle is not None else eps_gpu

    # roofline of the dominant kernel (evaluation passes)
    flops = work["flops"]
    phases = ["p2m", "m2m", "l2l", "s2l", "leaf", "l2p"]
    dom = max(phases, key=lambda p: timing[p][0])
    ms_dom, launches = timing[dom]
    achieved = flops[dom] / (ms_dom / 1e3 / args.steps) / 1e12 if ms_dom > 0 else 0.0
    traffic = read_traffic(dom)
    # the matrix-core S2L is bound by the FP64 MFMA rate (the same 78.6
    # TFLOP/s on MI355X as the vector FMA rate); everything else by the vector ALU
    bound = "mfma" if dom == "s2l" and tile == 0 else "alu"
    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": PEAK_FP64_VALU_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VALU_TFLOPS, 4),
                "traffic": traffic, "kernel": dom,
                "avg_launch_ms": round(ms_dom / max(launches, 1), 4),
                "launches_per_step": launches // max(args.steps, 1)}

    # the kernels on their own: the same plan with the near field after the
    # downward pass on one stream (AXF_NO_OVERLAP), so that each kernel's
    # launch time is not shared with the other's
    t_ser = {}
    if not args.no_standalone:
        ser = axf.Plan(rs, zs, rf, zf, nm, args.order, depth=depth, tile=tile, overlap=False)
        ser.evaluate(S)
        torch.cuda.synchronize()
        ser.set_timing(True)
        for _ in range(args.steps):
            ser.evaluate(S)
        torch.cuda.synchronize()
        t_ser = ser.read_timing()
        ser.set_timing(False)
        ser.close()
    standalone = {}
    for ph in [p for p in ("s2l", "leaf") if p in t_ser]:
        ms_ph, n_ph = t_ser[ph]
        if ms_ph > 0:
            a = flops[ph] / (ms_ph / 1e3 / args.steps) / 1e12
            standalone[ph] = {"achieved": round(a, 3), "frac": round(a / PEAK_FP64_VALU_TFLOPS, 4),
                              "avg_launch_ms": round(ms_ph / max(n_ph, 1), 4),
                              "ms_per_eval": round(ms_ph / args.steps, 4)}
    roofline["standalone"] = standalone
    roofline["note"] = ("achieved/frac/avg_launch_ms are from the timed (headline) evaluations, where the "
                        "near field runs beside the S2L passes on a second stream; 'standalone' times the "
                        "same kernels with the near field after the downward pass on one stream")

    secondary = None
    if not args.no_secondary and args.order != CONFIG_ORDER:
        d2, tb2 = autotune_depth(torch, axf, coords, S, nm, CONFIG_ORDER, [4, 5, 6, 7], (0, 2, 4, 8))
        p2, phi2, ts2, te2, _ = measure(torch, axf, coords, S, nm, CONFIG_ORDER, d2, args.steps, args.warmup, tb2)
        phi2_s = phi2[..., sample].cpu().numpy()
        refs = ref_cpu if eps_oracle is not None else ref_gpu_s
        e2 = (np.abs(phi2_s - refs).max(axis=-1) / np.abs(refs).max(axis=-1)).max()
        secondary = {"order": CONFIG_ORDER, "depth": d2, "tile": tb2, "value": units / ts2,
                     "eval_only_value": units / te2, "ms_per_step": ts2 * 1e3,
                     "max_rel_err": float(e2), "fmm_vs_direct_speedup": t_direct / ts2}
        p2.close()

    # the tree of config's leaf rule (<= max_leaf points of each set per leaf)
    leaf_rule = None
    rule_plan = axf.Plan(rs, zs, rf, zf, nm, 0, depth=0, max_leaf=args.max_leaf)
    d_rule = rule_plan.info()["depth"]
    rule_plan.close()
    if d_rule != depth and not args.no_leaf_rule:
        pr, phir, tsr, ter, _ = measure(torch, axf, coords, S, nm, args.order, d_rule, args.steps, args.warmup, tile)
        phir_s = phir[..., sample].cpu().numpy()
        refs = ref_cpu if eps_oracle is not None else ref_gpu_s
        er = (np.abs(phir_s - refs).max(axis=-1) / np.abs(refs).max(axis=-1)).max()
        leaf_rule = {"depth": d_rule, "max_points_per_leaf": leaf_occupancy(pr.info(), coords_np),
                     "value": units / tsr, "ms_per_step": tsr * 1e3, "eval_only_value": units / ter,
                     "max_rel_err": float(er)}
        pr.close()

    adjoint = None if args.no_adjoint else measure_adjoint(torch, axf, inputs, dev)
    curve = None if args.no_curve else measure_curve(torch, axf, inputs, dev)
    batch = None if args.no_batch else measure_batch(torch, axf, inputs, dev)

    line = {
        "metric": "modal ring-pair interactions/s at <=1e-10 rel err; FMM vs direct speedup",
        "value": units / t_step,
        "unit": "modal ring-pair interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"annulus: {ns} ring sources + {nf} distinct field points, r in [0.1,1], "
                               f"z in [-1,1], modes 0..{nm - 1}, complex N(0,1) strengths",
                   "order": args.order, "depth": depth,
                   "s2l_kernel": "matrix cores, tiles of up to 16 boxes" if tile == 0
                   else f"vector units, tiles of {tile} boxes",
                   "depth_choice": "fastest of depths 3..7 x S2L kernels (matrix cores; vector units with "
                                   "tiles of 2, 4, 8) (timed plan + evaluate)"
                   if args.depth == 0 else "given",
                   "max_points_per_leaf": leaf_occupancy(info, coords_np), "nrhs": 1,
                   "step": "plan (tree + tables) + evaluate",
                   "memory": "library arena cache enabled (axf_set_cache_limit): a step's plan reuses the "
                             "previous step's device blocks"},
        "max_rel_err": float(eps.max()),
        "meets_1e-10": bool(eps.max() <= 1e-10),
        "rel_err_per_mode": [float(f"{x:.3g}") for x in eps],
        "error_reference": "FP64 CPU oracle" if eps_oracle is not None else "GPU direct sum",
        "eval_only_value": units / t_eval,
        "ms_eval_only": t_eval * 1e3,
        "phase_ms_per_eval": {p: round(timing[p][0] / args.steps, 4) for p in timing},
        "gpu_direct_value": units / t_direct,
        "ms_gpu_direct": t_direct * 1e3,
        "fmm_vs_direct_speedup": t_direct / t_step,
        "fmm_vs_direct_speedup_eval_only": t_direct / t_eval,
        "near_pairs": work["near_pairs"], "s2l_box_pairs": work["s2l_pairs"], "s2l_units": work["s2l_units"],
        "near_census": {"backward_fraction": census["backward"] / max(census["pairs"], 1.0),
                        "agm_iterations_per_pair": census["agm_iterations"] / max(census["pairs"], 1.0),
                        "recursion_steps_per_pair": census["steps"] / max(census["pairs"], 1.0),
                        "model_flops_per_pair": work["flops"]["leaf"] / max(census["pairs"], 1.0)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "config_order_result": secondary,
        "leaf_rule_result": leaf_rule,
        "adjoint_result": adjoint,
        "curve_result": curve,
        "batch_result": batch,
    }
    if eps_oracle is not None:
        line["gpu_direct_vs_oracle"] = direct_parity
    plan.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
