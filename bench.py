"""Benchmark of the batched MBE-FCI hot path on one MI355X.

Default workload (--workload large): the 60-orbital problem, reference
CAS(8e,8o), screening a = 5.0, orders 1-4, energies and density-matrix
gradients.  Orders 0-3 (23,479 tuples) are the set-up, timed and reported per
order but outside the timed steps; order 4 (270,725 tuples, about 99 % of the
work) is opened as a streamed order and a step solves one stratified slice of
it, tuples s, s + B, s + 2B, ... (B = --slices): the whole path for those
tuples -- shape classes and batches, integral gather, string tables, diagonal,
P-space guess and preconditioner, Davidson with the sigma kernels, increments
against the completed lower orders (Eq. 3), and the density matrices of the
converged vectors embedded into the gradient with their adjoint weight 1.  The
slices of the warm-up and timed steps are disjoint, every one with the class
mix of the whole order.  Integrals are resident on the device before the timed
region.  Prints one JSON line.

Other workloads (--workload sweep | plain | hubbard): one step is one whole
expansion (no gradient), as the per-config figures need.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload large] [--slices 400]
                    [--no-per-solve] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CASCI increments/s + sigma FP64 GFLOP/s, batched vs per-solve, |ΔE|≤1e-9 Eh"
FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {0: "k_sigma_strip", 1: "k_sigma_linked_gat", 2: "k_sigma_linked_res", 3: "k_sigma_linked_dv",
                4: "k_sigma_w", 5: "k_linked_wr", 6: "k_whole"}
# Calibrated HBM bytes per sigma application of the dominant kernel from the
# FETCH_SIZE / WRITE_SIZE passes of profiles/ (the dispatches' bytes over the
# applications they carried; a launch carries as many applications as tuples
# still running), valid only while the kernel sources hash to the value they
# were taken on.  The reported traffic per launch is this times the timed
# run's applications per launch.
TRAFFIC = {
    # kernel id -> (sources sha1, calibrated bytes per application), from
    # profiles/hbm-traffic-large-n60-order4.md
    "large": {3: ("585e181301a003da4f6be845fb36597025553baf", 6583818.2),
              5: ("585e181301a003da4f6be845fb36597025553baf", 245659318.1)},
    # profiles/hbm-traffic-sweep-n24-cas66-orders1-5.md
    "sweep": {2: ("585e181301a003da4f6be845fb36597025553baf", 1360333.7)},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=["large", "sweep", "plain", "hubbard"])
    ap.add_argument("--slices", type=int, default=400, help="order-4 slices of the large workload")
    ap.add_argument("--ws-gib", type=float, default=200.0)
    ap.add_argument("--no-per-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="large workload without the gradient")
    ap.add_argument("--kernels-only", action="store_true",
                    help="large workload: energies of stratified order-4 slices of all C(52, 4) tuples (the list "
                         "screening leaves at a = 5.0), no lower orders, increments or gradient -- for profiler "
                         "runs of the order-4 kernels, not a headline figure")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="bytes of a plain device-to-device copy run 3 times first (HBM counter calibration)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sources_sha1():
    """sha1 over the alpha-beta kernel sources (strip.hip, then device.h)."""
    import hashlib
    h = hashlib.sha1()
    for name in ("strip.hip", "device.h"):
        with open(os.path.join(ROOT, "paper_1905_02786_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def merge_classes(acc, cls):
    for c in cls:
        key = (c["n_active"], c["n_alpha"], c["n_beta"])
        a = acc.setdefault(key, {k: 0 for k in c})
        for k, v in c.items():
            if k in ("n_active", "n_alpha", "n_beta", "kernel", "dim"):
                a[k] = v
            else:
                a[k] += v
    return acc


def class_table(acc):
    out = []
    for key in sorted(acc):
        c = acc[key]
        tf = c["sigma_flops"] / (c["sigma_ms"] / 1e3) / 1e12 if c["sigma_ms"] > 0 else 0.0
        row = {"cas": f"({c['n_alpha'] + c['n_beta']}e,{c['n_active']}o)", "dim": c["dim"],
               "kernel": KERNEL_NAMES[c["kernel"]], "tuples": c["tuples"],
               "iterations_mean": c["iterations"] / max(1, c["tuples"]), "sigma_applications": c["sigma_calls"],
               "sigma_launches": c["sigma_launches"], "alpha_beta_ms": c["sigma_ms"],
               "sigma_all_ms": c["sigma_total_ms"], "wall_ms": c["wall_ms"], "alpha_beta_tflops": tf,
               "frac": tf / FP64_MFMA_PEAK_TFLOPS, "flops": c["sigma_flops"]}
        if c["kernel"] == 5 and c["gather_ms"] > 0:
            row.update(gather_bytes_and_rate(c))
        out.append(row)
    return out


def gather_bytes_and_rate(c):
    """The gather of the W-in-HBM form: per application it reads the 1 +
    n_a (n_A - n_a) W rows of every determinant and c, and writes sigma."""
    rows = 1 + c["n_alpha"] * (c["n_active"] - c["n_alpha"])
    by = (rows + 2) * 8.0 * c["dim"] * c["sigma_calls"]
    gbs = by / (c["gather_ms"] / 1e3) / 1e9
    return {"gather_ms": c["gather_ms"], "gather_bytes": by, "gather_gbs": gbs, "gather_hbm_frac": gbs / HBM_PEAK_GBS}


def roofline(acc, workload):
    """The alpha-beta kernel with the largest HIP-event time over the timed
    steps: its FLOPs (rows formed) over that time."""
    by_k = {}
    for c in acc.values():
        b = by_k.setdefault(c["kernel"], {"ms": 0.0, "flops": 0.0, "launches": 0, "bytes": 0.0, "apps": 0})
        b["apps"] += c["sigma_calls"]
        b["ms"] += c["sigma_ms"]
        b["flops"] += c["sigma_flops"]
        b["launches"] += c["sigma_launches"]
        b["bytes"] += c["sigma_calls"] * algorithmic_bytes(c)
    kid = max(by_k, key=lambda k: by_k[k]["ms"])
    b = by_k[kid]
    achieved = b["flops"] / (b["ms"] / 1e3) / 1e12 if b["ms"] > 0 else 0.0
    tr = TRAFFIC.get(workload, {}).get(kid)
    traffic = tr[1] * b["apps"] / max(1, b["launches"]) if (tr and tr[0] == sources_sha1()) else None
    return {"bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": traffic, "kernel": KERNEL_NAMES[kid],
            "launches": b["launches"], "avg_launch_ms": b["ms"] / max(1, b["launches"]),
            "per_launch_flops": b["flops"] / max(1, b["launches"]),
            "algorithmic_bytes_per_launch": b["bytes"] / max(1, b["launches"]),
            "time_share_of_alpha_beta": b["ms"] / max(1e-9, sum(x["ms"] for x in by_k.values())),
            "flops_counted": "2 x rows formed x P_A x dim per sigma application (rows: 1 + n_a (n_A - n_a) for the "
                             "linked-row kernels, P_A for the all-pairs kernel)"}


def algorithmic_bytes(c):
    """HBM bytes one sigma application of the class's alpha-beta kernel must
    move: read c and write sigma (16 dim) plus the pair matrix (8 P_A^2); for
    the W-in-HBM form read c and write its 1 + n_a (n_A - n_a) W rows."""
    nA, na = c["n_active"], c["n_alpha"]
    P = nA * (nA + 1) // 2
    if c["kernel"] == 5:
        return 8.0 * c["dim"] * (2 + na * (nA - na))
    return 16.0 * c["dim"] + 8.0 * P * P


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def oracle_threads():
    """Threads the oracle's OpenMP matvec runs on (OMP_NUM_THREADS or all)."""
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


# ------------------------------------------------------------- large --------

def bench_order4_kernels(args, M, torch, out):
    """Profiler mode: the order-4 kernels on stratified slices of the order-4
    list, each step's progress printed (no set-up phase without output)."""
    import itertools
    import numpy as np
    import synth
    P = synth.config_large(0)
    ws = M.workspace(int(args.ws_gib * (1 << 30)))
    allt = np.array(list(itertools.combinations(P.expansion_space(), 4)), dtype=np.int16)
    ctx = M.Context.from_problem(P, device=0, profile=1, batched=1)
    B, acc, times = args.slices, {}, []
    for s in range(args.warmup + args.steps):
        tl = allt[s::B]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        e, st = ctx.solve_tuples(4, tl, ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        log(f"slice {s}: {len(tl)} tuples in {dt:.2f} s")
        if s >= args.warmup:
            times.append(dt)
            merge_classes(acc, ctx.class_stats())
    out.update({"value": sum(len(allt[s::B]) for s in range(args.warmup, args.warmup + args.steps)) / sum(times),
                "ms_per_step": 1e3 * sum(times) / len(times), "kernels_only": True,
                "config": {"workload": "order-4 energies only (profiler mode)"},
                "classes": class_table(acc), "roofline": roofline(acc, "large")})
    return out


def bench_large(args, M, torch, out):
    import numpy as np
    import synth
    if args.kernels_only:
        return bench_order4_kernels(args, M, torch, out)
    P = synth.config_large(0)
    ws = M.workspace(int(args.ws_gib * (1 << 30)))
    grad = 0 if args.no_grad else 1
    opts = dict(profile=1, batched=1, gradient=grad, stream_last=1)
    ctx = M.Context.from_problem(P, device=0, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    part, handle = ctx.run(ws, keep=True)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    setup_cls = ctx.class_stats()
    o4 = part.orders[-1]
    n4 = len(o4.tuples)
    log(f"set-up: orders 0-{len(part.orders) - 2} in {t_setup:.1f} s, order 4 opened with {n4} tuples")
    B = args.slices
    nstep = args.warmup + args.steps
    if nstep > B:
        raise SystemExit(f"--warmup + --steps ({nstep}) exceeds --slices ({B}): slices must stay disjoint")
    times, ntup, acc = [], 0, {}
    for s in range(nstep):
        cnt = len(range(s, n4, B))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.order_solve(handle, s, B, cnt, ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        if s >= args.warmup:
            times.append(dt)
            ntup += cnt
            merge_classes(acc, ctx.class_stats())
        log(f"{'warmup' if s < args.warmup else 'step'} {s}: {cnt} tuples in {dt:.2f} s")
    t_tot = sum(times)
    value = ntup / t_tot
    res = ctx.result(handle)
    o4 = res.orders[-1]
    solved = o4.status != M.TUPLE_PENDING
    assert (o4.status[solved] == 0).all(), "a tuple did not converge"
    flops = sum(c["sigma_flops"] for c in acc.values())
    sig_ms = sum(c["sigma_ms"] for c in acc.values())
    sig_all_ms = sum(c["sigma_total_ms"] for c in acc.values())
    out.update({
        "value": value, "unit": "increments/s", "ms_per_step": 1e3 * t_tot / len(times),
        "config": {"workload": "60 orbitals, 6a+6b electrons, reference CAS(8e,8o) = orbitals 2-9, MBE orders 1-4 "
                               "over 52 expansion orbitals, a = 5.0, energies and RDM gradients, seed 0; a step is a "
                               f"stratified 1/{B} slice of order 4 (tuples s + {B} i)",
                   "orders": [len(o.tuples) for o in res.orders], "tuples_per_step": ntup / len(times),
                   "gradient": bool(grad), "batched": True},
        "setup": {"seconds": t_setup, "per_order_ms": [o.wall_ms for o in part.orders[:-1]],
                  "tuples": sum(len(o.tuples) for o in part.orders[:-1]),
                  "classes": class_table(merge_classes({}, setup_cls))},
        "whole_job_estimate_s": t_setup + n4 / value,
        "sigma": {"alpha_beta_tflops": flops / (sig_ms / 1e3) / 1e12 if sig_ms else 0.0,
                  "sigma_all_kernels_gflops": flops / (sig_all_ms / 1e3) / 1e9 if sig_all_ms else 0.0,
                  "alpha_beta_ms": sig_ms, "sigma_all_ms": sig_all_ms,
                  "applications": sum(c["sigma_calls"] for c in acc.values())},
        "classes": class_table(acc),
        "roofline": roofline(acc, "large"),
        "order_sums_so_far": [o.order_sum for o in res.orders[:-1]],
    })
    if not args.no_per_solve:
        # the one-solve-per-launch path on unsolved tuples of the same class
        # mix: residue nstep mod B, spread over the whole list
        ctx.set_options(a=P.a, max_order=P.max_order, profile=0, batched=0, gradient=grad, stream_last=1)
        m = max(1, math.ceil(n4 / (B * 12)))
        cnt = len(range(nstep, n4, B * m))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.order_solve(handle, nstep, B * m, cnt, ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        v1 = cnt / dt
        out["per_solve"] = {"value": v1, "unit": "increments/s", "tuples": cnt, "seconds": dt,
                            "sample": f"order-4 tuples {nstep} + {B * m} i, one tuple per launch sequence",
                            "batched_over_per_solve": value / v1}
        log(f"per-solve: {cnt} tuples in {dt:.1f} s")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_large(P, o4)
    return out


def cpu_large(P, o4):
    """Oracle time per order-4 tuple, extrapolated: the oracle's whole CASCI
    (ARPACK on its matrix-free Slater-Condon product) timed on one order-1
    tuple, scaled per order-4 shape class by the time of one oracle product
    there; averaged with the class mix of order 4."""
    import numpy as np
    from oracle import fci
    log("cpu baseline (oracle) ...")
    X = P.expansion_space()
    S1 = (X[5],)
    sp1 = fci.cas_space(P, S1)
    x1 = np.random.default_rng(0).standard_normal(sp1.dim)
    t0 = time.perf_counter()
    fci.matvec(P, sp1, x1)
    t_mv1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    fci.casci_energy(P, S1)
    t_full1 = time.perf_counter() - t0
    classes = {}
    for t in o4.tuples:
        S = tuple(int(x) for x in t)
        nocc = sum(1 for x in S if x < P.nbeta)
        classes.setdefault(nocc, [S, 0])
        classes[nocc][1] += 1
    total, detail, spent = 0.0, [], t_mv1 + t_full1
    for nocc, (S, cnt) in sorted(classes.items()):
        sp = fci.cas_space(P, S)
        x = np.random.default_rng(1).standard_normal(sp.dim)
        t0 = time.perf_counter()
        fci.matvec(P, sp, x)
        t_mv = time.perf_counter() - t0
        spent += t_mv
        per = t_full1 * t_mv / t_mv1
        total += per * cnt
        detail.append({"class": f"({sp.na + sp.nb}e,{len(sp.active)}o)", "dim": sp.dim, "tuples": cnt,
                       "matvec_s": t_mv, "est_s_per_tuple": per})
    n = sum(c[1] for c in classes.values())
    model, ncpu = host_info()
    return {"value": n / total, "unit": "increments/s", "cores": oracle_threads(), "kind": "oracle",
            "sample": (f"oracle CASCI of order-1 tuple {S1} (dim {sp1.dim}) timed whole ({t_full1:.1f} s, "
                       f"{t_full1 / t_mv1:.0f} products' worth); per order-4 class one oracle product timed and the "
                       f"whole CASCI scaled by the product-time ratio (extrapolated); {spent:.1f} s of CPU work"),
            "classes": detail, "host_cpu": model, "host_nproc": ncpu}


# ------------------------------------------------------ whole expansions ----

def problem_for(workload):
    import synth
    if workload == "sweep":
        return synth.config_sweep(0), ("24 orbitals (orbital 0 frozen), 6a+6b electrons, reference CAS(6e,6o) = "
                                       "orbitals 3-8, MBE orders 1-5 over 17 expansion orbitals, a = 5.0, seed 0")
    if workload == "plain":
        return synth.config_plain(0), ("10 orbitals, 4a+4b, reference CAS(2e,2o) = orbitals 3-4, full order over 8 "
                                       "expansion orbitals (256 tuples), no screening, seed 0")
    return synth.config_hubbard(4.0), ("10-site open Hubbard chain, U/t = 4, half filling, MO basis, reference "
                                       "CAS(2e,2o), full order (256 tuples), no screening")


def bench_expansion(args, M, torch, out):
    P, desc = problem_for(args.workload)
    ws = M.workspace(int(min(args.ws_gib, 96.0) * (1 << 30)))
    # timed steps without per-kernel events (Davidson iterations in blocks,
    # replayed as captured hipGraphs); then one profiled step (one host round
    # trip per iteration, every sigma launch timed) for the kernel figures
    ctx = M.Context.from_problem(P, device=0, profile=0, batched=1)
    for i in range(args.warmup):
        t0 = time.perf_counter()
        ctx.run(ws)
        log(f"warmup step {i}: {time.perf_counter() - t0:.3f} s")
    times, res = [], None
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.run(ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log(f"step {i}: {times[-1]:.3f} s")
    graph_batches = ctx.stats()["graph_batches"]
    whole_batches = ctx.stats()["whole_batches"]
    pctx = M.Context.from_problem(P, device=0, profile=1, batched=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pres = pctx.run(ws)
    torch.cuda.synchronize()
    t_prof = time.perf_counter() - t0
    acc = merge_classes({}, pctx.class_stats())
    # (the profiled pass keeps every class batched; the timed pass runs the
    # small classes in whole-tuple mode: each tuple's energy within the
    # Davidson tolerances, about 1e-11 apart, and the total, a signed sum of
    # thousands of increments, within 1e-8)
    d_prof = abs(pres.total - res.total)
    assert d_prof <= 1e-8, d_prof
    ntup = sum(len(o.tuples) for o in res.orders)
    t_step = sum(times) / len(times)
    value = ntup / t_step
    flops = sum(c["sigma_flops"] for c in acc.values())
    sig_ms = sum(c["sigma_ms"] for c in acc.values())
    sig_all_ms = sum(c["sigma_total_ms"] for c in acc.values())
    out.update({
        "value": value, "unit": "increments/s", "ms_per_step": 1e3 * t_step,
        "config": {"workload": desc, "tuples": ntup, "orders": [len(o.tuples) for o in res.orders], "batched": True},
        "total_energy": res.total, "per_order_ms": [o.wall_ms for o in res.orders],
        "graph_batches_per_step": graph_batches, "profiled_step_s": t_prof,
        "whole_batches_per_step": whole_batches, "profiled_vs_timed_total_dE": d_prof,
        "sigma": {"alpha_beta_tflops": flops / (sig_ms / 1e3) / 1e12 if sig_ms else 0.0,
                  "sigma_all_kernels_gflops": flops / (sig_all_ms / 1e3) / 1e9 if sig_all_ms else 0.0},
        "classes": class_table(acc), "roofline": roofline(acc, args.workload),
    })
    if not args.no_per_solve:
        ctx1 = M.Context.from_problem(P, device=0, profile=0, batched=0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r1 = ctx1.run(ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter() - t0
        import numpy as np
        worst = max(float(np.abs(a.eps - b.eps).max()) for a, b in zip(r1.orders, res.orders))
        out["per_solve"] = {"value": ntup / t1, "unit": "increments/s", "tuples": ntup, "seconds": t1,
                            "sample": "the whole expansion, one tuple per launch sequence",
                            "batched_over_per_solve": value / (ntup / t1), "max_abs_deps_vs_batched": worst}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_expansion(P, res)
    return out


def cpu_expansion(P, res, budget=20.0):
    """Oracle time per tuple on one tuple per (order, shape class) while the
    budget lasts, smallest first; the rest priced by dim x connectivity."""
    from oracle import fci
    log("cpu baseline (oracle) ...")
    classes = {}
    for o in res.orders:
        for t in o.tuples:
            S = tuple(int(x) for x in t)
            sp = fci.cas_space(P, S)
            key = (o.k, len(sp.active), sp.na, sp.nb)
            classes.setdefault(key, [S, sp.dim, 0])
            classes[key][2] += 1

    def conn(nA, na, nb):
        def sd(n_e):
            v = nA - n_e
            return n_e * v + math.comb(n_e, 2) * math.comb(v, 2)
        return 1 + sd(na) + sd(nb) + (na * (nA - na)) * (nb * (nA - nb))
    measured, spent, ref = {}, 0.0, None
    for key in sorted(classes, key=lambda k: classes[k][1]):
        S, dim, cnt = classes[key]
        if spent > budget:
            continue
        t0 = time.perf_counter()
        fci.casci_energy(P, S)
        dt = time.perf_counter() - t0
        spent += dt
        measured[key] = dt
        ref = (key, dt, dim)
    total, n_extra = 0.0, 0
    for key, (S, dim, cnt) in classes.items():
        if key in measured:
            total += measured[key] * cnt
        else:
            rk, rdt, rdim = ref
            total += rdt * (dim * conn(*key[1:])) / (rdim * conn(*rk[1:])) * cnt
            n_extra += cnt
    ntot = sum(c[2] for c in classes.values())
    model, ncpu = host_info()
    return {"value": ntot / total, "unit": "increments/s", "cores": oracle_threads(), "kind": "oracle",
            "sample": (f"one tuple per (order, shape class) solved by the oracle ({len(measured)} of {len(classes)} "
                       f"classes, {spent:.1f} s); whole-run time = per-class time x class count"
                       + (f", {n_extra} tuples priced by dim x connectivity scaling (extrapolated)" if n_extra else "")),
            "host_cpu": model, "host_nproc": ncpu}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the tuple-parallel path would shard "
              "each order's tuples across GPUs, which this build does not do.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1905_02786_amd as M
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        src = torch.ones(args.copy_probe // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: 3 x {args.copy_probe} bytes")
        del src, dst
    out = {"metric": METRIC, "value": None, "unit": "increments/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    if args.workload == "large":
        bench_large(args, M, torch, out)
    else:
        bench_expansion(args, M, torch, out)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
