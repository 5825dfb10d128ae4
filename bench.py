"""Benchmark: exact top-K users/sec on one MI355X.

Workload: 480,000 users x 17,770 items, f = 50 (the Netflix shape of the
paper's Table I), MF-shaped synthetic factors (rows r g/||g||, g ~ N(0, I),
r ~ LogNormal(0, 0.5)), K = 10.  One step = one full exact top-K of every
user (item preparation, matrix-core screen with fused streaming top-K,
certification + float64 rescore, fallback), inputs resident in HBM.

Prints one JSON line.  The headline `value` is the bf16-screen users/sec; the
float32-screen path is timed on the same inputs and reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16": 2516.6, "fp8": 5033.2, "fp32": 157.3}

# Sources whose content decides the screen kernel's machine code: measured
# traffic is reported only while their hash matches the one recorded with it.
SCREEN_SOURCES = ["include/mips.h", "paper_1706_01449_amd/csrc/internal.h",
                  "paper_1706_01449_amd/csrc/device_common.h",
                  "paper_1706_01449_amd/csrc/screen_core.h",
                  "paper_1706_01449_amd/csrc/screen_bf16.hip",
                  "paper_1706_01449_amd/csrc/api.cpp",
                  "paper_1706_01449_amd/build.py"]
TRAFFIC_FILE = "profiles/screen_kernel_mf_480000x17770_f50_bf16_K10_traffic.txt"


def precision_only(prec, steps, warmup):
    """The precision workload alone, one screen precision: calls timed with
    HIP events, for counter passes on its screen and certification kernels."""
    import torch
    import mipsgen
    import paper_1706_01449_amd as mips
    dev = torch.device("cuda:0")
    U, I = mipsgen.generate("precision", 0)
    Ut = torch.from_numpy(U).to(dev)
    It = torch.from_numpy(I).to(dev)
    ws = torch.empty(mips.lib().mips_bmm_topk_workspace_size(U.shape[0], I.shape[0], U.shape[1], 10,
                                                              mips.PRECISIONS[prec]),
                     dtype=torch.uint8, device=dev)
    for _ in range(warmup):
        mips.bmm_topk(Ut, It, 10, prec, workspace=ws)
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        mips.bmm_topk(Ut, It, 10, prec, workspace=ws)
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    ms.sort()
    print(json.dumps({"workload": "precision_1000000x136000_f100_K10", "precision": prec,
                      "calls": steps, "ms_per_call_median": ms[len(ms) // 2]}), flush=True)


def screen_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in SCREEN_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per screen launch from the committed counter summary, or None
    when the summary is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_hash") != screen_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mib):
    """A plain device-to-device copy of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 5}), flush=True)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_path(mips, torch, Ut, It, K, prec, steps, warmup):
    """Times `steps` back-to-back calls: the whole bracket by the host clock
    (synchronised on both sides) and each call by a HIP event pair on the
    call's stream; the library's own events give the per-kernel durations."""
    ws = torch.empty(mips.lib().mips_bmm_topk_workspace_size(Ut.shape[0], It.shape[0],
                                                              Ut.shape[1], K,
                                                              mips.PRECISIONS[prec]),
                     dtype=torch.uint8, device=Ut.device)
    for _ in range(warmup):
        mips.bmm_topk(Ut, It, K, prec, workspace=ws)
    torch.cuda.synchronize()
    mips.profile_read()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    mips.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record()
        out = mips.bmm_topk(Ut, It, K, prec, workspace=ws)
        e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mips.profile_enable(False)
    phases = mips.profile_read()
    calls = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    per_call = {"median": calls[len(calls) // 2], "min": calls[0], "mean": sum(calls) / len(calls)}
    _, _, st = mips.bmm_topk(Ut, It, K, prec, stats=True, workspace=ws)
    return (t1 - t0) / steps, phases, st, out, per_call


def timed(torch, fn, reps):
    """Median and min per-call time in ms: HIP events on the current stream
    around each call (inputs resident)."""
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def k_sweep(mips, torch, Ut, It, n_u):
    """users/s of the bfloat16 and float32 screens at K in {1, 5, 50}, and the
    E4M3 screen's exact-path users at K = 50."""
    out = {}
    for prec, steps in (("bf16", 10), ("fp32", 4)):
        for K in (1, 5, 50):
            log(f"k sweep: {prec} K={K}")
            t, ph, st, _, pc = time_path(mips, torch, Ut, It, K, prec, steps, 1)
            out[f"{prec}_K{K}"] = {"users_per_s": n_u / t, "ms_per_call_median": pc["median"],
                                   "ms_per_call_min": pc["min"],
                                   "screen_ms": ph["screen"][0] / max(1, ph["screen"][1]),
                                   "candidates_per_user": st["candidates_total"] / n_u,
                                   "exact_path_users": st["overflow_users"]}
    log("k sweep: fp8 K=50")
    t, ph, st, _, pc = time_path(mips, torch, Ut, It, 50, "fp8", 4, 1)
    out["fp8_K50"] = {"users_per_s": n_u / t, "ms_per_call_median": pc["median"],
                      "candidates_per_user": st["candidates_total"] / n_u,
                      "exact_path_users": st["overflow_users"],
                      "exact_path_fraction": st["overflow_users"] / n_u}
    return out


def extras(mips, torch, np, mipsgen, oracle_topk):
    """The other rows of the hot path, each on its own synthetic workload."""
    dev = torch.device("cuda:0")
    out = {}
    # --- Maximus on the clustered workload (480,000 x 17,770, f = 50, K = 10)
    log("extras: maximus")
    U, I = mipsgen.generate("clustered", 0)
    Ut = torch.from_numpy(U).to(dev)
    It = torch.from_numpy(I).to(dev)
    mx = {}
    t_bmm = timed(torch, lambda: mips.bmm_topk(Ut, It, 10, "bf16"), 5)
    for C in (8, 64, 256):
        holder = {}
        def build():
            holder["ix"] = mips.maximus_build(Ut, It, C, 3, 0, 0)
        tbs = []
        for _ in range(3):
            holder.pop("ix", None)        # the previous index is freed outside the timed call
            tbs.append(timed(torch, build, 1))
        tb = sorted(tbs)[1]
        ix = holder["ix"]
        tq = timed(torch, lambda: ix.query(10, "bf16"), 5)
        mips.profile_read()
        mips.profile_enable(True)
        ix.query(10, "bf16")
        torch.cuda.synchronize()
        mips.profile_enable(False)
        qph = {k: v[0] / max(1, v[1]) for k, v in mips.profile_read().items() if v[1]}
        idx, score, st = ix.query(10, "bf16", stats=True)
        tq32 = timed(torch, lambda: ix.query(10, "fp32"), 3)
        users = mipsgen.sample_users(U.shape[0], 200, seed=C)
        ri, _ = oracle_topk.topk(U[users], I, 10)
        walk_ms = qph.get("walk", 0.0)
        useful = 2.0 * U.shape[1] * st["items_scored"]          # 2 f sum_u w_u
        mx[f"C{C}"] = {"build_ms": tb, "query_ms": tq, "query_fp32_ms": tq32, "end_to_end_ms": tb + tq,
                       "tiles_per_user": st["mean_items_visited"] / 32.0,
                       "walk_useful_tflops": useful / (walk_ms * 1e-3) / 1e12 if walk_ms else None,
                       "walk_mfma_frac_bf16": (useful / (walk_ms * 1e-3) / 1e12 / PEAK_TFLOPS["bf16"]
                                               if walk_ms else None),
                       "users_per_s_query": U.shape[0] / (tq * 1e-3),
                       "users_per_s_end_to_end": U.shape[0] / ((tb + tq) * 1e-3),
                       "mean_items_visited": st["mean_items_visited"],
                       "exact_path_users": st["overflow_users"], "query_phases_ms": qph,
                       "index_match_sampled": float(np.mean(np.all(idx.cpu().numpy()[users] == ri, 1)))}
        del ix, holder
    mx["bmm_bf16_ms_same_data"] = t_bmm
    # new users: 10,000 fresh draws of the same mixture against the C=64 index
    ix = mips.maximus_build(Ut, It, 64, 3, 0, 0)
    # same seed, more users: the same mixture components, fresh draws
    Un = mipsgen.generate("clustered", 0, n_users=U.shape[0] + 10000)[0][U.shape[0]:]
    (Unt,) = [torch.from_numpy(Un).to(dev)]
    tn = timed(torch, lambda: ix.query_users(Unt, 10, "bf16"), 5)
    nidx, nsc, nst = ix.query_users(Unt, 10, "bf16", stats=True)
    ri, _ = oracle_topk.topk(Un[:200], I, 10)
    mx["new_users_10000_C64"] = {"query_ms": tn, "mean_items_visited": nst["mean_items_visited"],
                                 "exact_path_users": nst["overflow_users"],
                                 "index_match_sampled": float(np.mean(np.all(nidx.cpu().numpy()[:200] == ri, 1)))}
    del ix
    out["maximus_clustered_480000x17770_f50_K10"] = mx
    # Optimus (Section IV) on both 480,000 x 17,770 workloads
    log("extras: optimus")
    op = {}
    for wl in ("clustered", "mf"):
        if wl == "mf":
            del Ut, It
            U, I = mipsgen.generate("mf", 0)
            Ut = torch.from_numpy(U).to(dev)
            It = torch.from_numpy(I).to(dev)
        holder = {}
        def run():
            holder["r"] = mips.optimus_topk(Ut, It, 10, "bf16", n_clusters=64)
        t = timed(torch, run, 3)
        oidx, osc, rep = holder["r"]
        users = mipsgen.sample_users(U.shape[0], 200, seed=5)
        ri, _ = oracle_topk.topk(U[users], I, 10)
        rep["total_ms"] = t
        rep["index_match_sampled"] = float(np.mean(np.all(oidx.cpu().numpy()[users] == ri, 1)))
        op[wl] = rep
    out["optimus_480000x17770_f50_K10"] = op
    # norm-pruned brute force (stop test with theta_b = pi) on the MF workload
    ws = torch.empty(mips.lib().mips_bmm_topk_workspace_size(U.shape[0], I.shape[0], U.shape[1], 10,
                                                              mips.PRECISIONS["bf16"]),
                     dtype=torch.uint8, device=dev)
    tp = timed(torch, lambda: mips.norm_pruned_topk(Ut, It, 10, "bf16", workspace=ws), 5)
    pidx, psc, pst = mips.norm_pruned_topk(Ut, It, 10, "bf16", stats=True, workspace=ws)
    users = mipsgen.sample_users(U.shape[0], 200, seed=6)
    ri, _ = oracle_topk.topk(U[users], I, 10)
    out["norm_pruned_mf_480000x17770_f50_K10"] = {
        "ms": tp, "users_per_s": U.shape[0] / (tp * 1e-3),
        "mean_items_visited": pst["mean_items_visited"],
        "index_match_sampled": float(np.mean(np.all(pidx.cpu().numpy()[users] == ri, 1)))}
    del ws
    del Ut, It, U, I
    torch.cuda.empty_cache()
    # --- precision form: 1,000,000 x 136,000, f = 100, K = 10
    log("extras: precision form")
    U, I = mipsgen.generate("precision", 0)
    Ut = torch.from_numpy(U).to(dev)
    It = torch.from_numpy(I).to(dev)
    pf = {}
    users = mipsgen.sample_users(U.shape[0], 100, seed=1)
    ri, rk = oracle_topk.topk(U[users], I, 10)
    # "fp8_bf16": the E4M3 screen with the bfloat16 re-screen of its
    # candidates before the float64 rescore
    for name in ("bf16", "fp8", "fp8_bf16", "fp32"):
        prec = name
        ws = torch.empty(mips.lib().mips_bmm_topk_workspace_size(U.shape[0], I.shape[0], 100, 10,
                                                                  mips.PRECISIONS[prec]),
                         dtype=torch.uint8, device=dev)
        t = timed(torch, lambda: mips.bmm_topk(Ut, It, 10, prec, workspace=ws), 3)
        idx, score, st = mips.bmm_topk(Ut, It, 10, prec, stats=True, workspace=ws)
        gi = idx.cpu().numpy()[users]
        gs = score.cpu().numpy()[users]
        pf[name] = {"ms": t, "users_per_s": U.shape[0] / (t * 1e-3),
                    "index_match_sampled": float(np.mean(np.all(gi == ri, 1))),
                    "max_score_err_sampled": float(np.max(np.abs(gs - rk))),
                    "candidates_per_user": st["candidates_total"] / U.shape[0],
                    "rescored_per_user": st["rescored_pairs"] / U.shape[0],
                    "overflow_users": st["overflow_users"],
                    "max_screen_abs_err": st["max_screen_abs_err"],
                    "max_screen_rel_err": st["max_screen_rel_err"]}
        del ws
    out["precision_1000000x136000_f100_K10"] = pf
    del Ut, It, U, I
    torch.cuda.empty_cache()
    # --- differentiation form: 65,536 x 100,000, f = 64, K = 32
    log("extras: backward")
    U, I = mipsgen.generate("grad", 0)
    Ut = torch.from_numpy(U).to(dev)
    It = torch.from_numpy(I).to(dev)
    idx, score = mips.bmm_topk(Ut, It, 32, "bf16")
    G = torch.softmax(score.to(torch.float32), dim=1).contiguous()
    tf = timed(torch, lambda: mips.bmm_topk(Ut, It, 32, "bf16"), 5)
    tbk = timed(torch, lambda: mips.topk_backward(Ut, It, idx, G), 10)
    pairs = U.shape[0] * 32
    bytes_alg = pairs * 64 * 4 * 2 + U.shape[0] * 64 * 4 * 2 + I.shape[0] * 64 * 4
    # dI issues one float32 atomic per factor per run of equal items in each
    # wave's 64 grouped pairs (pairs sorted by item)
    it_sorted = np.sort(idx.cpu().numpy().reshape(-1), kind="stable")
    starts = np.ones(it_sorted.size, dtype=bool)
    starts[1:] = it_sorted[1:] != it_sorted[:-1]
    starts[::64] = True
    atomics = int(starts.sum()) * 64
    out["grad_65536x100000_f64_K32"] = {
        "forward_ms": tf, "backward_ms": tbk,
        "backward_pairs_per_s": pairs / (tbk * 1e-3),
        "backward_algorithmic_GBps": bytes_alg / (tbk * 1e-3) / 1e9,
        "backward_dI_atomics": atomics,
        "backward_dI_atomics_per_s": atomics / (tbk * 1e-3),
        "direct_scatter_atomics": pairs * 64}
    return out


def maximus_build_only(Cs, steps, warmup):
    """Maximus builds alone (480,000 x 17,770 clustered, f = 50, 3 k-means
    updates): median and min of per-build wall times, the index freed between
    builds."""
    import torch
    import mipsgen
    import paper_1706_01449_amd as mips
    U, I = mipsgen.generate("clustered", 0)
    Ut = torch.from_numpy(U).cuda()
    It = torch.from_numpy(I).cuda()
    torch.cuda.synchronize()
    for C in Cs:
        ts = []
        for rep in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ix = mips.maximus_build(Ut, It, C, 3, 0, 0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            del ix
            if rep >= warmup:
                ts.append((t1 - t0) * 1e3)
        ts.sort()
        print(json.dumps({"maximus_build_C": C, "build_ms_median": ts[len(ts) // 2],
                          "build_ms_min": ts[0], "builds": len(ts)}), flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(U, I, K, seconds_target=12.0, seconds_one=8.0):
    """The oracle as it stands, on bounded user samples: all host cores, and
    one core (the paper's setting)."""
    from oracle import topk as oracle_topk
    oracle_topk.build(force=False)
    cores = oracle_topk.num_threads()

    def rate(threads, target):
        probe = 256 if threads != 1 else 32
        t0 = time.perf_counter()
        oracle_topk.topk(U[:probe], I, K, nthreads=threads)
        dt = time.perf_counter() - t0
        n = int(min(U.shape[0], max(probe, probe * target / max(dt, 1e-6))))
        t0 = time.perf_counter()
        oracle_topk.topk(U[:n], I, K, nthreads=threads)
        dt = time.perf_counter() - t0
        return n, dt

    n, dt = rate(0, seconds_target)
    n1, dt1 = rate(1, seconds_one)
    return {"value": n / dt, "unit": "users/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} of {U.shape[0]} users x all {I.shape[0]} items, f={U.shape[1]}, "
                      f"K={K}, float64 keys + sorted K-list, {dt:.1f} s on {cores} threads",
            "cpu_model": cpu_model(),
            "one_core": {"value": n1 / dt1, "unit": "users/s", "cores": 1,
                         "sample": f"first {n1} users, {dt1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--K", type=int, default=10)
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the Maximus / precision-form / backward measurements")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--maximus-build", default="", metavar="C,C,...",
                    help="only time Maximus index builds on the clustered workload at these "
                         "cluster counts (one JSON line each) and exit")
    ap.add_argument("--precision-only", default="", metavar="PREC",
                    help="only run the 1,000,000 x 136,000 (f = 100, K = 10) workload with this "
                         "screen precision for --steps calls after --warmup, print one JSON line "
                         "and exit (the command the per-kernel counter passes profile)")
    ap.add_argument("--print-source-hash", action="store_true",
                    help="print the hash of the screen kernel sources and exit")
    args = ap.parse_args()
    if args.print_source_hash:
        print(screen_source_hash())
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.maximus_build:
        maximus_build_only([int(c) for c in args.maximus_build.split(",")], args.steps, args.warmup)
        return
    if args.precision_only:
        precision_only(args.precision_only, args.steps, args.warmup)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   "--gpus above 1 is not supported"}))
        sys.exit(2)

    import numpy as np
    import torch

    import mipsgen
    import paper_1706_01449_amd as mips

    K = args.K
    log("generating inputs")
    U, I = mipsgen.generate("mf", 0)
    n_u, f = U.shape
    n_i = I.shape[0]
    dev = torch.device("cuda:0")
    Ut = torch.from_numpy(U).to(dev)
    It = torch.from_numpy(I).to(dev)
    torch.cuda.synchronize()

    log(f"timing {args.precision} screen")
    t_main, ph_main, st_main, out, pc_main = time_path(mips, torch, Ut, It, K, args.precision,
                                                       args.steps, args.warmup)
    fp32 = None
    if not args.no_fp32 and args.precision != "fp32":
        log("timing fp32 screen")
        t32, ph32, st32, _, pc32 = time_path(mips, torch, Ut, It, K, "fp32", max(3, args.steps // 4), 1)
        fp32 = {"users_per_s": n_u / t32, "ms_per_step": t32 * 1e3,
                "ms_per_call_median": pc32["median"], "ms_per_call_min": pc32["min"],
                "screen_ms": ph32["screen"][0] / max(1, ph32["screen"][1])}

    # parity spot check on sampled users
    from oracle import topk as oracle_topk
    users = mipsgen.sample_users(n_u, 256, seed=123)
    ri, rk = oracle_topk.topk(U[users], I, K)
    gi = out[0].cpu().numpy()[users]
    gs = out[1].cpu().numpy()[users]
    match = float(np.mean(np.all(gi == ri, axis=1)))
    max_score_err = float(np.max(np.abs(gs - rk)))

    flops = 2.0 * n_u * n_i * f
    scr_ms = ph_main["screen"][0] / max(1, ph_main["screen"][1])
    achieved = flops / (scr_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    line = {
        "metric": "exact top-K users/sec (f=50,K=10): BF16-screen+rescore vs FP32 BMM; MFMA %",
        "value": n_u / t_main,
        "unit": "users/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_main * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "mf_480000x17770_f50", "n_users": n_u, "n_items": n_i, "f": f,
                   "K": K, "precision": args.precision, "parallelism": "single-gpu"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(), "kernel": "screen_kernel",
                     "kernel_ms": scr_ms},
        "ms_per_call": pc_main,
        "users_per_s_median_call": n_u / (pc_main["median"] * 1e-3),
        "phases_ms": {k: v[0] / max(1, v[1]) for k, v in ph_main.items() if v[1]},
        "fp32_screen": fp32,
        "index_match_sampled": match,
        "max_score_err_sampled": max_score_err,
        "stats": st_main,
    }
    if not args.no_extras:
        line["k_sweep"] = k_sweep(mips, torch, Ut, It, n_u)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(U, I, K)
    if not args.no_extras:
        del Ut, It, out
        torch.cuda.empty_cache()
        line["extras"] = extras(mips, torch, np, mipsgen, oracle_topk)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
