#!/usr/bin/env python
"""Benchmark of the Ozaki-II multiple-precision LU on one MI355X.

Workload: quad-double (4 x binary64 expansion, ~212 bits) LU with partial
pivoting of the Lotkin matrix of order n = 2048 (row 0 all ones, a_ij =
1/(i+j+1) below, each entry rounded greedily to QD), panel width b = 256,
Schur updates by the Ozaki-II INT8 path, followed by the solve with
b = A * ones.  One step = copy the resident input to the work buffer,
getrf, getrs.  Inputs are generated on the host and uploaded before the
timed region.

Also measured in the same run (not part of `value`):
  * the native QD LU on the same GPU -- the same panel and solve with the
    Schur update done by expansion multiply-subtracts (blocked naive, same b)
    and the unblocked b = 1 LU; the faster of the two is the comparator;
  * per-kernel times from HIP events on the library's stream, their
    algorithmic bytes / operations, and roofline fractions;
  * the CPU oracle on a bounded sample (rank 0 only).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from fractions import Fraction

METRIC = "QD LU n=2048 time vs native-QD GPU LU; Ozaki-II GEMM GOPS & % INT8 MFMA peak"
PEAK_HBM_GBS = 8000.0
PEAK_INT8_TOPS = 5000.0
# dense MFMA peaks of MI355X per back-end of the modular GEMM [TOP/s]
PEAK_MFMA = {"int8": 5000.0, "fp8": 5000.0, "f64": 78.6, "fp16": 2500.0}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def correct_bits(x_np):
    """min_i -log2 |x_i - 1| computed exactly (no binary64 underflow)."""
    worst = None
    for row in x_np.reshape(-1, x_np.shape[-1]):
        v = sum((Fraction(float(c)) for c in row), Fraction(0)) - 1
        if v == 0:
            continue
        v = abs(v)
        bits = v.denominator.bit_length() - v.numerator.bit_length()
        worst = bits if worst is None else min(worst, bits)
    return worst if worst is not None else 9999


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden")


def _qd_fraction(row):
    return sum((Fraction(float(c)) for c in row), Fraction(0))


def _ref_fraction(m, e, s, nl):
    mm = 0
    for q in range(nl - 1, -1, -1):
        mm = (mm << 64) | int(m[q])
    if mm == 0:
        return Fraction(0)
    v = Fraction(mm) * Fraction(2) ** (int(e) - 64 * nl)
    return -v if int(s) else v


def accuracy_vs_2p(ctx, n, nc, opts, method, block):
    """Error of the GPU's QD solve against the 2p-bit oracle solution of the
    same system (tests/golden/ref2p_*: the oracle's LU at p' = 448 bits,
    written by tests/golden/make_ref2p.py), for the well-conditioned R + n I
    and the graded D R D (c = 40) inputs: normwise relative error
    max_i |x_i - x'_i| / max_i |x'_i| as bits, computed exactly."""
    import numpy as np
    import torch

    import workloads as W
    out = {}
    for kind in ("wellcond", "graded40"):
        path = os.path.join(GOLDEN, f"ref2p_qd{n}_{kind}.npz")
        if nc != 4 or not os.path.exists(path):
            continue
        ref = np.load(path)
        rng = np.random.default_rng(int(ref["seed"]))
        A = W.wellcond(n, nc, rng) if kind == "wellcond" else W.graded(n, nc, 40.0, rng)
        rhs = W.rhs_ones(A)
        dA = torch.from_numpy(A).cuda()
        dx = torch.from_numpy(rhs).cuda()
        ipiv, info = ctx.getrf(dA, block=block, method=method, opts=opts)
        ctx.getrs(dA, ipiv, dx)
        ctx.sync_check()
        x = dx.cpu().numpy()[0]
        nl = int(ref["nl"])
        xr = [_ref_fraction(ref["m"][i], ref["e"][i], ref["s"][i], nl) for i in range(n)]
        num = max(abs(_qd_fraction(x[i]) - xr[i]) for i in range(n))
        den = max(abs(v) for v in xr)
        rel = num / den
        bits = (rel.denominator.bit_length() - rel.numerator.bit_length()) if rel else 9999
        out[kind] = {"err_bits_vs_2p": bits, "info": int(info.cpu()[0]),
                     "reference": f"oracle LU + solve at p'={64 * nl} bits"}
        log(f"accuracy {kind}: {bits} bits against the 2p oracle")
    return out


def schur_shapes(n, b):
    out = []
    for k in range(0, n, b):
        kb = min(b, n - k)
        if k + kb < n:
            out.append((n - k - kb, kb))
    return out


def op_counts(n, b):
    """Counts used to scale the oracle sample: panel + U12-solve multiply-
    subtracts, and Schur-update element x inner-index products."""
    P = 0.0
    U = 0.0
    for k in range(0, n, b):
        kb = min(b, n - k)
        nr = n - k
        m2 = n - k - kb
        P += nr * kb * kb / 2.0 + m2 * kb * kb / 2.0
        U += float(m2) * m2 * kb
    return P, U


PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
# kernels behind each profiled stage (one stage launch = one kernel dispatch
# for these stages)
STAGE_KERNELS = {"producer": ("k_producer_b", "k_producer", "k_producer_limbs"),
                 "gemm": ("k_gemm_i8_p", "k_gemm_i8", "k_gemm_f8", "k_gemm_f64"),
                 "consumer": ("k_consumer_mx", "k_consumer_b", "k_consumer", "k_consumer_limbs"),
                 "round": ("k_limb_round", "k_limb_sub")}


def traffic_of(stage, profile_md):
    """HBM bytes per launch of a stage's kernels from a committed rocprofv3
    counter summary (dispatch-weighted over the stage's kernels), or None
    when there is none or the kernel sources changed since it was taken."""
    from paper_2609_29554_amd import pmc
    s = pmc.load(os.path.join(PROFILES, profile_md))
    if not s or s.get("kernel_source_sha256") != pmc.source_sha():
        return None
    tot, n = 0.0, 0
    for fam in STAGE_KERNELS.get(stage, ()):
        rec = s["kernels"].get(fam)
        if rec and rec.get("hbm_bytes_per_launch") is not None:
            tot += rec["hbm_bytes_per_launch"] * rec["dispatches"]
            n += rec["dispatches"]
    return tot / n if n else None


def cpu_baseline(n_target, nc, b, n_sample):
    import oracle as O
    import workloads as W
    A = W.lotkin(n_sample, nc)
    rhs = W.rhs_ones(A)
    t0 = time.perf_counter()
    LU, ipiv, info, (tp, tu) = O.getrf(A, b, O.METHOD_OZAKI)
    t1 = time.perf_counter()
    O.getrs(LU, ipiv, rhs)
    t2 = time.perf_counter()
    Ps, Us = op_counts(n_sample, b)
    Pt, Ut = op_counts(n_target, b)
    scale_s = (n_target / n_sample) ** 2
    est = tp * Pt / Ps + tu * (Ut / Us if Us else 0.0) + (t2 - t1) * scale_s
    if n_sample == n_target:
        sample = (f"the whole workload: oracle getrf+getrs of the QD Lotkin matrix n={n_sample}, "
                  f"b={b} ({t2 - t0:.1f} s: panel+solve {tp:.1f} s, update {tu:.1f} s, getrs "
                  f"{t2 - t1:.1f} s)")
    else:
        sample = (f"full oracle getrf+getrs of the QD Lotkin matrix at n={n_sample}, b={b} "
                  f"({t2 - t0:.1f} s: panel+solve {tp:.1f} s, update {tu:.1f} s, getrs "
                  f"{t2 - t1:.1f} s), scaled to n={n_target} by panel op counts "
                  f"({Pt / Ps:.1f}x), Schur op counts ({Ut / max(Us, 1):.1f}x) and n^2 for getrs")
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": est, "unit": "s", "cores": min(threads, os.cpu_count() or threads),
            "kind": "oracle", "sample": sample}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--nc", type=int, default=4)
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--native-steps", type=int, default=1)
    ap.add_argument("--no-native", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probes", action="store_true",
                    help="skip the batched-LU, limb-LU and limb back-end probes of the default line")
    ap.add_argument("--cpu-sample-n", type=int, default=2048)
    ap.add_argument("--workload", choices=["lu", "gemm", "schur", "batch", "limb-schur", "limb-lu",
                                           "limb-gemm"],
                    default="lu",
                    help="lu: QD Lotkin LU (default); gemm: standalone TD product m=n=k=4096; "
                         "schur: only the LU's Ozaki-II Schur-update products (for profiling); "
                         "batch: 256 DD/QD systems n in [64, 512] in one persistent launch; "
                         "limb-schur: the Schur-update products of the Lotkin LU n=2048, "
                         "b=256 at p=4096 (64-limb numbers); limb-lu: the whole Lotkin LU + "
                         "solve on limb numbers (--limb-n, --limb-p, --limb-block; Table lotkin: "
                         "n=512, p=3136, b=256); limb-gemm: the limb product n=512 on the INT8 "
                         "and binary64 back-ends over p (--sweep-p; Table backend_hp)")
    ap.add_argument("--limb-n", type=int, default=512)
    ap.add_argument("--limb-p", type=int, default=3136)
    ap.add_argument("--limb-block", type=int, default=256)
    ap.add_argument("--limb-leaf", type=int, default=32,
                    help="recursive panel / U12 solve down to this width, inner updates by "
                         "Ozaki-II (0 = unblocked panel)")
    ap.add_argument("--limb-native", choices=["auto", "yes", "no"], default="auto",
                    help="also time the native limb LU (blocked and unblocked); auto: n <= 1024")
    ap.add_argument("--nlimb", type=int, default=64)
    ap.add_argument("--sweep-p", default="1024,2048,4096,8192,16384",
                    help="precisions of the limb-gemm back-end sweep")
    ap.add_argument("--limb-gemm-n", type=int, default=512)
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--gemm-n", type=int, default=4096)
    ap.add_argument("--gemm-backend", choices=["int8", "fp8", "f64", "fp16"], default="int8")
    ap.add_argument("--gemm-plan", choices=["literal", "rule"], default="literal",
                    help="standalone TD product: 'literal' = at 159-bit scaling as the workload "
                         "states it (one slice, N_mod covering 2 k 2^318); 'rule' = the plan "
                         "rule of Sec. 3.2")
    ap.add_argument("--sweep-n", type=int, default=1024,
                    help="order of the back-end comparison LU (0 = skip)")
    ap.add_argument("--sweep-block", type=int, default=128)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --block and the INT8 back-end instead of the autotuner's choice")
    ap.add_argument("--batch-block", type=int, default=64,
                    help="panel width of the batched Ozaki-II LU (at most 256)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device copy of this size first (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the LU would shard 2D block-cyclic over a process grid). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2609_29554_amd as Z
    import workloads as W

    if args.copy_calibration_mib > 0:
        src = torch.ones(args.copy_calibration_mib * (1 << 20) // 8, dtype=torch.float64,
                         device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload == "gemm":
        return bench_gemm(args)
    if args.workload == "schur":
        return bench_schur(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "limb-schur":
        return bench_limb_schur(args)
    if args.workload == "limb-lu":
        return bench_limb_lu(args)
    if args.workload == "limb-gemm":
        return bench_limb_gemm(args)

    n, nc, b = args.n, args.nc, args.block
    log(f"generating Lotkin n={n} nc={nc}")
    A0 = W.lotkin(n, nc)
    rhs0 = W.rhs_ones(A0)
    ctx = Z.Context(0)
    dev = torch.device("cuda", 0)
    dA0 = torch.from_numpy(A0).to(dev)
    db0 = torch.from_numpy(rhs0).to(dev)
    dA = torch.empty_like(dA0)
    dx = torch.empty_like(db0)
    names = {Z.BE_INT8: "int8", Z.BE_FP8_B17: "fp8", Z.BE_F64MOD: "f64", Z.BE_FP16: "fp16"}
    tuning = None
    if args.no_autotune:
        run_opts = Z.make_opts(block=b, backend=Z.BE_INT8)
    else:
        log("autotune")
        import tempfile
        run_opts, tuning = ctx.tune(nc, n, os.path.join(tempfile.gettempdir(), "ozii_tune.json"))
        b = run_opts.block
        log(f"autotuner: b={b} update={'native' if run_opts.method == Z.METHOD_NAIVE else names[run_opts.backend]}")
    run_method = run_opts.method
    update_name = "native" if run_method == Z.METHOD_NAIVE else names[run_opts.backend or Z.BE_INT8]
    ctx.reserve(nc, 0, 0, 0, n, run_opts)

    def step(method, blk, opts=None):
        dA.copy_(dA0)
        dx.copy_(db0)
        ipiv, info = ctx.getrf(dA, block=blk, method=method, opts=opts)
        ctx.getrs(dA, ipiv, dx)
        return ipiv, info

    log("warmup")
    for _ in range(args.warmup):
        step(run_method, b, run_opts)
    ctx.sync_check()
    ctx.set_profiling(True)
    ctx.profile_read()
    log(f"timing {args.steps} steps")
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record()
        ipiv, info = step(run_method, b, run_opts)
        evs[i][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = sorted(a.elapsed_time(z) for a, z in evs)
    prof = ctx.profile_read()
    ctx.set_profiling(False)
    ctx.sync_check()
    sec = (t1 - t0) / args.steps
    info_v = int(info.cpu()[0])
    bits = correct_bits(dx.cpu().numpy())
    log(f"ozaki step {sec * 1e3:.2f} ms, info={info_v}, correct bits={bits}")

    K = args.steps
    stages = {k: {"ms_per_step": v[0] / K, "launches_per_step": v[1] / K} for k, v in prof.items()
              if v[1]}

    def roof(name, bound):
        ms, launches, by, ops = prof[name]
        if not launches or ms <= 0:
            return None
        per_launch_ms = ms / launches
        traffic = (traffic_of(name, f"pmc_traffic_lu_qd{n}_lotkin_b{b}.md")
                   if update_name == "int8" else None)
        if bound == "mfma":
            peak = PEAK_MFMA[update_name]
            achieved = ops / launches / (per_launch_ms * 1e-3) / 1e12
            return {"bound": "mfma", "achieved": achieved, "peak": peak,
                    "unit": "TOP/s", "frac": achieved / peak, "traffic": traffic,
                    "kernel": name, "avg_launch_ms": per_launch_ms, "launches": launches / K,
                    "algorithmic_bytes_per_launch": by / launches}
        achieved = by / launches / (per_launch_ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": name,
                "avg_launch_ms": per_launch_ms, "launches": launches / K,
                "algorithmic_bytes_per_launch": by / launches}

    if run_method == Z.METHOD_NAIVE:
        rooflines = {}
        dominant = None
    else:
        rooflines = {"gemm": roof("gemm", "mfma"), "producer": roof("producer", "hbm"),
                     "consumer": roof("consumer", "hbm")}
        ozk = ("producer", "gemm", "consumer")
        if prof["fused"][1]:
            # (S4)-(S6) in one kernel: priced on its modular GEMM operations
            rooflines["fused"] = roof("fused", "mfma")
            ozk = ozk + ("fused",)
        ozk_ms = {k: prof[k][0] for k in ozk}
        dominant = max(ozk_ms, key=lambda k: ozk_ms[k])
    schur_ms = sum(prof[k][0] for k in ("exponents", "producer", "gemm", "consumer", "fused")) / K
    gemm_stage = "gemm" if prof["gemm"][1] or not prof["fused"][1] else "fused"
    gemm_ms, gemm_ops = prof[gemm_stage][0], prof[gemm_stage][3]
    gops = gemm_ops / (gemm_ms * 1e-3) / 1e9 if gemm_ms > 0 else None

    native = None
    if not args.no_native:
        # the paper's comparators: the same blocked LU with the native update
        # (same b; here under both schedules, the one the Ozaki-II run uses
        # first) and the unblocked LU; the speedup is against the fastest
        nat = {}
        same = run_opts.flags & Z.F_NO_LOOKAHEAD
        variants = [("blocked_naive" + ("" if same else "_lookahead"), b, same),
                    ("blocked_naive" + ("_lookahead" if same else ""), b, same ^ Z.F_NO_LOOKAHEAD),
                    ("unblocked", 1, Z.F_NO_LOOKAHEAD)]
        for label, blk, fl in variants:
            log(f"native {label}")
            nopts = Z.make_opts(flags=fl)
            step(Z.METHOD_NAIVE, blk, nopts)          # warm
            torch.cuda.synchronize()
            ctx.set_profiling(True)
            ctx.profile_read()
            tt0 = time.perf_counter()
            for _ in range(args.native_steps):
                step(Z.METHOD_NAIVE, blk, nopts)
            torch.cuda.synchronize()
            tt1 = time.perf_counter()
            p2 = ctx.profile_read()
            ctx.set_profiling(False)
            nat[label] = {"s": (tt1 - tt0) / args.native_steps,
                          "update_ms": p2["naive_update"][0] / args.native_steps,
                          "panel_ms": p2["panel"][0] / args.native_steps,
                          "lookahead": not (fl & Z.F_NO_LOOKAHEAD)}
            log(f"native {label}: {nat[label]['s'] * 1e3:.1f} ms")
        best_label = min(nat, key=lambda k: nat[k]["s"])
        best = nat[best_label]["s"]
        native = {**nat, "best": best_label, "best_s": best, "speedup_vs_native": best / sec,
                  "speedup_vs_same_schedule": nat[variants[0][0]]["s"] / sec}

    log("accuracy against the 2p-bit oracle")
    accuracy = accuracy_vs_2p(ctx, n, nc, run_opts, run_method, b)
    accuracy["lotkin"] = {"correct_bits_vs_ones": bits,
                          "note": "Lotkin n=2048 is far beyond QD's reach (log2 cond about "
                                  "5.1 n, Sec. 4.3): no correct bit is expected"}
    sweep = backend_sweep(ctx, args) if args.sweep_n > 0 else None
    td_gemm = td_gemm_probe(args.gemm_n) if args.gemm_n > 0 else None
    batch = limb = limb_gemm = None
    if not args.no_probes:
        log("batch probe")
        batch = batch_probe(args)
        log("limb LU probe (Table lotkin point)")
        limb = limb_lu_measure(512, 3136, 256, args.limb_leaf, 2, 1, "yes")
        log("limb product back-end sweep (Table backend_hp)")
        limb_gemm = limb_gemm_sweep(ctx, args.limb_gemm_n,
                                    [int(x) for x in args.sweep_p.split(",") if x], 2)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(n, nc, b, args.cpu_sample_n)

    out = {
        "metric": METRIC,
        "value": sec,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "step_ms": {"median": step_ms[len(step_ms) // 2], "min": step_ms[0], "max": step_ms[-1],
                    "how": "HIP events on the stream around each timed step"},
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"int8": "f64x4+i8", "fp8": "f64x4+fp8", "f64": "f64x4", "fp16": "f64x4+f16",
                  "native": "f64x4"}[update_name],
        "data": "synthetic",
        "config": {"workload": f"Lotkin quad-double LU n={n} (getrf+getrs), b={b}, Schur update "
                               f"{'Ozaki-II ' + update_name if update_name != 'native' else 'native'}"
                               f"{'' if run_opts.flags & Z.F_NO_LOOKAHEAD else ', look-ahead'}"
                               f"{', fused (S4)-(S6)' if run_opts.flags & Z.F_FUSED else ''}"
                               f"{' (autotuned)' if tuning else ''}",
                   "n": n, "nc": nc, "block": b, "update": update_name,
                   "lookahead": not (run_opts.flags & Z.F_NO_LOOKAHEAD),
                   "nslice": run_opts.nslice, "gemm_tile": run_opts.gemm_tile,
                   "fused": bool(run_opts.flags & Z.F_FUSED)},
        "autotune": tuning,
        "roofline": rooflines[dominant] if dominant else None,
        "rooflines": rooflines,
        "cpu_baseline": cpu,
        "native_qd_lu": native,
        "schur_update_ms": schur_ms,
        "gemm_gops": gops,
        "gemm_frac_peak": (gops / 1e3 / PEAK_MFMA.get(update_name, PEAK_INT8_TOPS)) if gops else None,
        "gemm_td": td_gemm,
        "stages": stages,
        "info": info_v,
        "correct_bits": bits,
        "accuracy": accuracy,
        "backend_sweep": sweep,
        "batch256": batch,
        "limb_lu_lotkin512_p3136": limb,
        "limb_gemm_backend_sweep": limb_gemm,
    }
    ctx.close()
    print(json.dumps(out))


def td_gemm_probe(n, steps=3):
    """The GEMM half of the headline metric on its own configuration: the
    standalone triple-double Ozaki-II product m = n = k = n (INT8) at 159-bit
    scaling as the workload states it (one slice, 48 moduli), and beside it
    with the plan rule of Sec. 3.2; modular GEMM GOPS and fraction of the INT8
    MFMA peak, timed with the library's HIP events (same recipe as
    --workload gemm)."""
    import numpy as np
    import torch

    import paper_2609_29554_amd as Z
    import workloads as W

    nc = 3
    rng = np.random.default_rng(20260932)
    dA = torch.from_numpy(W.random_expansions(n, n, nc, rng, exp_sigma=4.0)).cuda()
    dB = torch.from_numpy(W.random_expansions(n, n, nc, rng, exp_sigma=4.0)).cuda()
    dC = torch.zeros_like(dA)
    ctx = Z.Context(0)
    out = {"workload": f"Ozaki-II product C=AB, triple-double, m=n=k={n}, INT8"}
    for plan, qb in (("literal", 159), ("rule", 0)):
        opts = Z.make_opts(backend=Z.BE_INT8, qbits=qb)
        S, w, Q, nmod, _ = Z.plan_query(53 * nc, n, opts)
        ctx.gemm(0, dA, dB, dC, opts)
        ctx.sync_check()
        ctx.set_profiling(True)
        ctx.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.gemm(0, dA, dB, dC, opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = ctx.profile_read()
        ctx.set_profiling(False)
        ms, launches, _, ops = prof["gemm"]
        gops = ops / (ms * 1e-3) / 1e9
        out[plan] = {"S": S, "w": w, "nmod": nmod, "product_ms": (t1 - t0) / steps * 1e3,
                     "gemm_ms": ms / launches, "gemm_gops": gops,
                     "gemm_frac_int8_peak": gops / 1e3 / PEAK_INT8_TOPS,
                     "stages_ms": {k: v[0] / steps for k, v in prof.items() if v[1]}}
    ctx.close()
    return out


def backend_sweep(ctx, args):
    """Quad-double Lotkin LU + solve at n = sweep_n, b = sweep_block with the
    Schur update on each back-end of the modular GEMM (INT8, FP8 E4M3
    base-17, binary64 moduli, FP16) and natively; one timed step each after a
    warm-up step.  Reports seconds, Schur-update time and the modular GEMM
    rate against that engine's MFMA peak."""
    import torch

    import paper_2609_29554_amd as Z
    import workloads as W

    n, b, nc = args.sweep_n, args.sweep_block, args.nc
    A0 = torch.from_numpy(W.lotkin(n, nc)).cuda()
    r0 = torch.from_numpy(W.rhs_ones(W.lotkin(n, nc))).cuda()
    dA, dx = torch.empty_like(A0), torch.empty_like(r0)
    out = {"workload": f"Lotkin quad-double LU n={n} b={b} (getrf+getrs)"}
    for name, be, method in (("int8", Z.BE_INT8, Z.METHOD_OZAKI), ("fp8", Z.BE_FP8_B17, Z.METHOD_OZAKI),
                             ("f64", Z.BE_F64MOD, Z.METHOD_OZAKI), ("fp16", Z.BE_FP16, Z.METHOD_OZAKI),
                             ("native", Z.BE_INT8, Z.METHOD_NAIVE)):
        opts = Z.make_opts(backend=be)

        def run():
            dA.copy_(A0)
            dx.copy_(r0)
            ipiv, info = ctx.getrf(dA, block=b, method=method, opts=opts)
            ctx.getrs(dA, ipiv, dx)

        log(f"sweep {name}")
        run()
        ctx.sync_check()
        torch.cuda.synchronize()
        ctx.set_profiling(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = ctx.profile_read()
        ctx.set_profiling(False)
        ctx.sync_check()
        rec = {"s": t1 - t0, "correct_bits": correct_bits(dx.cpu().numpy())}
        if method == Z.METHOD_OZAKI:
            rec["schur_update_ms"] = sum(prof[k][0] for k in ("exponents", "producer", "gemm", "consumer"))
            ms, la, by, ops = prof["gemm"]
            if la and ms > 0:
                ach = ops / (ms * 1e-3) / 1e12
                rec["gemm"] = {"achieved": ach, "peak": PEAK_MFMA[name], "unit": "TOP/s",
                               "frac": ach / PEAK_MFMA[name], "ms": ms}
            S, w, Q, nmod, _ = Z.plan_query(53 * nc, b, opts)
            rec["plan"] = {"S": S, "w": w, "nmod": nmod}
        else:
            rec["schur_update_ms"] = prof["naive_update"][0]
        out[name] = rec
        log(f"sweep {name}: {rec['s'] * 1e3:.1f} ms, Schur {rec['schur_update_ms']:.2f} ms")
    return out


def _batch_run(ctx, systems, opts, args):
    """Upload, capture and replay one batch; returns (seconds per step,
    per-solve durations, completion times, info values)."""
    import numpy as np
    import torch

    src, work = [], []
    for nc, A, b in systems:
        n = A.shape[0]
        src.append((torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()))
        work.append((torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda(),
                     torch.zeros(n, dtype=torch.int64, device="cuda"),
                     torch.zeros(1, dtype=torch.int32, device="cuda")))
    ctx.batch_prepare(work, opts)
    times = torch.zeros(2 * len(work), dtype=torch.int64, device="cuda")
    ctx.batch_run(times)          # eager warm-up
    ctx.sync_check()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for (a0, b0), (a, bb, _, _) in zip(src, work):
                a.copy_(a0)
                bb.copy_(b0)
            ctx.batch_run(times)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync_check()
    t = times.cpu().numpy().reshape(-1, 2).astype(np.float64) / 100e6   # seconds
    dur = t[:, 1] - t[:, 0]
    done = t[:, 1] - t[:, 0].min()
    infos = [int(w[3].cpu()[0]) for w in work]
    return (t1 - t0) / args.steps, dur, done, infos


def bench_batch(args):
    """The batched configuration: count independent systems (orders uniform in
    [64, 512], half DD half QD, graded D R D) factored and solved in one
    persistent launch captured in a hipGraph; a step restores the inputs and
    replays the graph.  Reports the per-solve latency from device timestamps
    (the 100 MHz real-time counter at each system's start and end) for the
    blocked LU with the in-workgroup Ozaki-II update (block --batch-block),
    and beside it the unblocked LU with the native expansion update."""
    import numpy as np

    import paper_2609_29554_amd as Z
    import workloads as W

    rng = np.random.default_rng(20260934)
    log(f"generating {args.batch_count} systems")
    systems = W.batch_systems(args.batch_count, rng)
    ctx = Z.Context(0)
    ns = [A.shape[0] for _, A, _ in systems]

    ncs = np.array([nc for nc, _, _ in systems])

    def stats(sec, dur, done, infos):
        by_fmt = {{2: "DD", 3: "TD", 4: "QD"}[c]: {"p50": float(np.percentile(dur[ncs == c], 50)) * 1e3,
                                                  "p99": float(np.percentile(dur[ncs == c], 99)) * 1e3}
                  for c in sorted(set(ncs.tolist()))}
        return {"ms_per_step": sec * 1e3, "latency_by_format_ms": by_fmt,
                "latency_ms": {"p50": float(np.percentile(dur, 50)) * 1e3,
                               "p99": float(np.percentile(dur, 99)) * 1e3,
                               "max": float(dur.max()) * 1e3},
                "completion_ms": {"p50": float(np.percentile(done, 50)) * 1e3,
                                  "p99": float(np.percentile(done, 99)) * 1e3,
                                  "makespan": float(done.max()) * 1e3},
                "nonzero_info": int(sum(1 for v in infos if v != 0))}

    log(f"Ozaki-II update, b = {args.batch_block}")
    oz = stats(*_batch_run(ctx, systems, Z.make_opts(block=args.batch_block,
                                                     method=Z.METHOD_OZAKI), args))
    log("native update")
    nat = stats(*_batch_run(ctx, systems, None, args))
    out = {"metric": "batched DD/QD LU + solve: per-solve latency p50/p99",
           "value": oz["latency_ms"]["p99"], "unit": "ms (p99 per-solve latency)",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": oz["ms_per_step"],
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64x2/f64x4",
           "data": "synthetic",
           "config": {"workload": f"{len(systems)} independent systems, n in [64, 512] (mean "
                                  f"{np.mean(ns):.0f}), half DD half QD, graded D R D, one persistent "
                                  f"launch in a captured hipGraph; blocked LU b = {args.batch_block} "
                                  f"with the Ozaki-II update (INT8) inside each workgroup"},
           "latency_ms": oz["latency_ms"], "latency_by_format_ms": oz["latency_by_format_ms"],
           "completion_ms": oz["completion_ms"],
           "nonzero_info": oz["nonzero_info"],
           "native_update": dict(nat, config="unblocked LU, native expansion update")}
    ctx.close()
    print(json.dumps(out))


def bench_schur(args):
    """The Ozaki-II Schur updates of the QD Lotkin LU (n, b) alone: for every
    step, C = C - A B with the update's shape (M = N = n-k-b, K = b) on blocks
    of the Lotkin matrix.  Same kernels, shapes and plan as inside the LU, no
    panel; used to take hardware counters of the update kernels."""
    import torch

    import paper_2609_29554_amd as Z
    import workloads as W

    n, nc, b = args.n, args.nc, args.block
    A0 = torch.from_numpy(W.lotkin(n, nc)).cuda()
    ctx = Z.Context(0)
    shapes = schur_shapes(n, b)
    work = [(A0[:kb, b:b + m].clone(), A0[b:b + m, :kb].clone(), A0[b:b + m, b:b + m].clone())
            for m, kb in shapes]   # (K x M), (N x K), (N x M) blocks in (cols, rows, nc) layout
    ctx.reserve(nc, shapes[0][0], shapes[0][0], b, 0, None)
    for _ in range(max(args.warmup, 1)):
        for L21, U12, A22 in work:
            ctx.gemm(1, L21, U12, A22)
    ctx.sync_check()
    ctx.set_profiling(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for L21, U12, A22 in work:
            ctx.gemm(1, L21, U12, A22)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.set_profiling(False)
    sec = (t1 - t0) / args.steps
    out = {"metric": METRIC, "value": sec, "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64x4+i8", "data": "synthetic",
           "config": {"workload": f"Ozaki-II Schur updates of the QD Lotkin LU n={n} b={b}",
                      "shapes": shapes},
           "stages": {k: {"ms_per_step": v[0] / args.steps, "launches_per_step": v[1] / args.steps}
                      for k, v in prof.items() if v[1]}}
    ctx.close()
    print(json.dumps(out))


def bench_gemm(args):
    """Standalone Ozaki-II product C = A B, triple-double, m = n = k = N,
    entries with uniform mantissas and exponents round(N(0, 16))."""
    import numpy as np
    import torch

    import paper_2609_29554_amd as Z
    import workloads as W

    n, nc = args.gemm_n, 3
    log(f"generating TD operands n={n}")
    rng = np.random.default_rng(20260932)
    A = W.random_expansions(n, n, nc, rng, exp_sigma=4.0)
    B = W.random_expansions(n, n, nc, rng, exp_sigma=4.0)
    ctx = Z.Context(0)
    dA = torch.from_numpy(A).cuda()
    dB = torch.from_numpy(B).cuda()
    dC = torch.zeros_like(dA)
    be = {"int8": Z.BE_INT8, "fp8": Z.BE_FP8_B17, "f64": Z.BE_F64MOD, "fp16": Z.BE_FP16}[args.gemm_backend]
    opts = Z.make_opts(backend=be, qbits=159 if args.gemm_plan == "literal" else 0)
    peak = PEAK_MFMA[args.gemm_backend]
    S, w, Q, nmod, _ = Z.plan_query(53 * nc, n, opts)
    ctx.reserve(nc, n, n, n, 0, opts)
    for _ in range(args.warmup):
        ctx.gemm(0, dA, dB, dC, opts)
    ctx.sync_check()
    ctx.set_profiling(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.gemm(0, dA, dB, dC, opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.set_profiling(False)
    sec = (t1 - t0) / args.steps
    K = args.steps
    ms, launches, by, ops = prof["gemm"]
    ach = ops / launches / (ms / launches * 1e-3) / 1e12
    prof_md = (f"pmc_traffic_gemm_td{n}_{args.gemm_backend}"
               f"{'_literal' if args.gemm_plan == 'literal' else ''}.md")
    roof = {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TOP/s",
            "frac": ach / peak, "traffic": traffic_of("gemm", prof_md), "kernel": "gemm",
            "avg_launch_ms": ms / launches, "algorithmic_bytes_per_launch": by / launches}
    rooflines = {"gemm": roof}
    for k in ("producer", "consumer"):
        m2, l2, b2, _ = prof[k]
        a2 = b2 / l2 / (m2 / l2 * 1e-3) / 1e9
        rooflines[k] = {"bound": "hbm", "achieved": a2, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": a2 / PEAK_HBM_GBS, "traffic": traffic_of(k, prof_md), "kernel": k,
                        "avg_launch_ms": m2 / l2, "algorithmic_bytes_per_launch": b2 / l2}
    out = {
        "metric": METRIC, "value": sec, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64x3+i8", "data": "synthetic",
        "config": {"workload": f"Ozaki-II product C=AB, triple-double, m=n=k={n}"
                               f"{', 159-bit scaling' if args.gemm_plan == 'literal' else ', plan rule'}",
                   "backend": args.gemm_backend, "plan": args.gemm_plan, "S": S, "w": w,
                   "nmod": nmod},
        "roofline": roof, "rooflines": rooflines,
        "effective_gflops_td": 2.0 * n ** 3 / sec / 1e9,
        "stages": {k: {"ms_per_step": v[0] / K} for k, v in prof.items() if v[1]},
    }
    ctx.close()
    print(json.dumps(out))


def limb_cpu_baseline(nl, shapes, sample_mn=16):
    """The limb oracle on one update of sample_mn x sample_mn x b, timed per
    phase and scaled to the workload: residues by (M+N)K, modular products
    by MNK, CRT and rounding by MN."""
    import numpy as np

    import oracle as O
    import oracle.limbs as OL
    import workloads as W

    K = shapes[0][1]
    rng = np.random.default_rng(20260933)
    A = W.random_limbs(sample_mn, K, nl, rng, exp_sigma=2.0)
    B = W.random_limbs(K, sample_mn, nl, rng, exp_sigma=2.0)
    Cz = W.random_limbs(sample_mn, sample_mn, nl, rng, exp_sigma=2.0)
    pl = O.make_plan(64 * nl, K)
    t0 = time.perf_counter()
    ea, eb = OL.exponents(A, True), OL.exponents(B, False)
    pa = OL.residues(A, True, ea, pl)
    pb = OL.residues(B, False, eb, pl)
    t1 = time.perf_counter()
    tpl = O.modgemm(pa, pb, pl)
    t2 = time.perf_counter()
    OL.ozgemm(1, A, B, Cz, pl)   # the whole product again: CRT and rounding are its remainder
    t3 = time.perf_counter()
    t_rest = max((t3 - t2) - (t2 - t0), 0.0)
    s_mn = float(sample_mn * sample_mn)
    res = sum(2.0 * m * kb for m, kb in shapes) / (2.0 * sample_mn * K)
    mnk = sum(float(m) * m * kb for m, kb in shapes) / (s_mn * K)
    mn = sum(float(m) * m for m, _ in shapes) / s_mn
    est = (t1 - t0) * res + (t2 - t1) * mnk + t_rest * mn
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": est, "unit": "s", "cores": min(threads, os.cpu_count() or threads),
            "kind": "oracle",
            "sample": (f"limb oracle on one {sample_mn}x{sample_mn}x{K} update at p={64 * nl} "
                       f"(residues {t1 - t0:.1f} s, modular products {t2 - t1:.1f} s, CRT and "
                       f"rounding {t_rest:.1f} s), scaled to the seven updates by (M+N)K "
                       f"({res:.0f}x), MNK ({mnk:.0f}x) and MN ({mn:.0f}x)")}


def bench_limb_schur(args):
    """The Ozaki-II Schur updates of a blocked LU of the Lotkin matrix at
    p = 64 nlimb bits (n, b): for every step, C = RN_p(C - RN_p(A B)) with
    A = A[k+b:, k:k+b], B = A[k:k+b, k+b:], C = A[k+b:, k+b:] of the Lotkin
    matrix, updated in place through sub-block descriptors (no copies)."""
    import ctypes
    import numpy as np
    import torch

    import paper_2609_29554_amd as Z
    import workloads as W

    n, b, nl = args.n, args.block, args.nlimb
    log(f"generating Lotkin limbs n={n} p={64 * nl}")
    limb, ex, sg = W.lotkin_limbs(n, nl)
    dl = torch.from_numpy(limb.view(np.int64)).cuda()
    de = torch.from_numpy(ex).cuda()
    ds = torch.from_numpy(sg).cuda()
    del limb, ex, sg
    ctx = Z.Context(0)
    shapes = schur_shapes(n, b)

    def desc(r0, c0):
        off = r0 + c0 * n
        return Z.Limbs(dl.data_ptr() + 8 * off, de.data_ptr() + 4 * off, ds.data_ptr() + off,
                       n, n * n)

    work = []
    for k in range(0, n - b, b):
        m = n - k - b
        work.append((m, b, desc(k + b, k), desc(k, k + b), desc(k + b, k + b)))

    def step():
        for m, kb, A, B, Cd in work:
            ctx._call(Z.lib().ozII_gemm_limbs(ctx._h, 1, nl, m, m, kb, ctypes.byref(A),
                                              ctypes.byref(B), ctypes.byref(Cd), None))

    ctx._bind()
    for _ in range(max(args.warmup, 1)):
        step()
    ctx.sync_check()
    ctx.set_profiling(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.set_profiling(False)
    ctx.sync_check()
    sec = (t1 - t0) / args.steps
    S, w, Q, nmod, _ = Z.plan_query(64 * nl, b)
    ms, launches, by, ops = prof["gemm"]
    ach = ops / launches / (ms / launches * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": ach, "peak": PEAK_MFMA["int8"], "unit": "TOP/s",
            "frac": ach / PEAK_MFMA["int8"],
            "traffic": traffic_of("gemm", f"pmc_traffic_limb_schur_p{64 * nl}.md"),
            "kernel": "gemm", "avg_launch_ms": ms / launches, "launches": launches / args.steps,
            "algorithmic_ops_per_launch": ops / launches}
    rooflines = {"gemm": roof}
    for k in ("producer", "consumer", "round"):
        m2, l2, b2, _ = prof[k]
        if not l2:
            continue
        a2 = b2 / l2 / (m2 / l2 * 1e-3) / 1e9
        rooflines[k] = {"bound": "hbm", "achieved": a2, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": a2 / PEAK_HBM_GBS,
                        "traffic": traffic_of(k, f"pmc_traffic_limb_schur_p{64 * nl}.md"),
                        "kernel": k,
                        "avg_launch_ms": m2 / l2, "algorithmic_bytes_per_launch": b2 / l2}
    out = {"metric": METRIC, "value": sec, "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64 limbs+i8", "data": "synthetic",
           "config": {"workload": f"Ozaki-II Schur updates of the Lotkin LU n={n} b={b} at "
                                  f"p={64 * nl} (limb format)", "S": S, "w": w, "nmod": nmod,
                      "shapes": shapes},
           "roofline": roof, "rooflines": rooflines,
           "stages": {k: {"ms_per_step": v[0] / args.steps,
                          "launches_per_step": v[1] / args.steps}
                      for k, v in prof.items() if v[1]}}
    ctx.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (limb oracle sample)")
        out["cpu_baseline"] = limb_cpu_baseline(nl, shapes)
    print(json.dumps(out))


# Sec. 4.1.6, Table backend_hp, GPU block (H100): product of n = 512 limb
# matrices, time [ms] on INT8 and on binary64 moduli, modulus counts
PAPER_BACKEND_HP = {1024: (12.7, 7.4, 45, 15), 2048: (40.0, 22.6, 49, 16),
                    4096: (132.8, 74.8, 54, 16), 8192: (511.5, 272.7, 53, 16),
                    16384: (1900.8, 1046.5, 54, 16)}


def limb_gemm_sweep(ctx, n, ps, steps):
    """C = RN_p(A B) for random n x n limb matrices (exponents spread by
    N(0, 4), 5 % zeros) at each p, on the INT8 and the binary64 back-ends:
    HIP-event time per product, plan, modular-GEMM rate; returns a dict."""
    import numpy as np
    import torch

    import paper_2609_29554_amd as Z
    import workloads as W

    rows = {}
    for p in ps:
        nl = p // 64
        rng = np.random.default_rng(p)
        dev = []
        for _ in range(2):
            limb, ex, sg = W.random_limbs(n, n, nl, rng, exp_sigma=4.0, zero_frac=0.05)
            dev.append((torch.from_numpy(limb.view(np.int64)).cuda(), torch.from_numpy(ex).cuda(),
                        torch.from_numpy(sg).cuda()))
            del limb, ex, sg
        dA, dB = dev
        dC = tuple(torch.empty_like(x) for x in dA)
        row = {"paper_h100_ms": {"int8": PAPER_BACKEND_HP.get(p, (None,) * 4)[0],
                                 "f64": PAPER_BACKEND_HP.get(p, (None,) * 4)[1]},
               "paper_moduli": {"int8": PAPER_BACKEND_HP.get(p, (None,) * 4)[2],
                                "f64": PAPER_BACKEND_HP.get(p, (None,) * 4)[3]}}
        for name, be in (("int8", Z.BE_INT8), ("f64", Z.BE_F64MOD)):
            log(f"limb product n={n} p={p} {name}")
            opts = Z.make_opts(backend=be)
            ctx.gemm_limbs(0, dA, dB, dC, opts)       # warm: plan, workspace
            ctx.sync_check()
            ctx.set_profiling(True)
            ctx.profile_read()
            for _ in range(steps):
                ctx.gemm_limbs(0, dA, dB, dC, opts)
            ctx.sync_check()
            prof = ctx.profile_read()
            ctx.set_profiling(False)
            total = sum(v[0] for v in prof.values()) / steps
            gms, gl, _, gops = prof["gemm"]
            S, w, Q, nmod, _ = Z.plan_query(p, n, opts)
            ach = gops / (gms * 1e-3) / 1e12
            row[name] = {"ms": total, "gemm_ms": gms / steps,
                         "gemm_tops": ach, "gemm_frac": ach / PEAK_MFMA[name],
                         "S": S, "w": w, "nmod": nmod,
                         # (group, modulus) products: S (S + 1) / 2 slice pairs
                         "products": nmod * S * (S + 1) // 2,
                         "stages_ms": {k: v[0] / steps for k, v in prof.items() if v[1]}}
        row["ratio_int8_over_f64"] = row["int8"]["ms"] / row["f64"]["ms"]
        rows[p] = row
        del dA, dB, dC, dev
        torch.cuda.empty_cache()
    return rows


def bench_limb_gemm(args):
    import torch

    import paper_2609_29554_amd as Z

    ps = [int(x) for x in args.sweep_p.split(",") if x]
    ctx = Z.Context(0)
    rows = limb_gemm_sweep(ctx, args.limb_gemm_n, ps, args.steps)
    ctx.close()
    top = rows[max(ps)]
    best = min(top["int8"]["ms"], top["f64"]["ms"])
    out = {"metric": "limb product n=512 on INT8 vs binary64 moduli over p (Table backend_hp)",
           "value": best, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "ms_per_step": best, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "u64 limbs+i8/f64", "data": "synthetic",
           "config": {"workload": f"C = RN_p(A B), random n={args.limb_gemm_n} limb matrices, "
                                  f"p = {ps}", "value_at_p": max(ps)},
           "sweep": rows}
    print(json.dumps(out))


def host_limbs(X):
    """A device limb matrix back on the host, limbs as uint64."""
    import numpy as np
    lb, ex, sg = (x.cpu().numpy() for x in X)
    return lb.view(np.uint64), ex, sg


def limb_correct_bits(limb, ex, sg):
    """min_i floor(-log2 |x_i - 1|) of a limb vector, exactly (no binary64
    conversion, which would underflow at these precisions)."""
    from fractions import Fraction
    nl, n = limb.shape[0], limb.shape[-1]
    p = 64 * nl
    worst = None
    for i in range(n):
        m = 0
        for q in range(nl - 1, -1, -1):
            m = (m << 64) | int(limb[q, 0, i])
        v = Fraction(0) if m == 0 else Fraction(m) * Fraction(2) ** (int(ex[0, i]) - p)
        if sg[0, i]:
            v = -v
        d = abs(v - 1)
        if d == 0:
            continue
        bits = d.denominator.bit_length() - d.numerator.bit_length()
        if Fraction(2) ** (-bits) < d:
            bits -= 1
        worst = bits if worst is None else min(worst, bits)
    return worst if worst is not None else 1 << 30


# Table lotkin, GPU rows (total time of getrf + getrs in seconds, correct bits)
PAPER_LOTKIN = {(512, 3136): {"H100": {"naive_b1": 1.323, "naive_blk": 1.345, "ozaki": 1.308},
                              "GB10": {"naive_b1": 2.171, "naive_blk": 2.08, "ozaki": 1.651},
                              "bits": 545, "b": 256}}


def limb_lu_measure(n, p, b, leaf, steps, warmup, native_mode="auto"):
    """The Lotkin LU + solve on limb numbers (Sec. 4.3, Table lotkin): getrf
    with the Ozaki-II Schur update at panel width b (recursive panel down to
    `leaf` columns when leaf > 0), then getrs, timed together (median of
    `steps`); the same with the unblocked panel, the native variants
    (blocked naive at the same b, unblocked) and the correct bits of x
    against the true solution 1."""
    import numpy as np
    import torch

    import paper_2609_29554_amd as Z
    import workloads as W

    if p % 64 or not 64 <= p <= 4096:
        raise SystemExit("--limb-p must be a multiple of 64 in [64, 4096]")
    nl = p // 64
    log(f"generating Lotkin limbs n={n} p={p}")
    A = W.lotkin_limbs(n, nl)
    B = W.lotkin_rhs_limbs(n, nl)

    def up(X):
        return tuple(torch.from_numpy(np.ascontiguousarray(x).view(np.int64) if x.dtype == np.uint64
                                      else np.ascontiguousarray(x)).cuda() for x in X)

    dA0, dB0 = up(A), up(B)
    ctx = Z.Context(0)

    def run(method, blk, lf=0):
        dA = tuple(x.clone() for x in dA0)
        dX = tuple(x.clone() for x in dB0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ipiv, info = ctx.getrf_limbs(dA, block=blk, method=method, leaf=lf)
        ctx.getrs_limbs(dA, ipiv, dX)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.sync_check()
        return dt, dX, int(info.cpu()[0])

    log("warmup")
    for _ in range(max(warmup, 1)):
        run(Z.METHOD_OZAKI, b, leaf)
    ctx.set_profiling(True)
    ctx.profile_read()
    times = []
    for _ in range(steps):
        dt, dX, info = run(Z.METHOD_OZAKI, b, leaf)
        times.append(dt)
        log(f"ozaki step {dt:.3f} s")
    prof = ctx.profile_read()
    ctx.set_profiling(False)
    sec = sorted(times)[len(times) // 2]
    bits = limb_correct_bits(*host_limbs(dX))
    flat = None
    if leaf:
        dt, dXf, _ = run(Z.METHOD_OZAKI, b, 0)
        flat = {"s": dt, "correct_bits": limb_correct_bits(*host_limbs(dXf))}
        log(f"ozaki, unblocked panel {dt:.3f} s")
    native = None
    if native_mode == "yes" or (native_mode == "auto" and n <= 1024):
        native = {}
        for name, blk in (("naive_blk", b), ("naive_b1", n)):
            log(f"native {name}")
            dt, dXn, _ = run(Z.METHOD_NAIVE, blk)
            native[name] = {"s": dt, "block": blk,
                            "correct_bits": limb_correct_bits(*host_limbs(dXn))}
        best = min(v["s"] for v in native.values())
        native["speedup_vs_best_native"] = best / sec
    stages = {k: {"ms_per_step": v[0] / steps, "launches_per_step": v[1] / steps}
              for k, v in prof.items() if v[1]}
    roof = None
    if prof.get("gemm") and prof["gemm"][1]:
        ms, launches, _, ops = prof["gemm"]
        ach = ops / launches / (ms / launches * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": PEAK_MFMA["int8"], "unit": "TOP/s",
                "frac": ach / PEAK_MFMA["int8"], "traffic": None, "kernel": "gemm",
                "avg_launch_ms": ms / launches, "launches": launches / steps,
                "algorithmic_ops_per_launch": ops / launches}
    ctx.close()
    return {"s": sec, "steps_s": times, "n": n, "p": p, "block": b, "panel_leaf": leaf,
            "correct_bits": bits, "info": info, "ozaki_unblocked_panel": flat, "native": native,
            "roofline": roof, "stages": stages, "paper_context": PAPER_LOTKIN.get((n, p))}


def bench_limb_lu(args):
    """--workload limb-lu: limb_lu_measure at --limb-n / --limb-p /
    --limb-block / --limb-leaf, with the oracle timed on the host."""
    n, p, b = args.limb_n, args.limb_p, args.limb_block
    r = limb_lu_measure(n, p, b, args.limb_leaf, args.steps, args.warmup, args.limb_native)
    sec = r["s"]
    out = {"metric": METRIC, "value": sec, "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "u64 limbs+i8", "data": "synthetic",
           "config": {"workload": f"Lotkin LU + solve on limb numbers n={n} p={p} b={b} "
                                  f"(getrf_limbs Ozaki-II INT8 + getrs_limbs)",
                      "n": n, "p": p, "block": b, "panel_leaf": args.limb_leaf},
           **{k: r[k] for k in ("correct_bits", "info", "ozaki_unblocked_panel", "native",
                                "roofline", "stages", "paper_context")}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = limb_lu_cpu_baseline(n, p // 64)
    print(json.dumps(out))


def batch_probe(args, steps=2):
    """p50 / p99 per-solve latency and makespan of the batched configuration
    (the --workload batch recipe, fewer replays) for the main bench line."""
    import types

    import numpy as np

    import paper_2609_29554_amd as Z
    import workloads as W

    rng = np.random.default_rng(20260934)
    systems = W.batch_systems(args.batch_count, rng)
    ctx = Z.Context(0)
    a = types.SimpleNamespace(steps=steps, warmup=1)
    sec, dur, done, infos = _batch_run(ctx, systems, Z.make_opts(block=args.batch_block,
                                                                 method=Z.METHOD_OZAKI), a)
    ctx.close()
    return {"workload": f"{len(systems)} systems n in [64, 512], half DD half QD, graded D R D, "
                        f"one hipGraph-replayed persistent launch, Ozaki-II update b = "
                        f"{args.batch_block} (see --workload batch)",
            "latency_ms": {"p50": float(np.percentile(dur, 50)) * 1e3,
                           "p99": float(np.percentile(dur, 99)) * 1e3},
            "makespan_ms": float(done.max()) * 1e3,
            "nonzero_info": int(sum(1 for v in infos if v != 0))}


def limb_lu_cpu_baseline(n, nl, n_sample=256):
    """The p-bit oracle's LU + solve (unblocked, multiply-subtracts, as it
    stands) on the Lotkin matrix of order min(n, n_sample) at the same p,
    scaled by n^3 to the workload's order."""
    import oracle.lfloat as LF
    m = min(n, n_sample)
    A = LF.lotkin(m, nl)
    rhs = LF.rhs_times_ones(A)
    t0 = time.perf_counter()
    F, ip, _ = LF.getrf(A)
    LF.getrs(F, ip, rhs)
    t = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": t * (n / m) ** 3, "unit": "s", "cores": min(threads, os.cpu_count() or threads),
            "kind": "oracle",
            "sample": f"oracle getrf + getrs of the Lotkin matrix n={m} at p={64 * nl}: {t:.1f} s, "
                      f"scaled by (n/{m})^3"}


if __name__ == "__main__":
    main()
