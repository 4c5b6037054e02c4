"""Benchmark: panel-interactions/s of one FMM matvec y = P x on one MI355X.

Workload (default, --workload coils): two 5-turn square planar coils (trace
width 0.1, thickness 0.035, spacing 0.1, gap 0.5), ~200k flat triangle panels,
three current components as complex64 densities N(0,1), single right-hand
side, expansion order p = 8, leaves <= 64 panels, plain FP32 (M2L on the
vector ALUs).  The mixed-precision variant (FP32 M2L on MFMA, FP64 singular
integrals) and the surrogate + mixed variant (learned near-singular pairs)
run on the same inputs and are reported beside it.
--workload bga: the ~1M-panel BGA-like package with 6 ports x 3 components
= 18 complex columns, mixed precision as its own variant.

A step is one full matvec (gather, P2P, P2M, M2M, M2L, L2L, L2P, scatter)
with the near field already assembled and x, y resident in HBM.
panel-interactions per matvec = n_complex_columns * N^2.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12      # FP32 vector / FP32 MFMA (dense), MI355X
PEAK_FP64 = 78.6e12
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_variant(xrl, torch, tree, x, precision, steps, warmup, order=8, surrogate=None, engine="auto"):
    n_cols = x.shape[1]
    plan = xrl.Plan(tree, order=order, precision=precision, engine=engine, max_cols=n_cols)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = plan.assemble(surrogate=surrogate, audit_every=100 if surrogate is not None else 0)
    t_asm = time.perf_counter() - t0
    y = torch.empty_like(x)
    for _ in range(warmup):
        plan.matvec(x, y)
    torch.cuda.synchronize()
    # timed region: exactly `steps` matvecs, no profiling events inside
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.matvec(x, y)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    # per-phase device times from HIP events on the matvec stream
    plan.set_profiling(True)
    ph = {k: [] for k in xrl.PHASES}
    for _ in range(max(3, min(steps, 10))):
        plan.matvec(x, y)
        for k, v in plan.phase_ms().items():
            ph[k].append(v)
    plan.set_profiling(False)
    torch.cuda.synchronize()
    ph = {k: float(np.mean(v)) for k, v in ph.items()}
    return plan, y, t, t_asm, st, ph


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="coils", choices=["coils", "bga"])
    ap.add_argument("--n", type=int, default=200_000, help="target panel count of the coil mesh")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--variants", default=None, help="comma list of fp32, mixed, surrogate (first = headline); "
                    "name@engine overrides the translation engine (auto, mfma, valu, mfma_os, mfma_ts)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the matvec would shard).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2409_12375_amd import inputs as I
    from paper_2409_12375_amd import xrl

    torch.cuda.set_device(0)
    if args.workload == "coils":
        V, T = I.coils(args.n)
        n_c = 3
        variants = args.variants or "fp32,mixed,surrogate"
        desc = "two 5-turn square coils, %d triangle panels, 3 complex64 columns"
    else:
        V, T = I.bga()
        n_c = 18
        variants = args.variants or "mixed,fp32,surrogate"
        desc = "BGA-like package (10x10 plane, 400 holes, 100 vias, 100 balls), %d triangle panels, " \
               "18 complex64 columns (6 ports x 3 components)"
    N = len(T)
    xh = I.densities(N, n_c, np.complex64)
    x = torch.from_numpy(xh).cuda()
    log("%s: N=%d panels" % (args.workload, N))
    tree = xrl.Tree(V, T, max_leaf=64)
    sur_path = os.path.join(ROOT, "tests", "golden", "surrogate_mlp.npz")
    results = {}
    ys = {}
    for name in variants.split(","):
        base, _, engine = name.partition("@")
        prec = "mixed" if base == "surrogate" else base
        sur = None
        if base == "surrogate":
            if not os.path.exists(sur_path):
                log("no trained surrogate weights, skipping the surrogate variant")
                continue
            sur = xrl.Surrogate.load(sur_path)
        plan, y, t, t_asm, st, ph = run_variant(xrl, torch, tree, x, prec, args.steps, args.warmup, surrogate=sur,
                                                    engine=engine or "auto")
        info = plan.info()
        K = (8 + 1) ** 2
        C = 2 * n_c
        m2l_flops = 2.0 * K * K * C * info["n_m2l_pairs"]
        near_bytes = 4.0 * info["n_near_entries"] + 4.0 * info["n_near_rows"]
        results[name] = {
            "precision": prec, "ms_per_matvec": 1e3 * t, "assemble_s": t_asm,
            "panel_interactions_per_s": n_c * float(N) * N / t,
            "amortized_panel_interactions_per_s": n_c * float(N) * N / (t + t_asm / 36.0),
            "phase_ms": ph, "n_m2l_pairs": info["n_m2l_pairs"], "n_near_entries": info["n_near_entries"],
            "n_boxes": info["n_boxes"], "n_leaves": info["n_leaves"], "max_sep_ratio": info["max_sep_ratio"],
            "n_demoted_pairs": info["n_demoted_pairs"],
            "m2l_flops": m2l_flops, "m2l_tflops": m2l_flops / (ph["m2l"] * 1e-3) / 1e12,
            "p2p_gbps": near_bytes / (ph["p2p"] * 1e-3) / 1e9,
            "nearfield": {k: st[k] for k in ("n_self", "n_touching", "n_near_singular", "n_regular",
                                             "n_mlp_accepted", "n_mlp_fallback", "audit_max_rel_err",
                                             "audit_rms_rel_err", "ms")},
        }
        ys[name] = y.cpu().numpy()
        plan.close()
        log(name, json.dumps(results[name]))

    main_v = variants.split(",")[0]
    R = results[main_v]
    # dominant phase and its roofline
    dom = max(R["phase_ms"], key=R["phase_ms"].get)
    bound, achieved, peak, unit = "alu", R["m2l_tflops"], PEAK_FP32 / 1e12, "TFLOP/s"
    if dom == "p2p":
        bound, achieved, peak, unit = "hbm", R["p2p_gbps"], PEAK_HBM / 1e9, "GB/s"
    elif results[main_v]["precision"] == "mixed":
        bound = "mfma"
    roof = {"bound": bound, "kernel": "m2l" if dom != "p2p" else "p2p", "achieved": achieved, "peak": peak,
            "unit": unit, "frac": achieved / peak, "traffic": None}

    # accuracy and CPU baseline: the FP64 oracle on a bounded row sample
    cpu = None
    acc = {}
    if not args.no_cpu:
        import oracle as O
        rng = np.random.default_rng(7)
        order = rng.permutation(N)
        t0 = time.perf_counter()
        first = np.sort(order[:64])
        ref1, used = O.matvec(V, T, xh.astype(np.complex128), rows=first)
        t1 = time.perf_counter() - t0
        m_more = int(max(0, min(N - 64, (args.cpu_seconds - t1) / max(t1, 1e-3) * 64)))
        rows = np.sort(order[64:64 + m_more])
        if len(rows):
            ref2, _ = O.matvec(V, T, xh.astype(np.complex128), rows=rows)
        t_cpu = time.perf_counter() - t0
        allrows = np.concatenate([first, rows])
        ref = np.concatenate([ref1, ref2]) if len(rows) else ref1
        m = len(allrows)
        cpu = {"value": n_c * float(m) * N / t_cpu, "unit": "panel-interactions/s", "cores": int(used),
               "kind": "oracle",
               "sample": "%d random target rows x all %d source panels x %d complex columns, FP64 direct "
                         "summation, %.1f s" % (m, N, n_c, t_cpu)}
        for v, yv in ys.items():
            e = np.linalg.norm(yv[allrows] - ref, axis=0) / np.linalg.norm(ref, axis=0)
            acc[v] = float(e.max())
            results[v]["max_col_rel_l2"] = float(e.max())

    line = {
        "metric": "panel-interactions/s per FMM matvec at 1e-4 rel L2; surrogate+MP vs plain FP32",
        "value": R["panel_interactions_per_s"],
        "unit": "panel-interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": R["ms_per_matvec"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if main_v == "fp32" else ("f64" if main_v == "fp64" else "f32+f64"),
        "data": "synthetic",
        "config": {"workload": (desc % N) + ", p=8, leaf<=64, %s" % (
                       "plain FP32" if main_v == "fp32" else "mixed precision (FP32 MFMA M2L, FP64 singular)"),
                   "n_panels": N, "complex_columns": n_c, "order": 8, "max_leaf": 64},
        "roofline": roof,
        "cpu_baseline": cpu,
        "max_col_rel_l2": acc.get(main_v),
        "variants": results,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
