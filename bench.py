"""Benchmark of the HOBO hot path on one MI355X.

Workload: order-3 HOBO, N=128 variables, every a_i, b_ij, c_ijk present with
FP32 coefficients ~N(0,1)/N (seed 0); B=4096 replicas; 1000 single-flip
Metropolis sweeps with geometric temperatures 5.0 -> 0.01.

One step = the whole hot path over one batch, through the C-ABI:
  hobo_energy        (B energies of the batch)
  hobo_local_fields  (B energies + all N single-flip changes)
  hobo_anneal_batch  (B replicas x 1000 sweeps, random start, FP64 rescore)
in the split-BF16 (hi+lo) precision.  value = energy+dE evaluations per
second, counting one per replica-sweep of the annealer (a sweep computes all
N flip changes and tracks E) plus B for the fields call.

The JSON line also carries the roofline of the dominant kernel (the
annealer), the plain-FP32, BF16x3 and learned-proposal variants of the same
annealing run with their time to target, the evaluation kernels' rates and
roofline fractions at a saturating batch, and the CPU oracle's rate on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_VARS, ORDER, REPLICAS, SWEEPS, T0, T1 = 128, 3, 4096, 1000, 5.0, 0.01
PEAK_TFLOPS = {"fp32": 157.3, "bf16x2": 2500.0, "bf16x3": 2500.0}
PASSES = {"fp32": 1, "bf16x2": 2, "bf16x3": 3}
PREC_OF = {"fp32": 0, "bf16x2": 1, "bf16x3": 2}


def w_eval(n: int, k: int) -> int:
    """Flops of E plus all N flip changes for one state, dense triangle:
    2 * sum_r r * C(n, r) (each order-r monomial feeds r fields)."""
    return 2 * sum(r * math.comb(n, r) for r in range(1, k + 1))


def w_energy(n: int, k: int) -> int:
    """Flops of one energy: 2 * sum_r C(n, r)."""
    return 2 * sum(math.comb(n, r) for r in range(1, k + 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=SWEEPS)
    ap.add_argument("--replicas", type=int, default=REPLICAS)
    ap.add_argument("--precision", default="bf16x2", choices=list(PREC_OF))
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-eval-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mixed-instances", type=int, default=16,
                    help="instances of the mixed family for the persistent-vs-per-instance comparison (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device (scale for the HBM traffic counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the replicas are independent and "
              "would shard across GPUs, but only the one-GPU path is implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2407_19987_amd import hobo
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    B, S = args.replicas, args.sweeps
    terms = W.cfg_real3(seed=0, n=N_VARS)
    t = hobo.Tensor.from_terms(terms)
    t.prepare(hobo.FN_ENERGY | hobo.FN_FIELDS | hobo.FN_ANNEAL, 0b111)
    W_ = (N_VARS + 63) // 64
    xs = hobo.bits_to_device(W.pack_bits(W.random_states(N_VARS, B, seed=1000)))
    e1 = torch.empty(B, dtype=torch.float64, device=dev)
    e2 = torch.empty(B, dtype=torch.float64, device=dev)
    de = torch.empty((B, N_VARS), dtype=torch.float32, device=dev)
    x = torch.empty(W_ * B, dtype=torch.int64, device=dev)
    bx = torch.empty(W_ * B, dtype=torch.int64, device=dev)
    be = torch.empty(B, dtype=torch.float64, device=dev)
    tr = torch.empty(S, dtype=torch.float64, device=dev)

    def step(prec: int, learned=None):
        hobo.energy(t, xs, B, prec, e1)
        hobo.local_fields(t, xs, B, prec, de, e2)
        kw = {}
        if learned is not None:
            kw = dict(mlp=learned["mlp"], tau=learned["tau"], p_floor=learned["p_floor"], refresh=learned["refresh"])
        hobo.anneal_batch(t, B, x, bx, be, sweeps=S, t_start=T0, t_end=T1, seed=42, precision=prec,
                          init=hobo.INIT_RANDOM, trace_out=tr, launch_mode=hobo.LAUNCH_PERSISTENT, **kw)

    def timed(prec_name: str, warmup: int, steps: int, learned=None):
        prec = PREC_OF[prec_name]
        for _ in range(warmup):
            step(prec, learned)
        torch.cuda.synchronize()
        for k in (0, 1, 2):
            hobo.timing_read(k)  # drop warm-up records
        hobo.timing_enable(True)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(steps):
            step(prec, learned)
        b.record()
        torch.cuda.synchronize()
        hobo.timing_enable(False)
        ms = a.elapsed_time(b) / steps
        kt = {k: hobo.timing_read(k) for k in (0, 1, 2)}
        return dict(ms_per_step=ms, anneal_ms=kt[0][0] / steps, anneal_launches=kt[0][1] // steps,
                    fields_ms=kt[1][0] / max(kt[1][1], 1), energy_ms=kt[2][0] / max(kt[2][1], 1),
                    best=float(be.min().item()), trace=tr.cpu().numpy().copy(),
                    e_eval=e1.cpu().numpy().copy(), e_fields=e2.cpu().numpy().copy())

    main_res = timed(args.precision, args.warmup, args.steps)
    evals_per_step = B * S + B
    value = evals_per_step / (main_res["ms_per_step"] / 1e3)
    flops = w_eval(N_VARS, ORDER) * B * S
    achieved = flops / (main_res["anneal_ms"] / 1e3) / 1e12
    peak = PEAK_TFLOPS[args.precision]

    # FP64 reference energies of the batch (term-by-term on the GPU)
    e64 = torch.empty(B, dtype=torch.float64, device=dev)
    hobo.energy(t, xs, B, hobo.PREC_FP64, e64)
    torch.cuda.synchronize()
    e64 = e64.cpu().numpy()
    floor = float(np.median(np.abs(e64)))

    def err(v):
        return float(np.max(np.abs(v - e64) / np.maximum(np.abs(e64), floor)))

    def summary(r):
        return dict(evals_per_s=evals_per_step / (r["ms_per_step"] / 1e3), ms_per_step=r["ms_per_step"],
                    anneal_ms=r["anneal_ms"], best_energy=r["best"], energy_rel_err_vs_fp64=err(r["e_eval"]))

    variants = {args.precision: summary(main_res)}
    traces = {args.precision: (main_res["trace"], main_res["anneal_ms"])}
    if not args.no_variants:
        for name in ("fp32", "bf16x3", "bf16x2"):
            if name == args.precision:
                continue
            r = timed(name, 1, 2)
            variants[name] = summary(r)
            traces[name] = (r["trace"], r["anneal_ms"])
    learned_info = None
    if not args.no_learned:
        from paper_2407_19987_amd import learned as LP

        # transitions of plain runs on held-out-from-the-bench training instances
        tt0 = time.perf_counter()
        feats, labels = [], []
        for k in range(4):
            tk = hobo.Tensor.from_terms(W.cfg_real3(seed=100 + k, n=N_VARS))
            f, y = LP.record_transitions(tk, 1024, S, T0, T1, seed=7 + k,
                                         record=list(range(0, S, max(S // 16, 1))), precision=PREC_OF["bf16x2"])
            feats.append(f)
            labels.append(y)
        feats, labels = torch.cat(feats), torch.cat(labels)
        # shuffle once (fixed permutation) so minibatches mix temperatures
        perm = torch.from_numpy(np.random.default_rng(0).permutation(labels.numel())).to(dev)
        feats, labels = feats[perm].contiguous(), labels[perm].contiguous()
        state, losses = LP.train(feats, labels, W.mlp_init(1), batch=4096, epochs=2, lr=2e-3)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - tt0
        lp = dict(mlp=state[:hobo.MLP_PARAMS].contiguous(), tau=0.02, p_floor=0.02, refresh=20)
        r = timed("bf16x2", 1, 2, learned=lp)
        variants["learned_bf16x2"] = summary(r)
        traces["learned_bf16x2"] = (r["trace"], r["anneal_ms"])
        learned_info = dict(transitions=int(labels.numel()), train_steps=int(losses.numel()),
                            loss_first=float(losses[0]), loss_last=float(losses[-1]), record_train_s=train_s,
                            tau=lp["tau"], p_floor=lp["p_floor"], refresh=lp["refresh"])
    # time to within 1% of the best energy any variant reached
    e_best = min(v["best_energy"] for v in variants.values())
    target = e_best + 0.01 * abs(e_best)
    for name, (trace, ams) in traces.items():
        hit = np.nonzero(trace <= target)[0]
        variants[name]["ttt_ms"] = float((hit[0] + 1) / S * ams) if len(hit) else None

    # evaluation kernels: rate and roofline at the bench batch and at a saturating one
    eval_info = {}
    if not args.no_eval_sweep:
        for bb in (B, 65536):
            xe = hobo.bits_to_device(W.pack_bits(W.random_states(N_VARS, bb, seed=2000)))
            ee = torch.empty(bb, dtype=torch.float64, device=dev)
            dd = torch.empty((bb, N_VARS), dtype=torch.float32, device=dev)
            for pname in ("bf16x2", "fp32"):
                pr = PREC_OF[pname]
                for fn, kid in (("energy", 2), ("fields", 1)):
                    f = (lambda: hobo.energy(t, xe, bb, pr, ee)) if fn == "energy" else (
                        lambda: hobo.local_fields(t, xe, bb, pr, dd))
                    f()
                    torch.cuda.synchronize()
                    hobo.timing_read(kid)
                    hobo.timing_enable(True)
                    for _ in range(5):
                        f()
                    torch.cuda.synchronize()
                    hobo.timing_enable(False)
                    ms, n = hobo.timing_read(kid)
                    us = ms / n * 1e3
                    wf = (w_energy if fn == "energy" else w_eval)(N_VARS, ORDER) * bb
                    tfl = wf * PASSES[pname] / (us * 1e-6) / 1e12
                    eval_info[f"{fn}_{pname}_B{bb}"] = dict(
                        us=us, evals_per_s=bb / (us * 1e-6), issued_tflops=tfl,
                        frac_of_peak=tfl / PEAK_TFLOPS[pname])

    # many instances of uneven size and order in one persistent, graph-captured
    # launch against one launch sequence per instance (same kernels and shapes)
    multi = None
    if args.mixed_instances > 0:
        mi, mb, msw = args.mixed_instances, 256, 100
        th0 = time.perf_counter()
        mts = [hobo.Tensor.from_terms(W.cfg_mixed_instance(0, i)) for i in range(mi)]
        for mt in mts:
            mt.prepare(hobo.FN_ANNEAL, 1 << PREC_OF["fp32"])
        host_s = time.perf_counter() - th0
        words = sum(((mt.n_vars + 63) // 64) * mb for mt in mts)
        mx = torch.zeros(words, dtype=torch.int64, device=dev)
        mbx = torch.zeros_like(mx)
        mbe = torch.zeros(mi * mb, dtype=torch.float64, device=dev)
        mtr = torch.zeros(mi * msw, dtype=torch.float64, device=dev)
        res = {}
        for name, mode in (("per_instance", hobo.LAUNCH_PER_INSTANCE), ("persistent_graph", hobo.LAUNCH_GRAPH)):
            kw = dict(sweeps=msw, t_start=T0, t_end=T1, seed=3, precision=PREC_OF["fp32"], trace_out=mtr,
                      launch_mode=mode)
            hobo.anneal_batch(mts, [mb] * mi, mx, mbx, mbe, **kw)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(2):
                hobo.anneal_batch(mts, [mb] * mi, mx, mbx, mbe, **kw)
            b.record()
            torch.cuda.synchronize()
            res[name] = dict(ms=a.elapsed_time(b) / 2, best=mbe.cpu().numpy().copy())
        same = bool(np.array_equal(res["per_instance"]["best"], res["persistent_graph"]["best"]))
        multi = {"instances": mi, "replicas_each": mb, "sweeps": msw, "precision": "fp32",
                 "orders": [int(mt.order) for mt in mts], "n_vars": [int(mt.n_vars) for mt in mts],
                 "per_instance_ms": res["per_instance"]["ms"], "persistent_graph_ms": res["persistent_graph"]["ms"],
                 "speedup": res["per_instance"]["ms"] / res["persistent_graph"]["ms"],
                 "replica_sweeps_per_s": mi * mb * msw / (res["persistent_graph"]["ms"] / 1e3),
                 "identical_results": same, "host_build_pack_s": host_s,
                 "sample": f"instances 0..{mi - 1} of the mixed family (master seed 0)"}

    cpu = None
    if not args.no_cpu:
        import oracle

        c = oracle.canonicalize(terms)
        # a bounded sample: time a small run, then size the sample to ~15 s of host work
        nrep, nsw = 64, 10
        t0 = time.perf_counter()
        oracle.anneal(c, nrep, nsw, T0, T1, seed=42)
        probe = time.perf_counter() - t0
        nsw = int(max(10, min(S, nsw * 20.0 / max(probe, 1e-3))))
        t0 = time.perf_counter()
        oracle.anneal(c, nrep, nsw, T0, T1, seed=42, schedule_sweeps=S)
        dt = time.perf_counter() - t0
        cpu = {"value": nrep * nsw / dt, "unit": "evals/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"oracle annealer, {nrep} replicas x the first {nsw} sweeps of the same N=128 order-3 "
                         f"instance's {S}-sweep schedule (T {T0}->{T1}), {dt:.1f} s on "
                         f"{platform.processor() or platform.machine()}"}

    # HBM traffic of the dominant kernel from the committed counter summary,
    # valid only for the kernel source it was measured on
    traffic = None
    try:
        import hashlib
        import re

        src = os.path.join(ROOT, "paper_2407_19987_amd", "csrc", "anneal_block.hip")
        prof = os.path.join(ROOT, "profiles", "anneal_block_traffic_order3_n128_b4096.md")
        txt = open(prof).read()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        row = re.search(r"`anneal_block_kernel<1, \d+>` \(BF16x2\) \| \d+ \| ([0-9.]+) \| ([0-9.]+) \|", txt)
        fs = float(re.search(r"FETCH x ([0-9.]+)", txt).group(1))
        ws = float(re.search(r"WRITE x ([0-9.]+)", txt).group(1))
        if (digest in txt and row and args.precision == "bf16x2" and B == REPLICAS and S == SWEEPS
                and main_res["anneal_launches"] == 4):
            traffic = (float(row.group(1)) * fs + float(row.group(2)) * ws) * 1024.0
    except (OSError, AttributeError, ValueError):
        traffic = None

    rec = {
        "metric": "HOBO energy+ΔE evals/s; time-to-target energy, plain vs split/learned",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if args.precision.startswith("bf16") else "fp32",
        "data": "synthetic",
        "config": {"workload": f"order-3 HOBO, N={N_VARS}, dense FP32 N(0,1)/N coefficients, B={B} replicas, "
                               f"{S} Metropolis sweeps T {T0}->{T1}, energy + fields + anneal per step",
                   "n_vars": N_VARS, "order": ORDER, "replicas": B, "sweeps": S, "precision": args.precision},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic, "kernel": "anneal_block_kernel",
                     "flops_per_launch": flops // max(main_res["anneal_launches"], 1),
                     "avg_launch_ms": main_res["anneal_ms"] / max(main_res["anneal_launches"], 1),
                     "launches_per_step": main_res["anneal_launches"]},
        "variants": variants,
        "learned": learned_info,
        "eval_kernels": eval_info,
        "multi_instance": multi,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
