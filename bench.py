"""Benchmark of the HOBO hot path on one MI355X.

Workload: order-3 HOBO, N=128 variables, every a_i, b_ij, c_ijk present with
FP32 coefficients ~N(0,1)/N (seed 0); B=4096 replicas; 1000 single-flip
Metropolis sweeps with geometric temperatures 5.0 -> 0.01.

One step = the whole hot path over one batch, through the C-ABI:
  hobo_energy        (B energies of the batch)
  hobo_local_fields  (B energies + all N single-flip changes)
  hobo_anneal_batch  (B replicas x 1000 sweeps, random start, FP64 rescore)
in the split-FP16 (hi+lo, power-of-two scaled) precision, the split that
meets the 1e-5 energy tolerance at the two-pass rate.  value = energy+dE
evaluations per second, counting one per replica-sweep of the annealer (a
sweep computes all N flip changes and tracks E) plus B for the fields call.

The JSON line also carries the roofline of the dominant kernel (the
annealer), the plain-FP32, BF16x2, BF16x3 and learned-proposal variants of
the same annealing run (energy error against FP64 on the |E| / s(x) floor,
tracked-energy drift, time to target), the evaluation kernels' rates at the
bench batch and a saturating one, the integer-encoded order-4 workload's
INT8x4 rates, the mixed-instance launch comparison, and the CPU oracle's rate
on a bounded sample (all host threads and one).

Optional heavier measurements: --mixed-full (256 instances x 1024 replicas x
500 sweeps, autotuned against default shapes) and --ttt-seeds K (time to
within 1 % on K held-out instances, learned proposal against plain).
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
PREC_OF = {"fp32": 0, "bf16x2": 1, "bf16x3": 2, "fp16x2": 5}
ALG_OF = {"auto": 0, "slabs": 1, "blocks": 2}  # hobo_anneal_params.algorithm
PEAK_TFLOPS = {"fp32": 157.3, "bf16x2": 2500.0, "bf16x3": 2500.0, "fp16x2": 2500.0, "int8x4": 5000.0}
PASSES = {"fp32": 1, "bf16x2": 2, "bf16x3": 3, "fp16x2": 2}
DTYPE = {"fp32": "fp32", "bf16x2": "bf16", "bf16x3": "bf16", "fp16x2": "fp16"}


def w_eval(n: int, k: int) -> int:
    """Flops of E plus all N flip changes for one state, dense triangle:
    2 * sum_r r * C(n, r) (each order-r monomial feeds r fields)."""
    return 2 * sum(r * math.comb(n, r) for r in range(1, k + 1))


def w_energy(n: int, k: int) -> int:
    """Flops of one energy: 2 * sum_r C(n, r)."""
    return 2 * sum(math.comb(n, r) for r in range(1, k + 1))


def progress(msg: str) -> None:
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=SWEEPS)
    ap.add_argument("--replicas", type=int, default=REPLICAS)
    ap.add_argument("--precision", default="fp16x2", choices=list(PREC_OF))
    ap.add_argument("--algorithm", default="auto", choices=list(ALG_OF),
                    help="annealing kernel of the step: auto (the blocked kernel where it applies), or the "
                         "per-bit slab kernel")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-eval-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mixed-instances", type=int, default=16,
                    help="instances of the mixed family for the persistent-vs-per-instance comparison (0: skip)")
    ap.add_argument("--mixed-full", action="store_true",
                    help="the mixed workload at its full size: 256 instances x 1024 replicas")
    ap.add_argument("--mixed-sweeps", type=int, default=500,
                    help="sweeps of the --mixed-full runs (the time of 500 is extrapolated linearly when fewer)")
    ap.add_argument("--ttt-seeds", type=int, default=0,
                    help="held-out instances for the learned-vs-plain time-to-target comparison (0: skip)")
    ap.add_argument("--eval-only", action="store_true",
                    help="only the evaluation kernels' rates (energy and fields at B=4096 and 65536, INT8x4, TT)")
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
    if args.eval_only:
        t.prepare(hobo.FN_ENERGY | hobo.FN_FIELDS, sum(1 << p for p in PREC_OF.values()))
        info = eval_rates(hobo, W, torch, dev, t, B)
        info.update(int8_rates(hobo, W, torch, dev))
        info.update(tt_rates(hobo, W, torch, dev))
        info.update(gd_rates(hobo, torch, dev, t, B))
        print(json.dumps({"eval_kernels": info, "paper_problems": paper_problems(torch)}))
        return
    t.prepare(hobo.FN_ENERGY | hobo.FN_FIELDS | hobo.FN_ANNEAL, sum(1 << p for p in PREC_OF.values()))
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
                          init=hobo.INIT_RANDOM, trace_out=tr, launch_mode=hobo.LAUNCH_PERSISTENT,
                          algorithm=ALG_OF[args.algorithm], **kw)

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

    # FP64 energies of the batch and the tolerance floor s(x) = (sum of the
    # squared active terms)^(1/2): the FP64 energy of the squared-coefficient
    # tensor, both term by term on the GPU
    e64 = torch.empty(B, dtype=torch.float64, device=dev)
    hobo.energy(t, xs, B, hobo.PREC_FP64, e64)
    mp, mi, mw = t.monomials()
    tsq = hobo.Tensor(N_VARS, mp, mi, np.asarray(mw, dtype=np.float64) ** 2)
    s2 = torch.empty(B, dtype=torch.float64, device=dev)
    hobo.energy(tsq, xs, B, hobo.PREC_FP64, s2)
    torch.cuda.synchronize()
    e64 = e64.cpu().numpy()
    floor = np.sqrt(np.maximum(s2.cpu().numpy(), 0.0))

    def err(v):
        return float(np.max(np.abs(v - e64) / np.maximum(np.abs(e64), floor)))

    def summary(r):
        return dict(evals_per_s=evals_per_step / (r["ms_per_step"] / 1e3), ms_per_step=r["ms_per_step"],
                    anneal_ms=r["anneal_ms"], best_energy=r["best"],
                    energy_err_vs_fp64=err(r["e_eval"]), fields_energy_err_vs_fp64=err(r["e_fields"]),
                    tracked_drift=abs(float(r["trace"][-1]) - r["best"]))

    variants = {args.precision: summary(main_res)}
    traces = {args.precision: (main_res["trace"], main_res["anneal_ms"])}
    if not args.no_variants:
        for name in ("fp32", "bf16x3", "bf16x2", "fp16x2"):
            if name == args.precision:
                continue
            r = timed(name, 1, 2)
            variants[name] = summary(r)
            traces[name] = (r["trace"], r["anneal_ms"])
    learned_info = None
    if not args.no_learned:
        from paper_2407_19987_amd import learned as LP

        lp, learned_info = train_proposal(hobo, LP, W, torch, dev, S, PREC_OF[args.precision])
        r = timed(args.precision, 1, 2, learned=lp)
        key = f"learned_{args.precision}"
        variants[key] = summary(r)
        traces[key] = (r["trace"], r["anneal_ms"])
    # time to within 1% of the best energy any variant reached (kernel time
    # up to the first sweep whose trace reaches it; the annealer's sweeps all
    # cost the same)
    e_best = min(v["best_energy"] for v in variants.values())
    target = e_best + 0.01 * abs(e_best)
    for name, (trace, ams) in traces.items():
        hit = np.nonzero(trace <= target)[0]
        variants[name]["ttt_ms"] = float((hit[0] + 1) / S * ams) if len(hit) else None

    eval_info = {}
    if not args.no_eval_sweep:
        eval_info = eval_rates(hobo, W, torch, dev, t, B)
        eval_info.update(int8_rates(hobo, W, torch, dev))
        eval_info.update(tt_rates(hobo, W, torch, dev))
        eval_info.update(gd_rates(hobo, torch, dev, t, B))
    problems = None if args.no_eval_sweep else paper_problems(torch)

    multi = None
    if args.mixed_instances > 0:
        multi = mixed(hobo, W, torch, dev, args.mixed_instances, 256, 100, tune=False)
    mixed_full = None
    if args.mixed_full:
        mixed_full = mixed(hobo, W, torch, dev, 256, 1024, args.mixed_sweeps, tune=True)
        if args.mixed_sweeps != 500:  # every sweep costs the same: linear in the sweep count
            k = 500 / args.mixed_sweeps
            mixed_full["extrapolated_to_500_sweeps"] = {
                key: mixed_full[key] * k for key in ("per_instance_ms", "persistent_graph_ms", "tuned_graph_ms")
                if key in mixed_full}
    ttt = ttt_eval(hobo, W, torch, dev, args.ttt_seeds, S, PREC_OF[args.precision]) if args.ttt_seeds > 0 else None

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(terms, S)

    # the committed counter summaries are the blocked annealer's
    slabs = args.algorithm == "slabs"
    traffic = None if slabs else read_traffic(args.precision, B, S, main_res["anneal_launches"])
    cu_path = None if slabs else read_cu_path(args.precision, B, S, main_res["anneal_launches"], main_res["anneal_ms"])
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
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"order-3 HOBO, N={N_VARS}, dense FP32 N(0,1)/N coefficients, B={B} replicas, "
                               f"{S} Metropolis sweeps T {T0}->{T1}, energy + fields + anneal per step",
                   "n_vars": N_VARS, "order": ORDER, "replicas": B, "sweeps": S, "precision": args.precision,
                   "algorithm": args.algorithm},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic, "kernel": "anneal_kernel" if slabs else "anneal_block_kernel",
                     "flops_per_launch": flops // max(main_res["anneal_launches"], 1),
                     "avg_launch_ms": main_res["anneal_ms"] / max(main_res["anneal_launches"], 1),
                     "launches_per_step": main_res["anneal_launches"],
                     "measured_bound": cu_path},
        "variants": variants,
        "learned": learned_info,
        "eval_kernels": eval_info,
        "paper_problems": problems,
        "multi_instance": multi,
        "mixed_full": mixed_full,
        "ttt_heldout": ttt,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec))


def train_proposal(hobo, LP, W, torch, dev, S, prec):
    """Record transitions of plain runs on training instances (seeds 100+k),
    train the proposal network on them with the engine's kernels."""
    tt0 = time.perf_counter()
    feats, labels = [], []
    for k in range(4):
        tk = hobo.Tensor.from_terms(W.cfg_real3(seed=100 + k, n=N_VARS))
        f, y = LP.record_transitions(tk, 1024, S, T0, T1, seed=7 + k,
                                     record=list(range(0, S, max(S // 16, 1))), precision=prec)
        feats.append(f)
        labels.append(y)
    feats, labels = torch.cat(feats), torch.cat(labels)
    # shuffle once (fixed permutation) so minibatches mix temperatures
    perm = torch.from_numpy(np.random.default_rng(0).permutation(labels.numel())).to(dev)
    feats, labels = feats[perm].contiguous(), labels[perm].contiguous()
    state, losses = LP.train(feats, labels, W.mlp_init(1), batch=4096, epochs=2, lr=2e-3)
    torch.cuda.synchronize()
    lp = dict(mlp=state[:hobo.MLP_PARAMS].contiguous(), tau=0.02, p_floor=0.02, refresh=20)
    info = dict(transitions=int(labels.numel()), train_steps=int(losses.numel()), loss_first=float(losses[0]),
                loss_last=float(losses[-1]), record_train_s=time.perf_counter() - tt0, tau=lp["tau"],
                p_floor=lp["p_floor"], refresh=lp["refresh"])
    return lp, info


def _kernel_us(hobo, torch, f, kid, reps=5):
    f()
    torch.cuda.synchronize()
    hobo.timing_read(kid)
    hobo.timing_enable(True)
    for _ in range(reps):
        f()
    torch.cuda.synchronize()
    hobo.timing_enable(False)
    ms, n = hobo.timing_read(kid)
    return ms / n * 1e3


def eval_rates(hobo, W, torch, dev, t, B):
    """Energy and fields kernels on the headline instance: evaluations per
    second, issued matrix-core rate (stored tiles x passes, from the layout)
    against the precision's peak, and the dense-triangle algorithmic rate."""
    out = {}
    for bb in (B, 65536):
        xe = hobo.bits_to_device(W.pack_bits(W.random_states(N_VARS, bb, seed=2000)))
        ee = torch.empty(bb, dtype=torch.float64, device=dev)
        dd = torch.empty((bb, N_VARS), dtype=torch.float32, device=dev)
        for pname in ("fp16x2", "bf16x2", "fp32"):
            pr = PREC_OF[pname]
            for fn, kid, fmask in (("energy", 2, hobo.FN_ENERGY), ("fields", 1, hobo.FN_FIELDS)):
                f = (lambda: hobo.energy(t, xe, bb, pr, ee)) if fn == "energy" else (
                    lambda: hobo.local_fields(t, xe, bb, pr, dd))
                us = _kernel_us(hobo, torch, f, kid)
                issued = t.layout_info(fmask, pr).issued_flops * bb / (us * 1e-6) / 1e12
                alg = (w_energy if fn == "energy" else w_eval)(N_VARS, ORDER) * bb / (us * 1e-6) / 1e12
                out[f"{fn}_{pname}_B{bb}"] = dict(us=us, evals_per_s=bb / (us * 1e-6), issued_tflops=issued,
                                                  algorithmic_tflops=alg,
                                                  frac_of_peak=issued / PEAK_TFLOPS[pname])
    return out


def int8_rates(hobo, W, torch, dev, bb=8192):
    """The integer-encoded order-4 workload (8 six-bit integers, 12 pairs,
    N=48) with INT8x4 digits at B=8192: evaluations per second and the
    issued (stored tiles), dense-triangle and useful (non-zero monomial) op
    rates; useful ops per evaluation: 2 sum_r r nnz_r (fields), 2 nnz (energy)."""
    terms = W.cfg_intenc4(seed=0)
    t = hobo.Tensor.from_terms(terms)
    n, k = t.n_vars, t.order
    nnz = [int(v) for v in t.info().n_per_order]
    xe = hobo.bits_to_device(W.pack_bits(W.random_states(n, bb, seed=2100)))
    ee = torch.empty(bb, dtype=torch.int64, device=dev)
    dd = torch.empty((bb, n), dtype=torch.int64, device=dev)
    out = {}
    for fn, kid, fmask in (("energy", 2, hobo.FN_ENERGY), ("fields", 1, hobo.FN_FIELDS)):
        f = (lambda: hobo.energy(t, xe, bb, hobo.PREC_INT8X4, ee)) if fn == "energy" else (
            lambda: hobo.local_fields(t, xe, bb, hobo.PREC_INT8X4, dd, ee))
        us = _kernel_us(hobo, torch, f, kid)
        rate = bb / (us * 1e-6)
        issued = t.layout_info(fmask, hobo.PREC_INT8X4).issued_flops * rate / 1e12
        dense = (w_energy if fn == "energy" else w_eval)(n, k) * rate / 1e12
        useful = (2 * sum(nnz) if fn == "energy" else 2 * sum(r * c for r, c in enumerate(nnz))) * rate / 1e12
        out[f"intenc4_{fn}_int8x4_B{bb}"] = dict(us=us, evals_per_s=rate, issued_tops=issued, dense_tops=dense,
                                                 useful_tops=useful, frac_of_peak=issued / PEAK_TFLOPS["int8x4"])
    return out


def paper_problems(torch, shots=10000, sweeps=300):
    """The three worked problems of Sec. V end to end through the front-end:
    compile (host), sample `shots` replicas on the GPU, aggregate; the time of
    each part, the best energy and the number of distinct optimal states."""
    import numpy as np

    from paper_2407_19987_amd import frontend as F

    def seating():
        q = F.symbols_list([5, 5], "bq{}_{}")
        wins = [[(i, j + d) for d in range(3)] for i in range(5) for j in range(3)]
        wins += [[(i + d, j) for d in range(3)] for j in range(5) for i in range(3)]
        return 10 * sum(q[w[0]] * q[w[1]] * q[w[2]] for w in wins) - sum(q[i, j] for i in range(5) for j in range(5))

    def pythagorean():
        q = F.symbols_list([3, 4], "bp{}_{}")
        v = [sum((1 << k) * q[p, k] for k in range(4)) for p in range(3)]
        return (v[0] ** 2 + v[1] ** 2 - v[2] ** 2) ** 2 + 10 * sum(np.prod(1 - q[p, :]) for p in range(3))

    def tsp():
        q = F.symbols_list([4, 2], "bt{}_{}")
        v = [2 * q[p, 0] + q[p, 1] for p in range(3)]
        return 10 * (v[0] * v[1] * v[2] - 6) ** 2

    out = {}
    for name, make in (("seating_5x5", seating), ("pythagorean_4bit", pythagorean), ("tsp_intenc", tsp)):
        t0 = time.perf_counter()
        cp = F.compile_hobo(make())
        t1 = time.perf_counter()
        rows = F.sample(cp, shots, sweeps=sweeps, seed=1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        best = rows[0].energy
        out[name] = dict(n_vars=cp.n_vars, order=int(cp.tensor.order), offset=cp.offset, compile_ms=(t1 - t0) * 1e3,
                         sample_and_aggregate_ms=(t2 - t1) * 1e3, shots=shots, sweeps=sweeps, best_energy=best,
                         optimal_states=sum(1 for r in rows if r.energy == best), distinct_states=len(rows))
    return out


def tt_rates(hobo, W, torch, dev, bb=65536):
    """Energies through the tensor-train cores (Sec. VI.F) of the integer-
    encoded TSP instance (N=6, order 6, ranks 2-4) and of a dense order-3
    N=16 instance: evaluations per second and the FP64 rate of the core
    contraction (2 N sum_k r_{k-1} r_k flops per state) against the FP64
    vector peak (78.6 TFLOP/s)."""
    out = {}
    for name, terms in (("tsp_n6_k6", W.paper_tsp_intenc()), ("real3_n16", W.cfg_real3(seed=0, n=16))):
        tt = hobo.TensorTrain(hobo.Tensor.from_terms(terms))
        xe = hobo.bits_to_device(W.pack_bits(W.random_states(tt.n_vars, bb, seed=2200)))
        ee = torch.empty(bb, dtype=torch.float64, device=dev)
        tt.energy(xe, bb, ee)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(10):
            tt.energy(xe, bb, ee)
        b.record()
        torch.cuda.synchronize()
        us = a.elapsed_time(b) / 10 * 1e3
        flops = 2 * tt.n_vars * sum(tt.ranks[k] * tt.ranks[k + 1] for k in range(tt.order))
        tfl = flops * bb / (us * 1e-6) / 1e12
        out[f"tt_{name}_B{bb}"] = dict(us=us, evals_per_s=bb / (us * 1e-6), ranks=tt.ranks, fp64_tflops=tfl,
                                       frac_of_fp64_vector_peak=tfl / 78.6)
    return out


def gd_rates(hobo, torch, dev, t, B, iters=100):
    """Gradient-descent search (Sec. II.D.2) on the headline instance: B
    replicas x `iters` projected FP64 steps, then rounding and exact
    energies.  Gradient evaluations (replica-steps) per second and the FP64
    rate of the record walk, sum_r r^2 nnz_r flops per replica-step (each
    order-r monomial feeds r gradients, each r - 1 products and one sum),
    against the FP64 vector peak (78.6 TFLOP/s)."""
    n = t.n_vars
    nnz = [int(v) for v in t.info().n_per_order]
    p = torch.empty(n * B, dtype=torch.float64, device=dev)
    x = torch.empty(((n + 63) // 64) * B, dtype=torch.int64, device=dev)
    e = torch.empty(B, dtype=torch.float64, device=dev)
    hobo.gd_batch(t, B, p, x, e, iterations=2, eta=0.05, seed=1)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    hobo.gd_batch(t, B, p, x, e, iterations=iters, eta=0.05, seed=1)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    flops = sum(r * r * c for r, c in enumerate(nnz)) * B * iters
    return {f"gd_real3_n{n}_B{B}_{iters}steps": dict(
        ms=ms, replica_steps_per_s=B * iters / (ms * 1e-3), fp64_tflops=flops / (ms * 1e-3) / 1e12,
        frac_of_fp64_vector_peak=flops / (ms * 1e-3) / 1e12 / 78.6, best_rounded_energy=float(e.min().item()),
        median_rounded_energy=float(e.median().item()))}


def mixed(hobo, W, torch, dev, mi, mb, msw, tune):
    """Many instances of uneven size and order (N in [24, 160], order 2-4,
    density 0.3, FP32) annealed in one persistent, graph-captured launch
    against one launch sequence per instance (same kernels and shapes); with
    `tune`, also the persistent launch after hobo_autotune of each instance's
    annealer shape against the default shapes."""
    th0 = time.perf_counter()
    mts = []
    for i in range(mi):
        mts.append(hobo.Tensor.from_terms(W.cfg_mixed_instance(0, i)))
        mts[-1].prepare(hobo.FN_ANNEAL, 1 << PREC_OF["fp32"])
        if (i + 1) % 32 == 0:
            progress(f"mixed instances built and packed: {i + 1} of {mi}")
    host_s = time.perf_counter() - th0
    words = sum(((mt.n_vars + 63) // 64) * mb for mt in mts)
    mx = torch.zeros(words, dtype=torch.int64, device=dev)
    mbx = torch.zeros_like(mx)
    mbe = torch.zeros(mi * mb, dtype=torch.float64, device=dev)
    mtr = torch.zeros(mi * msw, dtype=torch.float64, device=dev)
    res = {}

    def run(name, mode, reps):
        progress(f"mixed {mi} x {mb} x {msw}: {name}")
        kw = dict(sweeps=msw, t_start=T0, t_end=T1, seed=3, precision=PREC_OF["fp32"], trace_out=mtr,
                  launch_mode=mode)
        hobo.anneal_batch(mts, [mb] * mi, mx, mbx, mbe, **kw)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            hobo.anneal_batch(mts, [mb] * mi, mx, mbx, mbe, **kw)
        b.record()
        torch.cuda.synchronize()
        res[name] = dict(ms=a.elapsed_time(b) / reps, best=mbe.cpu().numpy().copy())

    reps = 2 if mi * mb * msw <= (1 << 24) else 1
    run("per_instance", hobo.LAUNCH_PER_INSTANCE, reps)
    run("persistent_graph", hobo.LAUNCH_GRAPH, reps)
    out = {"instances": mi, "replicas_each": mb, "sweeps": msw, "precision": "fp32",
           "orders": [int(mt.order) for mt in mts], "n_vars": [int(mt.n_vars) for mt in mts],
           "per_instance_ms": res["per_instance"]["ms"], "persistent_graph_ms": res["persistent_graph"]["ms"],
           "speedup": res["per_instance"]["ms"] / res["persistent_graph"]["ms"],
           "replica_sweeps_per_s": mi * mb * msw / (res["persistent_graph"]["ms"] / 1e3),
           # useful work: each order-r monomial feeds r fields, 2 flops each, per replica-sweep
           "useful_tflops": sum(2 * sum(r * int(c) for r, c in enumerate(mt.info().n_per_order)) for mt in mts)
                            * mb * msw / (res["persistent_graph"]["ms"] / 1e3) / 1e12,
           "identical_results": bool(np.array_equal(res["per_instance"]["best"], res["persistent_graph"]["best"])),
           "host_build_pack_s": host_s, "sample": f"instances 0..{mi - 1} of the mixed family (master seed 0)"}
    if tune:
        # the library shapes each kernel kind's persistent launch by the
        # tuned width of its costliest instance (stored tiles x replicas):
        # tune those two (blocked: order <= 3; per-bit: order 4)
        tt0 = time.perf_counter()
        tuned = {}
        for kind in (0, 1):
            cand = [mt for mt in mts if (mt.order <= 3) == bool(kind)]
            if not cand:
                continue
            mt = max(cand, key=lambda m: m.layout_info(hobo.FN_ANNEAL, PREC_OF["fp32"]).tiles)
            xb = hobo.bits_to_device(W.pack_bits(W.random_states(mt.n_vars, mb, seed=5)))
            tuned["blocked" if kind else "per_bit"] = dict(
                n_vars=int(mt.n_vars), order=int(mt.order),
                waves=hobo.autotune(mt, xb, mb, hobo.FN_ANNEAL, PREC_OF["fp32"])[2])
        tune_s = time.perf_counter() - tt0
        out["tuned_shapes"] = tuned
        # a fresh setup per call argument set: the tuned shapes are read when the setup is built
        mx2 = torch.zeros_like(mx)
        mx = mx2
        run("tuned_graph", hobo.LAUNCH_GRAPH, reps)
        out.update(tuned_graph_ms=res["tuned_graph"]["ms"], tune_host_s=tune_s,
                   tuned_vs_default=res["persistent_graph"]["ms"] / res["tuned_graph"]["ms"],
                   tuned_identical_results=bool(np.array_equal(res["tuned_graph"]["best"],
                                                               res["persistent_graph"]["best"])))
    return out


def ttt_eval(hobo, W, torch, dev, n_seeds, S, prec):
    """Time to within 1 % of the best energy found (over both methods, FP64
    rescored) on held-out instances (seeds 10000+k), learned proposal against
    plain Metropolis; the run is timed in windows of 25 sweeps and the time to
    target is the elapsed kernel time at the end of the first window whose
    trace reaches the target."""
    from paper_2407_19987_amd import learned as LP

    lp, info = train_proposal(hobo, LP, W, torch, dev, S, prec)
    B, win = REPLICAS, 25
    W_ = (N_VARS + 63) // 64
    x = torch.empty(W_ * B, dtype=torch.int64, device=dev)
    bx = torch.empty(W_ * B, dtype=torch.int64, device=dev)
    be = torch.empty(B, dtype=torch.float64, device=dev)
    tr = torch.empty(win, dtype=torch.float64, device=dev)
    rows = []
    for k in range(n_seeds):
        if k % 8 == 0:
            progress(f"time to target: held-out instance {k} of {n_seeds}")
        tk = hobo.Tensor.from_terms(W.cfg_real3(seed=10000 + k, n=N_VARS))
        tk.prepare(hobo.FN_ANNEAL | hobo.FN_FIELDS, 1 << prec)
        curves = {}
        for name, kw in (("plain", {}), ("learned", dict(mlp=lp["mlp"], tau=lp["tau"], p_floor=lp["p_floor"],
                                                          refresh=lp["refresh"]))):
            elapsed, curve = 0.0, []
            for s0 in range(0, S, win):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                hobo.anneal_batch(tk, B, x, bx, be, sweeps=win, t_start=T0, t_end=T1, seed=42, precision=prec,
                                  init=hobo.INIT_RANDOM if s0 == 0 else hobo.INIT_GIVEN, trace_out=tr,
                                  launch_mode=hobo.LAUNCH_PERSISTENT, first_sweep=s0, schedule_sweeps=S,
                                  continue_best=s0 > 0, **kw)
                b.record()
                torch.cuda.synchronize()
                elapsed += a.elapsed_time(b)
                curve.append((elapsed, float(be.min().item())))
            curves[name] = curve
        e_best = min(c[-1][1] for c in curves.values())
        target = e_best + 0.01 * abs(e_best)
        row = {"seed": 10000 + k}
        for name, curve in curves.items():
            hit = [ms for ms, e in curve if e <= target]
            row[name] = hit[0] if hit else None
            row[name + "_total_ms"] = curve[-1][0]
        rows.append(row)
    out = {"seeds": n_seeds, "window_sweeps": win, "precision": prec, "training": info}
    for name in ("plain", "learned"):
        v = np.array([r[name] for r in rows if r[name] is not None])
        out[name] = dict(reached=int(len(v)), median_ms=float(np.median(v)) if len(v) else None,
                         iqr_ms=[float(np.percentile(v, 25)), float(np.percentile(v, 75))] if len(v) else None,
                         median_total_ms=float(np.median([r[name + "_total_ms"] for r in rows])))
    out["learned_wins"] = int(sum(1 for r in rows if r["learned"] is not None and
                                  (r["plain"] is None or r["learned"] < r["plain"])))
    out["rows"] = rows
    return out


def cpu_baseline(terms, S):
    """The oracle annealer on a bounded sample of the same instance, on all
    host threads and on one."""
    import oracle

    c = oracle.canonicalize(terms)
    nrep, nsw = 64, 10
    all_threads = oracle.num_threads()
    t0 = time.perf_counter()
    oracle.anneal(c, nrep, nsw, T0, T1, seed=42)
    probe = time.perf_counter() - t0
    # a bounded sample: about 15 s of host work on all threads
    nsw = int(max(10, min(S, nsw * 15.0 / max(probe, 1e-3))))
    t0 = time.perf_counter()
    oracle.anneal(c, nrep, nsw, T0, T1, seed=42, schedule_sweeps=S)
    dt = time.perf_counter() - t0
    # one thread: 16 replicas x 4 sweeps
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.anneal(c, 16, 4, T0, T1, seed=42, schedule_sweeps=S)
    dt1 = time.perf_counter() - t1
    oracle.set_threads(all_threads)
    model = cpu_model()
    return {"value": nrep * nsw / dt, "unit": "evals/s", "cores": all_threads, "kind": "oracle",
            "single_core_value": 16 * 4 / dt1, "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": f"oracle annealer, {nrep} replicas x the first {nsw} sweeps of the same N=128 order-3 "
                      f"instance's {S}-sweep schedule (T {T0}->{T1}), {dt:.1f} s on {all_threads} threads of "
                      f"{model}; single core: 16 replicas x 4 sweeps, {dt1:.1f} s"}


# what the blocked annealer streams is set by its kernel, the layout packer
# and the work schedule: a counter summary holds for these sources only
ANNEALER_SOURCES = ("anneal_block.hip", "pack.cpp", "schedule.cpp")


def annealer_digest() -> str:
    """sha256 over the blocked annealer's sources, in ANNEALER_SOURCES order."""
    import hashlib

    h = hashlib.sha256()
    for name in ANNEALER_SOURCES:
        with open(os.path.join(ROOT, "paper_2407_19987_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_cu_path(precision, B, S, launches, anneal_ms):
    """The annealer's measured bound: each compute unit's vector-memory
    return path, which carries the coefficient tiles into registers.  The
    bytes returned to registers per launch (from the schedule, checked
    against the counted vector-memory reads), the L1 -> L2 read requests
    (128 B) and the data-return unit's busy share come from the committed
    counter summary of the same annealer sources; the bytes are taken over
    this run's launch time, against 64 B per clock per CU (256 CUs,
    2.4 GHz)."""
    try:
        import re

        prof = os.path.join(ROOT, "profiles", "anneal_block_cu_path_order3_n128_fp16x2.md")
        txt = open(prof).read()
        if annealer_digest() not in txt:
            return None
        ret = float(re.search(r"\*\*([0-9.e+]+) bytes returned to registers per\s+launch\*\*", txt).group(1))
        req = float(re.search(r"`TCP_TCC_READ_REQ_sum`[^|]*\| ([0-9.e+]+) \|", txt).group(1))
        busy = float(re.search(r"\| data return \(TD\) busy \| ([0-9.]+) %", txt).group(1)) / 100
        wait = float(re.search(r"stalled waiting for the L1[^|]*\| ([0-9.]+) %", txt).group(1)) / 100
        if precision != "fp16x2" or B != REPLICAS or S != SWEEPS or launches != 4:
            return None
        sec = anneal_ms / launches * 1e-3
        tbps = ret / sec / 1e12
        peak = 64 * 256 * 2.4e9 / 1e12
        return {"resource": "per-CU vector-memory return path (coefficient tiles into registers)",
                "achieved": tbps, "peak": peak, "unit": "TB/s", "frac": tbps / peak,
                "returned_bytes_per_launch": ret, "l1_fill_tbps": req * 128 / sec / 1e12,
                "data_return_busy": busy, "data_return_waiting_on_l1": wait,
                "source": "profiles/anneal_block_cu_path_order3_n128_fp16x2.md"}
    except (OSError, AttributeError, ValueError):
        return None


def read_traffic(precision, B, S, launches):
    """HBM traffic of the dominant kernel from the committed counter summary,
    valid only for the annealer sources and precision it was measured on."""
    try:
        import re

        prof = os.path.join(ROOT, "profiles", f"anneal_block_traffic_order3_n128_b4096_{precision}.md")
        txt = open(prof).read()
        digest = annealer_digest()
        row = re.search(r"`anneal_block_kernel<%d, \d+>` \| \d+ \| ([0-9.]+) \| ([0-9.]+) \|" % PREC_OF[precision],
                        txt)
        fs = float(re.search(r"FETCH x ([0-9.]+)", txt).group(1))
        ws = float(re.search(r"WRITE x ([0-9.]+)", txt).group(1))
        if digest in txt and row and B == REPLICAS and S == SWEEPS and launches == 4:
            return (float(row.group(1)) * fs + float(row.group(2)) * ws) * 1024.0
    except (OSError, AttributeError, ValueError):
        pass
    return None


if __name__ == "__main__":
    main()
