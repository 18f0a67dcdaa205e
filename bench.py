#!/usr/bin/env python3
"""Benchmark of the FSS hot path on one MI355X.

Default workload: the GELU operator over one BERT-base FFN activation
(128 x 3072 elements, 24-bit inputs with 12 fractional bits, 16 degree-2
intervals on [-6, 6) plus two tails, outputs in Z_2^64).  One step is one
pass of the whole hot path over the batch:
    dealer key generation for both parties (fresh one-time keys every step)
    -> masked opening xhat = x + r_in
    -> both parties' evaluation of both FSS calls and the local combination.
`value` counts element-evals (one party x one element x both calls) per second
of the timed steps.  The plain evaluator (two launches per party) is timed on
the same inputs for comparison.

Prints ONE JSON line.  --gpus N with N > 1 exits: evaluation runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "element-evals/sec (GELU spec, Z_2^64) + p50/p99 latency, fused vs plain"
# MI355X CU local memory serves 32 lane addresses per clock: a wave64 ds_read
# of 4 or 8 bytes per lane holds it for 2 clocks.  T-table AES needs one such
# lookup per state byte and round, so 256 CUs x 32 x 2.4 GHz bounds the path.
LOOKUP_PEAK_T = 256 * 32 * 2.4e9 / 1e12
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz of 32-bit integer VALU issue.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic 32-bit integer ops of one T-table AES-128 block: 10 rounds x
# (16 table-index extractions + 8 three-input XORs) + 16 for whitening,
# last-round byte merge and the Matyas-Meyer-Oseas feed-forward.
OPS_PER_AES = 256
# MI355X HBM3E bandwidth, GB/s.
HBM_PEAK_GBPS = 8000.0


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return 0.0
    k = (len(xs) - 1) * q
    lo, hi = int(k), min(int(k) + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(op, n_bits, f_bits, lookup_r, gpu_shares) -> dict:
    """The oracle (dealer keygen + both parties' evaluation) on fixed samples of
    the workload: the first 131,072 elements (2,048 tiles) on every host thread
    and the first 4,096 on one.  The all-thread sample's shares and masks are
    compared with the GPU's for the same seed (`gpu_shares(count)` runs the
    fused path once at the operator's seed and returns its first `count`
    elements)."""
    import numpy as np

    import oracle as O

    S = O.compile_spec(op.spec, n_bits, f_bits, lookup_r=lookup_r)
    out = {"unit": "element-evals/s", "kind": "oracle"}
    rates = {}
    for label, count, threads in (("single_core", 4096, 1), ("all_cores", 131072, 0)):
        count = min(count, len(op.x))
        elems = np.arange(count, dtype=np.int64)
        a0 = O.aes_blocks()
        t0 = time.perf_counter()
        y0, y1, z0, z1, r_in, r_out, used = O.full(S, op.seed, elems, op.x[:count], threads=threads, masks=True)
        dt = time.perf_counter() - t0
        aes = O.aes_blocks() - a0
        rates[label] = {"element_evals_per_s": round(2 * count / dt, 1), "aes_blocks_per_s": round(aes / dt, 1),
                        "threads": int(used), "elements": count, "wall_s": round(dt, 3)}
        if label == "all_cores":
            g = gpu_shares(count)
            ok = all(np.array_equal(a, b) for a, b in ((g["y0"], y0), (g["y1"], y1), (g["z0"], z0),
                                                         (g["z1"], z1), (g["r_in"], r_in), (g["r_out"], r_out)))
            out["verified_elements"] = count if ok else 0
            out["verified"] = bool(ok)
    allc = rates["all_cores"]
    out.update({"value": allc["element_evals_per_s"], "cores": allc["threads"],
                "aes_blocks_per_s": allc["aes_blocks_per_s"],
                "single_core": rates["single_core"],
                "sample": (f"first {allc['elements']} of {len(op.x)} elements on {allc['threads']} threads "
                           f"({allc['wall_s']} s) and first {rates['single_core']['elements']} on one thread "
                           f"({rates['single_core']['wall_s']} s): dealer keygen + both parties' evaluation; "
                           "the all-thread sample's shares and masks compared with the GPU's at the same seed")})
    return out


KERNEL_SOURCES = ["paper_2606_09551_amd/csrc/fss_kernels_impl.hpp", "paper_2606_09551_amd/csrc/fss_common.hpp",
                  "paper_2606_09551_amd/csrc/fss_kernels.hpp", "paper_2606_09551_amd/csrc/fss_aes_bs.hpp"]


def measured_traffic(workload: str, lookup_r: int):
    """HBM bytes per fused launch from the committed rocprofv3 counter summary,
    or None when the kernel sources or the lookup radix differ from those the
    counters were taken with."""
    import hashlib

    if workload != "c2":
        return None
    path = os.path.join(ROOT, "profiles", "k_fused_gelu_128x3072_traffic.md")
    if not os.path.exists(path):
        return None
    want = f"traffic_bytes_per_launch_r{lookup_r}"
    kv = {}
    for line in open(path):
        if ":" in line and line.split(":")[0].strip() in ("kernel_sources_sha256_16", want):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in KERNEL_SOURCES)
    if kv.get("kernel_sources_sha256_16") != hashlib.sha256(src).hexdigest()[:16] or want not in kv:
        return None
    return int(kv[want])


def hbm_view(alg_bytes: float, traffic, launch_s: float) -> dict:
    """The fused launch against the HBM roofline: algorithmic bytes and, where
    the counters are on record, the measured bytes, per launch and as GB/s."""
    out = {"algorithmic_bytes": int(alg_bytes), "algorithmic_gbps": round(alg_bytes / launch_s / 1e9, 1),
           "peak_gbps": HBM_PEAK_GBPS, "traffic_bytes": traffic, "traffic_gbps": None, "frac": None}
    if traffic:
        gbps = traffic / launch_s / 1e9
        out["traffic_gbps"] = round(gbps, 1)
        out["frac"] = round(gbps / HBM_PEAK_GBPS, 4)
    return out


def build_ops(workload: str):
    from paper_2606_09551_amd import workloads as W

    if workload == "c1":
        return W.config1(), 16, 8, "clip_relu_4096"
    if workload == "c2":
        return W.config2(), W.N_BITS, W.F_BITS, "gelu_bert_base_ffn_128x3072"
    if workload == "c3":
        return W.config3(), W.N_BITS, W.F_BITS, "softmax_exp_12x128x128_recip_12x128"
    if workload == "c4":
        return W.config4(), W.N_BITS, W.F_BITS, "gpt2_small_seq256_12_layers_gelu_exp_recip_rsqrt"
    raise SystemExit(f"unknown workload {workload}")


def layer_groups(ops) -> list:
    """Indices of ops grouped per transformer layer (name prefix 'L<k>.')."""
    groups, keyed = [], {}
    for i, op in enumerate(ops):
        key = op.name.split(".")[0] if op.name.startswith("L") and "." in op.name else "all"
        if key not in keyed:
            keyed[key] = len(groups)
            groups.append([])
        groups[keyed[key]].append(i)
    return groups


def main() -> None:
    import tempfile

    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--requests", type=int, default=64, help="c5: requests in the Poisson stream")
    ap.add_argument("--rate", type=float, default=50.0, help="c5: mean arrival rate (req/s)")
    ap.add_argument("--no-graphs", action="store_true", help="launch each layer's plan directly (no HIP graph)")
    ap.add_argument("--autotune", default=os.path.join(tempfile.gettempdir(), "fusefss_tune_cache.txt"),
                    metavar="CACHE", help="autotuner cache file (the fused launch is tuned on the first layer)")
    ap.add_argument("--no-autotune", action="store_true", help="use the planner's default launch")
    ap.add_argument("--tune", default=None, metavar="V,BPC,ORDER,PARTS,PRED[,LANES]",
                    help="fix the fused launch: AES variant, blocks per CU, unit order, parts per tile, "
                         "call-1 unit, lanes per element (as fss_tune; replaces the autotuner)")
    ap.add_argument("--latency-reps", type=int, default=None,
                    help="fused/plain step pairs, alternating, for the latency percentiles and ratios "
                         "(default: as many as fit about 5 s of steps, 60 to 500)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--lookup-r", type=int, default=None, choices=[2, 3, 4],
                    help="input bits per level of call 2's DCF (default: the library's)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one copy kernel of this size (HBM counter calibration)")
    ap.add_argument("--ablation", choices=["reuse"], default=None,
                    help="reuse: compiled program cached vs rebuilt per layer (12 GELU layers)")
    ap.add_argument("--study", choices=["literal"], default=None,
                    help="literal: the compilation protocol's literal interval lookup (one DCF per boundary) "
                         "with Horner's rule on shares, against the single-key lookup (GELU 128x3072)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: evaluation runs on one GPU; --gpus {args.gpus} is not supported "
              "(elements are independent, so the path would shard by element range, one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2606_09551_amd import fss as F
    from paper_2606_09551_amd import runtime as R

    torch.cuda.set_device(0)
    if args.ablation == "reuse":
        reuse_ablation(args)
        return
    if args.study == "literal":
        literal_study(args)
        return
    if args.workload == "c5":
        serve_bench(args)
        return
    ops, n_bits, f_bits, wname = build_ops(args.workload)
    insts = []
    tuned_r = {}
    for op in ops:
        spec = F.Spec(op.spec, args.lookup_r)
        if args.lookup_r is None and not (args.no_autotune or args.tune):
            # the key-layout knob: lookup radix per spec and size, timed once and cached
            key = (op.spec.name, len(op.x))
            if key not in tuned_r:
                tuned_r[key] = spec.autotune_radix(n_bits, f_bits, len(op.x), args.autotune)
            F.lib.fss_spec_set_lookup_radix(spec.handle, tuned_r[key])
        inst = R.OpInstanceGPU(spec, n_bits, f_bits, len(op.x))
        inst.set_input(op.x)
        insts.append(inst)
    n_elems = sum(i.n for i in insts)
    stream = torch.cuda.current_stream()
    for inst, op in zip(insts, ops):       # the plan reads each key buffer's header
        inst.keygen(op.seed)
    torch.cuda.synchronize()
    groups = layer_groups(ops)
    tune = None
    if args.tune:
        v, bpc, order, parts, pred, *lanes = (int(t) for t in args.tune.split(","))
        tune = F.Tune(0, bpc, v, order, parts, pred, lanes[0] if lanes else 0)
    elif not args.no_autotune:
        tune = F.fss_autotune([insts[i].item(b) for i in groups[0] for b in (0, 1)], args.autotune)
    plans = [F.Plan([insts[i].item(b) for i in g for b in (0, 1)], tune) for g in groups]
    graphs = None if args.no_graphs else [F.Graph([p]) for p in plans]
    cfg = plans[0].config()
    cfg["parts"] = max(p.parts() for p in plans)
    eval_aes = sum(p.aes_blocks() for p in plans)
    eval_lookups = sum(p.table_lookups() for p in plans)
    # algorithmic HBM bytes of the evaluation launches: both parties' keys read
    # once, x-hat read, y and the predicate bit-planes written
    eval_bytes = sum(2 * (i.key_bytes + 16 * i.n + 8 * i.ell * ((i.n + 63) // 64)) for i in insts)
    kg_work = [i.spec.keygen_work(n_bits, f_bits, i.n) for i in insts]
    kg_aes = sum(w[0] for w in kg_work)
    kg_lookups = sum(w[1] for w in kg_work)

    # Dealer work of different operators is independent: with several operators
    # it is spread over side streams (joined before evaluation), so the
    # keygen of a small operator overlaps that of a large one.
    dealers = [torch.cuda.Stream() for _ in range(min(4, len(insts)))] if len(insts) > 1 else []

    def step(k: int, fused: bool, ev, seeds=None):
        base = 0xB3C4 + 7919 * k
        ev[0].record(stream)
        seed_of = (lambda j, op: op.seed) if seeds == "op" else (lambda j, op: (op.seed ^ base) + j)
        if dealers:
            for d in dealers:
                d.wait_event(ev[0])
            for j, (inst, op) in enumerate(zip(insts, ops)):
                with torch.cuda.stream(dealers[j % len(dealers)]):
                    inst.keygen(seed_of(j, op))
                    inst.mask()
            for d in dealers:
                done = torch.cuda.Event()
                done.record(d)
                stream.wait_event(done)
        else:
            for j, (inst, op) in enumerate(zip(insts, ops)):
                inst.keygen(seed_of(j, op))
                inst.mask()
        ev[1].record(stream)
        if fused:
            if graphs:
                for g in graphs:
                    g.launch()
            else:
                for p in plans:
                    p.launch()
        else:
            for inst in insts:
                inst.eval_plain(0)
                inst.eval_plain(1)
        ev[2].record(stream)

    def events():
        return [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def check_status():
        code = F.fss_status()
        if code != 0:
            raise SystemExit(f"device status {code}")

    # Both paths are warmed up before either is timed, so neither run carries
    # the first launches' start-up (clock ramp, first-touch of the buffers).
    for k in range(args.warmup):
        step(k, True, events())
        if not args.no_plain:
            step(k, False, events())
    torch.cuda.synchronize()

    # The timed steps: K fused steps back to back between two synchronisations.
    evs = [events() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + k, True, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    check_status()
    fused = {"wall_s": wall, "keygen_ms": statistics.mean(e[0].elapsed_time(e[1]) for e in evs),
             "eval_ms": statistics.mean(e[1].elapsed_time(e[2]) for e in evs),
             "lat": [e[0].elapsed_time(e[2]) for e in evs]}

    # Fused against plain: pairs of steps with the same seeds, the order
    # alternating from pair to pair so that neither path always follows the
    # other (the part carries its clock from one kernel to the next); every
    # step is bracketed by synchronisations.  Latency percentiles come from
    # these repetitions.
    cmp = None
    if not args.no_plain:
        import gc

        if args.latency_reps is None:  # a p99 over more samples is less a maximum
            step_ms = wall * 1e3 / max(1, args.steps)
            reps = min(500, max(60, int(5000.0 / (2.0 * step_ms))))
        else:
            reps = max(args.latency_reps, 50)
        rec = {True: [], False: []}
        pair_events = [[events(), events()] for _ in range(reps)]
        gc.collect()
        gc.disable()  # no collector pause inside a timed step
        try:
            for k in range(reps):
                for i, fz in enumerate((True, False) if k % 2 == 0 else (False, True)):
                    ev = pair_events[k][i]
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    step(1000 + k, fz, ev)
                    torch.cuda.synchronize()
                    rec[fz].append((time.perf_counter() - t1, ev))
        finally:
            gc.enable()
        rec = {fz: [(w, ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[0].elapsed_time(ev[2]))
                    for w, ev in rows] for fz, rows in rec.items()}
        check_status()

        def summary(rows):
            lat = [r[3] for r in rows]
            ev_ = [r[2] for r in rows]
            return {"step_wall_ms": round(1e3 * statistics.mean(r[0] for r in rows), 4),
                    "step_wall_p50_ms": round(1e3 * pct([r[0] for r in rows], 0.5), 4),
                    "keygen_ms": round(statistics.mean(r[1] for r in rows), 4),
                    "eval_ms": round(statistics.mean(ev_), 4),
                    "latency_ms": {"p50": round(pct(lat, 0.5), 4), "p99": round(pct(lat, 0.99), 4)},
                    "eval_latency_ms": {"p50": round(pct(ev_, 0.5), 4), "p99": round(pct(ev_, 0.99), 4)}}
        cmp = {"reps": reps, "fused": summary(rec[True]), "plain": summary(rec[False])}

    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 0, out=dst)
        torch.cuda.synchronize()

    evals = 2 * n_elems
    value = evals * args.steps / fused["wall_s"]
    eval_s = fused["eval_ms"] / 1e3
    achieved = eval_lookups / eval_s / 1e12
    valu_achieved = eval_aes * OPS_PER_AES / eval_s / 1e12
    kg_s = fused["keygen_ms"] / 1e3
    kg_achieved = kg_lookups / kg_s / 1e12
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "element-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(fused["wall_s"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": wname, "elements": n_elems, "parties": 2, "n_bits": n_bits,
                   "frac_bits": f_bits, "ops": len(ops),
                   "path": "fused persistent work-list" + (", HIP graph per layer" if graphs else ""),
                   "launches_per_step": len(plans),
                   "step": "keygen (both parties) + masked opening + eval (both parties)",
                   "launch": cfg, "autotuned": tune is not None and not args.tune,
                   "lookup_r": insts[0].lookup_r,
                   "lookup_r_autotuned": bool(tuned_r),
                   "key_bytes_per_party": sum(i.key_bytes for i in insts)},
        "breakdown_ms": {"keygen": round(fused["keygen_ms"], 4), "eval": round(fused["eval_ms"], 4)},
        "aes_blocks_per_s": round((eval_aes + kg_aes) * args.steps / fused["wall_s"], 1),
        "eval_only_element_evals_per_s": round(evals / eval_s, 1),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(LOOKUP_PEAK_T, 3),
                     "unit": "T table-lookups/s", "frac": round(achieved / LOOKUP_PEAK_T, 4),
                     "traffic": measured_traffic(args.workload, insts[0].lookup_r),
                     "kernel": "k_fused", "ceiling": "CU local-memory lookup rate (T-table AES)",
                     "lookups_per_launch": eval_lookups / len(plans),
                     "aes_blocks_per_launch": eval_aes / len(plans),
                     "valu": {"achieved": round(valu_achieved, 3), "peak": round(VALU_PEAK_TOPS, 3),
                              "unit": "Tops/s", "frac": round(valu_achieved / VALU_PEAK_TOPS, 4),
                              "ops_per_aes_block": OPS_PER_AES},
                     "hbm": hbm_view(eval_bytes / len(plans), measured_traffic(args.workload, insts[0].lookup_r),
                                     eval_s / len(plans)),
                     "keygen": {"kernel": "k_keygen", "achieved": round(kg_achieved, 3),
                                "peak": round(LOOKUP_PEAK_T, 3), "unit": "T table-lookups/s",
                                "frac": round(kg_achieved / LOOKUP_PEAK_T, 4),
                                "lookups_per_step": kg_lookups, "aes_blocks_per_step": kg_aes,
                                "ms": round(fused["keygen_ms"], 4)}},
    }
    if cmp is None:
        out["latency_ms"] = {"p50": round(pct(fused["lat"], 0.5), 4), "p99": round(pct(fused["lat"], 0.99), 4),
                             "samples": args.steps, "of": "the timed steps (keygen + opening + eval), HIP events"}
    else:
        f_, p_ = cmp["fused"], cmp["plain"]
        out["latency_ms"] = dict(f_["latency_ms"], samples=cmp["reps"],
                                 of="step (keygen + opening + eval), HIP events, over the fused/plain pairs "
                                    "run after the timed steps")
        out["eval_latency_ms"] = dict(f_["eval_latency_ms"], samples=cmp["reps"])
        out["plain"] = {"value": round(evals / (p_["step_wall_ms"] / 1e3), 1), "step_wall_ms": p_["step_wall_ms"],
                        "keygen_ms": p_["keygen_ms"], "eval_ms": p_["eval_ms"],
                        "latency_ms": p_["latency_ms"], "eval_latency_ms": p_["eval_latency_ms"]}
        out["fused_paired"] = {"value": round(evals / (f_["step_wall_ms"] / 1e3), 1),
                               "step_wall_ms": f_["step_wall_ms"], "keygen_ms": f_["keygen_ms"],
                               "eval_ms": f_["eval_ms"]}
        out["fused_over_plain"] = round(p_["step_wall_ms"] / f_["step_wall_ms"], 4)
        out["fused_over_plain_p50"] = round(p_["step_wall_p50_ms"] / f_["step_wall_p50_ms"], 4)
        out["eval_fused_over_plain"] = round(p_["eval_ms"] / f_["eval_ms"], 4)
        out["comparison"] = (f"{cmp['reps']} pairs of one fused and one plain step with the same seeds, "
                             "order alternating, each step between synchronisations")

    if not args.no_cpu_baseline:
        def gpu_shares(count):
            # one fused step at the operator's own seed, first `count` elements
            step(0, True, events(), seeds="op")
            torch.cuda.synchronize()
            check_status()
            h = insts[0].host()
            return {"y0": h["y0"][:count], "y1": h["y1"][:count], "r_in": h["r_in"][:count],
                    "r_out": h["r_out"][:count], "z0": R.unpack_bits(h["z0"], insts[0].n)[:count],
                    "z1": R.unpack_bits(h["z1"], insts[0].n)[:count]}
        out["cpu_baseline"] = cpu_baseline(ops[0], n_bits, f_bits, insts[0].lookup_r, gpu_shares)
    print(json.dumps(out), flush=True)


def serve_bench(args) -> None:
    """Config 5: a Poisson stream of BERT-base requests (L ~ U{16..512}) served
    by the continuous-batching server, fused and plain evaluators on the same
    stream.  Party 0's server is evaluated; each request's keys are generated
    on the device at admission (dealer time reported separately)."""
    import gc

    import torch

    from paper_2606_09551_amd import serving as S
    from paper_2606_09551_amd import workloads as W

    reqs = W.config5_requests(args.requests, args.rate)
    stream = [(r.rid, r.L, r.arrival) for r in reqs]
    free, total = torch.cuda.mem_get_info()
    arena = int(min(free * 0.85, 230 * 2**30))
    out = {}
    for path in ("fused", "plain"):
        srv = S.Server(arena, layers=12, path=path)
        st = srv.run(stream)
        st.pop("_requests")
        out[path] = st
        print(f"served {len(stream)} requests ({path}): {st['makespan_s']:.1f} s", file=sys.stderr, flush=True)
        del srv
        gc.collect()
        torch.cuda.empty_cache()
    f, p = out["fused"], out["plain"]
    line = {
        "metric": METRIC,
        "value": round(f["element_evals_per_s"], 1),
        "unit": "element-evals/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": round(f["makespan_s"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"serving_bert_base_poisson_{args.rate:g}rps_{args.requests}req_L16_512",
                   "party": 0, "layers": 12, "ops_per_layer": "gelu, exp, reciprocal, rsqrt x2 tokens",
                   "arena_bytes": arena, "keys": "generated on the device at admission"},
        "latency_s": f["latency_s"],
        "admission_to_done_s": f["admission_to_done_s"],
        "requests_per_s": round(f["requests_per_s"], 3),
        "dealer_s": round(f["dealer_s"], 3),
        "mean_batch_requests": round(f["mean_batch_requests"], 3),
        "batches": f["batches"],
        "plain": {"value": round(p["element_evals_per_s"], 1), "latency_s": p["latency_s"],
                  "admission_to_done_s": p["admission_to_done_s"], "makespan_s": round(p["makespan_s"], 3)},
        "fused_over_plain": round(f["element_evals_per_s"] / p["element_evals_per_s"], 4),
        "offered_rps": args.rate,
    }
    print(json.dumps(line), flush=True)


def reuse_ablation(args) -> None:
    """Program reuse across layers (the paper's ablation "Program Reuse Across
    Layers"): 12 BERT-base GELU layers of 128x3072, both parties, fresh keys for
    every layer.  `cached` compiles the spec, builds the work-list plan and
    captures its HIP graph once and replays it for every layer (the key, input
    and output buffers are reused; keys are regenerated into them);
    `per_layer` compiles, plans and captures again for every layer.  Init is
    the host wall time of compile + spec tables + plan + capture; eval is the
    HIP-event time of the layers' fused launches."""
    import torch

    from paper_2606_09551_amd import fss as F
    from paper_2606_09551_amd import runtime as R
    from paper_2606_09551_amd import workloads as W

    op = W.config2()[0]
    n_bits, f_bits, layers = W.N_BITS, W.F_BITS, 12
    stream = torch.cuda.current_stream()
    inst = R.OpInstanceGPU(F.Spec(op.spec), n_bits, f_bits, len(op.x))
    inst.set_input(op.x)

    def run(cached: bool) -> dict:
        init_s, eval_ms, keep = 0.0, [], []
        spec = plan = graph = None
        for layer in range(layers):
            if not cached or spec is None:
                t0 = time.perf_counter()
                spec = F.Spec(op.spec)
                spec.query(n_bits, f_bits)
                init_s += time.perf_counter() - t0
                inst.spec = spec
            inst.keygen(op.seed + 7919 * layer)
            inst.mask()
            torch.cuda.synchronize()
            if not cached or plan is None:
                t0 = time.perf_counter()
                plan = F.Plan([inst.item(0), inst.item(1)])
                graph = F.Graph([plan])
                torch.cuda.synchronize()
                init_s += time.perf_counter() - t0
                keep.append((spec, plan, graph))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            graph.launch()
            e1.record(stream)
            torch.cuda.synchronize()
            eval_ms.append(e0.elapsed_time(e1))
        for _, p, g in keep:
            g.free()
            p.free()
        return {"program_inits": len(keep), "init_ms": round(init_s * 1e3, 3),
                "eval_ms_total": round(sum(eval_ms), 3), "eval_ms_per_layer": round(statistics.mean(eval_ms), 4)}

    run(True)  # warm-up: first compile, first launch, allocator
    out = {"ablation": "program_reuse", "workload": "gelu_bert_base_ffn_128x3072_x12_layers",
           "parties": 2, "cached": run(True), "per_layer": run(False)}
    print(json.dumps(out), flush=True)


def literal_study(args) -> None:
    """Call 2 as the compilation protocol states it against this library's
    single-key form, GELU over 128x3072 at n = 24, f = 12, both parties.
    literal: keys of the literal lookup (one vector DCF per inner boundary
    of the translated partition) plus the Beaver triples of Horner's rule,
    then both parties' lookups and the d rounds of Horner's rule on shares
    (openings between the parties' steps).  single_key: fss_keygen (both
    calls' keys) and fss_eval_coeff for both parties (lookup and local
    combination at the public x-hat).  Both produce shares of P(x) + r_out
    from the same seed; the openings are compared element by element.  HIP
    events on the launch stream; steps alternate between the two paths."""
    import numpy as np
    import torch

    from paper_2606_09551_amd import fss as F
    from paper_2606_09551_amd import runtime as R
    from paper_2606_09551_amd import workloads as W

    op = W.config2()[0]
    n_bits, f_bits = W.N_BITS, W.F_BITS
    spec = F.Spec(op.spec, args.lookup_r)
    N = len(op.x)
    single = R.OpInstanceGPU(spec, n_bits, f_bits, N)
    lit = R.LiteralGPU(spec, n_bits, f_bits, N)
    single.set_input(op.x)
    lit.set_input(op.x)
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        return e0, e1

    def single_step(seed):
        k = timed(lambda: (single.keygen(seed), single.mask()))
        ev = timed(lambda: [F.fss_eval_coeff(b, single.keys[b], single.xhat, N, single.y[b]) for b in (0, 1)])
        return k, ev

    def lit_step(seed):
        k = timed(lambda: (lit.keygen(seed), lit.mask()))
        ev = timed(lit.eval)
        return k, ev

    rows = {"single_key": [], "literal": []}
    for s in range(args.warmup + args.steps):
        seed = op.seed + 104729 * s
        pair = (single_step(seed), lit_step(seed))
        torch.cuda.synchronize()
        if F.fss_status() != 0:
            raise RuntimeError("device status after a study step")
        if s >= args.warmup:
            for name, (k, ev) in zip(("single_key", "literal"), pair):
                rows[name].append((k[0].elapsed_time(k[1]), ev[0].elapsed_time(ev[1])))
    sh, lh = single.host(), lit.host()
    same = bool(np.array_equal(sh["y0"] + sh["y1"], lh["y0"] + lh["y1"]))
    out = {"study": "literal_lookup", "workload": "gelu_bert_base_ffn_128x3072", "elements": N, "parties": 2,
           "n_bits": n_bits, "frac_bits": f_bits, "lookup_r": spec.lookup_r, "steps": args.steps,
           "openings_equal": same}
    for name, key_bytes in (("single_key", single.key_bytes), ("literal", lit.key_bytes)):
        kg = statistics.median(r[0] for r in rows[name])
        ev = statistics.median(r[1] for r in rows[name])
        out[name] = {"keygen_ms": round(kg, 4), "eval_ms": round(ev, 4),
                     "element_evals_per_s": round(2 * N / ((kg + ev) * 1e-3), 1),
                     "key_bytes_per_party": key_bytes}
    out["single_key"]["keygen_covers"] = "both calls' keys (predicate atoms included)"
    out["single_key"]["eval_covers"] = "call 2 and the combination at x-hat, both parties"
    out["literal"]["keygen_covers"] = "literal lookup keys and the Horner triples"
    out["literal"]["eval_covers"] = f"both parties' lookups and {lit.d} Beaver rounds of Horner's rule"
    out["literal"]["intervals_after_padding"] = spec.query(n_bits, f_bits)["m"] + 1
    out["literal_over_single_eval"] = round(out["literal"]["eval_ms"] / out["single_key"]["eval_ms"], 3)
    out["literal_over_single_keygen"] = round(out["literal"]["keygen_ms"] / out["single_key"]["keygen_ms"], 3)
    print(json.dumps(out), flush=True)
    if not same:
        sys.exit(1)


if __name__ == "__main__":
    main()
