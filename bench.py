"""Throughput benchmark of the RRS depth hot path on one MI355X.

A step is one full RRS depth computation (every refinement of every query:
directions, projection, univariate depth, argmin/pole update) over the
workload's queries, with X and Z already resident in HBM (device pointers).
The default workload is halfspace depth on 100,000 x 100 Gaussian-mixture
data, 500 queries, K = 5000, r = 25, alpha = 0.6, in the bfloat16
matrix-core form with binary64 recheck (results identical to binary64).

Prints ONE JSON line:
  value     query x direction x point projections per second (whole job)
  roofline  the dominant kernel's achieved rate against its bound, from its
            average launch duration measured with HIP events on its launch
            stream during the timed steps
  cpu_baseline  the FP64 oracle on a bounded query sample on the host cores
  forms     (default workload) the same workload in the plain binary32 form
            (with its error against binary64) and the binary32 recheck form,
            and projection depth on the same data (binary32 recheck form)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3, "f32_plain": 157.3}   # dense matrix cores

# workload -> (generator, notion, default precision: the fastest exact form)
WORKLOADS = {
    "c2": ("c2", "projection", "f32"),
    "c1": ("c1", "halfspace", "f64"),
    "c1b": ("c1b", "halfspace", "f64"),
    "c3": ("c3", "apd", "bf16"),
    "c5h": ("c5", "halfspace", "bf16"),
    "c5p": ("c5", "projection", "f32"),
}


def kernel_sources_hash() -> str:
    """sha256 (first 16 hex digits) of the HIP sources and headers of librrs:
    recorded HBM traffic is used only while the kernels are unchanged."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_08262_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    with open(os.path.join(ROOT, "include", "rrs.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch of `kernel` on this workload from the rocprofv3
    counter runs summarised under profiles/ (FETCH_SIZE and WRITE_SIZE, each
    scaled by what the counter reads for a copy of known size), or None when
    there is no record or the kernel sources changed since it was taken."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    cur = kernel_sources_hash()
    for f in sorted(os.listdir(pdir)):
        if not f.endswith(".md"):
            continue
        with open(os.path.join(pdir, f)) as fh:
            for ln in fh:
                if not ln.startswith("traffic-record:"):
                    continue
                kv = dict(t.split("=", 1) for t in ln.split(":", 1)[1].split() if "=" in t)
                if (kv.get("kernel") == kernel and kv.get("workload") == workload
                        and kv.get("precision") == precision and kv.get("sources") == cur):
                    return {"bytes": float(kv["fetch_bytes"]) + float(kv["write_bytes"]),
                            "fetch_bytes": float(kv["fetch_bytes"]),
                            "write_bytes": float(kv["write_bytes"]), "record": f"profiles/{f}"}
    return None


def kernel_model(name: str, notion: str, d: int, precision: str = "f64"):
    """Algorithmic cost per work unit of each kernel (bytes or flops the method needs)."""
    if name == "k_gemm" and notion != "halfspace":
        # projection / APD: the GEMM writes each binary32 projection once
        return {"bound": "hbm", "per_unit": 4.0, "unit": "GB/s", "peak": HBM_PEAK_GBS,
                "scale": 1e-9, "what": "4 B written per projection (binary32 column)"}
    if name == "k_gemm":
        # one projection is a d-term dot product: 2d flops, whatever the
        # padding of K and the number of split products the kernel issues
        kp = (d + 2 + 15) // 16 * 16 if precision == "bf16" else (d + 1 + 7) // 8 * 8
        issued = 2 * kp * (3 if precision == "bf16" else 1)
        return {"bound": "mfma", "per_unit": 2.0 * d, "unit": "TFLOP/s",
                "peak": MFMA_PEAK_TFLOPS[precision], "scale": 1e-12,
                "what": f"2d = {2 * d} algorithmic flops per projection "
                        f"({issued} matrix-core flops issued)",
                "issued_per_unit": float(issued)}
    if name == "k_proj_f64":
        if notion == "halfspace":
            return {"bound": "alu", "per_unit": 2.0 * d, "unit": "TFLOP/s",
                    "peak": FP64_VALU_PEAK_TFLOPS, "scale": 1e-12,
                    "what": f"2d = {2 * d} FP64 flops per projection"}
        return {"bound": "hbm", "per_unit": 8.0, "unit": "GB/s", "peak": HBM_PEAK_GBS,
                "scale": 1e-9, "what": "8 B written per projection (binary64 column)"}
    if name == "k_select" and precision != "f64":
        return {"bound": "hbm", "per_unit": 4.0, "unit": "GB/s", "peak": HBM_PEAK_GBS,
                "scale": 1e-9, "what": "4 B read per projection (binary32 column)"}
    if name == "k_select":
        return {"bound": "hbm", "per_unit": 8.0, "unit": "GB/s", "peak": HBM_PEAK_GBS,
                "scale": 1e-9, "what": "8 B read per projection (binary64 column)"}
    return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, notion, max_queries, per_thread_budget=1.2e8, runs=3):
    """The FP64 oracle on a bounded sample of the workload: whole queries when
    one query costs at most `per_thread_budget` projections, else only the
    first refinement (the m sphere directions of l = 1) of each sampled query,
    which is the same per-projection work.  The median of `runs` runs."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    threads = oracle.max_threads()
    nq = max(1, min(threads, max_queries, w.nq))
    qs = np.arange(nq)
    full = w.n_refine * w.m_dirs * w.n <= per_thread_budget
    K, r = (w.K, w.n_refine) if full else (w.m_dirs, 1)
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        oracle.rrs_depth_idx(notion, w.X, w.Z[qs], qs, K, r, w.cap_shrink, w.rrs_seed,
                             nthreads=nq)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    proj = nq * r * w.m_dirs * w.n
    what = (f"all {w.n_refine} refinements ({w.n_refine * w.m_dirs} directions each)" if full
            else f"refinement 1 only ({w.m_dirs} sphere directions each)")
    return {"value": proj / dt, "unit": "projections/s", "cores": int(nq), "kind": "oracle",
            "sample": f"queries 0..{nq - 1} of {w.nq}, {what}, one OpenMP thread per query, "
                      f"{proj:.3g} projections per run, median of {runs} runs "
                      f"({', '.join(f'{t:.1f}' for t in times)} s) on {cpu_model()}; "
                      f"oracle built with {oracle.CFLAGS_TEXT}",
            "seconds": dt}


def run_form(fn, X, Z, w, precision, steps):
    """Times `steps` calls of one precision form (after one warm-up call)."""
    import torch
    fn(X, Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn(X, Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed, precision=precision)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    return out, sec


def error_vs(out, ref):
    """Error of one form's outputs against the binary64 form's."""
    depth = out["depth"].cpu().numpy()
    dref = ref["depth"].cpu().numpy()
    rel = np.abs(depth - dref) / np.maximum(np.abs(dref), 1e-300)
    err = {"queries": int(depth.size),
           "queries_differing": int(np.count_nonzero(depth != dref)),
           "max_rel": float(rel.max()), "mean_rel": float(rel.mean()),
           "max_abs": float(np.abs(depth - dref).max())}
    if out.get("count") is not None:
        c = out["count"].cpu().numpy()
        cr = ref["count"].cpu().numpy()
        err["count_mismatches"] = int(np.count_nonzero(c != cr))
        err["max_count_diff"] = int(np.abs(c - cr).max())
    return err


def serve_main(args):
    """Serving stream: requests arrive at their Poisson times and go through
    one serving context (resident data sets, admission by memory, several
    requests on the device at once).  Reports whole-stream throughput and
    the p50/p99 of the submit-to-result latency."""
    import numpy as np
    import torch

    from paper_2506_08262_amd import rrs, workloads
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = workloads.c4_stream(args.requests, max_queries=args.max_queries)
    offered = sum(r.projections for r in stream) / stream[-1].arrival
    print(f"[bench] serving stream: {len(stream)} requests over {stream[-1].arrival:.3f} s, "
          f"offered {offered:.3g} projections/s", file=sys.stderr, flush=True)
    prec = {"halfspace": args.serve_h_precision, "projection": args.serve_p_precision}
    with rrs.Context(device=0, slots=args.slots, hbm_budget=args.hbm_budget << 30) as ctx:
        dss = [ctx.put(r.X) for r in stream]
        print("[bench] data sets resident", file=sys.stderr, flush=True)
        # warm-up: one small request per notion (kernel loading, operand prep)
        for notion in ("halfspace", "projection"):
            ctx.submit(dss[0], notion, stream[0].Z[:1], 100, 2, 0.5, 0,
                       precision=prec[notion]).wait()
        t0 = time.monotonic()
        reqs = []
        for i, r in enumerate(stream):
            delay = t0 + r.arrival - time.monotonic()
            if delay > 0:
                time.sleep(delay)
            reqs.append(ctx.submit(dss[i], r.notion, r.Z, r.K, r.n_refine, r.cap_shrink, i,
                                   precision=prec[r.notion]))
        outs = []
        for i, q in enumerate(reqs):
            outs.append(q.wait())
            if (i + 1) % 16 == 0:
                print(f"[bench] {i + 1}/{len(reqs)} requests done", file=sys.stderr, flush=True)
        stats = ctx.stats()
    info = [o["info"] for o in outs]
    lat = np.array([i["done_s"] - i["submit_s"] for i in info])
    qwait = np.array([i["admit_s"] - i["submit_s"] for i in info])
    t_first = min(i["submit_s"] for i in info)
    t_last = max(i["done_s"] for i in info)
    proj = float(sum(i["projections"] for i in info))
    value = proj / (t_last - t_first)
    line = {
        "metric": "query·direction·point projections/s; p50/p99 request latency",
        "value": value,
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": (t_last - t_first) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"halfspace {prec['halfspace']}, projection {prec['projection']}",
        "data": "synthetic",
        "config": {"workload": f"c4: serving stream of {len(stream)} requests, Poisson 200/s, "
                               "halfspace/projection 1/2 each, own data set per request "
                               "(n log-uniform [1e3,1e5], d U{3..100}, N(0,I) or t3), "
                               f"1..{args.max_queries} queries, K in {{1k,5k,10k}}, r=10, "
                               "alpha=0.5",
                   "requests": len(stream), "slots": args.slots,
                   "hbm_budget_gib": args.hbm_budget},
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3),
                       "mean": float(lat.mean() * 1e3),
                       "queue_wait_p50": float(np.percentile(qwait, 50) * 1e3)},
        "offered_load": offered,
        "achieved_over_offered": value / offered,
        "serving_stats": stats,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def sec_main_ms(t0, t1, steps):
    return (t1 - t0) / steps * 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5h", choices=sorted(WORKLOADS) + ["c4"])
    ap.add_argument("--requests", type=int, default=64, help="c4: requests in the stream")
    ap.add_argument("--max-queries", type=int, default=1000, help="c4: query cap per request")
    ap.add_argument("--slots", type=int, default=4, help="c4: concurrent requests")
    ap.add_argument("--hbm-budget", type=int, default=64, help="c4: serving budget in GiB")
    ap.add_argument("--serve-h-precision", default="bf16", help="c4: halfspace precision")
    ap.add_argument("--serve-p-precision", default="f32", help="c4: projection precision")
    ap.add_argument("--precision", default=None, choices=["f64", "f32", "bf16", "f32_plain"],
                    help="projection arithmetic (default: the workload's fastest exact form)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other precision forms and projection depth on the "
                         "default workload")
    ap.add_argument("--cpu-queries", type=int, default=32)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run three plain 1 GiB device-to-device copies (reference "
                         "kernel of known size for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (queries shard "
              f"across GPUs without communication; run one process per GPU)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c4":
        serve_main(args)
        return

    import torch

    from paper_2506_08262_amd import rrs, workloads
    wname, notion, default_prec = WORKLOADS[args.workload]
    if args.precision is None:
        args.precision = default_prec
    w = workloads.make(wname, **({"notion": notion} if wname == "c5" else {}))
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print("[bench] copy calibration: 3 x 1 GiB read + 1 GiB written", file=sys.stderr,
              flush=True)
    X = torch.from_numpy(w.X).to(dev)
    Z = torch.from_numpy(w.Z).to(dev)
    fn = rrs.DEPTH_FUNCS[notion]
    print(f"[bench] workload {args.workload} ({notion}) n={w.n} d={w.d} queries={w.nq} "
          f"K={w.K} r={w.n_refine} alpha={w.cap_shrink} precision={args.precision}",
          file=sys.stderr, flush=True)
    prec = {"precision": args.precision}

    for i in range(args.warmup):
        fn(X, Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed, **prec)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    rrs.rrs_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = fn(X, Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed, **prec)
        print(f"[bench] step {i + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = rrs.rrs_profile_read()
    counters = {c: rrs.rrs_profile_counter(c)
                for c in ("select_fast", "select_fallback", "recheck_pairs", "gemm_pairs",
                          "shared_full", "shared_median", "shared_none")}
    rrs.rrs_profile_enable(False)
    depth = out["depth"].cpu().numpy()

    err = None
    forms = None
    want_forms = args.workload == "c5h" and not args.no_forms
    ref = None
    if args.precision == "f32_plain" or want_forms:
        # binary64 result of the same workload (untimed): the reference for
        # the error of the approximate form and the check of the exact ones
        print("[bench] binary64 reference run ...", file=sys.stderr, flush=True)
        ref = fn(X, Z, w.K, w.n_refine, w.cap_shrink, w.rrs_seed, precision="f64")
        torch.cuda.synchronize()
    if args.precision == "f32_plain":
        err = error_vs(out, ref)
    if want_forms:
        forms = {args.precision: {"ms_per_step": sec_main_ms(t0, t1, args.steps),
                                  "value": w.projections / ((t1 - t0) / args.steps),
                                  "identical_to_f64": error_vs(out, ref)["queries_differing"] == 0
                                  and error_vs(out, ref).get("count_mismatches", 0) == 0}}
        for prec_name in ("f32_plain", "f32"):
            print(f"[bench] form {prec_name} ...", file=sys.stderr, flush=True)
            o2, s2 = run_form(fn, X, Z, w, prec_name, 2)
            e2 = error_vs(o2, ref)
            forms[prec_name] = {"ms_per_step": s2 * 1e3, "value": w.projections / s2,
                                "error_vs_f64": e2}
        wp = workloads.make("c5", notion="projection")
        print("[bench] projection depth, same data, f32 ...", file=sys.stderr, flush=True)
        _, s3 = run_form(rrs.DEPTH_FUNCS["projection"], X, Z, wp, "f32", 1)
        forms["c5p_projection_f32"] = {"ms_per_step": s3 * 1e3, "value": wp.projections / s3}

    sec = (t1 - t0) / args.steps
    proj = w.projections
    value = proj / sec

    # dominant kernel's roofline from its live HIP-event timings
    roof = None
    modelled = {k: v for k, v in prof.items() if kernel_model(k, notion, w.d, args.precision)}
    dom = max(modelled.items(), key=lambda kv: kv[1]["total_ms"]) if modelled else None
    if dom is not None:
        name, st = dom
        model = kernel_model(name, notion, w.d, args.precision)
        if model is not None:
            units_per_launch = st["work_units"] / st["launches"]
            timing = "per launch: algorithmic cost of one launch / its average HIP-event time"
            if name == "k_gemm" and notion == "halfspace" and counters.get("gemm_pairs"):
                # with cap culling the sign GEMM evaluates only the pairs of the
                # points not decided by the cap bound: its algorithmic work is
                # those pairs (counted by the library), not every projection
                units_per_launch = counters["gemm_pairs"] / st["launches"]
                timing += ("; units = (query, direction, point) pairs the GEMM evaluated "
                           "(the other projections are decided by the cap bound)")
            achieved = model["per_unit"] * units_per_launch / (st["avg_ms"] * 1e-3) * model["scale"]
            kernel_ms_per_step = st["total_ms"] / args.steps
            if kernel_ms_per_step > 1.02 * sec * 1e3:
                # launches of this kernel overlapped (the library split the
                # queries over streams): per-launch times include the others'
                # share of the GPU, so rate the kernel over the whole step
                # instead (a lower bound on its rate)
                achieved = (model["per_unit"] * units_per_launch * st["launches"] / args.steps
                            / sec * model["scale"])
                timing = (f"aggregate: launches overlapped (sum of launch times "
                          f"{kernel_ms_per_step:.0f} ms per step > step {sec * 1e3:.0f} ms), "
                          f"so the rate is the step's algorithmic cost of this kernel / the step time")
            roof = {"kernel": name, "bound": model["bound"], "achieved": achieved,
                    "peak": model["peak"], "unit": model["unit"], "frac": achieved / model["peak"],
                    "traffic": None, "avg_launch_ms": st["avg_ms"],
                    "units_per_launch": units_per_launch, "per_unit": model["what"],
                    "timing": timing}
            rec = recorded_traffic(name, args.workload, args.precision)
            if rec is not None:
                # HBM bytes per launch (counter runs), beside the algorithmic bytes
                roof["traffic"] = rec["bytes"]
                roof["traffic_detail"] = rec
                if model["unit"] == "GB/s":
                    roof["algorithmic_bytes"] = model["per_unit"] * units_per_launch
            if "issued_per_unit" in model:
                roof["issued_frac"] = (roof["frac"] * model["issued_per_unit"]
                                       / model["per_unit"])

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, notion, args.cpu_queries)

    line = {
        "metric": "query·direction·point projections/s",
        "value": value,
        "unit": "projections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f32_plain": "f32",
                  "bf16": "bf16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {notion} depth, {w.recipe}; K={w.K}, "
                               f"n_refine={w.n_refine}, cap_shrink={w.cap_shrink}",
                   "notion": notion, "n": w.n, "d": w.d, "queries": w.nq, "K": w.K,
                   "n_refine": w.n_refine, "cap_shrink": w.cap_shrink,
                   "precision": args.precision,
                   "projections_per_step": proj},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": {k: {"avg_ms": v["avg_ms"], "launches_per_step": v["launches"] / args.steps,
                        "ms_per_step": v["total_ms"] / args.steps} for k, v in prof.items()},
        "counters": counters,
        "depth_mean": float(depth.mean()),
    }
    if counters.get("gemm_pairs"):
        gp = counters["gemm_pairs"] / args.steps
        line["cull"] = {"gemm_pairs_per_step": gp, "gemm_fraction": gp / proj,
                        "what": "pairs the sign GEMM evaluated; the rest were decided by the "
                                "cap bound of refinements l >= 2 (exact)"}
    if err is not None:
        line["error_vs_f64"] = err
    if forms is not None:
        line["forms"] = forms
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
