"""Benchmark of the TT-RBKI sweep on one MI355X.

Workload: the 256^4 tensor (2^32 entries): the orthogonally decomposable signal
sum_{i<=50} i^-1 u_i o v_i o w_i o z_i (Haar factors; every unfolding has singular values
1/i) plus Gaussian noise at 5e-2 relative norm, scaled to RMS 1; target ranks 32,
oversampling p = 8, Krylov depth q = 4, Omega seed 0.  The tensor is built on the GPU in
float64 and rounded once into each storage tier: bfloat16 (bf16 products, float32
accumulation, float32 carries, float64 small factorisations), float32 and float64.  Each
tier's relative error is measured against the float64 tensor and compared with the float64
sweep's ("matched" when they agree to 1% of the float64 error).  The headline is the
bfloat16 sweep when it is matched (the float32 sweep otherwise): algorithmic TFLOP/s.

One step = one full sweep (every mode of Algorithm 3) over the resident tensor.
``roofline`` reports the dominant kernel of the headline sweep (timed standalone with HIP
events on the library's stream, same shape and launch configuration as inside the sweep)
against MI355X peaks; ``cpu_baseline`` times the float64 CPU oracle on a bounded sample of
the same workload on the host cores (rank 0, N = 1 only).  The 48^5 workload's sweeps are
reported alongside (``tt48x5``).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
WORKLOAD = "odeco256x4"
SIDE_WORKLOAD = "tt48x5"
TIERS = ("bf16", "f32", "f64")
CPU_SAMPLE_SLICES = 48   # oracle sample: X[..., :48] of the 256^4 tensor (about 12 s on 16 cores)


def _dtype(tier):
    import torch
    return {"bf16": torch.bfloat16, "f32": torch.float32, "f64": torch.float64}[tier]


def sweep_flops_bytes(pl, elem_bytes_x: int, elem_bytes_carry: int):
    """Algorithmic flops and HBM bytes of one sweep (streaming part only), counted for the
    streamed Krylov form whatever form the library takes (the same count for every tier):

    regular mode  : flops m n (2s + 4s(q+1) + 2r), reads (q+3) m n, writes r n
    saturated     : flops min(m,n)(min(m,n)+1) max(m,n) + 2 r m n, reads 2 m n, writes r n
    identity      : nothing
    """
    flops = 0.0
    nbytes = 0.0
    eb = elem_bytes_x
    for k in range(pl.d - 1):
        m, n, s, r = pl.m[k], pl.n[k], pl.s[k], pl.ranks[k + 1]
        kind = int(pl.kind[k])
        if kind == 2:
            flops += m * n * (2 * s + 4 * s * (pl.q + 1) + 2 * r)
            nbytes += (pl.q + 3) * m * n * eb + r * n * elem_bytes_carry
        elif kind == 1:
            sh, lo = min(m, n), max(m, n)
            flops += sh * (sh + 1) * lo + 2 * r * m * n
            nbytes += 2 * m * n * eb + r * n * elem_bytes_carry
        if kind != 0:
            eb = elem_bytes_carry
    return flops, nbytes


def time_sweeps(ttr, x, w, steps: int, warmup: int):
    import torch
    pl = ttr.plan(list(x.shape), w.ranks, w.q, w.p, x.dtype)
    ws = torch.empty(pl.workspace_bytes, dtype=torch.uint8, device=x.device)
    for _ in range(warmup):
        cores = ttr.tt_rbki(x, w.target_ranks(), w.q, w.p, seed=w.omega_seed, workspace=ws)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        cores = ttr.tt_rbki(x, w.target_ranks(), w.q, w.p, seed=w.omega_seed, workspace=ws)
    stop.record()
    torch.cuda.synchronize()
    return pl, cores, start.elapsed_time(stop) / steps


def rel_error(ttr, x64, cores):
    e = ttr.tt_error(x64, cores).cpu().numpy()
    return math.sqrt(e[0] / e[1])


def run_tiers(ttr, x64, w, steps: int, warmup: int, label: str):
    """Time every storage tier's sweep; the error of each against the float64 tensor."""
    import torch
    out = {}
    for tier in TIERS:
        print(f"[bench] {label} {tier} sweeps", file=sys.stderr, flush=True)
        x = x64 if tier == "f64" else x64.to(_dtype(tier))
        pl, cores, ms = time_sweeps(ttr, x, w, steps, warmup)
        if tier != "f64":
            del x
        eps = rel_error(ttr, x64, cores)
        del cores
        torch.cuda.empty_cache()
        eb = {"bf16": 2, "f32": 4, "f64": 8}[tier]
        flops, nbytes = sweep_flops_bytes(pl, eb, 8 if tier == "f64" else 4)
        out[tier] = {"ms_per_step": ms, "tflops": flops / ms / 1e9, "eps": eps,
                     "hbm_gbs_sweep_streamed_form": nbytes / ms / 1e6, "plan": pl}
    e64 = out["f64"]["eps"]
    for tier in ("bf16", "f32"):
        out[tier]["matched"] = abs(out[tier]["eps"] - e64) <= 1e-2 * e64
        out[tier]["speedup_vs_f64"] = out["f64"]["ms_per_step"] / out[tier]["ms_per_step"]
    return out


def dominant_kernel(ttr, xb, w, reps: int = 10):
    """The bfloat16 sweep's dominant kernel: the one-pass Gram-and-sketch kernel of mode 1
    (A A^T and A Omega_1 over the 256 x 16,777,216 unfolding, Omega_1 drawn inside the
    kernel), launched `reps` times back to back between two HIP events on the library's
    stream (the partial reductions fall outside them).  Algorithmic work per launch: 2 m n
    bytes (A read once) and m (m + 1) n + 2 m n S matrix-core flops (S = s rounded up to 16)."""
    pl = ttr.plan(list(xb.shape), w.ranks, w.q, w.p, xb.dtype)
    m, n, s = int(pl.m[0]), int(pl.n[0]), int(pl.s[0])
    if not int(pl.gram_first[0]):
        raise RuntimeError("mode 1 does not take the Gram-first form")
    a = xb.reshape(m, n)
    ttr.gram_sketch_timed(a, w.omega_seed, 1, s, 2)
    _, _, ms = ttr.gram_sketch_timed(a, w.omega_seed, 1, s, reps)
    # One elementwise copy of A (reads and writes 2 m n bytes): the reference dispatch
    # against which the HBM byte counters of a profiled run are scaled.
    import torch
    torch.neg(a, out=torch.empty_like(a))
    torch.cuda.synchronize()
    S = (s + 15) // 16 * 16
    alg_bytes = 2.0 * m * n
    alg_flops = float(m * (m + 1) * n + 2 * m * n * S)
    return {"m": m, "n": n, "s": s, "ms": ms, "launches": reps, "bytes": alg_bytes, "flops": alg_flops,
            "gbs": alg_bytes / ms / 1e6, "tflops": alg_flops / ms / 1e9}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gram_sketch_bf16_256x16777216_traffic.txt")
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2308_01480_amd", "csrc", f)
                   for f in ("bf16_kernels.hip", "omega.h", "convert.h", "common.h", "kernels.h")] + \
                  [os.path.join(ROOT, "paper_2308_01480_amd", "build.py")]  # the compiler flags


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the timed kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs, each scaled by a copy kernel of known size), or
    None when the summary is absent or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            kv = dict(line.split("=", 1) for line in (l.strip() for l in fh) if "=" in line and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("source_digest") != kernel_source_digest():
        return None
    return float(kv["hbm_bytes_per_launch"])


def host_info():
    info = {"nproc": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    info["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


def cpu_baseline(x64, w, slices: int = CPU_SAMPLE_SLICES):
    """The float64 oracle sweep, run once on the host cores, on the sample X[..., :slices]
    of the workload's tensor (same ranks, p, q and Omega seed); TFLOP/s of its algorithmic
    work."""
    import torch
    from oracle import ttrbki
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    xs = x64[..., :slices].contiguous().cpu().numpy()
    torch.cuda.empty_cache()
    pl = ttrbki.plan_modes(xs.shape, w.target_ranks(), w.q, w.p)
    flops = 0.0
    for mi in pl:
        if mi.kind == "regular":
            flops += mi.m * mi.n * (2 * mi.s + 4 * mi.s * (w.q + 1) + 2 * mi.r)
        elif mi.kind == "saturated":
            sh, lo = min(mi.m, mi.n), max(mi.m, mi.n)
            flops += sh * (sh + 1) * lo + 2 * mi.r * mi.m * mi.n
    t0 = time.perf_counter()
    ttrbki.tt_rbki(xs, w.target_ranks(), w.q, w.p, seed=w.omega_seed)
    dt = time.perf_counter() - t0
    out = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"one float64 oracle sweep of X[..., :{slices}] of the {WORKLOAD} tensor "
                     f"(dims {list(xs.shape)}, mode kinds {[mi.kind for mi in pl]}), {dt:.1f} s",
           "seconds": dt, "sample_gflop": flops / 1e9}
    out.update(host_info())
    return out


def side_workload(ttr, synth, steps: int, warmup: int):
    """The 48^5 workload's sweeps in the three tiers (reported beside the headline)."""
    import torch
    w = synth.workload(SIDE_WORKLOAD)
    x64 = synth.build_device(w, dtype=torch.float64)
    tiers = run_tiers(ttr, x64, w, steps, warmup, SIDE_WORKLOAD)
    del x64
    torch.cuda.empty_cache()
    return {"workload": f"{SIDE_WORKLOAD}: 48^5 TT-rank-20 N(0,1) cores + Student-t(2) noise 1e-2; r=20 p=10 q=3",
            **{t: {k: v for k, v in d.items() if k != "plan"} for t, d in tiers.items()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="skip the 48^5 workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the TT-RBKI sweep here is a single-GPU build "
              "(sharding along the last mode is described in the design notes, not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2308_01480_amd as ttr
    import synth

    w = synth.workload(WORKLOAD)
    print(f"[bench] building {WORKLOAD} dims={w.dims} on cuda:0", file=sys.stderr, flush=True)
    x64 = synth.build_device(w, dtype=torch.float64)
    torch.cuda.synchronize()
    tiers = run_tiers(ttr, x64, w, args.steps, args.warmup, WORKLOAD)
    head = "bf16" if tiers["bf16"]["matched"] else "f32"
    h = tiers[head]
    pl = h["plan"]
    f_flops, _ = sweep_flops_bytes(pl, 2, 4)
    out = {
        "metric": "TT-RBKI sweep time & TFLOP/s, BF16/FP32 vs FP64 at matched rel. error",
        "value": h["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}: 256^4 odeco signal sum_(i<=50) i^-1 (Haar factors) + Gaussian noise "
                               f"5e-2; r=32 p=8 q=4; headline tier {head}",
                   "dims": list(w.dims), "ranks": w.ranks, "p": w.p, "q": w.q, "mode_kinds": pl.kinds,
                   "gram_first": [int(pl.gram_first[i]) for i in range(pl.d - 1)],
                   "sweep_gflop_streamed_form": f_flops / 1e9},
        "tiers": {t: {k: v for k, v in d.items() if k != "plan"} for t, d in tiers.items()},
        "speedup_bf16_vs_f64": tiers["bf16"]["speedup_vs_f64"],
        "speedup_f32_vs_f64": tiers["f32"]["speedup_vs_f64"],
        "matched_rel_error": {"bf16": tiers["bf16"]["matched"], "f32": tiers["f32"]["matched"]},
    }
    if not args.no_roofline:
        print("[bench] dominant kernel", file=sys.stderr, flush=True)
        xb = x64.to(torch.bfloat16)
        dk = dominant_kernel(ttr, xb, w)
        del xb
        torch.cuda.empty_cache()
        # 2 bytes per element streamed against (m + 1) + 2 S flops per element: 206 flop/B at
        # m = 256, S = 48, below the bf16 matrix-core ridge (2500 / 8 = 312), so HBM bounds it.
        out["roofline"] = {"bound": "hbm", "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic(),
                           "kernel": f"kb_gram_sb: A A^T and A Omega_1 in one pass, bf16, mode-1 unfolding "
                                     f"{dk['m']}x{dk['n']}, s={dk['s']}, Omega drawn in the kernel",
                           "ms_per_launch": dk["ms"], "launches": dk["launches"],
                           "alg_bytes_per_launch": dk["bytes"], "alg_flops_per_launch": dk["flops"],
                           "mfma_tflops": dk["tflops"], "mfma_frac": dk["tflops"] / MFMA_PEAK_TFLOPS["bf16"]}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (float64 oracle on a sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(x64, w)
    del x64
    torch.cuda.empty_cache()
    if not args.no_side:
        out[SIDE_WORKLOAD] = side_workload(ttr, synth, args.steps, args.warmup)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
