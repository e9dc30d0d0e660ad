#!/usr/bin/env python3
"""Benchmark of SOGRAND product-code decoding on one MI355X.

Workload: the (4096, 3249) = [64,57]^2 eBCH product code over BPSK-AWGN at
Eb/N0 = 2.5, 3.0 and 3.5 dB, 10^4 frames per Eb/N0 (seeds 1, 2, 3), list size
L = 4, query cap 10^4, 6 row+column iterations, alpha = 0.5.  One step decodes
all 3x10^4 frames (every step of the hot path: ranking, query loop, soft
output, exchange, validity checks) with inputs already resident in HBM.

Prints one JSON line.  `value` is decoded information bits per second of the
fastest form whose BLER matches the plain binary64 form at every Eb/N0.
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

PEAK_ALU_TOPS = 256 * 64 * 2.4e9 / 1e12   # VALU lane-operations: 256 CUs x 64 lanes/clk x 2.4 GHz
SNRS = ((2.5, 1), (3.0, 2), (3.5, 3))
N, K, L, QCAP, ITERS = 64, 57, 4, 10000, 6


def ops_per_word(n: int, lst: int) -> int:
    """Algorithmic lane-operations of one component decode outside the query loop.

    hard decision + syndrome 2n; ranking n*ceil(log2 n) comparisons; rho = e^-|lambda| n;
    parity-class masses 3n; Corollary 1 2L+4; eq. (LLRi) n(L+8) (L list terms, the
    soft-input terms and two logarithms); extrinsic LLR and alpha scaling 2n.
    """
    lg = math.ceil(math.log2(n))
    return 2 * n + n * lg + n + 3 * n + (2 * lst + 4) + n * (lst + 8) + 2 * n


def wilson(k: int, n: int, z: float = 1.96):
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=10000, help="frames per Eb/N0")
    ap.add_argument("--cpu-frames", type=int, default=10000, help="oracle sample: frames per Eb/N0")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="plain_f64,plain_f32,batched_f64,batched_f32")
    ap.add_argument("--tune", action="store_true",
                    help="pick the batched launch shape by timing a few candidates on a sample first")
    ap.add_argument("--no-count", action="store_true",
                    help="skip the work-counting run (for profiler runs that average kernel durations)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a device copy of this many MiB (HBM byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(frames shard across GPUs with no communication; see the design notes).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2310_10737_amd as sg
    import synth

    dev = torch.device("cuda:0")
    code = synth.ebch(N, K)
    gcode = sg.Code.ebch(N, K)
    F = args.frames
    llr_parts, cw_parts = [], []
    for snr, seed in SNRS:
        llr, cw, _ = synth.product_frames(code, snr, seed, np.arange(F))
        llr_parts.append(llr)
        cw_parts.append(cw)
    llr_all = np.concatenate(llr_parts)
    cw_all = torch.from_numpy(np.concatenate(cw_parts)).to(dev)
    del cw_parts
    x64 = torch.from_numpy(llr_all).to(dev)
    x32 = x64.float()
    total = x64.shape[0]
    info_bits_per_step = total * K * K

    def outputs(dt):
        return dict(
            hard=torch.empty((total, N, N), dtype=torch.uint8, device=dev), llr_app=None,
            success=torch.empty(total, dtype=torch.uint8, device=dev),
            half_iters=torch.empty(total, dtype=torch.int16, device=dev),
            sum_queries=torch.empty(total, dtype=torch.int64, device=dev),
            sum_max_queries=torch.empty(total, dtype=torch.int64, device=dev))

    def run_plain(x, out):
        sg.sogrand_decode_product(gcode, x, list_max=L, query_cap=QCAP, max_iter=ITERS, outputs=out)

    fcode = torch.zeros(total, dtype=torch.uint8, device=dev)
    foff = torch.arange(total, dtype=torch.int64, device=dev) * (N * N)
    shape = sg.sched()

    def run_batched(x, out, sc):
        sg.sogrand_decode_batched([gcode], fcode, foff, x.view(-1), list_max=L, query_cap=QCAP, max_iter=ITERS,
                                  sched_=sc, outputs=out)

    def tune(x):
        """Times candidate launch shapes on the first 3000 frames; returns the fastest."""
        m = min(3000, total)
        xs = x[:m].contiguous().view(-1)
        fc, fo = fcode[:m], foff[:m]
        best = None
        for w, f, ch, g in [(8, 2, 1, 3), (4, 2, 1, 6), (8, 3, 1, 3), (4, 2, 1, 8), (8, 2, 2, 3), (4, 1, 1, 6)]:
            sc = sg.sched(w, f, ch, g)
            sg.sogrand_decode_batched([gcode], fc, fo, xs, L, QCAP, ITERS, sched_=sc)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sg.sogrand_decode_batched([gcode], fc, fo, xs, L, QCAP, ITERS, sched_=sc)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, sc)
        return best[1]

    forms = {}
    for form in args.forms.split(","):
        if form == "plain_f64":
            x, out = x64, outputs(torch.float64)
            step = lambda: run_plain(x64, out)  # noqa: E731
        elif form == "plain_f32":
            x, out = x32, outputs(torch.float32)
            step = lambda: run_plain(x32, out)  # noqa: E731
        elif form in ("batched_f64", "batched_f32"):
            x = x64 if form == "batched_f64" else x32
            out = outputs(x.dtype)
            out["hard"] = out["hard"].view(-1)
            out["status"] = torch.zeros(1, dtype=torch.int32, device=dev)
            sc = tune(x) if args.tune else shape
            step = lambda: run_batched(x, out, sc)  # noqa: E731
        else:
            raise SystemExit(f"unknown form {form}")
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # work counted once in a separate run (the counters add atomics); decoding is deterministic
        work = {}
        if not args.no_count:
            sg.profile_begin(count_work=True)
            step()
            torch.cuda.synchronize()
            work = sg.profile_end()
        sg.profile_begin(count_work=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kern = sg.profile_end()
        ms = (t1 - t0) * 1e3 / args.steps
        if "status" in out and int(out["status"].item()) != 0:
            raise SystemExit(f"{form}: batched kernel reported status {int(out['status'].item())}")
        err = torch.any((out["hard"].view(total, N, N) != cw_all).view(total, -1), dim=1).cpu().numpy()
        hi = out["half_iters"].double().cpu().numpy()
        sq = out["sum_queries"].double().cpu().numpy()
        smq = out["sum_max_queries"].double().cpu().numpy()
        per_snr = {}
        for j, (snr, _) in enumerate(SNRS):
            sl = slice(j * F, (j + 1) * F)
            k_err = int(err[sl].sum())
            per_snr[str(snr)] = dict(
                bler=k_err / F, bler_ci95=wilson(k_err, F), frames=F,
                avg_iterations=float(hi[sl].mean() / 2), queries_per_bit=float(sq[sl].mean() / (N * N)),
                parallel_queries_per_bit=float(smq[sl].mean() / (N * N)))
        forms[form] = dict(ms_per_step=ms, info_bits_per_s=info_bits_per_step / (ms / 1e3),
                           per_snr=per_snr, kernels=kern, work=work)
        if form.startswith("batched"):
            forms[form]["sched"] = dict(waves_per_group=sc.waves_per_group, frames_per_group=sc.frames_per_group,
                                        steal_chunk=sc.steal_chunk, groups_per_cu=sc.groups_per_cu)

    # matched BLER: every Eb/N0 inside the plain binary64 form's 95% interval
    base = forms.get("plain_f64")
    best_name, best = None, None
    for name, f in forms.items():
        ok = True
        if base is not None:
            for snr in base["per_snr"]:
                lo, hi_ = base["per_snr"][snr]["bler_ci95"]
                b = f["per_snr"][snr]["bler"]
                ok &= (lo - 1e-12) <= b <= (hi_ + 1e-12)
        f["bler_matches_plain_f64"] = ok
        if ok and (best is None or f["info_bits_per_s"] > best["info_bits_per_s"]):
            best_name, best = name, f

    # roofline of the dominant kernel of the chosen form: the row/column pass kernel of the
    # plain forms, the persistent kernel of the batched forms
    kname = "batched" if best_name.startswith("batched") else "product_pass"
    kp = best["kernels"].get(kname, {})
    wk = best["work"].get(kname, {})
    roof = None
    if kp.get("launches") and wk:
        avg_ms = kp["total_ms"] / kp["launches"]
        launches_per_step = kp["launches"] / args.steps
        ops_step = wk["words"] * ops_per_word(N, L) + 2 * wk["queries"] + 2 * wk["ranks"]
        ops_launch = ops_step / launches_per_step
        achieved = ops_launch / (avg_ms / 1e3) / 1e12
        roof = dict(bound="alu", achieved=achieved, peak=PEAK_ALU_TOPS, unit="Top/s",
                    frac=achieved / PEAK_ALU_TOPS, traffic=None,
                    kernel="k_batched (persistent)" if kname == "batched" else
                    "k_product_pass (row and column instantiations)",
                    avg_launch_ms=avg_ms, ops_per_launch=ops_launch,
                    words_per_step=wk["words"], queries_per_step=wk["queries"],
                    ranks_per_step=wk["ranks"], exact_rank_words_per_step=wk.get("exact_rank"))

    if args.copy_mib > 0:
        src = torch.empty(args.copy_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu and args.cpu_frames > 0:
        import oracle
        threads = min(16, len(os.sched_getaffinity(0)))
        cf = min(args.cpu_frames, F)
        sample = np.concatenate([llr_all[j * F:j * F + cf] for j in range(len(SNRS))])
        t0 = time.perf_counter()
        oracle.decode_product(code, sample, L, QCAP, ITERS, nthreads=threads)
        dt = time.perf_counter() - t0
        cpu = dict(value=sample.shape[0] * K * K / dt, unit="info bits/s", cores=threads, kind="oracle",
                   sample=f"first {cf} frames of each Eb/N0 ({sample.shape[0]} frames), {dt:.1f} s wall")

    line = {
        "metric": "decoded info bits/s at matched BLER",
        "value": best["info_bits_per_s"],
        "unit": "info bits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "eBCH [64,57]^2 product code, BPSK-AWGN 2.5/3.0/3.5 dB, 1e4 frames each, "
                               "L=4, query cap 1e4, 6 iterations, alpha 0.5",
                   "form": best_name, "frames_per_step": total, "info_bits_per_frame": K * K,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": {k: {kk: vv for kk, vv in v.items() if kk not in ("work",)} for k, v in forms.items()},
        "p99_frame_latency_ms": None,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
