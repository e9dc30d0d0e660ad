#!/usr/bin/env python3
"""Benchmark of SOGRAND product-code decoding on one MI355X.

Default workload (--workload headline): the metric "decoded info bits/s (batched/served vs
plain) at matched BLER; p99 frame latency", one JSON line combining
  * the mixed stream (the line's `value`): 3x10^4 frames, codes uniform over the eBCH
    [32,26]^2, [64,57]^2 and [128,120]^2 product codes, Eb/N0 uniform in [2, 4] dB (seed 4),
    binary32 LLR storage, L = 4, query cap 10^5, 6 iterations, alpha 0.5: one persistent
    batched launch per step against per-code plain calls on the same frames, resident in HBM;
  * the serving form (`served`, `p50_frame_latency_ms`, `p99_frame_latency_ms`): 10^5
    requests arriving as a Poisson process of rate 2x10^5/s (seed 6), codes uniform over the
    three, Eb/N0 uniform in [2.5, 4.0] dB, the same decoder settings, continuous batching;
  * the [64,57]^2 workload's forms (`product_64x57`): 10^4 frames at each of 2.5, 3.0, 3.5 dB
    (seeds 1-3), L = 4, cap 10^4, 6 iterations; plain and batched, binary64 and binary32.

Other workloads, each printing its own line:
  product    the [64,57]^2 workload above, with the oracle as CPU baseline.
  mixed      the mixed stream alone.
  component  2^20 independent [128,120] words at 4.0 dB (seed 5), cap 10^5,
             L = 1 and 4, FP32 and FP64 storage.
  serve      the serving workload alone.
  gldpc      the (1024, 640) QC-GLDPC code with [32,26] eBCH check nodes at
             Eb/N0 = 2.0, 2.25 and 2.5 dB, 10^4 frames each (seeds 11-13),
             L = 4, cap 10^4, alpha = 0.6, 20 iterations, list-BLER stop 10^-5
             (the paper's GLDPC settings); plain FP64 and FP32 storage and the
             batched form with FP32 storage.
  rician     [64,57]^2 over block Rician fading (N_c = 256, t = 8, K = 6) with
             Gray QPSK and a random interleaver, Eb/N0 = 6, 8, 10 dB, 10^4
             frames each (seeds 21-23), L = 4, cap 10^4, alpha = 0.5, 20
             iterations, list-BLER stop 10^-5 (the paper's fading settings).

Every decode computes in binary64; `dtype` names that arithmetic, and the LLR storage of the
timed form is given in the config.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import math
import os
import re
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ALU_TOPS = 256 * 64 * 2.4e9 / 1e12   # VALU lane-operations: 256 CUs x 64 lanes/clk x 2.4 GHz
SNRS = ((2.5, 1), (3.0, 2), (3.5, 3))
N, K, L, QCAP, ITERS = 64, 57, 4, 10000, 6
MIX_CODES = ((32, 26), (64, 57), (128, 120))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "product_64x57_hbm_bytes.md")
MIXED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batched_mixed_hbm_bytes.md")
KERNEL_SOURCES = ("word.hpp", "pair.hpp", "decode.hip", "batched.hip", "internal.hpp")


def ops_per_word(n: int, lst: int) -> int:
    """Algorithmic lane-operations of one component decode outside the query loop.

    hard decision + syndrome 2n; ranking n*ceil(log2 n) comparisons; rho = e^-|lambda| n;
    parity-class masses 3n; Corollary 1 2L+4; eq. (LLRi) n(L+8) (L list terms, the
    soft-input terms and two logarithms); extrinsic LLR and alpha scaling 2n.
    """
    lg = math.ceil(math.log2(n))
    return 2 * n + n * lg + n + 3 * n + (2 * lst + 4) + n * (lst + 8) + 2 * n


def algorithmic_ops(work: dict, n: int, lst: int) -> float:
    """Per query: one syndrome XOR and one mass multiply per rank, plus the zero test and the
    accumulation (2 + 2w); per word: ops_per_word."""
    return work["words"] * ops_per_word(n, lst) + 2 * work["queries"] + 2 * work["ranks"]


def wilson(k: int, n: int, z: float = 1.96):
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


def kernel_digest() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2310_10737_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(form: str, path: str = None):
    """HBM bytes per launch of the form's dominant kernel (the row/column pass kernel, or the
    persistent kernel), from a committed counter summary (the [64,57]^2 one by default), if it
    was taken on the current kernel sources (else None)."""
    try:
        text = open(path or TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    if not m or m.group(1) != kernel_digest():
        return None
    m = re.search(rf"bytes_per_launch\[{form}\]:\s*([0-9.eE+]+)", text)
    return float(m.group(1)) if m else None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads for the oracle: every core this process may run on, at most 16 (the host share
    of one GPU on the machines measured here, whatever the affinity mask shows)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def timed(step, steps, warmup, sg, count=True):
    """Runs warmup steps, a work-counting step (separate: its atomics perturb timing), then the
    timed steps under HIP-event profiling; returns (ms per step, kernel stats, work stats)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    work = {}
    if count:
        sg.profile_begin(count_work=True)
        step()
        torch.cuda.synchronize()
        work = sg.profile_end()
    sg.profile_begin(count_work=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = sg.profile_end()
    return (t1 - t0) * 1e3 / steps, kern, work


def roofline(kname, label, kern, work, steps, n, lst, traffic=None):
    kp, wk = kern.get(kname, {}), work.get(kname, {})
    if not kp.get("launches") or not wk:
        return None
    avg_ms = kp["total_ms"] / kp["launches"]
    launches_per_step = kp["launches"] / steps
    ops_launch = algorithmic_ops(wk, n, lst) / launches_per_step
    achieved = ops_launch / (avg_ms / 1e3) / 1e12
    return dict(bound="alu", achieved=achieved, peak=PEAK_ALU_TOPS, unit="Top/s", frac=achieved / PEAK_ALU_TOPS,
                traffic=traffic, kernel=label, avg_launch_ms=avg_ms, ops_per_launch=ops_launch,
                words_per_step=wk["words"], queries_per_step=wk["queries"], ranks_per_step=wk["ranks"],
                exact_rank_words_per_step=wk.get("exact_rank"))


def base_line(args, metric, value, unit, ms, dtype, config, roof, cpu, **extra):
    line = {
        "metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config,
        "roofline": roof, "cpu_baseline": cpu,
    }
    line.update(extra)
    return line


def _mixed_chunk(job):
    import numpy as np
    from threadpoolctl import threadpool_limits
    import synth
    nks, lo, hi, seed, a, b = job
    with threadpool_limits(1):   # one BLAS thread per worker process
        codes = [synth.ebch(*nk) for nk in nks]
        cidx, eb, offs, llr, cw = synth.mixed_product_frames(codes, lo, hi, seed, np.arange(a, b))
    return cidx, eb, offs, llr.astype(np.float32), cw


_FRAME_SETS = {}


def mixed_frames_f32(nks, lo, hi, seed, F, np):
    """synth.mixed_product_frames over frames 0..F-1 with FP32 LLRs, generated by a process pool
    in chunks of frames (each frame's values depend only on (seed, frame), so the result is the
    same as one call).  The pool forks, so a run that needs several sets generates them all
    before the GPU is touched; a set is generated once per process."""
    key = (tuple(nks), lo, hi, seed, F)
    if key not in _FRAME_SETS:
        _FRAME_SETS[key] = _mixed_frames_f32(nks, lo, hi, seed, F, np)
    return _FRAME_SETS[key]


def _mixed_frames_f32(nks, lo, hi, seed, F, np):
    import multiprocessing as mp
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    step = 1000
    jobs = [(nks, lo, hi, seed, a, min(F, a + step)) for a in range(0, F, step)]
    pool = mp.get_context("fork").Pool(workers)
    try:
        parts = pool.map(_mixed_chunk, jobs)
    finally:
        # the workers exit on their own; terminating them would signal them while a
        # profiler's handlers are installed
        pool.close()
        pool.join()
    cidx = np.concatenate([p[0] for p in parts])
    eb = np.concatenate([p[1] for p in parts])
    base, offs = 0, []
    for p in parts:
        offs.append(p[2] + base)
        base += p[3].shape[0]
    return cidx, eb, np.concatenate(offs), np.concatenate([p[3] for p in parts]), np.concatenate([p[4] for p in parts])


# --------------------------------------------------------------------------------------------
# frame workloads (product, gldpc, rician): frames of one code at a few Eb/N0, several forms
# --------------------------------------------------------------------------------------------
def frame_outputs(torch, total, n, dev):
    return dict(hard=torch.empty((total, n, n), dtype=torch.uint8, device=dev), llr_app=None,
                success=torch.empty(total, dtype=torch.uint8, device=dev),
                half_iters=torch.empty(total, dtype=torch.int16, device=dev),
                sum_queries=torch.empty(total, dtype=torch.int64, device=dev),
                sum_max_queries=torch.empty(total, dtype=torch.int64, device=dev))


def per_snr_stats(out, cw_all, snrs, F, n):
    """BLER (with its 95 % Wilson interval), iterations and queries per coded bit for each Eb/N0
    group of F consecutive frames."""
    import torch
    total = cw_all.shape[0]
    err = torch.any((out["hard"].view(total, n, n) != cw_all).view(total, -1), dim=1).cpu().numpy()
    hi = out["half_iters"].double().cpu().numpy()
    sq = out["sum_queries"].double().cpu().numpy()
    smq = out["sum_max_queries"].double().cpu().numpy()
    res = {}
    for j, (snr, _) in enumerate(snrs):
        sl = slice(j * F, (j + 1) * F)
        k_err = int(err[sl].sum())
        res[str(snr)] = dict(bler=k_err / F, bler_ci95=wilson(k_err, F), frames=F,
                             avg_iterations=float(hi[sl].mean() / 2),
                             queries_per_bit=float(sq[sl].mean() / (n * n)),
                             parallel_queries_per_bit=float(smq[sl].mean() / (n * n)))
    return res


def time_forms(args, sg, names, make_step, out_of, cw_all, snrs, F, n, info_bits_per_step):
    """Times each form's step; make_step(form, out) returns (step, sched or None)."""
    forms = {}
    for form in names:
        out = out_of(form)
        step, sc = make_step(form, out)
        ms, kern, work = timed(step, args.steps, args.warmup, sg, count=not args.no_count)
        if "status" in out and int(out["status"].item()) != 0:
            raise SystemExit(f"{form}: batched kernel reported status {int(out['status'].item())}")
        forms[form] = dict(ms_per_step=ms, info_bits_per_s=info_bits_per_step / (ms / 1e3),
                           per_snr=per_snr_stats(out, cw_all, snrs, F, n), kernels=kern, work=work)
        if sc is not None:
            forms[form]["sched"] = dict(waves_per_group=sc.waves_per_group, frames_per_group=sc.frames_per_group,
                                        steal_chunk=sc.steal_chunk, groups_per_cu=sc.groups_per_cu)
    return forms


def choose_form(forms):
    """The fastest form whose BLER lies inside the plain binary64 form's 95 % interval at every
    Eb/N0; adds bler_matches_plain_f64 and, for batched forms, speedup_vs_plain."""
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
    for prec in ("f64", "f32"):
        if f"plain_{prec}" in forms and f"batched_{prec}" in forms:
            forms[f"batched_{prec}"]["speedup_vs_plain"] = (forms[f"plain_{prec}"]["ms_per_step"]
                                                            / forms[f"batched_{prec}"]["ms_per_step"])
    return best_name, best


def dominant_roofline(args, best_name, best, n, traffic=None):
    """Roofline of the chosen form's dominant kernel: the pass kernel of the plain forms, the
    persistent kernel of the batched forms."""
    if best_name.startswith("batched"):
        return roofline("batched", "k_batched (persistent)", best["kernels"], best["work"], args.steps, n, L,
                        traffic=traffic)
    return roofline("product_pass", "k_product_pass (both word families)", best["kernels"], best["work"],
                    args.steps, n, L, traffic=traffic)


def oracle_baseline(args, np, llr_all, ngroups, F, decode, info_bits_per_frame):
    """The oracle over the first cpu_frames frames of each Eb/N0 group, on up to 16 threads."""
    if args.no_cpu or args.cpu_frames <= 0:
        return None
    threads = host_threads()
    cf = min(args.cpu_frames, F)
    sample = np.concatenate([llr_all[j * F:j * F + cf] for j in range(ngroups)])
    t0 = time.perf_counter()
    decode(sample, threads)
    dt = time.perf_counter() - t0
    c1 = max(1, cf // 20)
    s1 = np.concatenate([llr_all[j * F:j * F + c1] for j in range(ngroups)])
    t1 = time.perf_counter()
    decode(s1, 1)
    dt1 = time.perf_counter() - t1
    return dict(value=sample.shape[0] * info_bits_per_frame / dt, unit="info bits/s", cores=threads, kind="oracle",
                sample=f"first {cf} frames of each Eb/N0 ({sample.shape[0]} frames), {dt:.1f} s wall",
                cpu_model=cpu_model(), affinity_cores=len(os.sched_getaffinity(0)),
                one_thread=dict(value=s1.shape[0] * info_bits_per_frame / dt1,
                                sample=f"first {c1} frames of each Eb/N0, {dt1:.1f} s wall"))


def load_frames(np, torch, make, snrs, F, dev):
    llr_parts, cw_parts = [], []
    for snr, seed in snrs:
        llr, cw = make(snr, seed)
        llr_parts.append(llr)
        cw_parts.append(cw)
    llr_all = np.concatenate(llr_parts)
    cw_all = torch.from_numpy(np.concatenate(cw_parts)).to(dev)
    x64 = torch.from_numpy(llr_all).to(dev)
    return llr_all, cw_all, x64, x64.float()


def plain_or_batched(sg, torch, gcode, total, n, dev, x64, x32, iters, stop, alpha=0.5, decode=None, sched_of=None,
                     batched=None):
    """(out_of, make_step) for the forms plain_f64/f32 (decode: sogrand_decode_product or
    sogrand_decode_gldpc) and batched_f64/f32 (batched: sogrand_decode_batched or
    sogrand_decode_batched_gldpc)."""
    decode = decode or sg.sogrand_decode_product
    batched = batched or sg.sogrand_decode_batched
    fcode = torch.zeros(total, dtype=torch.uint8, device=dev)
    foff = torch.arange(total, dtype=torch.int64, device=dev) * (n * n)

    def out_of(form):
        out = frame_outputs(torch, total, n, dev)
        if form.startswith("batched"):
            out["hard"] = out["hard"].view(-1)
            out["status"] = torch.zeros(1, dtype=torch.int32, device=dev)
        return out

    def make_step(form, out):
        x = x64 if form.endswith("f64") else x32
        if form.startswith("plain"):
            return (lambda: decode(gcode, x, list_max=L, query_cap=QCAP, max_iter=iters, alpha=alpha, outputs=out,
                                   list_bler_stop=stop)), None
        if form.startswith("batched"):
            sc = sched_of(x) if sched_of else sg.sched()
            return (lambda: batched([gcode], fcode, foff, x.view(-1), list_max=L, query_cap=QCAP, max_iter=iters,
                                    alpha=alpha, sched_=sc, outputs=out, list_bler_stop=stop)), sc
        raise SystemExit(f"unknown form {form}")
    return out_of, make_step, fcode, foff


# --------------------------------------------------------------------------------------------
# product: [64,57]^2 at three Eb/N0, plain and batched forms
# --------------------------------------------------------------------------------------------
def bench_product(args, sg, np, torch, synth):
    dev = torch.device("cuda:0")
    code = synth.ebch(N, K)
    gcode = sg.Code.ebch(N, K)
    F = args.frames
    llr_all, cw_all, x64, x32 = load_frames(
        np, torch, lambda snr, seed: synth.product_frames(code, snr, seed, np.arange(F))[:2], SNRS, F, dev)
    total = x64.shape[0]
    iters, stop = args.iters, args.list_bler_stop

    def tune(x):
        """The library's launch-shape tuner on the step's own frames (a smaller sample weighs the
        end of a launch, where the last frames drain, more than the full step does)."""
        best, _ = sg.sched_tune([gcode], fcode, foff, x.contiguous().view(-1), L, QCAP, iters, list_bler_stop=stop)
        return best

    out_of, make_step, fcode, foff = plain_or_batched(sg, torch, gcode, total, N, dev, x64, x32, iters, stop,
                                                      sched_of=tune if args.tune else None)
    forms = time_forms(args, sg, args.forms.split(","), make_step, out_of, cw_all, SNRS, F, N, total * K * K)
    best_name, best = choose_form(forms)
    # the recorded HBM bytes were counted on the default configuration only
    default_cfg = iters == ITERS and stop == 0.0 and F == 10000
    roof = dominant_roofline(args, best_name, best, N, traffic=recorded_traffic(best_name) if default_cfg else None)

    def oracle_decode(sample, threads):
        import oracle
        oracle.decode_product(code, sample, L, QCAP, iters, nthreads=threads, pstop=stop)
    cpu = oracle_baseline(args, np, llr_all, len(SNRS), F, oracle_decode, K * K)

    storage = "f32" if best_name.endswith("f32") else "f64"
    settings = f"L=4, query cap 1e4, {iters} iterations, alpha 0.5"
    if stop > 0:
        settings += f", list-BLER stop {stop:g}"
    config = {"workload": "eBCH [64,57]^2 product code, BPSK-AWGN 2.5/3.0/3.5 dB, 1e4 frames each, " + settings,
              "form": best_name, "llr_storage": storage, "frames_per_step": total,
              "info_bits_per_frame": K * K, "parallelism": "single GPU"}
    return base_line(args, "decoded info bits/s at matched BLER", best["info_bits_per_s"], "info bits/s",
                     best["ms_per_step"], "f64", config, roof, cpu,
                     forms={k: {kk: vv for kk, vv in v.items() if kk != "work"} for k, v in forms.items()},
                     p99_frame_latency_ms=None)


# --------------------------------------------------------------------------------------------
# mixed: one persistent launch over three codes vs per-code plain calls
# --------------------------------------------------------------------------------------------
def bench_mixed(args, sg, np, torch, synth):
    """The mixed stream: one persistent batched launch per step against per-code plain calls
    on the same HBM-resident frames; BLER per code for both forms."""
    dev = torch.device("cuda:0")
    F, qcap = (args.frames if args.frames_set else 30000), (args.qcap or 100000)
    codes = [synth.ebch(*nk) for nk in MIX_CODES]
    cidx, eb, offs, llr, cw = mixed_frames_f32(MIX_CODES, 2.0, 4.0, 4, F, np)
    gcodes = [sg.Code.ebch(*nk) for nk in MIX_CODES]
    x = torch.from_numpy(llr).to(dev)
    fc = torch.from_numpy(cidx).to(dev)
    fo = torch.from_numpy(offs).to(dev)
    info = int(sum(codes[c].k ** 2 for c in cidx))
    groups = []
    for c, code in enumerate(codes):
        sel = np.nonzero(cidx == c)[0]
        nn = code.n * code.n
        idx = (offs[sel][:, None] + np.arange(nn)[None, :]).reshape(-1)
        groups.append((c, sel, idx))
    plain_in = [x[torch.from_numpy(idx).to(dev)].view(-1, codes[c].n, codes[c].n).contiguous()
                for c, sel, idx in groups]

    pouts = []

    def plain_step():
        pouts.clear()
        for (c, sel, idx), xi in zip(groups, plain_in):
            pouts.append(sg.sogrand_decode_product(gcodes[c], xi, list_max=L, query_cap=qcap, max_iter=ITERS))

    bout = {}

    def batched_step(sc):
        bout.update(sg.sogrand_decode_batched(gcodes, fc, fo, x, list_max=L, query_cap=qcap, max_iter=ITERS,
                                              sched_=sc))

    # launch shape: the library's tuner on the step's own frames, since a smaller sample weighs the
    # end of a launch more than the full step does (--no-tune: the library default, for profiler
    # runs that should see only full-size launches)
    sc = sg.sched()
    if not args.no_tune:
        sc, _ = sg.sched_tune(gcodes, fc, fo, x, list_max=L, query_cap=qcap, max_iter=ITERS)
    ms_b, kern_b, work_b = timed(lambda: batched_step(sc), args.steps, args.warmup, sg, count=not args.no_count)
    if int(bout["status"].item()) != 0:
        raise SystemExit(f"batched kernel reported status {int(bout['status'].item())}")
    ms_p, _, _ = (None, None, None) if args.no_plain else timed(plain_step, args.steps, args.warmup, sg, count=False)
    torch.cuda.synchronize()
    same = True
    bhard = bout["hard"].cpu().numpy()
    bsucc = bout["success"].cpu().numpy()
    bhalf = bout["half_iters"].double().cpu().numpy()
    bq = bout["sum_queries"].double().cpu().numpy()
    bmq = bout["sum_max_queries"].double().cpu().numpy()
    per_code, matched = {}, True
    for (c, sel, idx), po in zip(groups, pouts or [None] * len(groups)):
        nn = codes[c].n ** 2
        if po is None:   # --no-plain: the batched form's own statistics only
            po = dict(hard=bout["hard"][torch.from_numpy(idx).to(dev)], success=bout["success"][torch.from_numpy(sel).to(dev)])
        phard = po["hard"].cpu().numpy().reshape(-1)
        same &= bool(np.array_equal(bsucc[sel], po["success"].cpu().numpy()))
        same &= bool(np.array_equal(bhard[idx], phard))
        k_b = int(np.any(bhard[idx].reshape(-1, nn) != cw[idx].reshape(-1, nn), axis=1).sum())
        k_p = int(np.any(phard.reshape(-1, nn) != cw[idx].reshape(-1, nn), axis=1).sum())
        ci_p = wilson(k_p, int(sel.size))
        matched &= ci_p[0] - 1e-12 <= k_b / max(1, sel.size) <= ci_p[1] + 1e-12
        per_code[f"[{codes[c].n},{codes[c].k}]^2"] = dict(
            frames=int(sel.size), bler_batched=k_b / max(1, sel.size), bler_plain=k_p / max(1, sel.size),
            bler_plain_ci95=ci_p, avg_iterations=float(bhalf[sel].mean() / 2),
            queries_per_bit=float(bq[sel].mean() / nn), parallel_queries_per_bit=float(bmq[sel].mean() / nn))
    roof = None
    kp, wk = kern_b.get("batched", {}), work_b.get("batched", {})
    if kp.get("launches") and wk:
        # ops per word depend on n: weight by each code's share of the decoded words
        share = {c: float(bhalf[sel].sum()) * codes[c].n for c, sel, _ in groups}
        tw = sum(share.values())
        per_word = sum(ops_per_word(codes[c].n, L) * w for c, w in share.items()) / max(1.0, tw)
        ops = wk["words"] * per_word + 2 * wk["queries"] + 2 * wk["ranks"]
        avg_ms = kp["total_ms"] / kp["launches"]
        ops_launch = ops / (kp["launches"] / args.steps)
        achieved = ops_launch / (avg_ms / 1e3) / 1e12
        default_cfg = F == 30000 and qcap == 100000
        traffic = recorded_traffic("batched_f32", MIXED_TRAFFIC_FILE) if default_cfg else None
        roof = dict(bound="alu", achieved=achieved, peak=PEAK_ALU_TOPS, unit="Top/s", frac=achieved / PEAK_ALU_TOPS,
                    traffic=traffic, kernel="k_batched<float, 8 waves, n <= 128> (persistent)",
                    avg_launch_ms=avg_ms, ops_per_launch=ops_launch, words_per_step=wk["words"],
                    queries_per_step=wk["queries"], ranks_per_step=wk["ranks"],
                    exact_rank_words_per_step=wk.get("exact_rank"))
    cpu = None
    if not args.no_cpu and args.cpu_frames > 0:
        import oracle
        threads = host_threads()

        def oracle_rate(count, nthreads):
            t0 = time.perf_counter()
            bits = 0
            for c, code in enumerate(codes):
                sel = np.nonzero(cidx[:count] == c)[0]
                if sel.size == 0:
                    continue
                nn = code.n * code.n
                fr = np.stack([llr[o:o + nn] for o in offs[sel]]).astype(np.float64)
                oracle.decode_product(code, fr.reshape(-1, code.n, code.n), L, qcap, ITERS, store_f32=True,
                                      nthreads=nthreads)
                bits += sel.size * code.k ** 2
            dt = time.perf_counter() - t0
            return bits / dt, dt

        cf = min(args.cpu_frames, F)
        rate, dt = oracle_rate(cf, threads)
        c1 = min(max(1, cf // 10), F)
        rate1, dt1 = oracle_rate(c1, 1)
        cpu = dict(value=rate, unit="info bits/s", cores=threads, kind="oracle",
                   sample=f"first {cf} frames of the mixed stream, {dt:.1f} s wall on {threads} threads",
                   cpu_model=cpu_model(), affinity_cores=len(os.sched_getaffinity(0)),
                   one_thread=dict(value=rate1, sample=f"first {c1} frames, {dt1:.1f} s wall"))
    config = {"workload": "mixed eBCH product frames [32,26]^2/[64,57]^2/[128,120]^2 uniform, BPSK-AWGN Eb/N0 "
                          f"U[2,4] dB (seed 4), {F} frames, L=4, query cap {qcap}, 6 iterations, alpha 0.5",
              "form": "batched_f32", "llr_storage": "f32", "frames_per_step": F,
              "sched": dict(waves_per_group=sc.waves_per_group, frames_per_group=sc.frames_per_group,
                            steal_chunk=sc.steal_chunk, groups_per_cu=sc.groups_per_cu),
              "parallelism": "single GPU"}
    line = base_line(args, "decoded info bits/s (batched/served vs plain) at matched BLER; p99 frame latency",
                     info / (ms_b / 1e3), "info bits/s", ms_b, "f64", config, roof, cpu,
                     plain_f32=None if ms_p is None else dict(ms_per_step=ms_p, info_bits_per_s=info / (ms_p / 1e3)),
                     speedup_vs_plain=None if ms_p is None else ms_p / ms_b,
                     identical_to_plain=None if ms_p is None else same,
                     bler_matches_plain=None if ms_p is None else bool(matched),
                     per_code=per_code)
    del x, fc, fo, plain_in, pouts
    bout.clear()
    return line


def bench_headline(args, sg, np, torch, synth):
    """The metric's own line: the mixed stream (value), the served form (latency) and the
    [64,57]^2 forms, each under its own config."""
    # the served form first, as a serving process would start: its four lanes' streams then get
    # hardware queues of their own (HIP gives a process four; once other streams hold one, two
    # lanes share a queue and their steps serialise: 0.20 ms mean steps against 0.15)
    srv = bench_serve(args, sg, np, torch, synth)
    torch.cuda.empty_cache()
    line = bench_mixed(args, sg, np, torch, synth)
    torch.cuda.empty_cache()
    line["served"] = {k: srv[k] for k in ("value", "unit", "config", "p50_frame_latency_ms", "p99_frame_latency_ms",
                                          "offered_info_bits_per_s", "p99_frame_latency_ms_middle_80pct_arrivals",
                                          "mean_step_ms", "max_step_ms", "admission_retries", "per_code")}
    line["served"]["vs_plain"] = srv["value"] / line["plain_f32"]["info_bits_per_s"]
    line["p50_frame_latency_ms"] = srv["p50_frame_latency_ms"]
    line["p99_frame_latency_ms"] = srv["p99_frame_latency_ms"]
    pargs = argparse.Namespace(**vars(args))
    pargs.frames, pargs.no_cpu = 10000, True
    prod = bench_product(pargs, sg, np, torch, synth)
    torch.cuda.empty_cache()
    line["product_64x57"] = dict(
        config=prod["config"], value=prod["value"], unit=prod["unit"], roofline=prod["roofline"],
        forms={k: {kk: vv for kk, vv in v.items() if kk not in ("kernels", "per_snr")} | {"per_snr": v["per_snr"]}
               for k, v in prod["forms"].items()})
    line["plan_small_batches"] = bench_plan(sg, np, torch, synth)
    return line


def bench_plan(sg, np, torch, synth):
    """Small batches, where launches cost: the plain path's decode of 100 [32,26]^2 frames (3 dB,
    L=4, cap 1e3, FP64) called eagerly and replayed from its recorded graph (sogrand_plan_*),
    each timed call to completion, at I_max 4 and 20."""
    code = synth.ebch(32, 26)
    g = sg.Code.ebch(32, 26)
    llr = synth.product_frames(code, 3.0, 0, np.arange(100))[0]
    x = torch.from_numpy(llr).to("cuda:0").contiguous()
    res = {}
    for iters in (4, 20):
        out = sg.sogrand_decode_product(g, x, list_max=4, query_cap=1000, max_iter=iters)
        plan = sg.Plan(g, x, list_max=4, query_cap=1000, max_iter=iters)
        torch.cuda.synchronize()

        def median_ms(fn, reps=50):
            fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            return 1e3 * float(np.median(ts))
        eager = median_ms(lambda: sg.sogrand_decode_product(g, x, list_max=4, query_cap=1000, max_iter=iters,
                                                            outputs=out))
        graph = median_ms(plan.launch)
        same = all(bool(torch.equal(plan.outputs[k], out[k])) for k in ("hard", "success", "half_iters"))
        plan.close()
        res[f"I_max_{iters}"] = dict(launches=4 * iters + 1, eager_ms=eager, plan_ms=graph,
                                     speedup=eager / graph, identical=same)
    return dict(config={"workload": "100 eBCH [32,26]^2 frames, BPSK-AWGN 3 dB (seed 0), L=4, query cap 1e3, "
                                    "FP64, alpha 0.5", "form": "plain path, eager vs recorded graph"}, **res)


# --------------------------------------------------------------------------------------------
# component: 2^20 independent [128,120] words
# --------------------------------------------------------------------------------------------
def bench_component(args, sg, np, torch, synth):
    dev = torch.device("cuda:0")
    W = args.words
    qcap = args.qcap or 100000
    code = synth.ebch(128, 120)
    g = sg.Code.ebch(128, 120)
    llr, cw, _ = synth.component_words(code, 4.0, 5, np.arange(W))
    x64 = torch.from_numpy(llr).to(dev)
    x32 = x64.float()
    cwt = torch.from_numpy(cw).to(dev)
    forms = {}
    for name, x, lst in (("L4_f32", x32, 4), ("L1_f32", x32, 1), ("L4_f64", x64, 4), ("L1_f64", x64, 1)):
        out = dict(llr_app=None, llr_ext=torch.empty_like(x),
                   hard=torch.empty((W, 128), dtype=torch.uint8, device=dev),
                   n_queries=torch.empty(W, dtype=torch.int32, device=dev), n_found=None, found_q=None,
                   p_found=None, p_notfound=None)
        step = (lambda x_, l_, o_: lambda: sg.sogrand_decode_component(g, x_, list_max=l_, query_cap=qcap,
                                                                       outputs=o_))(x, lst, out)
        ms, kern, work = timed(step, args.steps, args.warmup, sg, count=not args.no_count)
        werr = torch.any(out["hard"] != cwt, dim=1).double().mean().item()
        q = out["n_queries"].double()
        forms[name] = dict(ms_per_step=ms, words_per_s=W / (ms / 1e3), info_bits_per_s=W * 120 / (ms / 1e3),
                           queries_per_s=q.sum().item() / (ms / 1e3), mean_queries=q.mean().item(),
                           max_queries=q.max().item(), word_error_rate=werr,
                           roofline=roofline("component", "k_component", kern, work, args.steps, 128, lst))
    head = forms["L4_f32"]
    cpu = None
    if not args.no_cpu and args.cpu_words > 0:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        m = min(args.cpu_words, W)
        threads = host_threads()
        sample = llr[:m].astype(np.float32).astype(np.float64)
        parts = np.array_split(sample, threads)
        t0 = time.perf_counter()
        # the oracle's C entry point releases the interpreter lock, so the threads run in parallel
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda part: oracle.decode_component(code, part, 4, qcap), parts))
        dt = time.perf_counter() - t0
        cpu = dict(value=m * 120 / dt, unit="info bits/s", cores=threads, kind="oracle",
                   sample=f"first {m} words in {threads} equal parts, L=4, {dt:.1f} s wall")
    config = {"workload": f"{W} independent eBCH [128,120] words, BPSK-AWGN 4.0 dB, query cap {qcap}, "
                          "L=4 FP32 storage (L=1 and FP64 in forms)", "form": "L4_f32", "parallelism": "single GPU"}
    return base_line(args, "decoded info bits/s (component words)", head["info_bits_per_s"], "info bits/s",
                     head["ms_per_step"], "f64", config, head["roofline"], cpu, forms=forms)


# --------------------------------------------------------------------------------------------
# gldpc: the (1024, 640) QC-GLDPC code with [32,26] eBCH check nodes
# --------------------------------------------------------------------------------------------
GLDPC_SNRS = ((2.0, 11), (2.25, 12), (2.5, 13))
GLDPC_ALPHA, GLDPC_ITERS, GLDPC_STOP = 0.6, 20, 1e-5


def bench_gldpc(args, sg, np, torch, synth):
    dev = torch.device("cuda:0")
    code = synth.ebch(32, 26)
    g = synth.gldpc(code)
    gcode = sg.Code.ebch(32, 26)
    n, F = code.n, args.frames
    llr_all, cw_all, x64, x32 = load_frames(
        np, torch, lambda snr, seed: synth.gldpc_frames(g, snr, seed, np.arange(F))[:2], GLDPC_SNRS, F, dev)
    total = x64.shape[0]
    out_of, make_step, _, _ = plain_or_batched(sg, torch, gcode, total, n, dev, x64, x32, GLDPC_ITERS, GLDPC_STOP,
                                               alpha=GLDPC_ALPHA, decode=sg.sogrand_decode_gldpc,
                                               batched=sg.sogrand_decode_batched_gldpc)
    names = [f for f in args.forms.split(",") if f in ("plain_f64", "plain_f32", "batched_f32")]
    forms = time_forms(args, sg, names, make_step, out_of, cw_all, GLDPC_SNRS, F, n, total * g.dim)
    best_name, best = choose_form(forms)
    roof = dominant_roofline(args, best_name, best, n)

    def oracle_decode(sample, threads):
        import oracle
        oracle.decode_gldpc(code, sample, L, QCAP, GLDPC_ITERS, GLDPC_ALPHA, pstop=GLDPC_STOP, nthreads=threads)
    cpu = oracle_baseline(args, np, llr_all, len(GLDPC_SNRS), F, oracle_decode, g.dim)
    config = {"workload": f"QC-GLDPC (1024, {g.dim}) with [32,26] eBCH check nodes (the paper's (1024,640)), "
                          f"BPSK-AWGN 2.0/2.25/2.5 dB, {F} frames each, L=4, query cap 1e4, alpha 0.6, "
                          "20 iterations, list-BLER stop 1e-5",
              "form": best_name, "info_bits_per_frame": g.dim, "frames_per_step": total,
              "parallelism": "single GPU"}
    return base_line(args, "decoded info bits/s (QC-GLDPC)", best["info_bits_per_s"], "info bits/s",
                     best["ms_per_step"], "f64", config, roof, cpu,
                     forms={k: {kk: vv for kk, vv in v.items() if kk != "work"} for k, v in forms.items()})


# --------------------------------------------------------------------------------------------
# rician: [64,57]^2 over block Rician fading with QPSK (N_c = 256, t = 8, K = 6)
# --------------------------------------------------------------------------------------------
RICIAN_SNRS = ((6.0, 21), (8.0, 22), (10.0, 23))
RICIAN_K, RICIAN_NC, RICIAN_ITERS, RICIAN_STOP = 6.0, 256, 20, 1e-5


def bench_rician(args, sg, np, torch, synth):
    dev = torch.device("cuda:0")
    code = synth.ebch(N, K)
    gcode = sg.Code.ebch(N, K)
    F = args.frames
    llr_all, cw_all, x64, x32 = load_frames(
        np, torch, lambda snr, seed: synth.rician_product_frames(code, snr, RICIAN_K, RICIAN_NC, seed,
                                                                 np.arange(F))[:2], RICIAN_SNRS, F, dev)
    total = x64.shape[0]
    out_of, make_step, _, _ = plain_or_batched(sg, torch, gcode, total, N, dev, x64, x32, RICIAN_ITERS, RICIAN_STOP)
    names = [f for f in args.forms.split(",") if f in ("plain_f64", "plain_f32", "batched_f32")]
    forms = time_forms(args, sg, names, make_step, out_of, cw_all, RICIAN_SNRS, F, N, total * K * K)
    best_name, best = choose_form(forms)
    roof = dominant_roofline(args, best_name, best, N)

    def oracle_decode(sample, threads):
        import oracle
        oracle.decode_product(code, sample, L, QCAP, RICIAN_ITERS, pstop=RICIAN_STOP, nthreads=threads)
    cpu = oracle_baseline(args, np, llr_all, len(RICIAN_SNRS), F, oracle_decode, K * K)
    config = {"workload": f"eBCH [64,57]^2 product code, block Rician fading (N_c 256, t 8, K 6) with Gray QPSK "
                          f"and a random interleaver, Eb/N0 6/8/10 dB, {F} frames each, L=4, query cap 1e4, "
                          "alpha 0.5, 20 iterations, list-BLER stop 1e-5",
              "form": best_name, "frames_per_step": total, "parallelism": "single GPU"}
    return base_line(args, "decoded info bits/s (block Rician fading)", best["info_bits_per_s"], "info bits/s",
                     best["ms_per_step"], "f64", config, roof, cpu,
                     forms={k: {kk: vv for kk, vv in v.items() if kk != "work"} for k, v in forms.items()})


# --------------------------------------------------------------------------------------------
# serve: open-loop Poisson arrivals through continuous batching
# --------------------------------------------------------------------------------------------
def bench_serve(args, sg, np, torch, synth):
    R = args.requests
    rate = args.rate
    qcap = args.qcap or 100000
    codes = [synth.ebch(*nk) for nk in MIX_CODES]
    cidx, eb, offs, x, cw = mixed_frames_f32(MIX_CODES, 2.5, 4.0, 6, R, np)
    gcodes = [sg.Code.ebch(*nk) for nk in MIX_CODES]
    # exponential inter-arrival times from the counter generator (stream 3 of seed 6)
    u = (synth.splitmix_stream(6, np.arange(R, dtype=np.uint64), 3, 1)[:, 0] >> np.uint64(11)).astype(np.float64)
    arrival = np.cumsum(-np.log1p(-(u * 2.0 ** -53)) / rate)
    arrival_ns = np.round((arrival - arrival[0]) * 1e9).astype(np.uint64)
    budget = args.hbm_gib << 30
    srv = sg.Server(budget, list_max=L, query_cap=qcap, max_iter=ITERS, precision=sg.SOGRAND_F32)
    # build the codes' schedules and load the kernels with one frame of each code
    for c in range(len(codes)):
        f = int(np.nonzero(cidx == c)[0][0])
        n = codes[c].n
        srv.submit(gcodes[c], np.ascontiguousarray(x[offs[f]:offs[f] + n * n]), tag=0)
    while srv.poll(max_results=8, timeout_ns=-1, want_hard=False):
        pass
    # an untimed warm-up replay of the first requests at the same rate, so that every lane
    # has run steps (its first ones carry one-time costs) before the timed replay starts
    W = min(8192, R)
    tw = sg.sogrand_clock_ns() + 5_000_000
    warm = {}
    wth = threading.Thread(target=lambda: warm.update(r=srv.replay(gcodes, cidx[:W], offs[:W], x, arrival_ns[:W], tw)))
    wth.start()
    got = 0
    while got < W:
        batch = srv.poll(max_results=1024, timeout_ns=50_000_000, want_hard=False)
        got += len(batch)
        if not batch and not wth.is_alive() and "r" not in warm:
            raise SystemExit("the warm-up replay failed")
    wth.join()
    # the poll loop below keeps up to R results alive; a full collection over them (and over
    # whatever earlier workloads left) can hold the loop long enough to back up the server's
    # completions, so the collector is paused for the timed replay
    gc.collect()
    gc.disable()
    st0 = srv.stats()
    results = []
    t0 = sg.sogrand_clock_ns() + 20_000_000
    fed = {}

    def feed():
        try:
            fed["retries"] = srv.replay(gcodes, cidx, offs, x, arrival_ns, t0)
        except Exception as e:   # reported by the main thread
            fed["error"] = e

    th = threading.Thread(target=feed)
    th.start()
    last_print = time.time()
    while len(results) < R:
        results.extend(srv.poll(max_results=1024, timeout_ns=50_000_000, want_hard=True))
        if "error" in fed:
            raise SystemExit(f"replay failed: {fed['error']}")
        if time.time() - last_print > 30:
            print(f"[serve] {len(results)}/{R} results", file=sys.stderr, flush=True)
            last_print = time.time()
    th.join()
    gc.enable()
    st1 = srv.stats()
    srv.close()
    tags = np.array([r["user_tag"] for r in results])
    done = np.array([r["t_done_ns"] for r in results], dtype=np.float64)
    lat_ms = (done - (t0 + arrival_ns[tags].astype(np.float64))) / 1e6
    span_s = (done.max() - t0) / 1e9
    info = float(sum(codes[c].k ** 2 for c in cidx))
    errs = np.zeros(R, dtype=bool)
    for r in results:
        f = r["user_tag"]
        n = codes[cidx[f]].n
        errs[f] = not np.array_equal(r["hard"].reshape(-1), cw[offs[f]:offs[f] + n * n])
    per_code = {}
    ctag = cidx[tags]
    for c, code in enumerate(codes):
        sel = cidx == c
        k_err = int(errs[sel].sum())
        per_code[f"[{code.n},{code.k}]^2"] = dict(
            requests=int(sel.sum()), bler=k_err / max(1, int(sel.sum())), bler_ci95=wilson(k_err, int(sel.sum())),
            p50_ms=float(np.percentile(lat_ms[ctag == c], 50)), p99_ms=float(np.percentile(lat_ms[ctag == c], 99)))
    steps = st1["steps"] - st0["steps"]
    # frames finishing in one step share its completion time: the gaps between
    # distinct completion times are step durations (plus any idle time)
    ends = np.unique(done)
    gaps_ms = np.diff(ends) / 1e6 if ends.size > 1 else np.zeros(1)
    mid = (arrival_ns[tags] >= np.percentile(arrival_ns, 10)) & (arrival_ns[tags] <= np.percentile(arrival_ns, 90))
    config = {"workload": f"{R} requests, Poisson arrivals {rate:.0f}/s, eBCH [32,26]^2/[64,57]^2/[128,120]^2 "
                          f"uniform, Eb/N0 U[2.5,4.0] dB, L=4, query cap {qcap}, 6 iterations, FP32 storage "
                          f"(timed after an untimed replay of the first {W} requests)",
              "hbm_budget_bytes": budget, "form": "served (continuous batching)", "parallelism": "single GPU"}
    return base_line(args, "decoded info bits/s (served) and p99 frame latency", info / span_s, "info bits/s",
                     span_s * 1e3, "f64", config, None, None,
                     p50_frame_latency_ms=float(np.percentile(lat_ms, 50)),
                     p99_frame_latency_ms=float(np.percentile(lat_ms, 99)),
                     offered_info_bits_per_s=info / max(1e-9, float(arrival[-1] - arrival[0])),
                     p99_frame_latency_ms_middle_80pct_arrivals=float(np.percentile(lat_ms[mid], 99)),
                     max_step_gap_ms=float(gaps_ms.max()), p99_step_gap_ms=float(np.percentile(gaps_ms, 99)),
                     admission_retries=fed.get("retries"), serve_steps=steps,
                     mean_step_ms=(st1["step_ms"] - st0["step_ms"]) / max(1, steps),
                     max_step_ms=st1["max_step_ms"], max_frames_per_step=st1["max_active"],
                     host_ms_between_steps=st1["host_ms"] - st0["host_ms"], per_code=per_code)


PHASES = ["hard decision, syndrome, rho", "ranking", "class masses", "query loop", "soft output",
          "rest of the line (loads, writes, masks)", "finding work (between lines)",
          "half hand-over (validity, retire or reopen)"]


def bench_phases(args, sg, np, torch, synth):
    """Wave clock cycles per word, by decode phase, of the persistent kernel in the clocked
    measurement build (`build.py --phase-clocks`): on the mixed stream and on [64,57]^2 frames at
    Eb/N0 uniform in [2.5, 3.5] dB, one decode each at the default launch shape."""
    res = {}
    for tag, nks, lo, hi, seed, qcap in [("mixed", [(32, 26), (64, 57), (128, 120)], 2.0, 4.0, 4, 100000),
                                         ("product_64x57", [(64, 57)], 2.5, 3.5, 1, 10000)]:
        F = args.frames if args.frames_set else 30000
        codes = [synth.ebch(*nk) for nk in nks]
        cidx, eb, offs, llr, cw = synth.mixed_product_frames(codes, lo, hi, seed, np.arange(F))
        g = [sg.Code.ebch(*nk) for nk in nks]
        x = torch.from_numpy(llr.astype(np.float32)).to("cuda:0")
        fc, fo = torch.from_numpy(cidx).to("cuda:0"), torch.from_numpy(offs).to("cuda:0")

        def run():
            return sg.sogrand_decode_batched(g, fc, fo, x, list_max=L, query_cap=qcap, max_iter=ITERS)
        run()
        torch.cuda.synchronize()
        sg.profile_begin(count_work=True)
        run()
        torch.cuda.synchronize()
        k = sg.profile_end()["batched"]
        tot, words = float(sum(k["phase_cycles"])), float(k["words"])
        res[tag] = dict(
            config={"workload": f"{F} frames of {'/'.join(f'[{n},{kk}]^2' for n, kk in nks)} eBCH, BPSK-AWGN "
                                f"Eb/N0 U[{lo},{hi}] dB (seed {seed}), L={L}, query cap {qcap}, {ITERS} iterations, "
                                f"FP32 storage, default launch shape"},
            words=int(k["words"]), queries=int(k["queries"]), cycles_per_word=tot / words,
            phases={nm: dict(cycles_per_word=c / words, share=c / tot) for nm, c in zip(PHASES, k["phase_cycles"])})
        del x, fc, fo
    return {"metric": "wave clock cycles per word by decode phase (clocked measurement build)",
            "value": res["mixed"]["cycles_per_word"], "unit": "cycles/word", "n_gpus": 1, "steps": 1, "warmup": 1,
            "higher_is_better": False, "data": "synthetic", "dtype": "f64",
            "config": res["mixed"]["config"], "mixed": res["mixed"], "product_64x57": res["product_64x57"]}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "product", "mixed", "component", "serve", "gldpc", "rician", "phases"])
    ap.add_argument("--frames", type=int, default=None, help="frames per Eb/N0 (product) or in total (mixed)")
    ap.add_argument("--words", type=int, default=1 << 20, help="component words")
    ap.add_argument("--requests", type=int, default=100000, help="serving requests")
    ap.add_argument("--rate", type=float, default=2e5, help="serving arrival rate (1/s)")
    ap.add_argument("--hbm-gib", type=int, default=8, help="serving slot budget")
    ap.add_argument("--qcap", type=int, default=None, help="query cap (mixed, component, serve)")
    ap.add_argument("--iters", type=int, default=ITERS, help="product workload: row+column iterations")
    ap.add_argument("--list-bler-stop", type=float, default=0.0,
                    help="product workload: end a word's search once its predicted list-BLER is below this")
    ap.add_argument("--cpu-frames", type=int, default=None, help="oracle sample: frames (per Eb/N0 for product)")
    ap.add_argument("--cpu-words", type=int, default=1 << 20, help="oracle sample: component words")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--forms", default="plain_f64,plain_f32,batched_f64,batched_f32")
    ap.add_argument("--tune", action="store_true",
                    help="product workload: pick the batched launch shape with the library's tuner first")
    ap.add_argument("--no-count", action="store_true",
                    help="skip the work-counting run (for profiler runs that average kernel durations)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a device copy of this many MiB (HBM byte-counter calibration)")
    ap.add_argument("--no-tune", action="store_true",
                    help="mixed workload: the library's default launch shape, no candidate sweep")
    ap.add_argument("--no-plain", action="store_true",
                    help="mixed workload: time the batched form only (profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(frames shard across GPUs with no communication; see the design notes).", file=sys.stderr)
        return 2
    args.frames_set = args.frames is not None
    if args.frames is None:
        args.frames = 10000
    if args.cpu_frames is None:
        args.cpu_frames = {"product": 10000, "mixed": 3000, "headline": 3000, "gldpc": 3000,
                           "rician": 3000}.get(args.workload, 0)

    import numpy as np
    import torch

    import paper_2310_10737_amd as sg
    import synth

    if args.workload == "phases":
        # the clocked measurement build, loaded in place of the product library
        from paper_2310_10737_amd import build as sgbuild
        if not os.path.exists(sgbuild.CLOCKED_LIB):
            print(f"{sgbuild.CLOCKED_LIB} is missing: build it with "
                  "python3 paper_2310_10737_amd/build.py --phase-clocks", file=sys.stderr)
            return 2
        sg._LIBPATH = sgbuild.CLOCKED_LIB
    if args.workload == "headline":
        # the mixed stream's and the served trace's frames, generated before the GPU is touched
        mixed_frames_f32(MIX_CODES, 2.0, 4.0, 4, args.frames if args.frames_set else 30000, np)
        mixed_frames_f32(MIX_CODES, 2.5, 4.0, 6, args.requests, np)
    fn = dict(headline=bench_headline, product=bench_product, mixed=bench_mixed, component=bench_component,
              serve=bench_serve, gldpc=bench_gldpc, rician=bench_rician, phases=bench_phases)[args.workload]
    line = fn(args, sg, np, torch, synth)
    if args.copy_mib > 0:
        # a plain device copy of known size: calibrates the HBM byte counters of profiler runs
        src = torch.empty(args.copy_mib << 18, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    roof = line.get("roofline")
    if roof and roof.get("bound") == "alu":
        # the derived peak stays the reference; the measured issue rate is reported beside it
        measured = sg.measure_valu_rate() / 1e12
        roof["peak_measured"] = measured
        roof["frac_of_measured"] = roof["achieved"] / measured
    if roof and roof.get("traffic") and roof.get("avg_launch_ms"):
        # the dominant kernel's HBM rate from the recorded bytes per launch, against 8 TB/s
        rate = roof["traffic"] / (roof["avg_launch_ms"] / 1e3) / 1e9
        roof["traffic_gb_per_s"] = rate
        roof["traffic_frac_of_hbm"] = rate / 8000.0
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
