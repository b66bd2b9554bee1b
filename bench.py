#!/usr/bin/env python3
"""Benchmark of the F-statistic search on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step is one pass of the whole hot path over the mixed-precision batched
workload: a two-sidereal-day segment (N = 86164 samples at 2 s, nfft = 2^18)
searched over 4096 sky positions x 256 spindowns = 1 048 576 templates
(per-sky demodulation and resampling, then per template the spindown chirp,
two FFTs, 2F and the threshold crossings).  Inputs are synthetic (Gaussian
noise plus five injected signals), resident in HBM before timing starts.

Printed: one JSON line with templates/s, the per-kernel HIP-event timings,
the roofline of the dominant kernel, the plain one-template-per-launch path
(256 x 64 templates), the CPU oracle timed on a bounded sample, and the same
batched workload searched with interbinning (template transforms of nfft/2
points, odd bins from their neighbours) as a separate entry, and the batched
search driven by a lattice grid (sky points and spindowns from the integers of
a generator matrix, frequencies shifted onto the grid) as another.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "F-stat templates/s at N=86164 (mixed vs plain FP64-phase); F rel err vs FP64"
HBM_PEAK_GBS = 8000.0
CAND_BYTES = 32          # device candidate entry
CX32 = 8                 # complex FP32


# device sources of the search kernels whose HBM traffic profiles/template_kernels_traffic.txt
# records (the vetting network and the host code do not change what those kernels move)
SEARCH_KERNEL_SOURCES = ("fstat_fft.hpp", "fstat_kernels.hpp", "fstat_tmpl.hpp")


def source_digest() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1410_3677_amd", "csrc")
    for name in SEARCH_KERNEL_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, templates_per_launch: int, variants: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it is current."""
    path = os.path.join(ROOT, "profiles", "template_kernels_traffic.txt")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != source_digest() or kernel not in t.get("kernels", {}):
        return None
    k = t["kernels"][kernel]
    if k.get("templates_per_launch") != templates_per_launch or t.get("variants") != variants:
        return None
    return k["bytes_per_launch"]


def cache_has_line(path, nfft: int, precision_key: int) -> bool:
    """Whether a tuning cache holds a line for this FFT length and precision key (the
    precision plus 2 with interbinning); the device tag is the library's business."""
    if not path or not os.path.exists(path):
        return False
    with open(path) as f:
        for line in f:
            p = line.split()
            if len(p) == 6 and p[1] == str(nfft) and p[2] == str(precision_key):
                return True
    return False


def fit_capacity(cap: int, torch, log, share: float = 0.5) -> int:
    """Candidate entries for a plan's device buffer: `cap`, cut to `share` of the device
    memory free now (the plan reports the true count of crossings also beyond it)."""
    free, _ = torch.cuda.mem_get_info()
    fit = int(share * free) // CAND_BYTES
    if cap > fit:
        log(f"candidate capacity {cap} cut to {fit} entries ({free / 2**30:.1f} GiB free)")
        return max(fit, 1)
    return cap


def guarded(name, log, fn, *a, **k):
    """Run a side entry of the bench; a failure is recorded in its entry instead of ending the run."""
    try:
        return fn(*a, **k)
    except Exception as e:  # noqa: BLE001 - recorded in the JSON line
        log(f"{name}: failed: {type(e).__name__}: {e}")
        return {"error": f"{type(e).__name__}: {e}"}


def _oracle_sky_worker(job):
    """One sky of the oracle sample: its sky stage and every spindown template (2F + threshold)."""
    import numpy as np
    from oracle import fstat_oracle as ora
    seg, alpha, delta, fdots, nfft, thr = job
    t0 = time.perf_counter()
    sky = ora.sky_stage(seg, alpha, delta, nfft)
    n = 0
    for f in fdots:
        tf = ora.template_two_f(seg, sky, float(f), nfft)
        n += int(np.count_nonzero(tf > thr))
    return len(fdots), n, time.perf_counter() - t0


def cpu_multicore_leg(args, log):
    """The oracle on the host's cores: one process per core, each taking one sky position of
    the batched workload with all its spindowns.  Runs before the GPU is touched, so the
    worker processes are plain forks of a process without GPU state."""
    import multiprocessing as mp
    import synth
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    w = synth.workload("batched", workers, args.nfdot)
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    jobs = [(seg, float(w.alpha[i]), float(w.delta[i]), w.fdot, nfft, w.threshold) for i in range(workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_sky_worker, jobs)
    dt = time.perf_counter() - t0
    ntpl = sum(r[0] for r in res)
    log(f"cpu oracle on {workers} cores: {ntpl / dt:.4g} templates/s ({ntpl} templates in {dt:.1f} s)")
    return {"value": ntpl / dt, "unit": "templates/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} sky x {args.nfdot} spindown templates of the batched workload, one process "
                      f"per core (numpy FP64, one thread each), {dt:.1f} s wall"}


def timed_search(args, F, torch, seg, al, de, fd, templates, nfft, log, interbinning=0, steps=None, warmup=None,
                 full_drain=False):
    """Plan (autotuned, from the cache or fixed), warm up, time `steps` searches of the
    whole template list (each followed by its count drain), and read the per-kernel
    HIP-event timings of the timed steps."""
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    label = "interbinning" if interbinning else "mixed"
    tlen = nfft // 2 if interbinning else nfft          # template transform length
    # crossings at 2F > 20 on the batched workload: about 1.1e-3 of the bins (2.1e-3 with
    # interbinning, whose odd bins of noise have a larger mean); capacity for the timed
    # steps with a margin (entries are 32 bytes)
    rate = 2.1e-3 if interbinning else 1.1e-3
    # the buffer holds one step's crossings (every step is drained by count before the next)
    cap = fit_capacity(int(max(1 << 20, 1.3 * rate * (nfft // 2) * templates)), torch, log)
    fixed = bool(args.templates_per_launch or args.skies_per_batch or args.no_autotune)
    cache = args.tuning_cache or None
    have_cache = cache_has_line(cache, nfft, 1 + 2 * interbinning)
    plan = F.Plan([F.segment_to_device(seg)], candidate_capacity=cap, workspace_from_torch=False,
                  templates_per_launch=args.templates_per_launch, skies_per_batch=args.skies_per_batch,
                  use_graph=0 if args.no_graph else 1, tuning_cache_path=cache, interbinning=interbinning)
    tuned = "fixed" if fixed else ("cache" if have_cache else "autotune")
    if tuned == "autotune":
        t_tune = time.perf_counter()
        plan.autotune(0, budget_ms=args.autotune_ms)
        log(f"{label}: autotune {time.perf_counter() - t_tune:.1f} s -> {plan.info(0)}")
    else:
        plan._set_torch_workspace()
    info = plan.info(0)
    log(f"{label}: plan {info}, capacity {cap}")
    for i in range(warmup):
        plan.search_batch(0, al, de, fd)
        torch.cuda.synchronize()
        log(f"{label}: warmup {i} done, {plan.candidate_count(allow_overflow=True)} candidates")
    plan.profile_enable(not args.no_events)
    for c in range(4):
        plan.profile_read(c, reset=True)
    torch.cuda.synchronize()
    # one step = one search of every template plus the count drain of its crossings (which
    # waits for the search and resets the device counter for the next step)
    counts = []
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.search_batch(0, al, de, fd)
        counts.append(plan.candidate_count(allow_overflow=True))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_cand = sum(counts)
    ms_step = (t1 - t0) * 1e3 / steps
    value = templates / ((t1 - t0) / steps)
    log(f"{label}: {ms_step:.1f} ms/step, {value:.4g} templates/s, {n_cand / steps:.4g} candidates/step"
        f"{'' if len(set(counts)) == 1 else f' (varying: {sorted(set(counts))})'}")

    kernels = {}
    for c, name in enumerate(F.KERNEL_NAMES):
        n, ms = plan.profile_read(c, reset=True)
        kernels[name] = {"launches": n, "total_ms": ms, "avg_ms": ms / n if n else None}
    drain = None
    if full_drain and counts:
        # one more search, then a full drain of its crossings timed on its own: key ordering
        # on the device, copy of the ordered entries, records and keys formed on the host
        plan.profile_enable(False)
        plan.search_batch(0, al, de, fd)
        torch.cuda.synchronize()
        bufs = F.candidate_buffers(max(counts[-1], 1), pinned=True)
        d0 = time.perf_counter()
        _, dkeys, nd = plan.candidates(out=bufs, allow_overflow=True)
        d1 = time.perf_counter()
        drain = {"candidates": nd, "ms": (d1 - d0) * 1e3, "entries_per_s": nd / (d1 - d0),
                 "what": "fstat_candidates after one search of the workload: device key ordering (count, scan, "
                         "scatter, per-template order), records and keys formed on the device and copied into "
                         "page-locked host arrays"}
        del bufs, dkeys
        log(f"{label}: full drain of {nd} candidates {(d1 - d0) * 1e3:.0f} ms")
    B = info["templates_per_launch"]
    N = seg.n
    cand_per_template = n_cand / max(templates * steps, 1)
    # algorithmic bytes per launch of the two template kernels:
    #  pass A writes the 2 x tlen complex FP32 intermediate of each template and reads the
    #  resampled series (2 x N complex FP32) once per launch (one sky per launch);
    #  pass B reads the intermediate back and writes the crossings.
    algo = {"template_a": B * 2 * tlen * CX32 + 2 * N * CX32,
            "template_b": B * 2 * tlen * CX32 + B * cand_per_template * CAND_BYTES}
    roofline = None
    if not args.no_events:
        dom = max(("template_a", "template_b"), key=lambda k: kernels[k]["total_ms"] or 0.0)
        avg_s = kernels[dom]["avg_ms"] / 1e3
        achieved = algo[dom] / avg_s / 1e9
        variants = info["pass_a_variant"] + 2 * info["pass_b_variant"]
        traffic = measured_traffic(dom + ("_ib" if interbinning else ""), B, variants)
        roofline = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "algorithmic_bytes_per_launch": algo[dom], "templates_per_launch": B,
                    "avg_launch_ms": kernels[dom]["avg_ms"]}
        for k in ("template_a", "template_b"):
            kernels[k]["achieved_GBs"] = algo[k] / (kernels[k]["avg_ms"] / 1e3) / 1e9
    plan.destroy()
    return {"value": value, "unit": "templates/s", "ms_per_step": ms_step, "n_cand": n_cand, "steps": steps,
            "candidates_per_step": n_cand / steps, "info": info, "kernels": kernels, "roofline": roofline,
            "tuning": tuned, "template_fft": tlen, "candidate_capacity": cap, "full_drain": drain}


def lattice_leg(args, F, torch, seg, nfft, info, log):
    """The batched search on lattice templates: a synthetic constrained generator matrix
    with about args.nsky sky points on the northern ecliptic hemisphere, spindown
    integers 0 .. args.nfdot - 1 (0 to -1e-9 Hz/s plus each sky point's offset), every
    template's frequencies shifted onto its own fraction of a bin.  Batch sizes of the
    explicit-list plan; its own throughput, not the headline value."""
    import synth
    f_ref = seg.f_off + 0.5 / seg.dt
    M = synth.lattice_matrix(nfft, seg.dt, f_ref, args.nsky, -1e-9 / max(args.nfdot - 1, 1), 4242)
    lat = F.lattice(M, synth.OBLIQUITY, f_ref)
    F.lattice_sky(lat, 1)           # first call loads the kernel
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sky = F.lattice_sky(lat, 1)
    t_sky = time.perf_counter() - t0
    nsky = int(sky["alpha"].numel())
    templates = nsky * args.nfdot
    cap = fit_capacity(int(max(1 << 20, 1.3 * 1.1e-3 * (nfft // 2) * templates)), torch, log)
    steps, warmup = min(args.steps, args.side_steps), min(args.warmup, 1)
    plan = F.Plan([F.segment_to_device(seg)], candidate_capacity=cap,
                  templates_per_launch=info["templates_per_launch"], skies_per_batch=info["skies_per_batch"],
                  use_graph=0 if args.no_graph else 1)
    for _ in range(warmup):
        plan.search_lattice(0, lat, sky, 0, args.nfdot - 1)
        torch.cuda.synchronize()
        plan.candidate_count(allow_overflow=True)
    torch.cuda.synchronize()
    n_cand = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.search_lattice(0, lat, sky, 0, args.nfdot - 1)
        n_cand += plan.candidate_count(allow_overflow=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.destroy()
    value = templates / ((t1 - t0) / steps)
    log(f"lattice: {nsky} sky points (box {sky['count']} on the sky), {value:.4g} templates/s, sky loop "
        f"{t_sky * 1e3:.2f} ms including allocation and the count read-back")
    return {"value": value, "unit": "templates/s", "ms_per_step": (t1 - t0) * 1e3 / steps, "steps": steps,
            "candidates_per_step": n_cand / steps, "sky_points": nsky, "sky_loop_ms": t_sky * 1e3,
            "config": {"workload": f"lattice templates, N={seg.n}, nfft=2^{int(math.log2(nfft))}, {nsky} sky points "
                                   f"(northern ecliptic hemisphere) x {args.nfdot} spindown integers, 2F>20",
                       "templates": templates, "templates_per_launch": info["templates_per_launch"],
                       "skies_per_batch": info["skies_per_batch"]}}


def ib_summary(ib, templates, nfft):
    """The interbinning leg for the JSON line (its own throughput; not the headline value)."""
    if ib is None or "error" in ib:
        return ib
    keep = ("value", "unit", "ms_per_step", "candidates_per_step", "kernels", "roofline", "tuning",
            "f_rel_err_vs_fp64_interbinned", "even_bins_rel_dev_vs_zero_padded",
            "odd_bins_mean_2F_ratio_vs_zero_padded", "accuracy_sample")
    out = {k: ib[k] for k in keep if k in ib}
    i = ib["info"]
    out["config"] = {"workload": f"the same {templates} templates, template transforms of nfft/2 = {nfft // 2} "
                                 "points, odd bins interbinned", "templates_per_launch": i["templates_per_launch"],
                     "skies_per_batch": i["skies_per_batch"], "pass_a_variant": i["pass_a_variant"],
                     "template_fft": ib["template_fft"], "p": i["p"], "q": i["q"]}
    return out


def vetting_leg(args, F, torch, np, dev, log):
    """Train the vetting network on oracle-generated patches (N = 86164), report false-alarm and
    false-dismissal rates against the threshold alone on held-out shapes, then run the plain
    workload (256 sky x 64 spindown) with the network attached: patch capture right after each
    F kernel launch and scoring of every crossing on the device."""
    import synth
    from oracle import vet_data, vet_oracle
    t0 = time.perf_counter()
    x, y, st = vet_data.make_dataset(5000, 32, 1600, 24)
    xe, ye, ste = vet_data.make_dataset(5001, 8, 1300, 20)
    t_gen = time.perf_counter() - t0
    log(f"vetting data: train {len(y)}, held out {len(ye)} ({t_gen:.1f} s)")
    batch = 256
    v = F.Vetter(8192)
    v.set_params(vet_oracle.init_params(np.random.default_rng(21)).astype(np.float32))
    xg, yg = torch.as_tensor(x, device="cuda"), torch.as_tensor(y, device="cuda")
    rng = np.random.default_rng(22)
    loss = torch.empty(1, device="cuda")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    steps = 0
    for ep in range(args.vet_epochs):
        perm = torch.as_tensor(rng.permutation(len(y)), device="cuda")
        for i in range(0, len(y) - batch + 1, batch):
            idx = perm[i:i + batch]
            v.gradient(xg[idx].contiguous(), yg[idx].contiguous(), loss)
            v.adam_step(1e-3)
            steps += 1
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    le = torch.empty(len(ye), device="cuda")
    v.forward(torch.as_tensor(xe, device="cuda"), le)
    le = le.cpu().numpy()
    cut = float(np.quantile(le[ye == 1], 0.01))
    far = float(np.mean(le[ye == 0] >= cut))
    fdr_added = float(np.mean(le[ye == 1] < cut))
    log(f"vetting: trained {steps} steps in {t_train:.1f} s, loss {loss.item():.4f}; held out: network keeps "
        f"{far:.4f} of noise crossings at {fdr_added:.4f} added false dismissal")
    # fused: the plain workload with patch capture and device scoring
    w2 = synth.workload("full")
    seg2 = w2.segments[0]
    cap = 1 << 21
    # the same search without the network attached: the cost of the capture (the F kernel
    # stores its launch's 2F rows, a gather copies each crossing's window)
    a2, d2, f2 = dev(w2.alpha), dev(w2.delta), dev(w2.fdot)
    p0 = F.Plan([F.segment_to_device(seg2)], candidate_capacity=cap, use_graph=0)
    p0.search_batch(0, a2[:2], d2[:2], f2)
    p0.candidate_count(allow_overflow=True)
    torch.cuda.synchronize()
    n0 = time.perf_counter()
    p0.search_batch(0, a2, d2, f2)
    torch.cuda.synchronize()
    n1 = time.perf_counter()
    p0.candidate_count(allow_overflow=True)
    p0.destroy()
    p = F.Plan([F.segment_to_device(seg2)], candidate_capacity=cap, use_graph=0)
    p.attach_vetter(v, cap)
    p.search_batch(0, a2[:2], d2[:2], f2)
    p.vet_candidates()
    p.candidate_count(allow_overflow=True)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    p.search_batch(0, a2, d2, f2)
    torch.cuda.synchronize()
    s1 = time.perf_counter()
    p.vet_candidates()
    torch.cuda.synchronize()
    s2 = time.perf_counter()
    recs, keys, n = p.candidates(capacity=cap)
    kept = int(np.sum(keys["vet_score"] >= 1.0 / (1.0 + np.exp(-cut))))
    inj = seg2.injections[0]
    near = np.abs(recs["f_hz"] - (seg2.f_off + inj.f)) < 2e-4
    p.destroy()
    v.destroy()
    # matrix-core roofline of inference: FLOPs per patch (multiply-add = 2) of the layers
    conv1 = 2 * 256 * 32 * 7
    conv23 = 2 * (2 * 256 * 32 * 224)
    dense = 2 * (8192 * 128 + 128 * 128 + 128)
    flop_patch = conv1 + conv23 + dense
    infer_tflops = flop_patch * n / (s2 - s1) / 1e12 if n else 0.0
    roof = {"bound": "mfma", "achieved": infer_tflops, "peak": 2500.0, "unit": "TFLOP/s",
            "frac": infer_tflops / 2500.0, "flop_per_patch": flop_patch, "patches": int(n),
            "note": "BF16 products with FP32 accumulation; dense BF16 peak"}
    return {"train_patches": int(len(y)), "heldout_patches": int(len(ye)), "epochs": args.vet_epochs,
            "train_s": t_train, "data_s": t_gen, "threshold_false_dismissal": st["threshold_false_dismissal"],
            "heldout_noise_kept_by_network": far, "heldout_added_false_dismissal": fdr_added,
            "heldout_noise_kept_by_threshold": 1.0,
            "plain_search_with_capture_ms": (s1 - s0) * 1e3, "plain_search_without_capture_ms": (n1 - n0) * 1e3,
            "scoring_ms": (s2 - s1) * 1e3,
            "plain_crossings": int(n), "plain_crossings_kept_by_network": kept,
            "plain_crossings_near_injection": int(near.sum()),
            "plain_crossings_near_injection_kept": int(np.sum(near & (keys["vet_score"] >= 1.0 / (1.0 + np.exp(-cut))))),
            "inference_roofline": roof}


def plain_leg(args, F, torch, np, dev, log):
    """The plain FP64-phase path: the full-segment workload (256 sky x 64 spindown), one
    template per launch, eager; then a full drain of its crossings (device-to-host copy and
    key ordering) timed on its own, and its F error against the FP64 oracle on a sample."""
    import synth
    w2 = synth.workload("full")
    seg2 = w2.segments[0]
    cap = 1 << 22
    p2 = F.Plan([F.segment_to_device(seg2)], templates_per_launch=1, skies_per_batch=1,
                candidate_capacity=cap, use_graph=0)
    a2, d2, f2 = dev(w2.alpha), dev(w2.delta), dev(w2.fdot)
    p2.search_batch(0, a2[:2], d2[:2], f2)
    torch.cuda.synchronize()
    p2.candidate_count(allow_overflow=True)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    p2.search_batch(0, a2, d2, f2)
    torch.cuda.synchronize()
    s1 = time.perf_counter()
    bufs = F.candidate_buffers(cap, pinned=True)
    d0 = time.perf_counter()
    recs, keys, n2 = p2.candidates(out=bufs)
    d1 = time.perf_counter()
    t2 = len(w2.alpha) * len(w2.fdot)
    ordered = bool(np.all(np.diff(keys["sky"].astype(np.int64) * (1 << 40) + keys["fdot_idx"].astype(np.int64)
                                  * (1 << 20) + keys["bin"]) > 0)) if n2 > 1 else True
    plain = {"value": t2 / (s1 - s0), "unit": "templates/s", "ms_per_step": (s1 - s0) * 1e3,
             "workload": f"plain FP64-phase path, one template per launch, N=86164, {len(w2.alpha)} sky x "
                         f"{len(w2.fdot)} spindown", "candidates": n2,
             "drain": {"candidates": n2, "ms": (d1 - d0) * 1e3, "ordered_by_key": ordered,
                       "what": "fstat_candidates after the search: wait, device key ordering, records and keys "
                               "formed on the device and copied into page-locked host arrays"}}
    log(f"plain: {plain['value']:.4g} templates/s; full drain of {n2} candidates {(d1 - d0) * 1e3:.1f} ms")
    if not args.no_cpu:
        # F error of the plain path against the FP64 oracle: 1 sky x 16 spindowns, all bins
        from oracle import fstat_oracle as ora
        nf2 = synth.nfft_for(seg2.n)
        nb2 = nf2 // 2
        fsel = w2.fdot[:: max(1, len(w2.fdot) // 16)][:16]
        spec2 = torch.empty(len(fsel) * nb2, dtype=torch.float32, device="cuda")
        p2.twoF_spectrum(0, a2[:1], d2[:1], dev(fsel), spec2)
        g2 = spec2.view(len(fsel), nb2).cpu().numpy().astype(np.float64)
        sky2 = ora.sky_stage(seg2, float(w2.alpha[0]), float(w2.delta[0]), nf2)
        e2 = max(float(np.max(np.abs(g2[j] - ref) / np.maximum(ref, 4.0)))
                 for j, ref in enumerate(ora.template_two_f(seg2, sky2, float(f), nf2) for f in fsel))
        plain["f_rel_err_vs_fp64"] = e2
        plain["accuracy_sample"] = f"1 sky x {len(fsel)} spindown templates of the plain workload, all bins"
        log(f"plain: max F rel err vs FP64 {e2:.3e}")
    p2.destroy()
    return plain


def ragged_leg(args, F, torch, np, dev, log):
    """Ragged batching: 32 segments of uneven length (N ~ U{20000..172328}, nfft 2^16..2^19,
    each with its own band offset and injections), 1024 sky x 128 spindown templates per
    segment, all segments in one search call (segment = -1) under a workspace budget that
    the plan's admission shrinks its batch sizes to."""
    import synth
    w = synth.workload("ragged", args.ragged_nsky, args.ragged_nfdot)
    segs = [F.segment_to_device(s) for s in w.segments]
    per_seg = len(w.alpha) * len(w.fdot)
    templates = per_seg * len(segs)
    bins = sum(synth.nfft_for(s.n) // 2 for s in w.segments)
    # crossings at 2F > 20: about 1.1e-3 of the bins on whole sidereal days, more where
    # the simplified form leaves out a large <ab>
    cap = fit_capacity(int(max(1 << 20, 1.6e-3 * bins * per_seg)), torch, log)
    budget = int(args.ragged_budget_gib * 2**30)
    plan = F.Plan(segs, candidate_capacity=cap, workspace_budget_bytes=budget,
                  use_graph=0 if args.no_graph else 1)
    info = plan.info(0)
    ws = plan.workspace.numel() if plan.workspace is not None else 0
    a, d, f = dev(w.alpha), dev(w.delta), dev(w.fdot)
    steps, warmup = min(args.steps, args.ragged_steps), min(args.warmup, 1)
    for _ in range(warmup):
        plan.search_batch(-1, a, d, f)
        plan.candidate_count(allow_overflow=True)
    torch.cuda.synchronize()
    counts = []
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.search_batch(-1, a, d, f)
        counts.append(plan.candidate_count(allow_overflow=True))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.destroy()
    value = templates / ((t1 - t0) / steps)
    # the two template passes' algorithmic bytes: 2 nfft x 8 B written and read per template,
    # each segment with its own nfft (the per-sky stage and the candidates left out)
    tbytes = sum(per_seg * 2 * 2 * synth.nfft_for(s.n) * 8 for s in w.segments)
    ns = sorted(s.n for s in w.segments)
    log(f"ragged: {len(segs)} segments, {templates} templates, {value:.4g} templates/s, "
        f"{counts[-1]} candidates/step, batches {info['templates_per_launch']} x {info['skies_per_batch']}")
    return {"value": value, "unit": "templates/s", "ms_per_step": (t1 - t0) * 1e3 / steps, "steps": steps,
            "template_bytes_per_step": tbytes,
            "achieved_GBs_whole_step": tbytes / ((t1 - t0) / steps) / 1e9,
            "candidates_per_step": sum(counts) / steps, "overflowed": max(counts) > cap,
            "config": {"workload": f"{len(segs)} segments, N from {ns[0]} to {ns[-1]}, nfft 2^"
                                   f"{int(math.log2(synth.nfft_for(ns[0])))}..2^{int(math.log2(synth.nfft_for(ns[-1])))}, "
                                   f"{len(w.alpha)} sky x {len(w.fdot)} spindown per segment, one call, 2F>20",
                       "templates": templates, "workspace_budget_bytes": budget, "workspace_bytes": ws,
                       "templates_per_launch": info["templates_per_launch"],
                       "skies_per_batch": info["skies_per_batch"]}}


def cpu_sample_leg(args, F, torch, np, dev, log, w, seg, fd, nfft, ib, cpu_mc):
    """The oracle on one core over a bounded sample of the batched workload, and the GPU's
    F error against it there (and, with interbinning, against the interbinned oracle)."""
    from oracle import fstat_oracle as ora
    sk = list(range(args.cpu_skies))
    p3 = F.Plan([F.segment_to_device(seg)])
    nb = nfft // 2
    spec = torch.empty(len(sk) * args.nfdot * nb, dtype=torch.float32, device="cuda")
    p3.twoF_spectrum(0, dev(w.alpha[sk]), dev(w.delta[sk]), fd, spec)
    torch.cuda.synchronize()
    g = spec.view(len(sk), args.nfdot, nb).cpu().numpy()
    p3.destroy()
    gi = None
    ib_ok = ib is not None and "error" not in ib
    if ib_ok:
        p4 = F.Plan([F.segment_to_device(seg)], interbinning=1)
        p4.twoF_spectrum(0, dev(w.alpha[sk]), dev(w.delta[sk]), fd, spec)
        torch.cuda.synchronize()
        gi = spec.view(len(sk), args.nfdot, nb).cpu().numpy()
        p4.destroy()
    del spec
    errs = []
    ib_err, ib_even, ib_odd_mean, zp_odd_mean = [], [], 0.0, 0.0
    c0 = time.perf_counter()
    for i in sk:
        sky = ora.sky_stage(seg, float(w.alpha[i]), float(w.delta[i]), nfft)
        for s in range(args.nfdot):
            tf = ora.template_two_f(seg, sky, float(w.fdot[s]), nfft)
            np.nonzero(tf > w.threshold)
            errs.append(float(np.max(np.abs(g[i, s] - tf) / np.maximum(tf, 4.0))))
            if gi is not None:
                # outside the timed oracle sample's cost: parity of the interbinned GPU
                # spectrum and the method's deviation from the zero-padded transform
                c_ib = time.perf_counter()
                ti = ora.template_two_f_interbin(seg, sky, float(w.fdot[s]), nfft)
                ib_err.append(float(np.max(np.abs(gi[i, s] - ti) / np.maximum(ti, 4.0))))
                ib_even.append(float(np.max(np.abs(ti[0::2] - tf[0::2]) / np.maximum(tf[0::2], 4.0))))
                ib_odd_mean += float(np.mean(ti[1::2]))
                zp_odd_mean += float(np.mean(tf[1::2]))
                c0 += time.perf_counter() - c_ib
    c1 = time.perf_counter()
    ntpl = len(sk) * args.nfdot
    single = {"value": ntpl / (c1 - c0), "unit": "templates/s", "cores": 1,
              "sample": f"{len(sk)} sky x {args.nfdot} spindown templates of the same workload "
                        f"(numpy FP64, single thread), {c1 - c0:.1f} s"}
    cpu = dict(cpu_mc) if cpu_mc else {}
    cpu["single_core"] = single
    f_err = max(errs)
    log(f"cpu oracle, one core: {single['value']:.3g} templates/s, max F rel err vs FP64 {f_err:.3e}")
    if ib_ok and ib_err:
        ib["f_rel_err_vs_fp64_interbinned"] = max(ib_err)
        ib["even_bins_rel_dev_vs_zero_padded"] = max(ib_even)
        ib["odd_bins_mean_2F_ratio_vs_zero_padded"] = ib_odd_mean / zp_odd_mean
        ib["accuracy_sample"] = f"{len(sk)} sky x {args.nfdot} spindown templates, all bins, FP64 oracle"
        log(f"interbinning: max F rel err vs the FP64 interbinned oracle {max(ib_err):.3e}; oracle even bins vs "
            f"zero-padded {max(ib_even):.2e}; odd-bin mean 2F ratio {ib_odd_mean / zp_odd_mean:.3f}")
    return {"cpu": cpu, "f_err": f_err}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nsky", type=int, default=4096)
    ap.add_argument("--nfdot", type=int, default=256)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-skies", type=int, default=2)
    ap.add_argument("--no-events", action="store_true", help="time without per-launch HIP events")
    ap.add_argument("--templates-per-launch", type=int, default=0)
    ap.add_argument("--skies-per-batch", type=int, default=0)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--autotune-ms", type=float, default=3000.0)
    ap.add_argument("--tuning-cache", default="",
                    help="tuning cache file: reused if it exists, else written by the autotuner")
    ap.add_argument("--no-vetting", action="store_true")
    ap.add_argument("--no-interbinning", action="store_true")
    ap.add_argument("--no-lattice", action="store_true")
    ap.add_argument("--vet-epochs", type=int, default=3)
    ap.add_argument("--side-steps", type=int, default=5,
                    help="timed steps of the interbinning and lattice entries (at most --steps)")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-full-drain", action="store_true",
                    help="skip the timed full drain (ordered copy of every crossing) of one batched search")
    ap.add_argument("--ragged-nsky", type=int, default=1024)
    ap.add_argument("--ragged-nfdot", type=int, default=128)
    ap.add_argument("--ragged-steps", type=int, default=2)
    ap.add_argument("--ragged-budget-gib", type=float, default=4.0,
                    help="workspace budget of the ragged plan (admission shrinks its batch sizes to it)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the search shards by sky "
              "position across GPUs with no exchange in the hot loop, but only the one-GPU path is built.",
              file=sys.stderr)
        sys.exit(2)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    # the oracle on all host cores first, before anything touches the GPU
    cpu_mc = None if args.no_cpu else cpu_multicore_leg(args, log)

    import numpy as np
    import torch

    import synth
    from paper_1410_3677_amd import fstat as F

    torch.cuda.set_device(0)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    if args.copy_calibration_mb:
        # a plain copy kernel moving a known number of bytes: out = x * 1 (reads and writes N*4 B)
        nel = args.copy_calibration_mb * (1 << 20) // 4
        xc = torch.ones(nel, dtype=torch.float32, device="cuda")
        yc = torch.empty_like(xc)
        torch.mul(xc, 1.0, out=yc)
        torch.cuda.synchronize()
        del xc, yc
        log(f"copy calibration: {args.copy_calibration_mb} MiB read and written")

    # ---------------- mixed-precision batched workload
    w = synth.workload("batched", args.nsky, args.nfdot)
    seg = w.segments[0]
    nfft = synth.nfft_for(seg.n)
    al, de, fd = dev(w.alpha), dev(w.delta), dev(w.fdot)
    templates = args.nsky * args.nfdot
    main_leg = timed_search(args, F, torch, seg, al, de, fd, templates, nfft, log, interbinning=0,
                            full_drain=not args.no_full_drain)
    value, ms_step, n_cand = main_leg["value"], main_leg["ms_per_step"], main_leg["n_cand"]
    info, kernels, roofline, tuned = main_leg["info"], main_leg["kernels"], main_leg["roofline"], main_leg["tuning"]
    B, N = info["templates_per_launch"], seg.n

    # ---------------- side entries: each records its failure instead of ending the run
    side = min(args.steps, args.side_steps)
    ib = None
    if not args.no_interbinning:
        # the same workload with interbinning (template transforms of nfft/2 points)
        ib = guarded("interbinning", log, timed_search, args, F, torch, seg, al, de, fd, templates, nfft, log,
                     interbinning=1, steps=side, warmup=min(args.warmup, 1))
    lat_leg = None
    if not args.no_lattice:
        # the same search driven by a lattice grid (sky loop over grid integers)
        lat_leg = guarded("lattice", log, lattice_leg, args, F, torch, seg, nfft, info, log)
    plain = None
    if not args.no_plain:
        plain = guarded("plain", log, plain_leg, args, F, torch, np, dev, log)
    ragged = None
    if not args.no_ragged:
        ragged = guarded("ragged", log, ragged_leg, args, F, torch, np, dev, log)
    cpu, f_err = None, None
    if not args.no_cpu:
        res = guarded("cpu sample", log, cpu_sample_leg, args, F, torch, np, dev, log, w, seg, fd, nfft, ib, cpu_mc)
        if "error" in res:
            cpu = dict(cpu_mc)
            cpu["single_core"] = res
        else:
            cpu, f_err = res["cpu"], res["f_err"]
    vetting = None
    if not args.no_vetting:
        # learned vetting: train on oracle patches, then score the plain search's crossings
        vetting = guarded("vetting", log, vetting_leg, args, F, torch, np, dev, log)

    out = {
        "metric": METRIC, "value": value, "unit": "templates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"mixed-precision batched search, N={N}, nfft=2^{int(math.log2(nfft))}, "
                               f"{args.nsky} sky x {args.nfdot} spindown, 5 injections, 2F>20",
                   "n": N, "nfft": nfft, "nsky": args.nsky, "nfdot": args.nfdot, "templates": templates,
                   "templates_per_launch": B, "skies_per_batch": info["skies_per_batch"],
                   "pass_a_variant": info["pass_a_variant"], "pass_b_variant": info["pass_b_variant"],
                   "tuning": tuned},
        "roofline": roofline, "cpu_baseline": cpu, "plain": plain,
        "f_rel_err_vs_fp64": f_err, "candidates_per_step": n_cand / args.steps, "kernels": kernels,
        # the two template passes' algorithmic bytes (2 nfft x 8 B written and read per
        # template) over the whole step's time, per-sky stage and count drain included
        "achieved_GBs_whole_step": templates * 2 * 2 * nfft * 8 / (ms_step / 1e3) / 1e9,
        "candidate_capacity": main_leg["candidate_capacity"], "full_drain": main_leg["full_drain"],
        "vetting": vetting,
        "interbinning": ib_summary(ib, templates, nfft),
        "lattice": lat_leg,
        "ragged": ragged,
        "context": {"paper_cray_xe6": {
            "value": 1e4 / 1900.0, "unit": "templates/s per core",
            "note": "derived from the paper's weak-scaling test (Sect. 4, weak-scaling figure): one task of 1e4 "
                    "spindown loops took about 1900 s on one Cray XE6 core, FP64 CPU code, N = 344656 samples "
                    "at 0.5 s; a different data length and machine, quoted as context, not as the baseline"}},
        "source_sha256": source_digest(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
