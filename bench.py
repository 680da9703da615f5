#!/usr/bin/env python3
"""Throughput of the Flow Fields search on one MI355X.

A step is one pass of the whole search (luma, pyramid, descriptors, seed
search, every level's init / sweeps / random search, forward-backward check,
both directions) over one batch of KITTI-shaped 1242x375 RGB pairs, issued as
one ff_match_batch call.  Inputs are synthetic (seeded road-scene textures
with planar-expansion motion and translating boxes) and resident in HBM
before the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--batch B]

Prints ONE JSON line.  value = matched pixels per second (W*H*pairs/s, both
fields and the mask computed for every pixel); pairs/s rides along.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

W0, H0, LEVELS = 1242, 375, 4
HBM_PEAK_GBS = 8000.0

# Line-kernel schedule for this workload as picked by ff_autotune on MI355X:
# (chunks per window, lines per block, mode: 0 free-running, 1 staged, 2 lockstep)
# for row levels 0..3, then col
# levels 0..3.  Any schedule gives identical outputs; --autotune re-tunes.
SCHEDULE_C1 = [1, 4, 2, 1, 4, 0, 1, 2, 0, 1, 8, 0, 1, 8, 2, 1, 8, 2, 1, 4, 0, 1, 4, 0]
# The same for the Census cost on the Sintel-shaped batch (used by the
# profiler legs, which do not autotune).
SCHEDULE_CENSUS = [1, 4, 2, 1, 4, 0, 1, 2, 0, 1, 4, 0, 1, 8, 2, 1, 8, 0, 1, 4, 0, 1, 4, 0]

# HBM traffic of the col-phase kernel per launch (average over the 8
# launches of a step), from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE runs of
# this benchmark scaled by the copy calibration (x2.0 fetch, x1.0 write).
# Valid only for the kernel source it was measured on.
TRAFFIC = {"kernel_sha": "fc99365dee475289", "bytes_per_launch": 1689564396}


def kernel_sha(src=None):
    """sha256[:16] of the kernels' code: ff_kernels.hip (or the file `src`)
    with its // comments, trailing blanks and empty lines removed, so that
    editing a comment keeps a measurement taken on the same code and any code
    change retires it."""
    import hashlib
    src = src or os.path.join(ROOT, "paper_1805_03517_amd", "csrc", "ff_kernels.hip")
    code = []
    for line in open(src, encoding="utf-8"):
        line = line.split("//", 1)[0].rstrip()
        if line:
            code.append(line)
    return hashlib.sha256("\n".join(code).encode()).hexdigest()[:16]


def level_dims(w, h, levels):
    out = []
    for _ in range(levels):
        out.append((w, h))
        w, h = w >> 1, h >> 1
    return out


# Algorithmic bytes per pixel per direction per iteration of the two phases:
# every candidate's 16-byte descriptor gather plus one pass over the own
# descriptor (16), state read (8) and state write (8).
#   row phase: LR (1) + RL (1) + random search (5 trials) = 7 gathers
#   col phase: TB (1) + RS (5) + BT (1) + RS (5)          = 12 gathers
ROW_BYTES_PER_PX = 7 * 16 + 32
COL_BYTES_PER_PX = 12 * 16 + 32
INIT_BYTES_PER_PX = 8 + 16 + 16 + 8     # coarse state, own descriptor, candidate, state write


def step_bytes(shapes, levels, iters=2):
    """Algorithmic bytes per kernel of one pass over a batch of pairs, each
    (width, height, channels): what each step of the method must move, every
    candidate gather counted, no cache reuse.  The level init runs inside the
    row phase's first pass of iteration 0, so its bytes are charged there."""
    tot = {k: 0 for k in ("gray", "down2", "desc", "seed_records", "row_phase", "col_phase", "fb")}
    for w, h, c in shapes:
        px = [a * b for a, b in level_dims(w, h, levels)]
        p0, pall, pc = px[0], sum(px), px[-1]
        tot["gray"] += (c + 1) * p0 * 2                          # C B in, 1 B luma out, 2 images
        tot["down2"] += sum(5 * q for q in px[1:]) * 2           # 4 B in, 1 B out per output pixel
        tot["desc"] += 33 * pall * 2                             # 1 B luma in, 2 x 16 B out
        tot["seed_records"] += 80 * pc * 2                       # 16 B in, 64 B record out
        tot["row_phase"] += (iters * ROW_BYTES_PER_PX + INIT_BYTES_PER_PX) * pall * 2
        tot["col_phase"] += iters * COL_BYTES_PER_PX * pall * 2
        tot["fb"] += 25 * p0 * 2                                 # own 8 + other 8 in, 4 + 4 + 1 out
    return tot


def rooflines(prof, per_pass, passes):
    """Each kernel's algorithmic bytes per pass / its device time per pass,
    against the HBM peak."""
    out = {}
    for k, b in per_pass.items():
        if k not in prof:
            continue
        sec = prof[k][1] / 1000.0 / passes
        gbs = b / sec / 1e9
        out[k] = {"bytes_per_step": b, "us_per_step": sec * 1e6, "achieved": gbs, "peak": HBM_PEAK_GBS,
                  "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    return out


def kernel_rooflines(prof, batch, steps):
    """Every kernel of the benchmark step (a batch of 1242x375 RGB pairs)
    against HBM."""
    return rooflines(prof, step_bytes([(W0, H0, 3)] * batch, LEVELS), steps)


def make_inputs(torch, batch, distinct):
    from paper_1805_03517_amd import synth
    base = [synth.config1(seed=1 + k)[:2] for k in range(distinct)]
    pairs = []
    for k in range(batch):
        a, b = base[k % distinct]
        pairs.append((torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()))
    return base, pairs


def cpu_baseline(base, n_pairs, threads):
    """The oracle as it stands, single-threaded, on the first n_pairs pairs;
    then, when threads > 1, one pair per thread on that many host cores at
    once (the oracle's C entry point releases the GIL and keeps no global
    state, so the threads run it side by side unchanged); then, for context,
    two Sintel-shaped 1024x436 pairs single-threaded (eps 7)."""
    import oracle
    oracle.build(force=not os.path.exists(oracle._LIB))
    prm = oracle.params(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED)
    t0 = time.perf_counter()
    for k in range(n_pairs):
        a, b = base[k % len(base)]
        oracle.match(a, b, prm)
    dt = time.perf_counter() - t0
    out = {"value": n_pairs * W0 * H0 / dt, "unit": "px/s", "cores": 1, "kind": "oracle",
           "sample": f"{n_pairs} KITTI-shaped 1242x375 RGB pairs, whole search, one thread",
           "pairs_per_s": n_pairs / dt, "seconds": dt}
    if threads > 1:
        from concurrent.futures import ThreadPoolExecutor
        t0 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda k: oracle.match(base[k % len(base)][0], base[k % len(base)][1], prm), range(threads)))
        dt = time.perf_counter() - t0
        out["all_cores"] = {"value": threads * W0 * H0 / dt, "unit": "px/s", "cores": threads,
                            "sample": f"{threads} pairs, one per thread", "pairs_per_s": threads / dt,
                            "seconds": dt}
    from paper_1805_03517_amd import synth
    prm2 = oracle.params(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=7, seed=0x5EED)
    c2 = [synth.config2(seed=30 + k)[:2] for k in range(2)]
    t0 = time.perf_counter()
    for a, b in c2:
        oracle.match(a, b, prm2)
    dt = time.perf_counter() - t0
    out["sintel_1024x436"] = {"value": 2 * 1024 * 436 / dt, "unit": "px/s", "cores": 1,
                              "sample": "2 Sintel-shaped 1024x436 RGB pairs, whole search, one thread",
                              "pairs_per_s": 2 / dt, "seconds": dt}
    return out


def serve_bench(torch, ff, n_req, lanes, budget):
    """Config 3: a stream of mixed-size requests served (continuous batching
    over `lanes` concurrent cohorts) vs plain (each request in turn through
    ff_match_pair, FIFO).  Arrivals are Poisson at 0.7 x the plain path's
    measured service rate, plus an all-at-once burst.  Latency = completion
    seen by the host - arrival."""
    import numpy as np
    from paper_1805_03517_amd import synth
    reqs, pool = synth.config3_requests(seed=3, n=n_req, per_kind=2)
    dev = {k: (torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for k, (a, b) in pool.items()}
    # the served handle's lanes take the whole budget; the plain baseline
    # runs on a handle of its own under the same budget
    m = ff.Matcher(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED,
                   hbm_budget=budget)
    mp = ff.Matcher(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED,
                    hbm_budget=budget)
    outs = [m._outputs(r["size"][1], r["size"][0], True, True) for r in reqs]
    px = sum(r["size"][0] * r["size"][1] for r in reqs)
    # warm the plain path
    for r, o in list(zip(reqs, outs))[:8]:
        mp.match(*dev[r["pool_key"]], out=o)
    torch.cuda.synchronize()
    m.serve_config(lanes=lanes, lane_bytes=budget // lanes)

    def plain(arr):
        lat = []
        t0 = time.perf_counter()
        for r, o, a in zip(reqs, outs, arr):
            while time.perf_counter() - t0 < a:
                pass
            mp.match(*dev[r["pool_key"]], out=o)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0 - a)
        return lat, time.perf_counter() - t0

    def served(arr):
        lat = [None] * len(reqs)
        t0 = time.perf_counter()
        nxt = 0
        left = len(reqs)
        while left:
            now = time.perf_counter() - t0
            while nxt < len(reqs) and arr[nxt] <= now:
                m.submit(*dev[reqs[nxt]["pool_key"]], tag=nxt, out=outs[nxt])
                nxt += 1
            for t in m.poll():
                lat[t] = time.perf_counter() - t0 - arr[t]
                left -= 1
        return lat, time.perf_counter() - t0

    def summary(lat, span):
        lat = np.asarray(lat) * 1000.0
        return {"pairs_per_s": len(lat) / span, "px_per_s": px / span,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))}

    burst = [0.0] * len(reqs)
    lat, span = plain(burst)
    mu = len(reqs) / span
    rate = 0.7 * mu
    gaps = np.cumsum([r["unit_gap"] for r in reqs])
    arr = list(gaps / rate)
    out = {"requests": len(reqs), "sizes": [list(s) for s in synth.SERVE_SIZES], "lanes": lanes,
           "hbm_budget": budget, "plain_service_rate": mu, "arrival_rate": rate,
           "burst": {"plain": summary(lat, span)}}
    out["burst"]["served"] = summary(*served(burst))
    out["poisson"] = {"plain": summary(*plain(arr)), "served": summary(*served(arr))}
    # near saturation: arrivals at 0.9 x the served burst rate (about 3-4 x
    # what the plain path can serve), served only -- the plain queue would
    # grow without bound
    mu_s = out["burst"]["served"]["pairs_per_s"]
    arr9 = list(gaps / (0.9 * mu_s))
    out["poisson_near_capacity"] = {"arrival_rate": 0.9 * mu_s, "served": summary(*served(arr9))}
    m.close()
    mp.close()
    return out


I8_PEAK_TOPS = 5000.0      # MI355X dense i8 MFMA, 5.0 POP/s


def seed_counts(w, h, levels, stride=3):
    for _ in range(levels - 1):
        w, h = w >> 1, h >> 1
    q = -(-w // stride) * -(-h // stride)
    return q, w * h


def seednn_bench(torch, ff, pair, batch_prof):
    """Seed search on i8 MFMA.  Useful ops = 2*Q*N*16 per direction (multiply
    and add of the 16-deep dot products); the kernel issues 4x that (K = 64
    MFMA holding [a, a, g] . [b, b, beta]).  Reported for the grouped launch of
    the benchmark batch and for a large shape: one full-resolution 1242x375
    level (levels = 1), Q = 51750 seeds x N = 465750 pixels, both directions.
    The tie-resolving pass that follows it (one chunk of 256 entries per seed)
    is reported beside it as resolve_us."""
    q, n = seed_counts(W0, H0, LEVELS)
    launches, ms, nbatch, resolve_us = batch_prof
    per_launch = nbatch * 2 * q * n * 16 * 2
    grouped = {"useful_tops": per_launch / (ms / launches * 1e-3) / 1e12, "avg_us": 1000.0 * ms / launches,
               "resolve_us": resolve_us}
    grouped["issued_tops"] = 4 * grouped["useful_tops"]
    m = ff.Matcher(levels=1, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED)
    a, b = pair
    for _ in range(2):
        m.match(a, b)
    torch.cuda.synchronize()
    m.profile(True)
    for _ in range(3):
        m.match(a, b)
    prof = m.profile_read()
    m.close()
    ql, nl = seed_counts(W0, H0, 1)
    lw, lms = prof["seed_nn"]
    rw, rms = prof["seed_resolve"]
    useful = 2 * ql * nl * 16 * 2 / (lms / lw * 1e-3) / 1e12
    large = {"Q": ql, "N": nl, "avg_us": 1000.0 * lms / lw, "useful_tops": useful, "issued_tops": 4 * useful,
             "resolve_us": 1000.0 * rms / rw}
    for d in (grouped, large):
        d["useful_frac"] = d["useful_tops"] / I8_PEAK_TOPS
        d["issued_frac"] = d["issued_tops"] / I8_PEAK_TOPS
    return {"peak_tops": I8_PEAK_TOPS, "grouped_batch": grouped, "large_shape": large}


def sparse_bench(torch, ff, pairs, steps):
    """3x3-block sparsification (Sec. 3.1, s = 7 for KITTI in Table 3) on the
    benchmark batch: whole-step throughput with it on, and the selection
    kernel against HBM.  Algorithmic bytes per level-0 pixel and direction:
    4 (consistency error read) + 1 (keep byte written); the error plane the
    consistency kernel writes with it (4 B) is charged to that kernel."""
    W, H = W0, H0
    m = ff.Matcher(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED, sparse_min=7)
    m.set_tuning(SCHEDULE_C1)
    outs = [m._outputs(H, W, True, True) for _ in pairs]
    for _ in range(2):
        m.match_batch(pairs, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        m.match_batch(pairs, outs=outs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m.profile(True)
    for _ in range(steps):
        m.match_batch(pairs, outs=outs)
    prof = m.profile_read()
    m.profile(False)
    kept = float(sum(o["sparse_f"].float().mean().item() for o in outs[:8]) / 8)
    m.close()
    n, ms = prof["sparse"]
    avg_s = ms / n / 1000.0
    bytes_launch = 5 * W * H * 2 * len(pairs)
    gbs = bytes_launch / avg_s / 1e9
    # the paper's whole filter: two consistency checks (second search keyed
    # by another seed) followed by the sparsification
    m2 = ff.Matcher(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED, sparse_min=7,
                    seed2=0xBEEF)
    m2.set_tuning(SCHEDULE_C1)
    outs2 = [m2._outputs(H, W, True, True) for _ in pairs]
    for _ in range(2):
        m2.match_batch(pairs, outs=outs2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        m2.match_batch(pairs, outs=outs2)
    torch.cuda.synchronize()
    wall2 = time.perf_counter() - t0
    kept2 = float(sum(o["sparse_f"].float().mean().item() for o in outs2[:8]) / 8)
    m2.close()
    return {"s": 7, "pairs_per_s": len(pairs) * steps / wall, "kept_fraction_fwd": kept,
            "kernel": {"name": "sparse", "avg_us": avg_s * 1e6, "algorithmic_bytes_per_launch": bytes_launch,
                       "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS},
            "two_checks_and_sparsify": {"pairs_per_s": len(pairs) * steps / wall2, "kept_fraction_fwd": kept2}}


CEN_COL_BYTES_PER_PX = 12 * 8 + 32     # 12 Census gathers of 8 B, own strings 2 x 8, state in + out


def subpix_bench(torch, ff, pairs, steps, sub_iters=1, sub_radius=2):
    """Sub-pixel refinement (Sec. 3.1) on the benchmark batch: whole-step
    throughput with it on, and its two line kernels' rate of 16-byte
    descriptor loads.  A quarter-pixel candidate reads B's 2x2 neighbourhood
    (4 loads); with radius R the random search makes J = floor(log2 R) + 1
    trials, so per level-0 pixel, direction and iteration the row phase
    evaluates 2 + J candidates and the column phase 2 + 2J.  Neighbouring
    lanes' 2x2 blocks overlap, so most of these loads hit L1/L2: their bytes
    (64 per candidate) exceed what HBM could deliver, and the load rate, not
    a byte count, is what these kernels are measured by."""
    W, H = W0, H0
    J = sub_radius.bit_length()
    m = ff.Matcher(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED,
                   sub_iters=sub_iters, sub_radius=sub_radius)
    m.set_tuning(SCHEDULE_C1)
    outs = [m._outputs(H, W, True, True) for _ in pairs]
    for _ in range(2):
        m.match_batch(pairs, outs=outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        m.match_batch(pairs, outs=outs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    m.profile(True)
    for _ in range(steps):
        m.match_batch(pairs, outs=outs)
    prof = m.profile_read()
    m.profile(False)
    frac_px = float(sum(((o["flow_f"] & 3) != 0).any(-1).float().mean().item() for o in outs[:8]) / 8)
    consistent = float(sum(o["mask_f"].float().mean().item() for o in outs[:8]) / 8)
    m.close()
    kern = {}
    for k, cands in (("sub_row_phase", 2 + J), ("sub_col_phase", 2 + 2 * J)):
        n, ms = prof[k]
        avg_s = ms / n / 1000.0
        loads = 4 * cands * W * H * 2 * len(pairs)
        # algorithmic bytes: 64 B (the 2x2 neighbourhood) per candidate plus
        # own descriptor and state in and out (32 B) per pixel and direction
        nbytes = (64 * cands + 32) * W * H * 2 * len(pairs)
        kern[k] = {"avg_us": avg_s * 1e6, "candidates_per_px": cands, "loads_per_launch": loads,
                   "g_loads_per_s": loads / avg_s / 1e9, "algorithmic_bytes_per_launch": nbytes,
                   "achieved": nbytes / avg_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": nbytes / avg_s / 1e9 / HBM_PEAK_GBS}
    return {"sub_iters": sub_iters, "sub_radius_quarter_px": sub_radius, "pairs_per_s": len(pairs) * steps / wall,
            "fractional_flow_fraction_fwd": frac_px, "consistent_fraction_fwd": consistent, "kernels": kern}


def census_bench(torch, ff, n_pairs, distinct, steps):
    """Census cost (Sec. 3.1; the paper's Sintel cost, eps = 7 from Table 3)
    on a batch of Sintel-shaped 1024x436 RGB pairs, against the descriptor
    cost on the same batch; each with the schedule ff_autotune picks for it.
    Census col-phase algorithmic bytes per pixel, direction and iteration:
    12 candidate gathers x 8 B + own strings 2 x 8 B + state 8 B in and out."""
    from paper_1805_03517_amd import synth
    W, H = 1024, 436
    base = [synth.config2(seed=30 + k)[:2] for k in range(distinct)]
    pairs = [(torch.from_numpy(base[k % distinct][0]).cuda(), torch.from_numpy(base[k % distinct][1]).cuda())
             for k in range(n_pairs)]
    dims = level_dims(W, H, LEVELS)
    px_all = sum(w * h for w, h in dims)
    out = {"workload": f"{n_pairs} Sintel-shaped {W}x{H} RGB pairs ({distinct} distinct), L = {LEVELS}, eps = 7"}
    for cost in ("census", "wh"):
        m = ff.Matcher(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=7, seed=0x5EED, cost=cost)
        outs = [m._outputs(H, W, True, True) for _ in pairs]
        m.match_batch(pairs, outs=outs)
        tuning = m.autotune(pairs, outs=outs)
        for _ in range(2):
            m.match_batch(pairs, outs=outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            m.match_batch(pairs, outs=outs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        m.profile(True)
        for _ in range(steps):
            m.match_batch(pairs, outs=outs)
        prof = m.profile_read()
        m.profile(False)
        m.close()
        plain = None
        if cost == "wh":
            # the plain path on the same batch: one ff_match_pair per pair
            m2 = ff.Matcher(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=7, seed=0x5EED, cost=cost)
            m2.set_tuning(tuning)
            for (a, b), o in zip(pairs[:4], outs[:4]):
                m2.match(a, b, out=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for (a, b), o in zip(pairs, outs):
                m2.match(a, b, out=o)
            torch.cuda.synchronize()
            dtp = time.perf_counter() - t0
            m2.close()
            plain = {"pairs_per_s": n_pairs / dtp, "px_per_s": n_pairs * W * H / dtp}
        n, ms = prof["col_phase"]
        per_px = CEN_COL_BYTES_PER_PX if cost == "census" else COL_BYTES_PER_PX
        avg_bytes = per_px * px_all * 2 * n_pairs * 2 / (2 * LEVELS)
        avg_s = ms / n / 1000.0
        gbs = avg_bytes / avg_s / 1e9
        out[cost] = {"pairs_per_s": n_pairs * steps / wall, "px_per_s": n_pairs * steps * W * H / wall,
                     "ms_per_step": 1000.0 * wall / steps, "schedule": tuning,
                     "col_phase": {"avg_us": avg_s * 1e6, "algorithmic_bytes_per_launch": avg_bytes,
                                   "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS},
                     "kernels": {k: round(1000.0 * v[1] / max(v[0], 1), 1) for k, v in prof.items()}}
        if plain:
            out[cost]["plain"] = plain
    return out


def c4_bench(torch, ff, n_pairs):
    """Config 4: n uneven gray pairs (sides 96..256, translations up to
    +-24 px, 3 levels) as ONE batched call (replayed hipGraph, tuned schedule)
    vs one ff_match_pair call per pair; outputs compared bit for bit."""
    from paper_1805_03517_amd import synth
    pairs = synth.config4_batch(seed=4, n=n_pairs)
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b, _ in pairs]
    px = sum(a.shape[0] * a.shape[1] for a, _, _ in pairs)
    mb = ff.Matcher(levels=3, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED)
    mp = ff.Matcher(levels=3, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED)
    ob = [mb._outputs(a.shape[0], a.shape[1]) for a, _ in dev]
    op = [mp._outputs(a.shape[0], a.shape[1]) for a, _ in dev]
    for _ in range(2):                          # second call captures the graph
        mb.match_batch(dev, outs=ob)
    tuning = mb.autotune(dev, outs=ob)
    prep = mb.prepare_batch(dev, outs=ob)       # the ff_pair array, marshalled once
    for _ in range(2):
        mb.match_prepared(prep)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        mb.match_prepared(prep)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    # the same with the array rebuilt in Python for every call
    t0 = time.perf_counter()
    for _ in range(reps):
        mb.match_batch(dev, outs=ob)
    torch.cuda.synchronize()
    tb_marshal = (time.perf_counter() - t0) / reps
    # per-kernel device time of the batched call (events around every
    # launch); seed search of the batch on i8 MFMA: one grouped launch
    mb.profile(True)
    for _ in range(reps):
        mb.match_prepared(prep)
    prof = mb.profile_read()
    mb.profile(False)
    shapes = [(a.shape[1], a.shape[0], 1) for a, _, _ in pairs]
    per_call = step_bytes(shapes, 3)
    total_bytes = sum(per_call.values())
    kern = {k: {"launches_per_call": v[0] // reps, "us_per_call": 1000.0 * v[1] / reps} for k, v in prof.items()}
    roof = rooflines(prof, per_call, reps)
    useful = 0
    for a, _, _ in pairs:
        wc, hc = a.shape[1] >> 2, a.shape[0] >> 2              # coarsest of 3 levels
        useful += 2 * (-(-wc // 3)) * (-(-hc // 3)) * wc * hc * 16 * 2
    sn, sms = prof["seed_nn"]
    rn, rms = prof["seed_resolve"]
    seed = {"avg_us": 1000.0 * sms / sn, "resolve_us": 1000.0 * rms / rn,
            "resolve_share": rms / (rms + sms),
            "useful_tops": useful / (sms / sn * 1e-3) / 1e12}
    seed["issued_tops"] = 4 * seed["useful_tops"]
    seed["useful_frac"] = seed["useful_tops"] / I8_PEAK_TOPS
    seed["issued_frac"] = seed["issued_tops"] / I8_PEAK_TOPS
    for (a, b), o in zip(dev, op):              # warm the per-pair path (graphs per shape)
        mp.match(a, b, out=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (a, b), o in zip(dev, op):
        mp.match(a, b, out=o)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    same = all(torch.equal(x[k], y[k]) for x, y in zip(ob, op) for k in x)
    mb.close()
    mp.close()
    kernel_ms = sum(v["us_per_call"] for v in kern.values()) / 1000.0
    return {"pairs": n_pairs, "batched": {"pairs_per_s": n_pairs / tb, "px_per_s": px / tb, "ms": 1000 * tb,
                                          "algorithmic_bytes": total_bytes,
                                          "algorithmic_frac": total_bytes / tb / 1e9 / HBM_PEAK_GBS,
                                          "kernel_ms": kernel_ms,
                                          "ms_marshalling_every_call": 1000 * tb_marshal},
            "per_pair": {"pairs_per_s": n_pairs / tp, "px_per_s": px / tp, "ms": 1000 * tp},
            "bit_identical": bool(same), "schedule": tuning, "seed_nn": seed, "kernels": kern,
            "kernel_rooflines": roof}


def plain_bench(torch, m, pairs, outs, rounds, batched_ms_per_pair):
    """The plain path on the benchmark batch: one ff_match_pair call per pair
    (same handle, schedule and outputs), back to back for throughput, then
    each call synchronised on its own for its latency."""
    import numpy as np
    print("[bench] plain per-pair path", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(rounds):
        for (a, b), o in zip(pairs, outs):
            m.match(a, b, out=o)
    torch.cuda.synchronize()
    dtp = time.perf_counter() - t0
    lat = []
    for (a, b), o in zip(pairs, outs):
        t1 = time.perf_counter()
        m.match(a, b, out=o)
        torch.cuda.synchronize()
        lat.append(1000.0 * (time.perf_counter() - t1))
    n = len(pairs) * rounds
    return {"calls": n, "pairs_per_s": n / dtp, "px_per_s": n * W0 * H0 / dtp,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "batched_ms_per_pair": batched_ms_per_pair}


def profiler_leg(torch, ff, leg, steps):
    """A short fixed-schedule run of one leg, for rocprofv3 runs (`serve`,
    bench.py's serving leg alone, is dispatched in main): `census`
    (64 Sintel-shaped 1024x436 RGB pairs, Census cost, eps 7), `subpix` (the
    64-pair 1242x375 batch with one quarter-pixel refinement iteration) or
    `c4` (the 4096-pair config-4 batch).  Prints one JSON line."""
    from paper_1805_03517_amd import synth
    if leg == "census":
        base = [synth.config2(seed=30 + k)[:2] for k in range(8)]
        pairs = [(torch.from_numpy(base[k % 8][0]).cuda(), torch.from_numpy(base[k % 8][1]).cuda()) for k in range(64)]
        m = ff.Matcher(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=7, seed=0x5EED, cost="census")
        m.set_tuning(SCHEDULE_CENSUS)
    elif leg == "subpix":
        _, pairs = make_inputs(torch, 64, 8)
        m = ff.Matcher(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED, sub_iters=1,
                       sub_radius=2)
        m.set_tuning(SCHEDULE_C1)
    elif leg == "c4":
        pairs = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b, _ in synth.config4_batch(seed=4, n=4096)]
        m = ff.Matcher(levels=3, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED)
    else:
        raise SystemExit(f"unknown leg {leg}")
    prep = m.prepare_batch(pairs)
    for _ in range(2):
        m.match_prepared(prep)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        m.match_prepared(prep)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    m.close()
    print(json.dumps({"leg": leg, "pairs": len(pairs), "ms_per_call": 1000 * dt}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--distinct", type=int, default=8, help="distinct synthetic pairs in a batch")
    ap.add_argument("--cpu-pairs", type=int, default=5)
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads for the all-core oracle run (0: this process's CPUs, at most 16)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-pair ff_match_pair leg")
    ap.add_argument("--autotune", action="store_true", help="re-tune the line-kernel schedule first")
    ap.add_argument("--default-schedule", action="store_true", help="the handle's default schedule")
    ap.add_argument("--schedule", type=str, default="",
                    help="comma-separated line-kernel schedule (6 x levels ints, see ff_tune_set) instead of the tuned one")
    ap.add_argument("--seednn-only", action="store_true",
                    help="only time the seed search at the large shape (for counter runs)")
    ap.add_argument("--c4-pairs", type=int, default=4096, help="config-4 batch size (0 skips it)")
    ap.add_argument("--leg", choices=["census", "subpix", "c4", "serve"],
                    help="only a short fixed-schedule run of that leg (for profiler runs)")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-census", action="store_true", help="skip the Census-cost leg")
    ap.add_argument("--core", action="store_true",
                    help="only the timed steps and their per-kernel timing (for profiler runs): no seed-search "
                         "shape, sparsification, sub-pixel, Census, serving, config-4 or CPU legs")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (5 times), the reference "
                         "for scaling FETCH_SIZE / WRITE_SIZE counters, then exit")
    args = ap.parse_args()
    if args.copy_calib:
        import torch
        n = args.copy_calib << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": n, "copies": 5}), flush=True)
        return
    if args.seednn_only:
        import torch
        from paper_1805_03517_amd import ff, synth
        a, b = synth.config1(seed=1)[:2]
        pair = (torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
        print(json.dumps(seednn_bench(torch, ff, pair, (1, 1.0, 0, 0.0))["large_shape"]), flush=True)
        return
    if args.leg:
        import torch
        from paper_1805_03517_amd import ff
        if args.leg == "serve":
            print(json.dumps(serve_bench(torch, ff, args.serve_requests, lanes=4, budget=64 << 30)), flush=True)
        else:
            profiler_leg(torch, ff, args.leg, max(1, args.steps))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); pairs are independent and a "
              "multi-GPU run would shard them across processes, which is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1805_03517_amd import ff

    print(f"[bench] generating {args.distinct} distinct 1242x375 pairs, batch {args.batch}", file=sys.stderr,
          flush=True)
    base, pairs = make_inputs(torch, args.batch, args.distinct)
    m = ff.Matcher(levels=LEVELS, seed_stride=3, iters=2, rs_radius=16, fb_eps=1, seed=0x5EED)
    outs = [m._outputs(H0, W0, True, True) for _ in range(args.batch)]
    stream = torch.cuda.current_stream()

    print("[bench] warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        m.match_batch(pairs, outs=outs)
    torch.cuda.synchronize()
    if args.autotune:
        print("[bench] autotuning the line-kernel schedule on this batch", file=sys.stderr, flush=True)
        m.autotune(pairs, outs=outs)
    elif args.schedule:
        m.set_tuning([int(v) for v in args.schedule.split(",")])
    elif not args.default_schedule:
        m.set_tuning(SCHEDULE_C1)
    tuning = m.tuning()
    for _ in range(2):
        m.match_batch(pairs, outs=outs)
    torch.cuda.synchronize()

    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    prep = m.prepare_batch(pairs, outs=outs)    # the ff_pair array, marshalled once
    m.match_prepared(prep)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        m.match_prepared(prep)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = 1000.0 * wall / args.steps
    pairs_per_s = args.batch * args.steps / wall
    px_per_s = pairs_per_s * W0 * H0
    consistent = float(sum(o["mask_f"].float().mean().item() for o in outs[: args.distinct]) / args.distinct)

    # Per-kernel device time over the same number of steps, events around every launch.
    print("[bench] per-kernel timing", file=sys.stderr, flush=True)
    m.profile(True)
    for _ in range(args.steps):
        m.match_prepared(prep)
    prof = m.profile_read()
    m.profile(False)
    dims = level_dims(W0, H0, LEVELS)
    px_all_levels = sum(w * h for w, h in dims)
    col_launches, col_ms = prof.get("col_phase", (0, 0.0))
    # every col-phase launch covers one level, both directions, all pairs
    col_bytes_per_step = COL_BYTES_PER_PX * px_all_levels * 2 * args.batch * 2     # x2 iterations
    col_launches_per_step = LEVELS * 2
    avg_bytes = col_bytes_per_step / col_launches_per_step
    avg_s = (col_ms / max(col_launches, 1)) / 1000.0
    achieved = avg_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    kernels = {k: {"launches": v[0], "avg_us": 1000.0 * v[1] / max(v[0], 1),
                   "share": v[1] / max(sum(x[1] for x in prof.values()), 1e-9)} for k, v in prof.items()}

    if args.core:
        args.no_serve = args.no_census = args.no_cpu = True
        args.c4_pairs = 0
    seednn = None
    if not args.core:
        print("[bench] seed search MFMA utilisation", file=sys.stderr, flush=True)
        sl, sms = prof.get("seed_nn", (1, 0.0))
        rl, rms = prof.get("seed_resolve", (1, 0.0))
        seednn = seednn_bench(torch, ff, pairs[0], (sl, sms, args.batch, 1000.0 * rms / rl))

    plain = None
    if not args.no_plain and not args.core:
        plain = plain_bench(torch, m, pairs, outs, max(1, args.steps // 4), ms_per_step / args.batch)

    sparse = None
    if not args.core:
        print("[bench] sparsification leg", file=sys.stderr, flush=True)
        sparse = sparse_bench(torch, ff, pairs, max(2, args.steps // 4))

    subpix = None
    if not args.core:
        print("[bench] sub-pixel refinement leg", file=sys.stderr, flush=True)
        subpix = subpix_bench(torch, ff, pairs, max(2, args.steps // 4))

    census = None
    if not args.no_census:
        print("[bench] Census-cost leg (Sintel-shaped batch)", file=sys.stderr, flush=True)
        census = census_bench(torch, ff, args.batch, args.distinct, max(2, args.steps // 4))

    serving = None
    if not args.no_serve:
        print(f"[bench] serving: {args.serve_requests} mixed requests, served vs plain", file=sys.stderr, flush=True)
        serving = serve_bench(torch, ff, args.serve_requests, lanes=4, budget=64 << 30)

    batch_c4 = None
    if args.c4_pairs:
        print(f"[bench] config 4: {args.c4_pairs} uneven gray pairs, batched vs per-pair", file=sys.stderr,
              flush=True)
        batch_c4 = c4_bench(torch, ff, args.c4_pairs)

    cpu = None
    if not args.no_cpu:
        print(f"[bench] oracle on {args.cpu_pairs} pairs (cpu baseline)", file=sys.stderr, flush=True)
        threads = args.cpu_threads or min(16, len(os.sched_getaffinity(0)))
        cpu = cpu_baseline(base, args.cpu_pairs, threads)

    line = {
        "metric": "matched px/s & pairs/s (fwd+bwd) at 1242x375; p50/p99 latency served vs plain",
        "value": px_per_s,
        "unit": "px/s",
        "pairs_per_s": pairs_per_s,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "gpu_ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "KITTI-shaped 1242x375 RGB pairs (planar expansion up to 150 px, 4 boxes), "
                               f"4 levels, stride 3, 2 iterations, R 16, eps 1; {args.batch} pairs per "
                               f"step ({args.distinct} distinct)",
                   "global_batch": args.batch, "parallelism": "none (1 GPU)", "schedule": tuning,
                   "consistent_fraction": consistent},
        "consistent_px_per_s": px_per_s * consistent,
        "roofline": {"bound": "hbm", "kernel": "col_phase", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (TRAFFIC["bytes_per_launch"]
                                 if TRAFFIC["kernel_sha"] == kernel_sha() and tuning == SCHEDULE_C1 else None),
                     "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": avg_bytes},
        "kernels": kernels,
        "kernel_rooflines": kernel_rooflines(prof, args.batch, args.steps),
        "plain": plain,
        "seed_nn": seednn,
        "sparsify": sparse,
        "subpixel": subpix,
        "census": census,
        "serving": serving,
        "batch_c4": batch_c4,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    m.close()


if __name__ == "__main__":
    main()
