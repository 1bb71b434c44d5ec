#!/usr/bin/env python3
"""Benchmark: ACBM motion estimation on one MI355X.

Workload (the paper's method at HD size): a 60-frame 1920x1088 u8 luma
sequence from the seeded moving-scene generator (panned blurred-noise
background, 16 textured rectangles with velocities up to +-24 px/frame,
sigma = 2 noise), 16x16 blocks, p = 32, lambda = Qp = 8, the paper's
alpha = 1000, beta = 8, gamma = 1/4.  The 59 frame pairs are resident in HBM
before timing starts.

One step = the whole hot path over the sequence: full search (FSBM: SAD
window search + J argmin) for all 59 pairs, then ACBM (Intra_SAD, PBM,
the two tests, critical full searches) for all 59 pairs with the temporal
field carried from pair to pair.

value = algorithmic candidate-pixel SAD evaluations per second of the step:
one evaluation is one |cur - ref| accumulated for one pixel of one valid
candidate; FSBM counts #valid * N*M per block and ACBM counts its returned
`cands` * N*M per block.  Out-of-frame lanes the kernels compute and mask are
not counted.

The roofline object covers the dominant kernel (the window search): its
algorithmic evaluations per launch divided by its mean launch time, measured
with HIP events on its own stream, against the packed-SAD VALU peak.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

METRIC = "candidate-pixel SAD evals/s + 1080p p=32 frames/s (FSBM vs ACBM), % VALU peak"
# 256 CUs x 64 lanes x 2.4 GHz x 4 absolute differences per lane-clock:
# V_SAD_U8 (4 per op, full rate) and V_QSAD_PK_U16_U8 (16 per op, quarter
# rate) reach the same byte rate.
PEAK_TEVALS = 256 * 64 * 2.4e9 * 4 / 1e12


# HBM bytes per launch of the FSBM window search on the 1920x1088 p = 32
# sequence (59 pairs), from two rocprofv3 --pmc runs of
# `bench.py --steps 1 --warmup 0 --no-cpu --only fsbm --calib-copy-mib 256`:
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of k_search<16,16,6,false>,
# each scaled by what the same counter reads for the 256 MiB device copy in
# that run (FETCH_SIZE reads 131091.3 KiB for 262144 KiB moved, WRITE_SIZE
# 262144 KiB).  Valid for the kernel these counters were taken on; set to
# None when the search kernel changes.
SEARCH_TRAFFIC = {"kernel": "k_search<16,16,6,false>", "fetch_kib": 147165.6,
                  "write_kib": 15802.1, "fetch_scale": 262144.0 / 131091.3, "write_scale": 1.0}


def search_traffic_bytes():
    t = SEARCH_TRAFFIC
    if t is None:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=60)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", choices=["fsbm", "acbm", "halfpel", "batch", "serve"], default=None,
                    help="run only one leg (profiling runs)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 64-sequence leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-requests leg")
    ap.add_argument("--serve-seconds", type=float, default=1.5,
                    help="duration of each arrival rate of the served leg")
    ap.add_argument("--serve-lanes", type=int, default=4,
                    help="passes the server keeps in flight (HIP streams)")
    ap.add_argument("--walker-phases", action="store_true",
                    help="report the row walkers' per-phase times (needs the profiling build: "
                         "ACBM_LIB=paper_0710_4819_amd/libacbm_phases.so, built by "
                         "`python -m paper_0710_4819_amd.build --phases`)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB, so that "
                         "hardware byte counters can be scaled against a known transfer")
    return ap.parse_args()


def log(msg):
    """Progress of the run, on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    """The host the oracle is timed on: CPU model, cores, compiler and flags."""
    import subprocess
    from oracle import build as oracle_build
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    cc = os.environ.get("CC", "gcc")
    try:
        ver = subprocess.run([cc, "--version"], capture_output=True, text=True,
                             timeout=30).stdout.splitlines()[0]
    except (OSError, IndexError, subprocess.SubprocessError):
        ver = cc
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable,
            "compiler": ver, "flags": " ".join(oracle_build.CFLAGS)}


def cpu_baseline(wl, prm_oracle):
    """The plain C oracle (one thread) on a bounded sample: FSBM and ACBM of
    the first frame pair of the same sequence.  Returns the timing record and
    the two oracle result arrays."""
    import oracle
    cur, ref = wl.frames[1], wl.frames[0]
    t0 = time.perf_counter()
    f = oracle.fsbm_frame(cur, ref, 16, 16, 32, prm_oracle)
    a = oracle.acbm_frame(cur, ref, 16, 16, 32, prm_oracle)
    dt = time.perf_counter() - t0
    evals = (int(f["cands"].astype(np.int64).sum()) + int(a["cands"].astype(np.int64).sum())) * 256
    return ({"value": evals / dt, "unit": "candidate-pixel SAD evals/s", "cores": 1,
             "kind": "oracle",
             "sample": "FSBM + ACBM of pair 1 of the 1920x1088 p=32 sequence, single thread, "
                       f"{dt:.1f} s, {evals / 1e9:.2f} G evals",
             "seconds": round(dt, 2)}, f, a)


def cpu_baseline_parallel(wl, prm_oracle, threads=16):
    """The same oracle, unchanged, on several frame pairs at once: one pair
    per thread (ctypes releases the interpreter lock around each C call), as
    many threads as the host's share of cores allows, at most 16.  Returns the
    timing record and the oracle's FSBM result of every pair it ran."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    n = max(1, min(threads, os.cpu_count() or 1, len(wl.frames) - 1))

    def one(t):
        cur, ref = wl.frames[t], wl.frames[t - 1]
        f = oracle.fsbm_frame(cur, ref, 16, 16, 32, prm_oracle)
        a = oracle.acbm_frame(cur, ref, 16, 16, 32, prm_oracle)
        return f, (int(f["cands"].astype(np.int64).sum()) + int(a["cands"].astype(np.int64).sum())) * 256

    oracle.se_bits(0)  # load the library before the threads start
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=n) as ex:
        outs = list(ex.map(one, range(1, n + 1)))
    dt = time.perf_counter() - t0
    evals = sum(e for _, e in outs)
    return ({"value": evals / dt, "unit": "candidate-pixel SAD evals/s", "cores": n,
             "kind": "oracle",
             "sample": f"FSBM + ACBM of pairs 1..{n} of the 1920x1088 p=32 sequence, one pair per "
                       f"thread, {dt:.1f} s, {evals / 1e9:.2f} G evals",
             "seconds": round(dt, 2)}, [f for f, _ in outs])


RESULT_FIELDS = ("mv_x", "mv_y", "sad", "j", "rate_bits", "cands", "mode", "intra_x")


def count_mismatches(got, want):
    """Blocks of one frame pair where any result field differs."""
    bad = np.zeros(want.shape, dtype=bool)
    for f in RESULT_FIELDS:
        bad |= got[f].astype(np.int64) != want[f].astype(np.int64)
    return int(bad.sum())


def probe_peak():
    """Runs the SAD-instruction probe (probe/probe_sad, built by
    probe/build.py) when it is there, and returns its issue costs, byte-diff
    rates and measured shader clock: the evidence behind the peak."""
    import re
    import subprocess
    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "probe", "probe_sad")
    if not os.path.exists(exe):
        return None
    try:
        txt = subprocess.run([exe], capture_output=True, text=True, timeout=120).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    out = {"source": "probe/probe_sad"}
    m = re.search(r"issue cost relative to a full-rate op: sad_u8 ([0-9.]+), qsad ([0-9.]+)", txt)
    if m:
        out["issue_cost_sad_u8"], out["issue_cost_qsad"] = float(m.group(1)), float(m.group(2))
    for op in ("v_sad_u8", "v_qsad_pk_u16_u8"):
        m = re.search(op + r"\s+[0-9.]+ ms\s+[0-9.]+ T lane-ops/s\s+([0-9.]+) T byte-diffs/s", txt)
        if m:
            out[op + "_T_byte_diffs_per_s"] = float(m.group(1))
    m = re.search(r"min ([0-9.]+), median ([0-9.]+), max ([0-9.]+) MHz", txt)
    if m:
        out["clock_mhz"] = {"min": float(m.group(1)), "median": float(m.group(2)),
                            "max": float(m.group(3))}
    return out


def batched_leg(torch, acbm, synth, dev, reps=5):
    """64 sequences x 8 frames of mixed resolution, p and block size: the
    graph-recorded FSBM batch against the eager batch call and against one
    acbm_fsbm_frame call per frame pair, and the same sequences as one
    graph-recorded ACBM batch, all launched on one stream (the library forks
    its walker launches onto side streams and joins them back), inputs resident."""
    seqs = [synth.batch_sequence(s) for s in range(64)]
    # tune each (block size, p) on the largest frame that uses it
    largest = {}
    for w in seqs:
        key = (w.block_w, w.block_h, w.p)
        if key not in largest or w.width * w.height > largest[key][0] * largest[key][1]:
            largest[key] = (w.width, w.height)
    tuned = {}
    for key, (wd, ht) in sorted(largest.items()):
        R, ms = acbm.autotune(key[0], key[1], key[2], wd, ht)
        tuned[key] = {"R": R, "ms_per_pair": ms, "tuned_on": f"{wd}x{ht}"}
    st = torch.cuda.Stream(device=dev)
    b = acbm.Batch(dev)
    dframes, prms = [], []
    for w in seqs:
        fr = [torch.from_numpy(f).to(dev) for f in w.frames]
        prm = acbm.default_params(w.block_w, w.block_h, w.lam)
        b.add(fr, w.block_w, w.block_h, w.p, prm, acbm.ALGO_FSBM)
        dframes.append(fr)
        prms.append(prm)
    ws = torch.empty(max(256, b.workspace_size()), dtype=torch.uint8, device=dev)
    gr = acbm.BatchGraph(b, ws)
    # one workspace and result buffer per sequence for the per-frame calls
    pf_ws = [acbm.workspace(acbm.OP_FSBM, acbm.geom(fr[0], w.block_w, w.block_h, w.p), dev)
             for w, fr in zip(seqs, dframes)]
    torch.cuda.synchronize()

    def per_frame():
        outs = []
        for w, fr, prm, wsb in zip(seqs, dframes, prms, pf_ws):
            for t in range(1, len(fr)):
                outs.append(acbm.fsbm_frame(fr[t], fr[t - 1], w.block_w, w.block_h, w.p, prm,
                                            ws=wsb, stream=st))
        return outs

    def timed(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(st):
            fn()  # warm-up
            e0.record(st)
            t0 = time.perf_counter()
            for _ in range(n):
                fn()
            e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n, (time.perf_counter() - t0) * 1e3 / n

    g_ms, g_wall = timed(lambda: gr.launch(st), reps)
    res = [acbm.to_numpy(o) for o in b.outs]
    e_ms, e_wall = timed(lambda: b.run(ws, st), reps)
    pf_out = per_frame()
    torch.cuda.synchronize()
    k = 0
    for i, w in enumerate(seqs):  # per-frame results are the batch's, bit for bit
        for t in range(len(w.frames) - 1):
            assert np.array_equal(acbm.to_numpy(pf_out[k]), res[i][t]), (i, t)
            k += 1
    p_ms, p_wall = timed(per_frame, 2)
    evals = sum(int(r["cands"].astype(np.int64).sum()) * w.block_w * w.block_h
                for r, w in zip(res, seqs))
    gr.close()
    # the same sequences with ACBM: one row-walker launch per block size
    ba = acbm.Batch(dev)
    for w, fr, prm in zip(seqs, dframes, prms):
        ba.add(fr, w.block_w, w.block_h, w.p, prm, acbm.ALGO_ACBM)
    ws_a = torch.empty(max(256, ba.workspace_size()), dtype=torch.uint8, device=dev)
    gra = acbm.BatchGraph(ba, ws_a)
    a_ms, _ = timed(lambda: gra.launch(st), reps)
    assert ba.status(ws_a, st) == 0, "batched ACBM dependency wait timed out"
    res_a = [acbm.to_numpy(o) for o in ba.outs]
    gra.close()
    evals_a = sum(int(r["cands"].astype(np.int64).sum()) * w.block_w * w.block_h
                  for r, w in zip(res_a, seqs))
    crit_a = float(np.mean(np.concatenate([(r["mode"] == 3).ravel() for r in res_a])))
    return {"workload": "64 sequences x 8 frames: QCIF/CIF/1280x720/1920x1088, p 7/16/32, "
                        "16x16 and 8x8 blocks, lambda 8, FSBM",
            "pairs": sum(len(w.frames) - 1 for w in seqs), "evals": evals,
            "graph_ms": g_ms, "graph_evals_per_s": evals / (g_ms / 1e3),
            "graph_frac_of_peak": evals / (g_ms / 1e3) / (PEAK_TEVALS * 1e12),
            "eager_batch_ms": e_ms, "per_frame_fsbm_ms": p_ms,
            "per_frame_fsbm_wall_ms": p_wall,
            "speedup_graph_vs_per_frame": p_ms / g_ms,
            "acbm_graph_ms": a_ms, "acbm_evals": evals_a, "acbm_critical_frac": crit_a,
            "acbm_graph_speed_vs_fsbm_graph": g_ms / a_ms,
            "acbm_graph_speed_vs_per_frame_fsbm": p_ms / a_ms,
            "tuned_rows": {f"{k[0]}x{k[1]}_p{k[2]}": v for k, v in tuned.items()}}


def halfpel_leg(torch, acbm, frames, prm, stream, steps):
    """FSBM and ACBM with half-pel precision on the same sequence (Table 1
    counts the 8 half-pel positions of the full search): device time per
    step and per kernel, candidates per block."""
    import dataclasses
    hp = dataclasses.replace(prm, subpel=1)
    dev = frames[0].device
    out = {}
    for name, algo in (("fsbm", acbm.ALGO_FSBM), ("acbm", acbm.ALGO_ACBM)):
        b = acbm.Batch(dev)
        res = b.add(frames, 16, 16, 32, hp, algo)
        ws = torch.empty(max(256, b.workspace_size()), dtype=torch.uint8, device=dev)
        b.run(ws, stream)  # warm-up
        torch.cuda.synchronize()
        acbm.profile_enable(True)
        acbm.profile_reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            b.run(ws, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        kern = {}
        for k in ("search", "half", "resolve", "predictive"):
            ms, n = acbm.profile_read(k)
            if n:
                kern[k + "_ms_per_launch"] = ms / n
        acbm.profile_enable(False)
        if algo == acbm.ALGO_ACBM:
            assert b.status(ws, stream) == 0, "half-pel ACBM dependency wait timed out"
        r = acbm.to_numpy(res)
        ms = e0.elapsed_time(e1) / steps
        npairs = len(frames) - 1
        out[name] = {"ms": ms, "frames_per_s": npairs / (ms / 1e3),
                     "cands_per_block": float(r["cands"].mean()),
                     "evals": int(r["cands"].astype(np.int64).sum()) * 256, **kern}
        if algo == acbm.ALGO_ACBM:
            out[name]["critical_frac"] = float((r["mode"] == acbm.MODE_CRITICAL).mean())
    out["acbm"]["speedup_vs_fsbm"] = out["fsbm"]["ms"] / out["acbm"]["ms"]
    return out


def latency_leg(torch, acbm, frames, prm, stream, reps=5):
    """Device time of one frame pair alone (frames 30 and 31 of the sequence,
    temporal field zero): the latency a single pair sees, which for ACBM is
    its block-dependency path rather than throughput."""
    out = {}
    pair = frames[30:32]
    for name, algo in (("fsbm", acbm.ALGO_FSBM), ("acbm", acbm.ALGO_ACBM)):
        b = acbm.Batch(frames[0].device)
        b.add(pair, 16, 16, 32, prm, algo)
        ws = torch.empty(max(256, b.workspace_size()), dtype=torch.uint8, device=frames[0].device)
        b.run(ws, stream)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.run(ws, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        out[name + "_pair_ms"] = float(np.median(ts))
    return out


def served_leg(torch, acbm, synth, rates, seconds, algo_names=("fsbm", "acbm"), nstreams=32,
               nfr=3, sat_requests=3000, lanes=4):
    """Poisson arrivals of frame-pair requests over 32 streams whose
    resolution (640x480 .. 3840x2160) and p (16, 32, 64) are drawn per stream;
    each stream cycles over nfr generated frames.  The server gathers the
    requests into passes (continuous batching) on 4 lanes.  Latency is submit
    -> result on the host (it includes the frame upload and the result
    download).  Per algorithm: each offered rate, then saturation (every
    request submitted at once).  The same request mix run as plain
    acbm_fsbm_frame calls, one after another on one stream with the frames
    already on the device, gives the per-frame FSBM rate the served rates are
    compared with."""
    specs = synth.serve_streams(nstreams)
    frames = [synth.stream_frames(sp, nfr) for sp in specs]
    prm = acbm.default_params(16, 16, 8)
    out = {"workload": f"{nstreams} streams, 640x480..3840x2160, p 16/32/64, 16x16 blocks, "
                       "lambda 8, Poisson arrivals", "lanes": lanes, "max_inflight": 64}
    algos = {"fsbm": acbm.ALGO_FSBM, "acbm": acbm.ALGO_ACBM, "pbm": acbm.ALGO_PBM}

    def one_rate(algo, rate, n, nthreads=4):
        """Submitting threads: thread i owns the streams s % nthreads == i and
        submits their arrivals in time order (the copy into the server's
        staging runs outside the interpreter lock, so the threads copy in
        parallel)."""
        import threading
        times, sids = synth.serve_arrivals(rate if rate else 1e9, n, nstreams)
        srv = acbm.Server(pool_bytes=24 << 30, max_streams=nstreams, max_inflight=64,
                          queue_depth=16384, lanes=lanes, pinned_bytes=2 << 30)
        try:
            first = [srv.submit(s, frames[s][0], 16, 16, specs[s]["p"], prm, algo)
                     for s in range(nstreams)]
            for t in first:
                srv.wait(t)
            base = srv.stats()
            tickets = [[] for _ in range(nthreads)]
            busy = [0] * nthreads
            errors = []

            def submitter(i, t0):
                nxt = {}
                try:
                    for k in range(n):
                        s = int(sids[k])
                        if s % nthreads != i:
                            continue
                        if rate:
                            target = t0 + float(times[k])
                            while True:
                                now = time.perf_counter()
                                if now >= target:
                                    break
                                time.sleep(min(0.0005, target - now))
                        j = nxt.get(s, 1)
                        try:
                            tickets[i].append(srv.submit(s, frames[s][j % nfr], 16, 16,
                                                         specs[s]["p"], prm, algo))
                            nxt[s] = j + 1
                        except acbm.AcbmError as e:
                            if e.status != acbm.E_BUSY:
                                raise
                            busy[i] += 1
                except Exception as e:  # reported by the main thread
                    errors.append(e)

            t0 = time.perf_counter()
            th = [threading.Thread(target=submitter, args=(i, t0)) for i in range(nthreads)]
            for x in th:
                x.start()
            for x in th:
                x.join()
            if errors:
                raise errors[0]
            evals = 0
            for tl in tickets:
                for t in tl:
                    r = srv.wait(t)
                    evals += int(r["cands"].astype(np.int64).sum()) * 256
            t1 = time.perf_counter()
            stt = srv.stats()
            tickets = [t for tl in tickets for t in tl]
            busy = sum(busy)
        finally:
            srv.close()
        done = int(stt["completed"] - base["completed"])
        return {"offered_rps": rate if rate else "saturation", "requests": n, "completed": done,
                "rejected_busy": busy, "achieved_rps": len(tickets) / (t1 - t0),
                "evals_per_s": evals / (t1 - t0),
                "p50_ms": stt["p50_us"] / 1e3, "p99_ms": stt["p99_us"] / 1e3,
                "mean_ms": stt["mean_us"] / 1e3,
                "device_busy_frac": stt["device_busy_frac"],
                "passes": int(stt["passes"] - base["passes"]),
                "mean_batch": (done / max(1, stt["passes"] - base["passes"]))}

    for name in algo_names:
        algo = algos[name]
        res = {"rates": {}}
        for rate in rates:
            res["rates"][str(rate)] = one_rate(algo, rate, max(1, int(rate * seconds)))
            log(f"served {name} at {rate} req/s: {res['rates'][str(rate)]['achieved_rps']:.0f} req/s")
        res["saturation"] = one_rate(algo, 0, sat_requests)
        log(f"served {name} saturated: {res['saturation']['achieved_rps']:.0f} req/s")
        out[name] = res
    # the same mix as plain per-frame FSBM calls, frames resident, one stream
    dev = torch.device("cuda", 0)
    dfr = [[torch.from_numpy(f).to(dev) for f in fr] for fr in frames]
    wss = [acbm.workspace(acbm.OP_FSBM, acbm.geom(dfr[s][0], 16, 16, specs[s]["p"]), dev)
           for s in range(nstreams)]
    _, sids = synth.serve_arrivals(1000.0, 400, nstreams)
    st = torch.cuda.Stream(device=dev)
    outs = [torch.empty((f[0].shape[0] // 16, f[0].shape[1] // 16, 32), dtype=torch.uint8,
                        device=dev) for f in dfr]

    def per_frame(k0, k1):
        for k in range(k0, k1):
            s = int(sids[k])
            acbm.fsbm_frame(dfr[s][1 + k % (nfr - 1)], dfr[s][k % (nfr - 1)], 16, 16,
                            specs[s]["p"], prm, ws=wss[s], stream=st)

    with torch.cuda.stream(st):
        per_frame(0, 32)  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        per_frame(0, len(sids))
        e1.record(st)
    torch.cuda.synchronize()
    pf_rps = len(sids) / (e0.elapsed_time(e1) / 1e3)
    out["per_frame_fsbm_rps"] = pf_rps
    out["per_frame_fsbm_note"] = ("400 requests of the same mix through acbm_fsbm_frame, one "
                                  "after another on one stream, frames already on the device")
    for name in algo_names:
        out[name]["saturation_vs_per_frame_fsbm"] = out[name]["saturation"]["achieved_rps"] / pf_rps
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0710_4819_amd import acbm, synth

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    wl = synth.hd_scene(nframes=args.frames, lam=8)
    frames = [torch.from_numpy(f).to(dev) for f in wl.frames]
    prm = acbm.default_params(16, 16, 8)
    npairs = len(frames) - 1
    stream = torch.cuda.Stream(device=dev)
    if args.calib_copy_mib:
        n = args.calib_copy_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    fs = acbm.Batch(dev)
    fs_out = fs.add(frames, 16, 16, 32, prm, acbm.ALGO_FSBM)
    ac = acbm.Batch(dev)
    ac_out = ac.add(frames, 16, 16, 32, prm, acbm.ALGO_ACBM)
    ws_f = torch.empty(fs.workspace_size(), dtype=torch.uint8, device=dev)
    ws_a = torch.empty(max(256, ac.workspace_size()), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    do_f = args.only in (None, "fsbm")
    do_a = args.only in (None, "acbm")
    if args.only in ("halfpel", "batch", "serve"):
        do_f = do_a = False

    def step(evs=None):
        if evs:
            evs[0].record(stream)
        if do_f:
            fs.run(ws_f, stream)
        if evs:
            evs[1].record(stream)
        if do_a:
            ac.run(ws_a, stream)
        if evs:
            evs[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if do_a:
        assert ac.status(ws_a, stream) == 0, "ACBM dependency wait timed out"

    if args.walker_phases and acbm.phase_profile_read(reset=True) is None:
        print("--walker-phases needs the phase-profiling build (ACBM_LIB)", file=sys.stderr)
        sys.exit(2)
    acbm.profile_enable(True)
    acbm.profile_reset()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    search_ms, search_n = acbm.profile_read("search")
    resolve_ms, resolve_n = acbm.profile_read("resolve")
    pred_ms, pred_n = acbm.profile_read("predictive")
    acbm.profile_enable(False)

    ms_step = wall * 1e3 / args.steps
    ms_f = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    ms_a = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))

    res_f = acbm.to_numpy(fs_out) if do_f else None
    res_a = acbm.to_numpy(ac_out) if do_a else None
    nm = 256
    ev_f = int(res_f["cands"].astype(np.int64).sum()) * nm if do_f else 0
    ev_a = int(res_a["cands"].astype(np.int64).sum()) * nm if do_a else 0
    out = {
        "metric": METRIC,
        "value": (ev_f + ev_a) / (ms_step / 1e3),
        "unit": "candidate-pixel SAD evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"hd_scene_1920x1088_{args.frames}f_16x16_p32_lambda8", "frames": args.frames,
                   "pairs": npairs, "block": "16x16", "p": 32, "lambda": 8, "qp": 8,
                   "alpha": prm.alpha, "beta": prm.beta, "gamma": "1/4", "timed": args.only or "fsbm+acbm"},
    }
    if do_f:
        out["fsbm"] = {"ms": ms_f, "frames_per_s": npairs / (ms_f / 1e3), "evals": ev_f,
                       "evals_per_s": ev_f / (ms_f / 1e3),
                       "search_ms_per_launch": search_ms / max(1, search_n),
                       "resolve_ms_per_launch": resolve_ms / max(1, resolve_n)}
    if do_a:
        modes = np.bincount(res_a["mode"].ravel(), minlength=5)
        out["acbm"] = {"ms": ms_a, "frames_per_s": npairs / (ms_a / 1e3), "evals": ev_a,
                       "evals_per_s": ev_a / (ms_a / 1e3),
                       "cands_per_block": float(res_a["cands"].mean()),
                       "critical_frac": float(modes[3] / modes.sum()),
                       "mode_counts": {"c1": int(modes[1]), "c2": int(modes[2]), "critical": int(modes[3])},
                       "predictive_ms_per_launch": pred_ms / max(1, pred_n),
                       "speedup_vs_fsbm": (ms_f / ms_a) if do_f else None}
    if do_f and search_n:
        per_launch = ev_f / (search_n / args.steps)  # one search launch covers all 59 pairs
        achieved = per_launch / (search_ms / search_n / 1e3) / 1e12
        traffic = search_traffic_bytes()
        out["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_TEVALS,
                           "unit": "T evals/s", "frac": achieved / PEAK_TEVALS, "traffic": traffic,
                           "traffic_unit": "HBM bytes per launch",
                           "traffic_GBps": (traffic / (search_ms / search_n / 1e3) / 1e9
                                            if traffic else None),
                           "kernel": "k_search (FSBM window search, QSAD)",
                           "launch_ms": search_ms / search_n}
    log(f"timed steps done: {ms_step:.2f} ms per step")
    if args.walker_phases:
        ph = acbm.phase_profile_read(reset=True)
        nblk, ncrit = max(1, ph["blocks"]), max(1, ph["critical_blocks"])
        us = lambda k, n: ph[k] / 100.0 / n  # s_memrealtime ticks at 100 MHz -> us
        out["walker_phases"] = {
            "blocks": ph["blocks"], "critical_blocks": ph["critical_blocks"],
            "us_per_block": {k: us(k, nblk) for k in ("dependency_wait", "phase_a", "phase_b",
                                                      "phase_c")},
            "critical_search_us_per_critical_block": us("critical_search", ncrit),
            "row_setup_us_per_row": us("row_setup", max(1, ph["blocks"] // 120)),
            "note": "thread 0 of each walker, s_memrealtime stamps; profiling build"}
    if do_f and do_a and len(frames) >= 32:
        out["latency_one_pair"] = latency_leg(torch, acbm, frames, prm, stream)
    if args.only in (None, "halfpel"):
        out["halfpel"] = halfpel_leg(torch, acbm, frames, prm, stream, args.steps)
        log("half-pel leg done")
    if args.only in (None, "batch") and not args.no_batch:
        out["batched"] = batched_leg(torch, acbm, synth, dev)
        log("batched leg done")
    if args.only in (None, "serve") and not args.no_serve:
        out["served"] = served_leg(torch, acbm, synth, [200, 500, 1000, 2000], args.serve_seconds,
                                   lanes=args.serve_lanes)
    if do_f and "roofline" in out:
        ev = probe_peak()
        if ev:
            out["roofline"]["peak_evidence"] = ev
    mismatches = 0
    if not args.no_cpu:
        log("oracle baseline and parity check")
        import oracle
        oprm = oracle.Params(lam=prm.lam, qp=prm.qp, alpha=prm.alpha, beta=prm.beta,
                             gamma_num=prm.gamma_num, gamma_den=prm.gamma_den)
        out["cpu_baseline"], want_f, want_a = cpu_baseline(wl, oprm)
        out["cpu_baseline"].update(host_info())
        out["cpu_baseline_parallel"], want_fs = cpu_baseline_parallel(wl, oprm)
        # the oracle results the baseline computed are the timed run's parity check
        parity = {"fsbm_pairs": 0, "acbm_pairs": 0, "blocks_differing": 0}
        if do_f:
            for t, wf in enumerate(want_fs):
                parity["blocks_differing"] += count_mismatches(res_f[t], wf)
                parity["fsbm_pairs"] += 1
        if do_a:
            parity["blocks_differing"] += count_mismatches(res_a[0], want_a)
            parity["acbm_pairs"] += 1
        parity["ok"] = parity["blocks_differing"] == 0
        out["parity"] = parity
        mismatches = parity["blocks_differing"]
    print(json.dumps(out), flush=True)
    if mismatches:
        print(f"bench.py: {mismatches} blocks differ from the oracle", file=sys.stderr)
        sys.exit(3)


if __name__ == "__main__":
    main()
