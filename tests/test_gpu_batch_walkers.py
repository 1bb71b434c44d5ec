"""Batched PBM/ACBM: the jobs of a batch with one block size and precision
share one row-walker launch, their rows taken in level order across jobs.
Every job's result equals the oracle's run of that sequence alone, bit for
bit, for groups that mix p, frame size, frame count, algorithm and the
ACBM thresholds, for a group split at its job limit, and on graph replays."""
import numpy as np
import pytest
import torch

import oracle
from paper_0710_4819_amd import acbm, synth

pytestmark = pytest.mark.gpu

FIELDS = ("mv_x", "mv_y", "sad", "j", "rate_bits", "cands", "mode", "intra_x")


def say(*a):
    print(*a, flush=True)


def oparams(p: acbm.Params) -> oracle.Params:
    return oracle.Params(lam=p.lam, qp=p.qp, alpha=p.alpha, beta=p.beta,
                         gamma_num=p.gamma_num, gamma_den=p.gamma_den, subpel=p.subpel)


def params(bw, bh, lam, subpel=0, qp=None, alpha=None):
    p0 = acbm.default_params(bw, bh, lam, qp)
    return acbm.Params(lam=p0.lam, qp=p0.qp, alpha=p0.alpha if alpha is None else alpha,
                       beta=p0.beta, gamma_num=p0.gamma_num, gamma_den=p0.gamma_den,
                       subpel=subpel)


def assert_oracle(name, got, frames, bw, bh, p, prm, algo):
    want = oracle.sequence(frames, bw, bh, p, oparams(prm), algo)
    for f in FIELDS:
        g, w = got[f].astype(np.int64), want[f].astype(np.int64)
        if not np.array_equal(g, w):
            bad = np.argwhere(g != w)[0]
            raise AssertionError(f"{name}: field {f} differs at {tuple(bad)}: "
                                 f"{g[tuple(bad)]} vs {w[tuple(bad)]}")


def _walker_jobs():
    """Sequences of uneven geometry and length for every block size, integer
    and half-pel, PBM and ACBM (19 jobs in 8 groups; the integer 16x16 group
    has five jobs, enough for the smaller walkers of many-job groups)."""
    sc = synth.cif_scene(nframes=6, lam=8)
    hd = synth.hd_scene(nframes=3, lam=8)
    jobs = [([f[32:208, 48:304] for f in sc.frames[:5]], 16, 16, 12, acbm.ALGO_ACBM,
             params(16, 16, 8)),
            ([f[:288, :352] for f in sc.frames[:3]], 16, 16, 16, acbm.ALGO_ACBM,
             params(16, 16, 4, qp=20)),
            ([f[:128, :192] for f in hd.frames[:3]], 16, 16, 20, acbm.ALGO_PBM,
             params(16, 16, 8))]
    for bw, bh in ((16, 16), (16, 8), (8, 16), (8, 8)):
        for subpel in (0, 1):
            jobs.append(([f[:144, :176] for f in sc.frames[:6]], bw, bh, 7, acbm.ALGO_ACBM,
                         params(bw, bh, 8, subpel)))
            jobs.append(([f[:96, :128] for f in hd.frames[:3]], bw, bh, 16 if subpel else 24,
                         acbm.ALGO_PBM if bw == bh else acbm.ALGO_ACBM,
                         params(bw, bh, 4, subpel, qp=12, alpha=400)))
    return jobs


def _batch(dev, jobs):
    b = acbm.Batch(dev)
    for frames, bw, bh, p, algo, prm in jobs:
        b.add([torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in frames], bw, bh, p,
              prm, algo)
    return b


def test_walker_groups_match_the_oracle():
    dev = torch.device("cuda", 0)
    jobs = _walker_jobs()
    b = _batch(dev, jobs)
    say(f"batch of {len(jobs)} PBM/ACBM jobs")
    got = [acbm.to_numpy(o) for o in b.run()]
    torch.cuda.synchronize()
    assert b.status() == 0
    for i, (frames, bw, bh, p, algo, prm) in enumerate(jobs):
        say(f"job {i}: {frames[0].shape} {bw}x{bh} p={p} algo={algo} subpel={prm.subpel}")
        assert_oracle(f"job {i}", got[i], frames, bw, bh, p, prm, algo)


def test_walker_group_graph_replays():
    dev = torch.device("cuda", 0)
    jobs = _walker_jobs()[:9]
    b = _batch(dev, jobs)
    eager = [acbm.to_numpy(o.clone()) for o in b.run()]
    ws = torch.empty(max(256, b.workspace_size()), dtype=torch.uint8, device=dev)
    gr = acbm.BatchGraph(b, ws)
    try:
        for rep in range(3):
            for o in b.outs:
                o.fill_(0xA5)
            say(f"graph replay {rep}")
            outs = gr.launch()
            torch.cuda.synchronize()
            for i, o in enumerate(outs):
                assert np.array_equal(acbm.to_numpy(o), eager[i]), f"replay {rep}, job {i}"
            x = torch.randn(1 << 18, device=dev)
            _ = (x * 2).sum().item()
    finally:
        gr.close()
    for i, (frames, bw, bh, p, algo, prm) in enumerate(jobs):
        assert_oracle(f"job {i}", eager[i], frames, bw, bh, p, prm, algo)


def test_walker_group_split_at_its_job_limit():
    """More tiny jobs than one group holds: the second group gives the same
    bit-exact results; every job also matches the oracle."""
    dev = torch.device("cuda", 0)
    g = synth.rng(77)
    jobs = []
    for s in range(300):
        h, w = (32, 48) if s % 3 else (48, 64)
        base = g.integers(0, 256, size=(h, w)).astype(np.uint8)
        nfr = 2 + s % 3
        frames = [np.roll(base, (k * (s % 5 - 2), k * (s % 7 - 3)), axis=(0, 1)) for k in range(nfr)]
        frames = [np.clip(f.astype(np.int32) + g.integers(-3, 4, size=f.shape), 0, 255)
                  .astype(np.uint8) for f in frames]
        jobs.append((frames, 16, 16, 4 + s % 5, acbm.ALGO_ACBM if s % 2 else acbm.ALGO_PBM,
                     params(16, 16, 4)))
    b = _batch(dev, jobs)
    say(f"batch of {len(jobs)} tiny jobs")
    got = [acbm.to_numpy(o) for o in b.run()]
    torch.cuda.synchronize()
    assert b.status() == 0
    for i, (frames, bw, bh, p, algo, prm) in enumerate(jobs):
        assert_oracle(f"job {i}", got[i], frames, bw, bh, p, prm, algo)


def test_side_streams_match_one_stream(monkeypatch):
    """Walker launches run on side streams forked off the caller's stream,
    beside the FSBM searches.  A batch that mixes FSBM jobs with several walker
    groups gives the same results with every launch on one stream
    (ACBM_BATCH_STREAMS=0), eagerly and on graph replays, and its FSBM jobs
    match the oracle."""
    dev = torch.device("cuda", 0)
    sc = synth.cif_scene(nframes=4, lam=8)
    jobs = _walker_jobs()[:7]
    fsbm = [([f[:144, :176] for f in sc.frames[:4]], 16, 16, 7, acbm.ALGO_FSBM,
             params(16, 16, 8)),
            ([f[:96, :128] for f in sc.frames[:3]], 8, 8, 5, acbm.ALGO_FSBM,
             params(8, 8, 4, subpel=1))]
    jobs = fsbm[:1] + jobs + fsbm[1:]
    b = _batch(dev, jobs)
    ws = torch.empty(max(256, b.workspace_size()), dtype=torch.uint8, device=dev)
    monkeypatch.setenv("ACBM_BATCH_STREAMS", "0")
    say(f"mixed batch of {len(jobs)} jobs on one stream")
    one = [acbm.to_numpy(o.clone()) for o in b.run(ws)]
    torch.cuda.synchronize()
    assert b.status(ws) == 0
    monkeypatch.delenv("ACBM_BATCH_STREAMS")
    for o in b.outs:
        o.fill_(0x5A)
    say("the same batch on side streams, eager")
    side = [acbm.to_numpy(o.clone()) for o in b.run(ws)]
    torch.cuda.synchronize()
    assert b.status(ws) == 0
    for i in range(len(jobs)):
        assert np.array_equal(side[i], one[i]), f"eager, job {i}"
    gr = acbm.BatchGraph(b, ws)
    try:
        for rep in range(3):
            for o in b.outs:
                o.fill_(0xA5)
            say(f"side-stream graph replay {rep}")
            outs = gr.launch()
            torch.cuda.synchronize()
            for i, o in enumerate(outs):
                assert np.array_equal(acbm.to_numpy(o), one[i]), f"replay {rep}, job {i}"
            x = torch.randn(1 << 18, device=dev)
            _ = (x * 2).sum().item()
    finally:
        gr.close()
    for i in (0, len(jobs) - 1):
        frames, bw, bh, p, algo, prm = jobs[i]
        assert_oracle(f"job {i}", one[i], frames, bw, bh, p, prm, algo)


def test_global_mode_capture_after_init():
    """After acbm_init (which creates the side streams), an acbm_batch call
    whose walker launches fork onto side streams can be captured into a torch
    CUDA graph in global capture mode; every replay equals the eager run."""
    dev = torch.device("cuda", 0)
    assert acbm.lib().acbm_init() == 0
    sc = synth.cif_scene(nframes=4, lam=8)
    jobs = [([f[:144, :176] for f in sc.frames[:4]], 16, 16, 7, acbm.ALGO_FSBM,
             params(16, 16, 8))] + _walker_jobs()[:5]
    b = _batch(dev, jobs)
    ws = torch.empty(max(256, b.workspace_size()), dtype=torch.uint8, device=dev)
    eager = [acbm.to_numpy(o.clone()) for o in b.run(ws)]
    torch.cuda.synchronize()
    assert b.status(ws) == 0
    s = torch.cuda.Stream(device=dev)
    g = torch.cuda.CUDAGraph()
    say("capturing acbm_batch in global mode")
    with torch.cuda.graph(g, stream=s, capture_error_mode="global"):
        b.run(ws, s)
    for rep in range(3):
        for o in b.outs:
            o.fill_(0x3C)
        say(f"captured batch replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(b.outs):
            assert np.array_equal(acbm.to_numpy(o), eager[i]), f"replay {rep}, job {i}"
        x = torch.randn(1 << 18, device=dev)
        _ = (x * 2).sum().item()
    assert b.status(ws) == 0
    for i in (0, 1):
        frames, bw, bh, p, algo, prm = jobs[i]
        assert_oracle(f"job {i}", eager[i], frames, bw, bh, p, prm, algo)


def test_eager_batch_beside_an_open_capture():
    """While one thread holds a capture open whose batch forked onto the
    library's side streams, another thread's eager acbm_batch must not fork
    onto those streams (they stay in the capture until it ends): it runs on
    its own stream, completes and matches the eager results; the capture then
    replays correctly."""
    import threading
    dev = torch.device("cuda", 0)
    assert acbm.lib().acbm_init() == 0
    jobs = _walker_jobs()[:4]
    b1, b2 = _batch(dev, jobs), _batch(dev, jobs)
    ws1 = torch.empty(max(256, b1.workspace_size()), dtype=torch.uint8, device=dev)
    ws2 = torch.empty(max(256, b2.workspace_size()), dtype=torch.uint8, device=dev)
    eager = [acbm.to_numpy(o.clone()) for o in b1.run(ws1)]
    torch.cuda.synchronize()
    assert b1.status(ws1) == 0
    s1, s2 = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    got = {}

    def other():
        try:
            with torch.cuda.stream(s2):
                for o in b2.outs:
                    o.fill_(0x77)
                b2.run(ws2, s2)
                s2.synchronize()
                got["status"] = b2.status(ws2, s2)
                got["outs"] = [acbm.to_numpy(o) for o in b2.outs]
        except Exception as e:  # reported by the main thread
            got["error"] = e

    g = torch.cuda.CUDAGraph()
    say("capture open on one thread, eager batch on another")
    with torch.cuda.graph(g, stream=s1, capture_error_mode="thread_local"):
        b1.run(ws1, s1)
        t = threading.Thread(target=other)
        t.start()
        t.join()
    assert "error" not in got, got.get("error")
    assert got["status"] == 0
    for i, o in enumerate(got["outs"]):
        assert np.array_equal(o, eager[i]), f"eager batch beside the capture, job {i}"
    for rep in range(2):
        for o in b1.outs:
            o.fill_(0x3C)
        say(f"replay {rep} of the capture")
        g.replay()
        torch.cuda.synchronize()
        for i, o in enumerate(b1.outs):
            assert np.array_equal(acbm.to_numpy(o), eager[i]), f"replay {rep}, job {i}"
    assert b1.status(ws1) == 0
