"""Served requests (continuous batching): each result equals the same frame
pair run alone, however requests of different streams are gathered into
passes and however the passes overlap on the GPU; streams at p = 64 against
the oracle; error paths."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_0710_4819_amd import acbm, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _streams():
    sc = synth.cif_scene(nframes=5, lam=8)
    hd = synth.hd_scene(nframes=4, lam=8)
    return [
        # frames, block, p, lam, algo
        ([f[:144, :176].copy() for f in sc.frames], 16, 7, 8, acbm.ALGO_ACBM),
        ([f[:96, :128].copy() for f in sc.frames[:4]], 8, 5, 4, acbm.ALGO_FSBM),
        ([f[:256, :320].copy() for f in hd.frames], 16, 16, 8, acbm.ALGO_PBM),
        ([f[32:176, 16:192].copy() for f in sc.frames], 16, 9, 2, acbm.ALGO_ACBM),
        # half-pel precision (vectors and the stream's resident field in half-pel units)
        ([f[:144, :176].copy() for f in sc.frames], 16, 7, 8, ("half", acbm.ALGO_ACBM)),
        # p = 64, the largest served search range
        (synth.stream_frames({"stream": 0, "width": 640, "height": 480, "p": 64,
                              "seed": 5400}, 3), 16, 64, 8, acbm.ALGO_ACBM),
        (synth.stream_frames({"stream": 1, "width": 640, "height": 480, "p": 64,
                              "seed": 5401}, 3), 16, 64, 8, acbm.ALGO_FSBM),
    ]


def _prm(blk, lam, algo):
    p = acbm.default_params(blk, blk, lam)
    if isinstance(algo, tuple):
        return dataclasses.replace(p, subpel=1), algo[1]
    return p, algo


def _alone(frames, blk, p, prm, algo):
    b = acbm.Batch("cuda")
    b.add([torch.from_numpy(f).cuda() for f in frames], blk, blk, p, prm, algo)
    return acbm.to_numpy(b.run()[0])


@pytest.mark.parametrize("lanes,max_inflight", [(4, 64), (2, 3), (1, 64)])
def test_served_results_equal_alone_in_a_mix(lanes, max_inflight):
    """Every frame of every stream submitted up front, streams interleaved:
    the worker gathers several streams into each pass.  lanes and
    max_inflight change how requests are batched and overlapped, never the
    results."""
    streams = _streams()
    srv = acbm.Server(pool_bytes=2 << 30, max_streams=8, max_inflight=max_inflight,
                      queue_depth=64, lanes=lanes)
    try:
        tickets = {}
        nmax = max(len(s[0]) for s in streams)
        say(f"serve mix: {len(streams)} streams, up to {nmax} frames each")
        for t in range(nmax):  # interleave the streams frame by frame
            for sid, (frames, blk, p, lam, algo) in enumerate(streams):
                if t < len(frames):
                    prm, a = _prm(blk, lam, algo)
                    tickets[(sid, t)] = srv.submit(sid, frames[t], blk, blk, p, prm, a)
        got = {k: srv.wait(v, timeout_us=60_000_000) for k, v in tickets.items()}
        st = srv.stats()
    finally:
        srv.close()
    for sid, (frames, blk, p, lam, algo) in enumerate(streams):
        prm, a = _prm(blk, lam, algo)
        assert got[(sid, 0)] is None  # the first frame only becomes the reference
        alone = _alone(frames, blk, p, prm, a)
        for t in range(1, len(frames)):
            assert np.array_equal(got[(sid, t)], alone[t - 1]), (sid, t)
    # streams 0, 1, the half-pel one and the p = 64 ones against the oracle directly
    for sid in (0, 1, 4, 5, 6):
        frames, blk, p, lam, algo = streams[sid]
        prm, a = _prm(blk, lam, algo)
        oprm = oracle.Params(lam=prm.lam, qp=prm.qp, alpha=prm.alpha, beta=prm.beta,
                             gamma_num=prm.gamma_num, gamma_den=prm.gamma_den, subpel=prm.subpel)
        want = oracle.sequence(frames, blk, blk, p, oprm, a)
        for t in range(1, len(frames)):
            for f in ("mv_x", "mv_y", "sad", "j", "rate_bits", "cands", "mode", "intra_x"):
                assert np.array_equal(got[(sid, t)][f].astype(np.int64),
                                      want[t - 1][f].astype(np.int64)), (sid, t, f)
    total = sum(len(s[0]) - 1 for s in streams)
    assert st["completed"] == total
    assert 0 < st["p50_us"] <= st["p99_us"]
    assert st["throughput_rps"] > 0
    say(f"lanes {lanes}: {st['passes']} passes, {st['mean_batch']:.2f} requests a pass, "
        f"device busy {st['device_busy_frac']:.2f}")
    assert st["passes"] < total and st["mean_batch"] > 1  # requests were gathered
    assert 0 < st["device_busy_frac"] <= 1


def test_serve_rejects_what_can_never_fit_and_bad_requests():
    srv = acbm.Server(pool_bytes=1 << 20, max_streams=2, max_inflight=1, queue_depth=4)
    try:
        big = np.zeros((288, 352), np.uint8)  # p = 32: the FSBM workspace alone exceeds 1 MiB
        with pytest.raises(acbm.AcbmError) as e:
            srv.submit(0, big, 16, 16, 32, acbm.default_params(16, 16, 8), acbm.ALGO_FSBM)
        assert e.value.status == acbm.E_NOMEM
        small = np.zeros((48, 64), np.uint8)
        with pytest.raises(acbm.AcbmError) as e:
            srv.submit(5, small, 16, 16, 4, acbm.default_params(16, 16, 8), acbm.ALGO_ACBM)
        assert e.value.status == acbm.E_INVAL
        t0 = srv.submit(1, small, 16, 16, 4, acbm.default_params(16, 16, 8), acbm.ALGO_ACBM)
        assert srv.wait(t0, timeout_us=30_000_000) is None
        other = np.zeros((64, 64), np.uint8)
        with pytest.raises(acbm.AcbmError) as e:
            srv.submit(1, other, 16, 16, 4, acbm.default_params(16, 16, 8), acbm.ALGO_ACBM)
        assert e.value.status == acbm.E_SHAPE
        t1 = srv.submit(1, small, 16, 16, 4, acbm.default_params(16, 16, 8), acbm.ALGO_ACBM)
        r = srv.wait(t1, timeout_us=30_000_000)
        assert r is not None and (r["mv_x"] == 0).all() and (r["sad"] == 0).all()
        assert srv.stats()["rejected"] >= 1
    finally:
        srv.close()
