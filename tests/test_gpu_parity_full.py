"""GPU parity at the measured sizes: whole frames against the CPU oracle.

The oracle is single-threaded C; independent frame pairs and sequences run
on a thread pool (ctypes releases the interpreter lock around each call), so
whole 1920x1088 frames, the whole 64-sequence mix and p = 64 / p = 127
windows are compared block by block, every field, bit for bit.  Where even
that is too slow (3840x2160 at p = 64), sampled blocks are recomputed by the
oracle's single-block entry from the GPU's own neighbouring vectors.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_0710_4819_amd import acbm, synth

pytestmark = pytest.mark.gpu

FIELDS = ("mv_x", "mv_y", "sad", "j", "rate_bits", "cands", "mode", "intra_x")


def say(*a):
    print(*a, flush=True)


def threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def pool_map(fn, items):
    oracle.se_bits(0)  # load the library before the threads start
    with ThreadPoolExecutor(max_workers=threads()) as ex:
        return list(ex.map(fn, items))


def same(gpu: np.ndarray, ref: np.ndarray, what: str):
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    for f in FIELDS:
        g = gpu[f].astype(np.int64)
        o = ref[f].astype(np.int64)
        if not np.array_equal(g, o):
            bad = np.argwhere(g != o)
            i = tuple(bad[0])
            raise AssertionError(f"{what}: field {f} differs at {len(bad)} blocks, first {i}: "
                                 f"gpu {gpu[i]} oracle {ref[i]}")


def oparams(p: acbm.Params) -> oracle.Params:
    return oracle.Params(lam=p.lam, qp=p.qp, alpha=p.alpha, beta=p.beta,
                         gamma_num=p.gamma_num, gamma_den=p.gamma_den, subpel=p.subpel)


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def oracle_fsbm_pairs(frames, bw, bh, p, prm):
    """FSBM of every pair of a sequence, the pairs on the thread pool."""
    op = oparams(prm)
    outs = pool_map(lambda t: oracle.fsbm_frame(frames[t], frames[t - 1], bw, bh, p, op),
                    range(1, len(frames)))
    return np.stack(outs)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("subpel", [0, 1])
def test_hd_whole_frames(subpel):
    """1920x1088, 16x16, p = 32, lambda = 8 (the benchmark's workload and
    launch configuration): the first two pairs of the sequence, FSBM and ACBM
    with the paper's thresholds, every block of both pairs."""
    sc = synth.hd_scene(nframes=3)
    p0 = acbm.default_params(16, 16, 8)
    prm = acbm.Params(lam=p0.lam, qp=p0.qp, alpha=p0.alpha, beta=p0.beta,
                      gamma_num=p0.gamma_num, gamma_den=p0.gamma_den, subpel=subpel)
    fr = [dev(f) for f in sc.frames]
    got = {}
    for name, algo in (("fsbm", acbm.ALGO_FSBM), ("acbm", acbm.ALGO_ACBM)):
        say(f"hd whole frames subpel={subpel}: {name} on the GPU")
        b = acbm.Batch("cuda")
        out = b.add(fr, 16, 16, 32, prm, algo)
        b.run()
        torch.cuda.synchronize()
        if algo == acbm.ALGO_ACBM:
            assert b.status() == 0
        got[name] = acbm.to_numpy(out)
    say(f"hd whole frames subpel={subpel}: oracle")
    op = oparams(prm)
    tasks = [("fsbm", t) for t in (1, 2)] + [("acbm", 0)]

    def run(task):
        kind, t = task
        if kind == "fsbm":
            return oracle.fsbm_frame(sc.frames[t], sc.frames[t - 1], 16, 16, 32, op)
        return oracle.sequence(sc.frames, 16, 16, 32, op, oracle.ACBM)

    f1, f2, a = pool_map(run, tasks)
    same(got["fsbm"][0], f1, f"hd fsbm pair 1 subpel={subpel}")
    same(got["fsbm"][1], f2, f"hd fsbm pair 2 subpel={subpel}")
    same(got["acbm"], a, f"hd acbm pairs 1-2 subpel={subpel}")
    assert (a["mode"] == acbm.MODE_CRITICAL).any() and (a["mode"] != acbm.MODE_CRITICAL).any()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("algo", [acbm.ALGO_FSBM, acbm.ALGO_PBM, acbm.ALGO_ACBM])
def test_p64_whole_640x480(algo):
    """640x480, 16x16, p = 64 (the largest search range of the served mix):
    the single-pair entry points, with and without a previous field."""
    spec = {"stream": 0, "width": 640, "height": 480, "p": 64, "seed": 5200}
    frames = synth.stream_frames(spec, 2)
    prm = acbm.default_params(16, 16, 8)
    cur, ref = frames[1], frames[0]
    by, bx = 30, 40
    prev = synth.rng(64).integers(-64, 65, size=(by, bx, 2)).astype(np.int16)
    say(f"p=64 640x480 algo={algo}")
    for pf in ((None,) if algo == acbm.ALGO_FSBM else (None, prev)):
        if algo == acbm.ALGO_FSBM:
            got = acbm.to_numpy(acbm.fsbm_frame(dev(cur), dev(ref), 16, 16, 64, prm))
            want = oracle.fsbm_frame(cur, ref, 16, 16, 64, oparams(prm))
        else:
            fn = acbm.pbm_frame if algo == acbm.ALGO_PBM else acbm.acbm_frame
            ofn = oracle.pbm_frame if algo == acbm.ALGO_PBM else oracle.acbm_frame
            ws = acbm.workspace(acbm.OP_ACBM, acbm.geom(dev(cur), 16, 16, 64), "cuda")
            got_t = fn(dev(cur), dev(ref), 16, 16, 64, prm,
                       prev_field=None if pf is None else dev(pf), ws=ws)
            assert acbm.workspace_status(ws) == 0
            got = acbm.to_numpy(got_t)
            want = ofn(cur, ref, 16, 16, 64, oparams(prm), prev_field=pf)
        same(got, want, f"p=64 algo {algo} prev={'yes' if pf is not None else 'no'}")


def _sample_blocks(by, bx, n, seed):
    g = synth.rng(seed)
    pts = {(0, 0), (0, bx - 1), (by - 1, 0), (by - 1, bx - 1), (by // 2, bx // 2)}
    while len(pts) < n:
        pts.add((int(g.integers(0, by)), int(g.integers(0, bx))))
    return sorted(pts)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("algo", [acbm.ALGO_FSBM, acbm.ALGO_ACBM])
def test_p64_4k_sampled(algo):
    """3840x2160, 16x16, p = 64 (the largest served request, 134 G
    evaluations for a full search): IntraX on every block, and 48 blocks
    recomputed by the oracle from the GPU's own neighbouring vectors."""
    spec = {"stream": 0, "width": 3840, "height": 2160, "p": 64, "seed": 5300}
    frames = synth.stream_frames(spec, 2)
    prm = acbm.default_params(16, 16, 8)
    cur, ref = frames[1], frames[0]
    say(f"p=64 3840x2160 algo={algo}")
    if algo == acbm.ALGO_FSBM:
        got = acbm.to_numpy(acbm.fsbm_frame(dev(cur), dev(ref), 16, 16, 64, prm))
    else:
        ws = acbm.workspace(acbm.OP_ACBM, acbm.geom(dev(cur), 16, 16, 64), "cuda")
        got = acbm.to_numpy(acbm.acbm_frame(dev(cur), dev(ref), 16, 16, 64, prm, ws=ws))
        assert acbm.workspace_status(ws) == 0
    assert np.array_equal(got["intra_x"].astype(np.uint64), oracle.intra_table(cur, 16, 16))
    prev = None if algo == acbm.ALGO_FSBM else np.zeros(got.shape + (2,), np.int16)
    op = oparams(prm)
    pts = _sample_blocks(*got.shape, 48, 640 + algo)

    def one(rc):
        r, c = rc
        return oracle.block(cur, ref, 16, 16, 64, op, algo, got["mv_x"], got["mv_y"], r, c,
                            prev_field=prev)

    for (r, c), o in zip(pts, pool_map(one, pts)):
        for f in FIELDS:
            assert int(o[f]) == int(got[r, c][f]), (r, c, f, o, got[r, c])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("algo", [acbm.ALGO_FSBM, acbm.ALGO_ACBM])
@pytest.mark.parametrize("blk,h,w", [(16, 288, 320), (8, 272, 272)])
def test_p127_whole(blk, h, w, algo):
    """p = 127, the largest search range the library takes: frames just
    large enough that interior blocks see the whole 255x255 window; the full
    search, and ACBM (whose critical blocks search the same window)."""
    ref = synth.texture(h, w, 1.5, synth.rng(1270 + blk))
    cur = synth.add_noise(np.roll(ref, (7, -11), (0, 1)), 2.0, synth.rng(1271 + blk))
    p0 = acbm.default_params(blk, blk, 8)
    say(f"p=127 algo={algo} {w}x{h} block {blk}")
    if algo == acbm.ALGO_FSBM:
        got = acbm.to_numpy(acbm.fsbm_frame(dev(cur), dev(ref), blk, blk, 127, p0))
        want = oracle.fsbm_frame(cur, ref, blk, blk, 127, oparams(p0))
        assert int(want["cands"].max()) == 255 * 255
    else:
        ws = acbm.workspace(acbm.OP_ACBM, acbm.geom(dev(cur), blk, blk, 127), "cuda")
        got = acbm.to_numpy(acbm.acbm_frame(dev(cur), dev(ref), blk, blk, 127, p0, ws=ws))
        assert acbm.workspace_status(ws) == 0
        want = oracle.acbm_frame(cur, ref, blk, blk, 127, oparams(p0))
    same(got, want, f"p=127 algo {algo} block {blk}")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("subpel", [0, 1])
def test_resolve_state_in_workspace(subpel):
    """2560x1088 with 8x8 blocks: 43,520 blocks, more than the resolve keeps
    in LDS, so its per-block state lives in the workspace.  Whole frame."""
    sc = synth.moving_scene(1088, 2560, 2, 20, (64, 256), 12, 3, 2560)[0]
    p0 = acbm.default_params(8, 8, 8)
    prm = acbm.Params(lam=p0.lam, qp=p0.qp, alpha=p0.alpha, beta=p0.beta,
                      gamma_num=p0.gamma_num, gamma_den=p0.gamma_den, subpel=subpel)
    cur, ref = sc[1], sc[0]
    say(f"2560x1088 8x8 p=16 subpel={subpel}: 43520 blocks")
    got = acbm.to_numpy(acbm.fsbm_frame(dev(cur), dev(ref), 8, 8, 16, prm))
    want = oracle.fsbm_frame(cur, ref, 8, 8, 16, oparams(prm))
    same(got, want, f"2560x1088 8x8 subpel={subpel}")


@pytest.mark.timeout(900)
@pytest.mark.parametrize("algo", [acbm.ALGO_FSBM, acbm.ALGO_ACBM])
def test_batch_mix_whole(algo):
    """The 64-sequence mix at its real geometry (QCIF/CIF/1280x720/1920x1088,
    p 7/16/32, 16x16 and 8x8 blocks, 8 frames each) in one batch call, every
    pair of every sequence against the oracle."""
    seqs = [synth.batch_sequence(s) for s in range(64)]
    b = acbm.Batch("cuda")
    prms = []
    for w in seqs:
        prm = acbm.default_params(w.block_w, w.block_h, w.lam)
        prms.append(prm)
        b.add([dev(f) for f in w.frames], w.block_w, w.block_h, w.p, prm, algo)
    say(f"batch mix algo={algo}: 64 sequences on the GPU")
    outs = [acbm.to_numpy(o) for o in b.run()]
    torch.cuda.synchronize()
    if algo == acbm.ALGO_ACBM:
        assert b.status() == 0
    say(f"batch mix algo={algo}: oracle on {threads()} threads")
    if algo == acbm.ALGO_FSBM:
        tasks = [(i, t) for i in range(64) for t in range(1, len(seqs[i].frames))]
        # largest first, so the pool ends together
        tasks.sort(key=lambda it: -seqs[it[0]].width * seqs[it[0]].height * seqs[it[0]].p ** 2)

        def run(it):
            i, t = it
            w = seqs[i]
            return oracle.fsbm_frame(w.frames[t], w.frames[t - 1], w.block_w, w.block_h, w.p,
                                     oparams(prms[i]))

        for (i, t), want in zip(tasks, pool_map(run, tasks)):
            same(outs[i][t - 1], want, f"batch mix seq {i} pair {t}")
    else:
        order = sorted(range(64), key=lambda i: -seqs[i].width * seqs[i].height * seqs[i].p ** 2)

        def run(i):
            w = seqs[i]
            return oracle.sequence(w.frames, w.block_w, w.block_h, w.p, oparams(prms[i]),
                                   oracle.ACBM)

        for i, want in zip(order, pool_map(run, order)):
            same(outs[i], want, f"batch mix acbm seq {i}")
