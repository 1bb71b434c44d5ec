"""Batched execution: the persistent full-search launches shared by all FSBM
jobs of a block size and plan give every job exactly its results alone; the
graph-recorded batch gives the eager batch's results on every replay, with
other GPU work between replays; autotuning changes no result."""
import numpy as np
import pytest
import torch

from paper_0710_4819_amd import acbm, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def _mixed_batch(dev):
    """Sequences of uneven geometry: QCIF/CIF crops, 16x16 and 8x8 blocks,
    p from 4 to 32, all three algorithms."""
    sc = synth.cif_scene(nframes=5, lam=8)
    hd = synth.hd_scene(nframes=4, lam=8)
    seqs = [
        ([f[:144, :176] for f in sc.frames], 16, 7, acbm.ALGO_FSBM, 8),
        ([f for f in sc.frames[:4]], 16, 16, acbm.ALGO_FSBM, 8),
        ([f[:144, :176] for f in sc.frames[:3]], 8, 7, acbm.ALGO_FSBM, 4),
        ([f[:256, :320] for f in hd.frames], 16, 32, acbm.ALGO_FSBM, 8),
        ([f[:96, :128] for f in sc.frames], 8, 16, acbm.ALGO_FSBM, 2),
        ([f[:144, :176] for f in sc.frames], 16, 7, acbm.ALGO_FSBM, 32),   # same class as job 0
        ([f[:144, :176] for f in sc.frames], 16, 9, acbm.ALGO_ACBM, 8),
        ([f[:128, :160] for f in sc.frames[:4]], 8, 6, acbm.ALGO_PBM, 4),
        ([f[:32, :48] for f in sc.frames[:3]], 16, 4, acbm.ALGO_FSBM, 1),   # tiny frame
    ]
    b = acbm.Batch(dev)
    for frames, blk, p, algo, lam in seqs:
        b.add([torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in frames], blk, blk, p,
              acbm.default_params(blk, blk, lam), algo)
    return b


def test_graph_batch_equals_eager_and_survives_replays():
    dev = torch.device("cuda", 0)
    b = _mixed_batch(dev)
    say(f"batch of {len(b.jobs)} jobs")
    eager = [acbm.to_numpy(o.clone()) for o in b.run()]
    torch.cuda.synchronize()
    # per-sequence runs give the same results
    for i, job in enumerate(b.jobs):
        single = acbm.Batch(dev)
        frames = b._keep[i][0]
        single.add(frames, job.geom.block_w, job.geom.block_h, job.geom.p,
                   acbm.Params(job.params.lambda_, job.params.qp, job.params.alpha,
                               job.params.beta, job.params.gamma_num, job.params.gamma_den),
                   job.algo)
        got = acbm.to_numpy(single.run()[0])
        assert np.array_equal(got, eager[i]), f"job {i}: batch differs from the job run alone"
    ws = torch.empty(max(256, b.workspace_size()), dtype=torch.uint8, device=dev)
    gr = acbm.BatchGraph(b, ws)
    try:
        for rep in range(4):
            for o in b.outs:
                o.fill_(0xA5)  # stale values must be overwritten by every replay
            say(f"graph replay {rep}")
            outs = gr.launch()
            torch.cuda.synchronize()
            for i, o in enumerate(outs):
                assert np.array_equal(acbm.to_numpy(o), eager[i]), f"replay {rep}, job {i}"
            # unrelated eager GPU work between replays
            x = torch.randn(1 << 20, device=dev)
            _ = (x * 2).sum().item()
            b.run()
            torch.cuda.synchronize()
    finally:
        gr.close()


def test_batch_equals_jobs_alone():
    """The grouped persistent launches give each job exactly its results alone,
    twice in a row on the same workspace (the job tables are rewritten)."""
    dev = torch.device("cuda", 0)
    b = _mixed_batch(dev)
    say(f"batch of {len(b.jobs)} jobs")
    ws = torch.empty(max(256, b.workspace_size()), dtype=torch.uint8, device=dev)
    first = [acbm.to_numpy(o.clone()) for o in b.run(ws)]
    for o in b.outs:
        o.fill_(0xA5)
    second = [acbm.to_numpy(o.clone()) for o in b.run(ws)]
    for i, job in enumerate(b.jobs):
        single = acbm.Batch(dev)
        single.add(b._keep[i][0], job.geom.block_w, job.geom.block_h, job.geom.p,
                   acbm.Params(job.params.lambda_, job.params.qp, job.params.alpha,
                               job.params.beta, job.params.gamma_num, job.params.gamma_den),
                   job.algo)
        alone = acbm.to_numpy(single.run()[0])
        assert np.array_equal(first[i], alone), f"job {i}: batch differs from the job alone"
        assert np.array_equal(second[i], alone), f"job {i}: second batch run differs"


def test_graph_batch_rejects_a_short_workspace():
    dev = torch.device("cuda", 0)
    b = _mixed_batch(dev)
    with pytest.raises(acbm.AcbmError) as e:
        acbm.BatchGraph(b, torch.empty(256, dtype=torch.uint8, device=dev))
    assert e.value.status == acbm.E_NOMEM


def test_autotune_changes_time_not_results():
    dev = torch.device("cuda", 0)
    sc = synth.cif_scene(nframes=3, lam=8)
    frames = [torch.from_numpy(f).to(dev) for f in sc.frames]
    prm = acbm.default_params(16, 16, 8)
    b = acbm.Batch(dev)
    out = b.add(frames, 16, 16, 16, prm, acbm.ALGO_FSBM)
    before = acbm.to_numpy(b.run()[0].clone())
    table_before = acbm.sad_table(frames[1], frames[0], 16, 16, 16).cpu().numpy()
    R, ms = acbm.autotune(16, 16, 16, 352, 288)
    say(f"autotune CIF p=16 -> R={R}, {ms:.4f} ms/pair")
    assert R in (1, 2, 3, 4, 5, 6, 8, 11, 16) and ms > 0
    after = acbm.to_numpy(b.run()[0])
    assert np.array_equal(before, after)
    assert np.array_equal(table_before, acbm.sad_table(frames[1], frames[0], 16, 16, 16).cpu().numpy())
