"""GPU parity with half-pel precision (acbm_params.subpel = 1) against the
CPU oracle, bit-exact on every field: vectors in half-pel units, H.263
bilinear half-pel samples, FSBM's 8 half-pel positions around its integer
winner, the half-pel PBM refinement ring."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_0710_4819_amd import acbm, synth
from test_gpu_parity import FIELDS, _sample_blocks, dev, oparams, same, say, search_cases

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", list(search_cases()), ids=lambda c: c[0])
def test_fsbm_half_frame(case):
    name, cur, ref, bw, bh, p, lam, pitch = case
    say(f"half fsbm {name}: {cur.shape} block {bw}x{bh} p={p} lambda={lam}")
    prm = acbm.Params(lam=lam, qp=lam, subpel=1)
    w = cur.shape[1]
    got = acbm.to_numpy(acbm.fsbm_frame(dev(cur, pitch), dev(ref, pitch), bw, bh, p, prm, width=w))
    want = oracle.fsbm_frame(cur, ref, bw, bh, p, oparams(prm))
    same(got, want, f"half fsbm {name}")


def test_fsbm_half_table1_count():
    """Table 1's full-search count: 969 positions per interior macroblock at
    p = 15 with half-pel precision."""
    ref = synth.texture(96, 96, 1.5, synth.rng(631))
    cur = synth.add_noise(np.roll(ref, (1, -1), (0, 1)), 1.0, synth.rng(632))
    prm = acbm.Params(lam=2, qp=2, subpel=1)
    say("half fsbm table-1 count: 96x96 16x16 p=15")
    got = acbm.to_numpy(acbm.fsbm_frame(dev(cur), dev(ref), 16, 16, 15, prm))
    same(got, oracle.fsbm_frame(cur, ref, 16, 16, 15, oparams(prm)), "half fsbm p15")
    assert (got["cands"][1:5, 1:5] == 969).all()


def test_half_batch_mixed_precision():
    """Integer and half-pel FSBM jobs of several geometries in one batch (and
    in one captured graph, replayed) equal the oracle's sequence runs."""
    sc = synth.cif_scene(nframes=5, lam=8)
    specs = [(144, 176, 16, 16, 7, 8, 1), (96, 128, 8, 8, 5, 4, 1), (144, 176, 16, 16, 7, 8, 0),
             (64, 96, 16, 8, 9, 2, 1)]
    b = acbm.Batch("cuda")
    seqs = []
    for (h, w, bw, bh, p, lam, hp) in specs:
        frames = [f[:h, :w].copy() for f in sc.frames]
        prm = acbm.Params(lam=lam, qp=lam, subpel=hp)
        b.add([dev(f) for f in frames], bw, bh, p, prm, acbm.ALGO_FSBM)
        seqs.append((frames, bw, bh, p, prm))
    say(f"half batch: {len(seqs)} FSBM jobs, mixed precision")
    outs = b.run()
    torch.cuda.synchronize()
    wants = [oracle.sequence(f, bw, bh, p, oparams(prm), oracle.FSBM) for (f, bw, bh, p, prm) in seqs]
    for k, want in enumerate(wants):
        same(acbm.to_numpy(outs[k]), want, f"half batch job {k}")
    g = acbm.BatchGraph(b)
    for rep in range(3):
        for o in outs:
            o.fill_(0xA5)
        g.launch()
        torch.cuda.synchronize()
        for k, want in enumerate(wants):
            same(acbm.to_numpy(outs[k]), want, f"half graph replay {rep} job {k}")
    g.close()


def test_fsbm_half_hd_sampled():
    """1920x1088, 16x16, p = 32, lambda = 8, half-pel: IntraX on every block
    and 24 sampled blocks per pair recomputed by the oracle from the GPU's
    own neighbouring vectors."""
    sc = synth.hd_scene(nframes=3)
    prm = acbm.Params(lam=8, qp=8, subpel=1)
    b = acbm.Batch("cuda")
    b.add([dev(f) for f in sc.frames], 16, 16, 32, prm, acbm.ALGO_FSBM)
    say("half fsbm hd sampled")
    got = acbm.to_numpy(b.run()[0])
    for t in range(len(sc.frames) - 1):
        cur, ref = sc.frames[t + 1], sc.frames[t]
        assert np.array_equal(got[t]["intra_x"].astype(np.uint64), oracle.intra_table(cur, 16, 16))
        for (r, c) in _sample_blocks(*got.shape[1:], 24, 300 + t):
            one = oracle.block(cur, ref, 16, 16, 32, oparams(prm), oracle.FSBM, got[t]["mv_x"],
                               got[t]["mv_y"], r, c)
            for f in FIELDS:
                assert int(one[f]) == int(got[t][r, c][f]), (t, r, c, f, one, got[t][r, c])


def test_half_rejects_large_p_and_bad_flag():
    cur = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(acbm.AcbmError) as e:
        acbm.fsbm_frame(cur, cur, 16, 16, 64, acbm.Params(lam=1, subpel=1))
    assert e.value.status == acbm.E_RANGE
    with pytest.raises(acbm.AcbmError) as e:
        acbm.fsbm_frame(cur, cur, 16, 16, 8, acbm.Params(lam=1, subpel=2))
    assert e.value.status == acbm.E_INVAL


def _half_pred_params():
    yield "paper", lambda bw, bh, lam: dataclasses.replace(acbm.default_params(bw, bh, lam), subpel=1)
    yield "mixed", lambda bw, bh, lam: acbm.Params(lam=lam, qp=lam, alpha=bw * bh, beta=1,
                                                    gamma_num=1, gamma_den=3, subpel=1)
    yield "all_critical", lambda bw, bh, lam: acbm.Params(lam=lam, qp=lam, alpha=0, beta=0,
                                                          gamma_num=0, gamma_den=1, subpel=1)


@pytest.mark.parametrize("algo", ["pbm", "acbm"])
@pytest.mark.parametrize("pp", list(_half_pred_params()), ids=lambda x: x[0])
@pytest.mark.parametrize("case", list(search_cases()), ids=lambda c: c[0])
def test_predictive_half_frame(case, pp, algo):
    """PBM and ACBM with half-pel precision, with and without a previous
    field (random half-pel vectors over the whole +-2p range)."""
    name, cur, ref, bw, bh, p, lam, pitch = case
    if algo == "pbm" and pp[0] != "paper":
        pytest.skip("PBM does not read the thresholds")
    prm = pp[1](bw, bh, lam)
    by, bx = cur.shape[0] // bh, cur.shape[1] // bw
    prev = synth.rng(78).integers(-2 * p, 2 * p + 1, size=(by, bx, 2)).astype(np.int16)
    say(f"half {algo} {name} {pp[0]}: {cur.shape} block {bw}x{bh} p={p} {prm}")
    w = cur.shape[1]
    fn = acbm.pbm_frame if algo == "pbm" else acbm.acbm_frame
    ofn = oracle.pbm_frame if algo == "pbm" else oracle.acbm_frame
    for pf in (None, prev):
        ws = acbm.workspace(acbm.OP_ACBM, acbm.geom(dev(cur, pitch), bw, bh, p, w), "cuda")
        got_t = fn(dev(cur, pitch), dev(ref, pitch), bw, bh, p, prm,
                   prev_field=None if pf is None else torch.from_numpy(pf).cuda(), width=w, ws=ws)
        assert acbm.workspace_status(ws) == 0
        got = acbm.to_numpy(got_t)
        want = ofn(cur, ref, bw, bh, p, oparams(prm), prev_field=pf)
        same(got, want, f"half {algo} {name} {pp[0]} prev={'yes' if pf is not None else 'no'}")


@pytest.mark.parametrize("algo", [acbm.ALGO_PBM, acbm.ALGO_ACBM])
def test_half_predictive_sequences_in_batch(algo):
    """Half-pel and integer predictive sequences in one batch (pair t takes
    pair t-1's half-pel field) equal the oracle's sequence runs."""
    sc = synth.cif_scene(nframes=5, lam=8)
    specs = [(144, 176, 16, 16, 7, 8, 1), (96, 128, 8, 8, 5, 4, 1), (144, 176, 16, 16, 7, 8, 0),
             (64, 96, 16, 8, 9, 2, 1)]
    b = acbm.Batch("cuda")
    seqs = []
    for (h, w, bw, bh, p, lam, hp) in specs:
        frames = [f[:h, :w].copy() for f in sc.frames]
        prm = dataclasses.replace(acbm.default_params(bw, bh, lam), subpel=hp)
        b.add([dev(f) for f in frames], bw, bh, p, prm, algo)
        seqs.append((frames, bw, bh, p, prm))
    say(f"half predictive batch algo={algo}: {len(seqs)} jobs")
    outs = b.run()
    torch.cuda.synchronize()
    for k, (f, bw, bh, p, prm) in enumerate(seqs):
        same(acbm.to_numpy(outs[k]), oracle.sequence(f, bw, bh, p, oparams(prm), algo),
             f"half predictive batch job {k}")


def test_acbm_half_hd_sampled():
    """1920x1088, 16x16, p = 32, lambda = 8, half-pel ACBM with the paper's
    thresholds: sampled blocks recomputed by the oracle from the GPU's own
    neighbouring vectors and previous field."""
    sc = synth.hd_scene(nframes=3)
    prm = dataclasses.replace(acbm.default_params(16, 16, 8), subpel=1)
    b = acbm.Batch("cuda")
    b.add([dev(f) for f in sc.frames], 16, 16, 32, prm, acbm.ALGO_ACBM)
    say("half acbm hd sampled")
    got = acbm.to_numpy(b.run()[0])
    for t in range(len(sc.frames) - 1):
        cur, ref = sc.frames[t + 1], sc.frames[t]
        prev = (np.zeros(got.shape[1:] + (2,), np.int16) if t == 0
                else oracle.field_of(got[t - 1]).astype(np.int16))
        for (r, c) in _sample_blocks(*got.shape[1:], 24, 400 + t):
            one = oracle.block(cur, ref, 16, 16, 32, oparams(prm), oracle.ACBM, got[t]["mv_x"],
                               got[t]["mv_y"], r, c, prev_field=prev)
            for f in FIELDS:
                assert int(one[f]) == int(got[t][r, c][f]), (t, r, c, f, one, got[t][r, c])
