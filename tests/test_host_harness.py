"""Host logic of the statistics harnesses, on the CPU: the Fig. 3 generator
makes exactly the motion it reports, and the Fig. 4 summary counts what it
says it counts."""
import numpy as np

from paper_0710_4819_amd import fig4, synth


def test_global_motion_is_exact_without_noise():
    """With no noise, frame k at x equals frame k-1 at x + d_k everywhere the
    shifted pixel lies inside the frame (the Fig. 3 setup: every block of a
    pair has the same known vector)."""
    wl = synth.global_motion(h=96, w=128, nframes=10, max_shift=6, noise_sigma=0.0, seed=61)
    assert len(wl.frames) == 10 and wl.truth.shape == (9, 6, 8, 2)
    h, w = 96, 128
    for k in range(1, 10):
        dx, dy = wl.meta["shifts"][k - 1]
        assert (wl.truth[k - 1, ..., 0] == dx).all() and (wl.truth[k - 1, ..., 1] == dy).all()
        a, b = wl.frames[k].astype(int), wl.frames[k - 1].astype(int)
        ys, xs = np.mgrid[0:h, 0:w]
        inside = (ys + dy >= 0) & (ys + dy < h) & (xs + dx >= 0) & (xs + dx < w)
        assert np.array_equal(a[inside], b[(ys + dy)[inside], (xs + dx)[inside]])
    # texture strength spans flat to textured blocks
    f = wl.frames[0].astype(np.int64)
    blk = f.reshape(6, 16, 8, 16).transpose(0, 2, 1, 3).reshape(48, 256)
    isad = np.abs(256 * blk - blk.sum(1, keepdims=True)).sum(1) / 256
    assert isad.max() > 3 * isad.min()


def _rec(cls_err_valid_intra):
    r = np.zeros(len(cls_err_valid_intra), fig4.RECORD_DTYPE)
    for i, (err, tv, intra, dev) in enumerate(cls_err_valid_intra):
        r[i]["err"] = err
        r[i]["cls"] = fig4.error_class(np.array(err))
        r[i]["truth_valid"] = tv
        r[i]["intra_sad"] = intra
        r[i]["sad_deviation"] = dev
    return r


def test_error_classes_and_summary():
    assert list(fig4.error_class(np.array([0, 1, 4, 5, 9]))) == [0, 1, 4, 5, 5]
    rec = _rec([(0, 1, 10.0, 100), (0, 1, 20.0, 300), (2, 1, 1.0, 5), (7, 1, 2.0, 7),
                (0, 0, 50.0, 1)])
    s = fig4.summarize(rec)
    assert s["blocks"] == 5 and s["truth_invalid"] == 1
    c = s["classes"]
    assert c["error=0"]["blocks"] == 2 and c["error=0"]["intra_sad_median"] == 15.0
    assert c["error=0"]["sad_deviation_mean"] == 200.0
    assert c["error=2"]["blocks"] == 1 and c["error>=5"]["blocks"] == 1
    assert c["error=1"] == {"blocks": 0}
    # quartiles of the four valid blocks (1, 2, 10, 20): one block each, the
    # two textured ones hold the true vectors
    assert s["true_share_by_intra_quartile"] == [0.0, 0.0, 1.0, 1.0]


def test_sweep_aggregate_and_relation():
    """aggregate() reduces result records to Table 1's measure and the sums;
    relate_to_fsbm() divides by the FSBM row of the same lambda and step."""
    from paper_0710_4819_amd import acbm, sweep
    res = np.zeros((2, 1, 2), acbm.RESULT_DTYPE)
    res["cands"] = [[[10, 30]], [[20, 40]]]
    res["mode"] = [[[acbm.MODE_CRITICAL, acbm.MODE_PBM_C1]], [[acbm.MODE_PBM_C2, acbm.MODE_CRITICAL]]]
    res["sad"], res["rate_bits"], res["j"] = 5, 2, 9
    a = sweep.aggregate(res)
    assert a == {"blocks": 4, "cands_per_block": 25.0, "critical_frac": 0.5, "c1_frac": 0.25,
                 "c2_frac": 0.25, "sum_sad": 20, "sum_rate": 8, "sum_j": 36}
    rows = [dict(algo="FSBM", lam=2, step=1, cands_per_block=100.0, sum_sad=10, sum_j=20),
            dict(algo="ACBM", lam=2, step=1, cands_per_block=25.0, sum_sad=11, sum_j=30)]
    sweep.relate_to_fsbm(rows)
    assert rows[1]["cands_vs_fsbm"] == 0.25 and rows[1]["sad_vs_fsbm"] == 1.1
    assert rows[1]["j_vs_fsbm"] == 1.5 and rows[0]["cands_vs_fsbm"] == 1.0
    assert len(sweep.grid()) == 45 and sweep.PAPER in sweep.grid()
