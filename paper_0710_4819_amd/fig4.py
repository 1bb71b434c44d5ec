"""Section 3.1's statistics harness (the Fig. 3 setup and Fig. 4 plots).

The paper finds where full search can be skipped by running FSBM (minimum
SAD, so lambda = 0) over a sequence with known global motion and plotting,
for every 16x16 block, Intra_SAD against SAD_deviation, split by how far the
found vector lies from the true one (error 0, 1, 2, 3, 4 and >= 5).  This
module runs that experiment on the GPU library: acbm_fsbm_frame with
lambda = 0 for the vectors and acbm_sad_stats for SAD_min, SAD_deviation and
IntraX, one frame pair at a time, and returns one record per block.

A block whose true vector is not a valid candidate (the displaced block
would leave the frame, or a component exceeds p) cannot be recovered by any
search; such records carry truth_valid = 0 and summarize() leaves them out.

Reading: the error of a block is the L1 distance |mv_x - t_x| + |mv_y - t_y|
between its vector and the true vector t (the same measure the tie-break
uses for |mv|); the paper does not name the measure.  Intra_SAD is reported
as IntraX / (N*M), the real-valued sum of Section 3.1.
"""
from __future__ import annotations

import numpy as np
import torch

from . import acbm

RECORD_DTYPE = np.dtype([
    ("pair", "<i4"), ("r", "<i4"), ("c", "<i4"),
    ("mv_x", "<i2"), ("mv_y", "<i2"), ("true_x", "<i2"), ("true_y", "<i2"),
    ("truth_valid", "<i4"), ("err", "<i4"), ("cls", "<i4"),
    ("sad_min", "<u4"), ("valid", "<u4"), ("sad_deviation", "<u8"), ("intra_x", "<u8"),
    ("intra_sad", "<f8"),
])

N_CLASSES = 6  # errors 0, 1, 2, 3, 4 and >= 5


def error_class(err: np.ndarray) -> np.ndarray:
    return np.minimum(err, N_CLASSES - 1)


def run(frames, truth: np.ndarray, block_w: int, block_h: int, p: int, device="cuda:0",
        stream=None) -> np.ndarray:
    """One record per (pair, block) of the sequence.  `frames` are u8 numpy
    arrays (uploaded once), `truth` is [pairs, by, bx, 2] (x, y)."""
    dev = torch.device(device)
    fr = [torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in frames]
    prm = acbm.Params(lam=0, qp=0)
    g = acbm.geom(fr[0], block_w, block_h, p)
    ws = acbm.workspace(acbm.OP_FSBM, g, dev)
    by, bx = fr[0].shape[0] // block_h, fr[0].shape[1] // block_w
    out = np.empty((len(frames) - 1, by, bx), RECORD_DTYPE)
    for k in range(1, len(frames)):
        res = acbm.to_numpy(acbm.fsbm_frame(fr[k], fr[k - 1], block_w, block_h, p, prm, ws=ws,
                                            stream=stream))
        st = acbm.stats_to_numpy(acbm.sad_stats(fr[k], fr[k - 1], block_w, block_h, p,
                                                stream=stream))
        o = out[k - 1]
        o["pair"] = k - 1
        o["r"] = np.arange(by)[:, None]
        o["c"] = np.arange(bx)[None, :]
        o["mv_x"], o["mv_y"] = res["mv_x"], res["mv_y"]
        o["true_x"], o["true_y"] = truth[k - 1, ..., 0], truth[k - 1, ..., 1]
        o["err"] = (np.abs(res["mv_x"].astype(np.int32) - truth[k - 1, ..., 0])
                    + np.abs(res["mv_y"].astype(np.int32) - truth[k - 1, ..., 1]))
        o["cls"] = error_class(o["err"])
        x0 = np.arange(bx)[None, :] * block_w
        y0 = np.arange(by)[:, None] * block_h
        tx, ty = truth[k - 1, ..., 0].astype(np.int64), truth[k - 1, ..., 1].astype(np.int64)
        W, H = fr[0].shape[1], fr[0].shape[0]
        o["truth_valid"] = ((np.abs(tx) <= p) & (np.abs(ty) <= p) & (x0 + tx >= 0)
                            & (x0 + tx + block_w <= W) & (y0 + ty >= 0)
                            & (y0 + ty + block_h <= H))
        o["sad_min"], o["valid"] = st["sad_min"], st["valid"]
        o["sad_deviation"], o["intra_x"] = st["sad_deviation"], st["intra_x"]
        o["intra_sad"] = st["intra_x"].astype(np.float64) / (block_w * block_h)
    return out.reshape(-1)


def summarize(rec: np.ndarray) -> dict:
    """Per error class: block count, and the median and mean of Intra_SAD,
    SAD_deviation and SAD_min.  Also the share of true vectors in each
    quartile of Intra_SAD (the paper's first conclusion is that textured
    blocks get true vectors).  Only blocks whose true vector is a valid
    candidate count."""
    out = {"blocks": int(rec.size), "truth_invalid": int((rec["truth_valid"] == 0).sum()),
           "classes": {}}
    rec = rec[rec["truth_valid"] != 0]
    for k in range(N_CLASSES):
        sel = rec[rec["cls"] == k]
        name = f"error={k}" if k < N_CLASSES - 1 else f"error>={k}"
        if sel.size == 0:
            out["classes"][name] = {"blocks": 0}
            continue
        out["classes"][name] = {
            "blocks": int(sel.size),
            "intra_sad_median": float(np.median(sel["intra_sad"])),
            "intra_sad_mean": float(sel["intra_sad"].mean()),
            "sad_deviation_median": float(np.median(sel["sad_deviation"])),
            "sad_deviation_mean": float(sel["sad_deviation"].astype(np.float64).mean()),
            "sad_min_mean": float(sel["sad_min"].astype(np.float64).mean()),
        }
    if rec.size:
        q = np.quantile(rec["intra_sad"], [0.25, 0.5, 0.75])
        bins = np.searchsorted(q, rec["intra_sad"], side="right")
        out["true_share_by_intra_quartile"] = [
            float((rec["cls"][bins == i] == 0).mean()) if (bins == i).any() else None
            for i in range(4)]
    return out


def to_csv(rec: np.ndarray, path: str):
    """Writes the records as CSV (one block per line) for plotting."""
    names = RECORD_DTYPE.names
    with open(path, "w") as f:
        f.write(",".join(names) + "\n")
        for row in rec:
            f.write(",".join(str(row[n]) for n in names) + "\n")


def main(argv=None):
    import argparse
    import json

    from . import synth
    ap = argparse.ArgumentParser(description="Fig. 3 sequence -> Fig. 4 statistics on the GPU")
    ap.add_argument("--csv", help="write one line per block here")
    ap.add_argument("--seed", type=int, default=6000)
    a = ap.parse_args(argv)
    wl = synth.global_motion(seed=a.seed)
    rec = run(wl.frames, wl.truth, wl.block_w, wl.block_h, wl.p)
    if a.csv:
        to_csv(rec, a.csv)
    print(json.dumps({"workload": f"global_motion {wl.width}x{wl.height} 16x16 p={wl.p}",
                      "shifts": wl.meta["shifts"], **summarize(rec)}, indent=1))


if __name__ == "__main__":
    main()
