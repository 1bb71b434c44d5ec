"""ACBM threshold and frame-rate sweep (Sections 3.2 and 4).

ACBM's cost and quality are steered by alpha, beta and gamma (Section 3.2:
the thresholds can trade full searches for quality, down to no full search
at all), and the paper compares 30 and 10 frames per second (Section 4,
Figs. 5-6, Table 1: candidates per macroblock, lower at the higher frame
rate).  This module measures that trade-off on the GPU library: every
(lambda, frame step, setting) combination becomes one job of a single
acbm_batch launch, next to FSBM and PBM jobs on the same frames, and each job
is reduced to Table 1's measure (candidate positions per block) plus the
critical fraction and the summed SAD, rate and J.

Frame rate: a step of s keeps frames 0, s, 2s, ... of the sequence, so a
30 fps sequence at step 3 stands for 10 fps (the motion per pair triples).
Qp = lambda for every job.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import acbm


@dataclass(frozen=True)
class Setting:
    alpha: int
    beta: int
    gamma_num: int
    gamma_den: int

    @property
    def label(self) -> str:
        return f"a{self.alpha}_b{self.beta}_g{self.gamma_num}/{self.gamma_den}"


PAPER = Setting(1000, 8, 1, 4)  # Section 4's choice for 16x16 blocks


def grid(alphas=(250, 500, 1000, 2000, 4000), betas=(4, 8, 16),
         gammas=((1, 8), (1, 4), (1, 2))) -> list:
    return [Setting(a, b, gn, gd) for a in alphas for b in betas for (gn, gd) in gammas]


def aggregate(res: np.ndarray) -> dict:
    """Table 1's measure and the rate-distortion sums of one job's results
    ([pairs, by, bx] acbm_block_result records)."""
    n = int(res.size)
    mode = res["mode"]
    return {
        "blocks": n,
        "cands_per_block": float(res["cands"].astype(np.float64).mean()),
        "critical_frac": float((mode == acbm.MODE_CRITICAL).mean()),
        "c1_frac": float((mode == acbm.MODE_PBM_C1).mean()),
        "c2_frac": float((mode == acbm.MODE_PBM_C2).mean()),
        "sum_sad": int(res["sad"].astype(np.int64).sum()),
        "sum_rate": int(res["rate_bits"].astype(np.int64).sum()),
        "sum_j": int(res["j"].astype(np.int64).sum()),
    }


def run(frames, block_w: int, block_h: int, p: int, lams=(2, 8, 32), steps=(1, 3),
        settings=None, device="cuda:0", fps=30) -> list:
    """One row per job.  `frames` are u8 numpy arrays of one sequence (uploaded
    once and shared by every job).  Each row holds the job's key (algo,
    lambda, step, fps, setting) and aggregate(), plus its cost and sums
    relative to the FSBM job of the same lambda and step."""
    settings = grid() if settings is None else settings
    dev = torch.device(device)
    fr = [torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in frames]
    batch = acbm.Batch(dev)
    keys = []
    for lam in lams:
        for step in steps:
            seq = fr[::step]
            if len(seq) < 2:
                raise ValueError(f"step {step} leaves fewer than two frames")
            base = dict(lam=lam, step=step, fps=fps / step)
            batch.add(seq, block_w, block_h, p, acbm.Params(lam=lam, qp=lam), acbm.ALGO_FSBM)
            keys.append(dict(base, algo="FSBM", setting=None))
            batch.add(seq, block_w, block_h, p, acbm.Params(lam=lam, qp=lam), acbm.ALGO_PBM)
            keys.append(dict(base, algo="PBM", setting=None))
            for s in settings:
                prm = acbm.Params(lam=lam, qp=lam, alpha=s.alpha, beta=s.beta,
                                  gamma_num=s.gamma_num, gamma_den=s.gamma_den)
                batch.add(seq, block_w, block_h, p, prm, acbm.ALGO_ACBM)
                keys.append(dict(base, algo="ACBM", setting=s))
    outs = batch.run()
    torch.cuda.synchronize(dev)
    rows = []
    for k, out in zip(keys, outs):
        row = dict(k)
        row["setting"] = k["setting"].label if k["setting"] else None
        row.update(aggregate(acbm.to_numpy(out)))
        rows.append(row)
    relate_to_fsbm(rows)
    return rows


def relate_to_fsbm(rows: list):
    """Adds cands_vs_fsbm, sad_vs_fsbm and j_vs_fsbm (ratios to the FSBM row
    of the same lambda and step) to every row, in place."""
    ref = {(r["lam"], r["step"]): r for r in rows if r["algo"] == "FSBM"}
    for r in rows:
        f = ref[(r["lam"], r["step"])]
        r["cands_vs_fsbm"] = r["cands_per_block"] / f["cands_per_block"]
        r["sad_vs_fsbm"] = r["sum_sad"] / max(1, f["sum_sad"])
        r["j_vs_fsbm"] = r["sum_j"] / max(1, f["sum_j"])


def table(rows: list, setting: str | None = None) -> str:
    """Table 1's layout: candidates per block for each lambda (= Qp) and frame
    rate, for FSBM, PBM and one ACBM setting (the paper's by default), with
    ACBM's critical fraction and summed J relative to FSBM."""
    setting = setting or PAPER.label
    lines = ["lambda  fps   FSBM cands  PBM cands  ACBM cands  ACBM critical  ACBM J/FSBM J"]
    by = {}
    for r in rows:
        if r["algo"] == "ACBM" and r["setting"] != setting:
            continue
        by.setdefault((r["lam"], r["step"]), {})[r["algo"]] = r
    for (lam, step), d in sorted(by.items()):
        if not {"FSBM", "PBM", "ACBM"} <= d.keys():
            continue
        a = d["ACBM"]
        lines.append(f"{lam:6d} {a['fps']:5.1f} {d['FSBM']['cands_per_block']:11.1f} "
                     f"{d['PBM']['cands_per_block']:10.1f} {a['cands_per_block']:11.1f} "
                     f"{a['critical_frac']:14.3f} {a['j_vs_fsbm']:14.4f}")
    return "\n".join(lines)


TABLE1_QPS = (30, 28, 26, 24, 22, 20, 18, 16)


def table1(sequences: dict, qps=TABLE1_QPS, steps=(1, 3), fps=30, device="cuda:0") -> dict:
    """Table 1's layout on the given sequences (name -> Workload with
    16x16 blocks and p = 15): average candidate positions per macroblock of
    ACBM with the paper's thresholds, half-pel precision, lambda = Qp, at
    each Qp and frame rate, next to half-pel FSBM's count.  Every job of
    every sequence runs in one acbm_batch call."""
    dev = torch.device(device)
    batch = acbm.Batch(dev)
    keys = []
    for name, wl in sequences.items():
        fr = [torch.from_numpy(np.ascontiguousarray(f)).to(dev) for f in wl.frames]
        for step in steps:
            seq = fr[::step]
            for qp in qps:
                prm = acbm.Params(lam=qp, qp=qp, alpha=PAPER.alpha, beta=PAPER.beta,
                                  gamma_num=PAPER.gamma_num, gamma_den=PAPER.gamma_den, subpel=1)
                batch.add(seq, wl.block_w, wl.block_h, wl.p, prm, acbm.ALGO_ACBM)
                keys.append((name, "ACBM", qp, step))
            batch.add(seq, wl.block_w, wl.block_h, wl.p,
                      acbm.Params(lam=qps[-1], qp=qps[-1], subpel=1), acbm.ALGO_FSBM)
            keys.append((name, "FSBM", qps[-1], step))
    outs = batch.run()
    torch.cuda.synchronize(dev)
    table = {}
    for (name, algo, qp, step), out in zip(keys, outs):
        r = acbm.to_numpy(out)
        table[(name, algo, qp, fps / step)] = {
            "cands_per_block": float(r["cands"].astype(np.float64).mean()),
            "critical_frac": float((r["mode"] == acbm.MODE_CRITICAL).mean()),
            "interior_cands_max": int(r["cands"][:, 1:-1, 1:-1].max()) if algo == "FSBM" else None,
        }
    return table


def table1_text(table: dict) -> str:
    names = sorted({k[0] for k in table})
    rates = sorted({k[3] for k in table}, reverse=True)
    qps = sorted({k[2] for k in table if k[1] == "ACBM"}, reverse=True)
    head = "Qp   " + "".join(f"{n + ' ' + str(int(f)) + 'fps':>20s}" for n in names for f in rates)
    lines = [head]
    for qp in qps:
        lines.append(f"{qp:<5d}" + "".join(f"{table[(n, 'ACBM', qp, f)]['cands_per_block']:20.1f}"
                                           for n in names for f in rates))
    fs = [v["interior_cands_max"] for k, v in table.items() if k[1] == "FSBM"]
    lines.append(f"FSBM positions per interior macroblock: {max(fs)}")
    return "\n".join(lines)


def main(argv=None):
    import argparse
    import json
    import time

    from . import synth
    ap = argparse.ArgumentParser(description="ACBM threshold / frame-rate sweep on the GPU")
    ap.add_argument("--json", help="write every row here")
    ap.add_argument("--frames", type=int, default=30)
    ap.add_argument("--table1", action="store_true",
                    help="Table 1's layout on synthetic QCIF sequences (p = 15, half-pel)")
    a = ap.parse_args(argv)
    if a.table1:
        seqs = {k: synth.qcif_scene(k, nframes=a.frames) for k in ("smooth", "textured")}
        t0 = time.perf_counter()
        tab = table1(seqs)
        print(f"{len(tab)} jobs in one batch: {time.perf_counter() - t0:.2f} s")
        print(table1_text(tab))
        return
    wl = synth.cif_scene(nframes=a.frames)
    t0 = time.perf_counter()
    rows = run(wl.frames, wl.block_w, wl.block_h, wl.p)
    dt = time.perf_counter() - t0
    print(f"{len(rows)} jobs (CIF {a.frames} frames, p = {wl.p}) in one batch: {dt:.2f} s "
          f"including upload and read-back")
    print(table(rows))
    best = sorted((r for r in rows if r["algo"] == "ACBM" and r["lam"] == 8 and r["step"] == 1),
                  key=lambda r: r["cands_per_block"])
    print("lambda 8, 30 fps, settings by cost (cands/block, J/FSBM J):")
    for r in best[:5] + best[-5:]:
        print(f"  {r['setting']:>18s} {r['cands_per_block']:8.1f} {r['j_vs_fsbm']:.4f}")
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
