"""GPU parity of PBM and ACBM with previous fields that hold vectors the
search cannot use: components beyond +-p (and +-2p at half-pel precision),
beyond the +-127 a signed byte holds, and at the int16 limits.  The paper's
predictor set (Section 2.2) takes the previous frame's vectors as
candidates; a predictor that is not a valid candidate is dropped, never
clamped or wrapped (so (256, 1) must not turn into (0, 1)).  Every field of
every block is compared with the oracle, at integer and half-pel
precision."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_0710_4819_amd import acbm, synth
from test_gpu_parity import dev, oparams, same, say, search_cases

pytestmark = pytest.mark.gpu


def hostile_prev(by: int, bx: int, p: int, subpel: int, seed: int) -> np.ndarray:
    """A previous field where about 60 % of the blocks carry an unusable
    vector; several of them wrap to valid small vectors modulo 256."""
    s = 2 if subpel else 1
    special = [(256, 1), (200, 0), (-200, 3), (128, 0), (-128, 0), (129, 2), (-129, -1),
               (-32768, 0), (32767, 1), (0, -32768), (1, 32767), (-32768, -32768),
               (s * p + 1, 0), (0, -(s * p + 1)), (2 * s * p + 1, 1), (-(2 * s * p + 1), 0),
               (-253, 2), (259, -1), (1, 258), (-2, -254), (512, 512), (255, 0), (0, -255)]
    g = synth.rng(seed)
    prev = g.integers(-s * p, s * p + 1, size=(by, bx, 2)).astype(np.int16)
    pick = g.random((by, bx)) < 0.6
    idx = g.integers(0, len(special), size=(by, bx))
    for r in range(by):
        for c in range(bx):
            if pick[r, c]:
                prev[r, c] = special[int(idx[r, c])]
    return prev


def _cases():
    keep = {"planted_qcif_l4", "tex_8x8_p6_l8_pitch96", "cif_scene_p16_l32", "levels_16x8_p4_l1"}
    return [c for c in search_cases() if c[0] in keep]


@pytest.mark.parametrize("subpel", [0, 1])
@pytest.mark.parametrize("algo", ["pbm", "acbm"])
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_prev_field_out_of_range(case, algo, subpel):
    name, cur, ref, bw, bh, p, lam, pitch = case
    by, bx = cur.shape[0] // bh, cur.shape[1] // bw
    prev = hostile_prev(by, bx, p, subpel, 900 + p)
    fn = acbm.pbm_frame if algo == "pbm" else acbm.acbm_frame
    ofn = oracle.pbm_frame if algo == "pbm" else oracle.acbm_frame
    settings = [("paper", dataclasses.replace(acbm.default_params(bw, bh, lam), subpel=subpel))]
    if algo == "acbm":
        settings.append(("mixed", acbm.Params(lam=lam, qp=lam, alpha=bw * bh, beta=1,
                                              gamma_num=1, gamma_den=3, subpel=subpel)))
    w = cur.shape[1]
    for sname, prm in settings:
        say(f"prev out of range: {algo} {name} {sname} subpel={subpel} p={p}")
        ws = acbm.workspace(acbm.OP_ACBM, acbm.geom(dev(cur, pitch), bw, bh, p, w), "cuda")
        got_t = fn(dev(cur, pitch), dev(ref, pitch), bw, bh, p, prm,
                   prev_field=torch.from_numpy(prev).cuda(), width=w, ws=ws)
        assert acbm.workspace_status(ws) == 0
        want = ofn(cur, ref, bw, bh, p, oparams(prm), prev_field=prev)
        same(acbm.to_numpy(got_t), want, f"{algo} {name} {sname} subpel={subpel} hostile prev")
