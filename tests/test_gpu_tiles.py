"""FSBM of 8x8 blocks in 2x2 tiles (one workgroup searches four blocks over
their 16x16 window) against the oracle: even grids of blocks take the tiled
search, grids with an odd number of block columns or rows the one-block
search, and both must give the oracle's every field.  Edge cases: a single
tile, a tile count that fills no whole XCD band, a row pitch wider than the
frame, p = 0, 1, an
unaligned p and p = 64, lambda = 0 and a flat frame whose blocks keep their
whole row of SADs, half-pel precision, and a batch that mixes tiled and
one-block jobs."""
import numpy as np
import pytest

import oracle
from paper_0710_4819_amd import acbm, synth

from test_gpu_parity import dev, oparams, same, say

pytestmark = pytest.mark.gpu


def tex_pair(h, w, seed, shift=(2, -3), sigma=1.5, noise=2.0):
    ref = synth.texture(h, w, sigma, synth.rng(seed))
    cur = synth.add_noise(np.roll(ref, shift, (0, 1)), noise, synth.rng(seed + 1))
    return cur, ref


def cases():
    # name, (h, w), p, lambda, pitch, seed; whether tiles apply follows from
    # the grid: even bx and by
    yield "one_tile_16x16_p3", (16, 16), 3, 4, None, 1
    yield "even_64x96_p7", (64, 96), 7, 8, None, 2
    yield "even_96x48_p5_l4", (48, 96), 5, 4, None, 3          # 18 tiles: a partial XCD band
    yield "even_pitch_80x48_p6", (48, 80), 6, 8, 112, 4
    yield "even_p0", (48, 64), 0, 8, None, 5
    yield "even_p1_l32", (48, 64), 1, 32, None, 6
    yield "even_p13_unaligned", (64, 80), 13, 8, None, 7
    yield "even_l0", (64, 64), 9, 0, None, 8
    yield "even_p64_160x144", (144, 160), 64, 8, None, 9
    yield "odd_bx_72x64_p7", (64, 72), 7, 8, None, 10          # bx 9: one block a workgroup
    yield "odd_by_64x72_p7", (72, 64), 7, 8, None, 11          # by 9
    yield "odd_both_40x56_p5", (40, 56), 5, 4, None, 12


@pytest.mark.parametrize("case", list(cases()), ids=lambda c: c[0])
def test_tiled_and_one_block_fsbm(case):
    name, (h, w), p, lam, pitch, seed = case
    cur, ref = tex_pair(h, w, 500 + seed)
    prm = acbm.Params(lam=lam, qp=max(lam, 1))
    say(f"tiles {name}: {w}x{h} 8x8 p={p} lambda={lam} pitch={pitch}")
    got = acbm.to_numpy(acbm.fsbm_frame(dev(cur, pitch), dev(ref, pitch), 8, 8, p, prm, width=w))
    want = oracle.fsbm_frame(cur, ref, 8, 8, p, oparams(prm))
    same(got, want, f"tiles {name}")


def test_flat_frame_whole_rows():
    """Every candidate ties: each block keeps its whole row of SADs (more
    possible winners than the overflow list holds), in each of the tile's
    four blocks."""
    cur = np.full((48, 64), 90, np.uint8)
    ref = np.full((48, 64), 91, np.uint8)
    prm = acbm.Params(lam=2, qp=2)
    say("tiles flat 64x48 8x8 p=9")
    got = acbm.to_numpy(acbm.fsbm_frame(dev(cur), dev(ref), 8, 8, 9, prm))
    same(got, oracle.fsbm_frame(cur, ref, 8, 8, 9, oparams(prm)), "tiles flat")


@pytest.mark.parametrize("subpel", [1])
def test_tiled_half_pel(subpel):
    cur, ref = tex_pair(64, 96, 540, shift=(1, 2), sigma=3.0, noise=1.0)
    prm = acbm.Params(lam=8, qp=8, subpel=subpel)
    say("tiles half-pel 96x64 8x8 p=6")
    got = acbm.to_numpy(acbm.fsbm_frame(dev(cur), dev(ref), 8, 8, 6, prm))
    same(got, oracle.fsbm_frame(cur, ref, 8, 8, 6, oparams(prm)), "tiles half-pel")


def test_batch_mixes_tiled_and_one_block_jobs():
    """8x8 FSBM sequences with even and odd grids in one batch call: two
    search groups (tiled and one-block), one resolve."""
    sc = synth.cif_scene(nframes=4, lam=8)
    seqs = [([f[:96, :128].copy() for f in sc.frames], 5, 4),     # even: tiled
            ([f[:72, :120].copy() for f in sc.frames[:3]], 7, 8),  # by 9: one block
            ([f[:64, :80].copy() for f in sc.frames], 7, 8),       # even, same p: tiled
            ([f[:48, :64].copy() for f in sc.frames[:3]], 3, 2)]   # even, another p
    b = acbm.Batch("cuda")
    for frames, p, lam in seqs:
        b.add([dev(f) for f in frames], 8, 8, p, acbm.default_params(8, 8, lam), acbm.ALGO_FSBM)
    say(f"tiles batch: {len(seqs)} sequences")
    outs = b.run()
    for k, (frames, p, lam) in enumerate(seqs):
        want = oracle.sequence(frames, 8, 8, p, oparams(acbm.default_params(8, 8, lam)),
                               acbm.ALGO_FSBM)
        same(acbm.to_numpy(outs[k]), want, f"tiles batch seq {k}")
