"""Pins that hold the CPU oracle to something other than itself.

Each pin is a plain function that raises AssertionError when the oracle
disagrees with what the paper or the mathematics fixes: printed figures,
closed forms, textbook codewords, an independent numpy computation, planted
motion, brute force on tiny inputs, and identities between the three searches.
`test_oracle_pins.py` runs them on the real oracle; `test_oracle_mutations.py`
runs them on deliberately broken builds and requires each break to be caught.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

import oracle
import brute
from conftest import golden, read_kv
from paper_0710_4819_amd import synth


# ----------------------------------------------------------------------------
# inputs
# ----------------------------------------------------------------------------
def _noise(h, w, seed, hi=256):
    return synth.rng(seed).integers(0, hi, size=(h, w)).astype(np.uint8)


def _tiny_cases():
    """Tiny frames of several kinds: textured, few-level (many ties), flat,
    ramp and planted shifts; 4x4 and 8x8 blocks, p up to 3."""
    cases = []
    k = 0
    for (h, w, bw, bh, p) in [(16, 16, 4, 4, 2), (24, 32, 8, 8, 3), (12, 20, 4, 4, 3),
                              (16, 24, 8, 4, 2), (8, 8, 4, 4, 1), (16, 16, 4, 8, 0)]:
        for kind in ("tex", "levels", "flat", "ramp", "planted"):
            k += 1
            if kind == "tex":
                ref = synth.texture(h, w, 1.0, synth.rng(100 + k))
                cur = synth.add_noise(np.roll(ref, (1, -1), (0, 1)), 2.0, synth.rng(200 + k))
            elif kind == "levels":
                ref = _noise(h, w, 300 + k, hi=3)
                cur = _noise(h, w, 400 + k, hi=3)
            elif kind == "flat":
                ref = np.full((h, w), 77, np.uint8)
                cur = np.full((h, w), 80, np.uint8)
            elif kind == "ramp":
                ref = (np.add.outer(np.arange(h) * 3, np.arange(w) * 5) % 256).astype(np.uint8)
                cur = np.roll(ref, (0, 2), (0, 1))
            else:
                ref = _noise(h, w, 500 + k)
                cur = np.roll(ref, (-1, 1), (0, 1))
            cases.append((cur, ref, bw, bh, p))
    return cases


def _fields(res_dict, by, bx, keys=("mv_x", "mv_y", "sad", "j", "rate_bits", "cands", "mode", "intra_x")):
    return {k: np.array([[res_dict[(r, c)][k] for c in range(bx)] for r in range(by)]) for k in keys}


def _same(oracle_res, brute_res, what):
    by, bx = oracle_res.shape
    b = _fields(brute_res, by, bx)
    for k, v in b.items():
        got = oracle_res[k].astype(np.int64)
        assert np.array_equal(got, v.astype(np.int64)), f"{what}: field {k} differs"


def _numpy_sad_table(cur, ref, bw, bh, p):
    """All SADs by an independent route: numpy sliding windows."""
    h, w = cur.shape
    by, bx = h // bh, w // bw
    W = 2 * p + 1
    pad = np.full((h + 2 * p, w + 2 * p), -1, dtype=np.int64)
    pad[p:p + h, p:p + w] = ref
    out = np.full((by, bx, W, W), 0xFFFFFFFF, dtype=np.uint64)
    curb = cur.astype(np.int64).reshape(by, bh, bx, bw).transpose(0, 2, 1, 3)
    for v in range(-p, p + 1):
        for u in range(-p, p + 1):
            sh = pad[p + v:p + v + h, p + u:p + u + w]
            shb = sh.reshape(by, bh, bx, bw).transpose(0, 2, 1, 3)
            inside = (shb >= 0).all(axis=(2, 3))
            s = np.abs(curb - shb).sum(axis=(2, 3))
            out[:, :, v + p, u + p] = np.where(inside, s, 0xFFFFFFFF)
    return out


def _closed_form_valid(width, height, bw, bh, p):
    """#valid candidates per block as a product of two interval lengths."""
    by, bx = height // bh, width // bw
    cnt = np.zeros((by, bx), dtype=np.int64)
    for r in range(by):
        for c in range(bx):
            x0, y0 = c * bw, r * bh
            nu = min(p, width - bw - x0) - max(-p, -x0) + 1
            nv = min(p, height - bh - y0) - max(-p, -y0) + 1
            cnt[r, c] = max(nu, 0) * max(nv, 0)
    return cnt


# ----------------------------------------------------------------------------
# rate term
# ----------------------------------------------------------------------------
def pin_se_codewords():
    """Textbook signed Exp-Golomb codewords fix the bit counts."""
    with open(golden("se_codewords.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    for k, word in rows:
        k = int(k)
        assert brute.codeword_se(k) == word, f"brute codeword of {k}"
        assert oracle.se_bits(k) == len(word), f"se_bits({k})"
    # a stream of codewords decodes back to the values, and its length is the
    # sum of the oracle's bit counts
    vals = [int(x) for x in synth.rng(7).integers(-300, 301, size=400)]
    stream = "".join(brute.codeword_se(v) for v in vals)
    at, back = 0, []
    while at < len(stream):
        k, at = brute.decode_se(stream, at)
        back.append(k)
    assert back == vals
    assert len(stream) == sum(oracle.se_bits(v) for v in vals)


def pin_se_closed_form():
    """se_bits(0) = 1 and se_bits(k) = 2*floor(log2|k|) + 3 otherwise; the
    largest rate in a window is 2*se_bits(2p)."""
    for k in range(-10000, 10001):
        want = 1 if k == 0 else 2 * (abs(k).bit_length() - 1) + 3
        assert oracle.se_bits(k) == want, k
    for p, rmax in [(7, 18), (15, 22), (16, 26), (32, 30), (64, 34)]:
        assert 2 * oracle.se_bits(2 * p) == rmax


# ----------------------------------------------------------------------------
# geometry and counts
# ----------------------------------------------------------------------------
def pin_paper_counts():
    """Full search at p = 15 counts 969 positions with the 8 half-pel ones
    (Sections 2.3 and 4), so 961 integer positions on an interior block."""
    kv = read_kv("paper_counts.txt")
    p = int(kv["p"])
    interior = int(kv["fsbm_positions_p15_halfpel"]) - int(kv["halfpel_extra"])
    assert interior == (2 * p + 1) ** 2
    cur = _noise(48, 48, 11)
    ref = _noise(48, 48, 12)
    res = oracle.fsbm_frame(cur, ref, 16, 16, p, oracle.Params(lam=2))
    assert int(res["cands"][1, 1]) == interior
    prm = read_kv("paper_counts.txt")
    d = oracle.Params()
    assert (d.alpha, d.beta, d.gamma_num, d.gamma_den) == (
        int(prm["alpha"]), int(prm["beta"]), int(prm["gamma_num"]), int(prm["gamma_den"]))


def pin_valid_counts():
    """FSBM counts every valid candidate once: the interval-product closed
    form, on QCIF with the planted-shift frames, and at odd shapes."""
    wl = synth.planted_blocks()
    res = oracle.fsbm_frame(wl.frames[1], wl.frames[0], 16, 16, 7, oracle.Params(lam=4))
    cf = _closed_form_valid(176, 144, 16, 16, 7)
    assert np.array_equal(res["cands"].astype(np.int64), cf)
    assert int(cf.sum()) == 18271
    for (h, w, bw, bh, p) in [(24, 40, 8, 4, 5), (16, 16, 16, 16, 3), (20, 12, 4, 4, 9)]:
        cur, ref = _noise(h, w, 1), _noise(h, w, 2)
        r = oracle.fsbm_frame(cur, ref, bw, bh, p, oracle.Params(lam=1))
        assert np.array_equal(r["cands"].astype(np.int64), _closed_form_valid(w, h, bw, bh, p))
    # the larger workloads' totals, closed form only
    assert int(_closed_form_valid(352, 288, 16, 16, 16).sum()) == 390028


# ----------------------------------------------------------------------------
# SAD, Intra_SAD, predictor
# ----------------------------------------------------------------------------
def pin_sad_table_numpy():
    """The SAD table equals an independent numpy sliding-window computation,
    with invalid positions marked, including a pitch wider than the frame."""
    for (h, w, bw, bh, p, seed) in [(32, 48, 16, 16, 5, 1), (24, 24, 8, 8, 4, 2),
                                    (16, 40, 8, 4, 3, 3)]:
        cur = synth.texture(h, w, 1.5, synth.rng(seed))
        ref = synth.texture(h, w, 1.5, synth.rng(seed + 50))
        got = oracle.sad_table(cur, ref, bw, bh, p).astype(np.uint64)
        assert np.array_equal(got, _numpy_sad_table(cur, ref, bw, bh, p))
    # pitch wider than width: garbage in the padding must not matter
    h, w, pitch = 16, 24, 40
    cur = _noise(h, pitch, 5)
    ref = _noise(h, pitch, 6)
    got = oracle.sad_table(cur, ref, 8, 8, 3, width=w).astype(np.uint64)
    assert np.array_equal(got, _numpy_sad_table(cur[:, :w].copy(), ref[:, :w].copy(), 8, 8, 3))


def pin_sad_planted_zero():
    """Noise-free planted shifts: the SAD at the planted vector is zero
    whenever the displaced block is wholly inside the frame and unclamped."""
    wl = synth.planted_blocks(noise_sigma=0.0)
    tab = oracle.sad_table(wl.frames[1], wl.frames[0], 16, 16, 7)
    t = wl.truth[0]
    by, bx = t.shape[:2]
    hits = 0
    for r in range(by):
        for c in range(bx):
            dx, dy = int(t[r, c, 0]), int(t[r, c, 1])
            x0, y0 = c * 16, r * 16
            if 0 <= x0 + dx and x0 + dx + 16 <= 176 and 0 <= y0 + dy and y0 + dy + 16 <= 144:
                assert tab[r, c, dy + 7, dx + 7] == 0
                hits += 1
    assert hits > 50


def pin_intra_exact():
    """IntraX = N*M * sum |p - mean| with the mean as an exact fraction; flat
    blocks give 0 and a half-0 / half-255 block gives N*M * N*M * 127.5."""
    cur = synth.texture(32, 48, 1.2, synth.rng(9))
    tab = oracle.intra_table(cur, 16, 8)
    for r in range(tab.shape[0]):
        for c in range(tab.shape[1]):
            blk = cur[r * 8:(r + 1) * 8, c * 16:(c + 1) * 16].astype(int).ravel().tolist()
            mu = Fraction(sum(blk), len(blk))
            want = sum(abs(Fraction(q) - mu) for q in blk) * len(blk)
            assert want.denominator == 1 and int(tab[r, c]) == int(want)
    flat = np.full((16, 16), 200, np.uint8)
    assert int(oracle.intra_table(flat, 16, 16)[0, 0]) == 0
    half = np.zeros((16, 16), np.uint8)
    half[:, 8:] = 255
    assert int(oracle.intra_table(half, 16, 16)[0, 0]) == 256 * 256 * 255 // 2


def pin_median_rules():
    """Median-of-three predictor with the picture-edge substitutions."""
    fx = np.array([[1, 5, -3, 7], [2, 9, 4, -6]], np.int32)
    fy = np.array([[-1, 0, 2, 3], [6, -2, -5, 8]], np.int32)
    # first block: everything missing -> (0, 0)
    assert oracle.median_pred(fx, fy, 0, 0) == (0, 0)
    # first row: B and C take A's value -> predictor is A
    assert oracle.median_pred(fx, fy, 0, 2) == (5, 0)
    # first column of a later row: A = (0,0), B = top, C = top-right
    assert oracle.median_pred(fx, fy, 1, 0) == (1, 0)          # med(0,1,5), med(0,-1,0)
    # interior: A = (9,-2), B = (-3,2), C = (7,3)
    assert oracle.median_pred(fx, fy, 1, 2) == (7, 2)
    # last column: C = (0,0); A = (4,-5), B = (7,3)
    assert oracle.median_pred(fx, fy, 1, 3) == (4, 0)


# ----------------------------------------------------------------------------
# the searches
# ----------------------------------------------------------------------------
def pin_fsbm_lambda0_global_min():
    """With lambda = 0, FSBM is the textbook full search: the global SAD
    minimum of the window, ties to smaller |u|+|v| then raster order."""
    for seed, (h, w, bw, bh, p) in enumerate([(32, 48, 16, 16, 6), (24, 32, 8, 8, 4)]):
        ref = synth.texture(h, w, 1.0, synth.rng(60 + seed))
        cur = synth.add_noise(np.roll(ref, (2, -1), (0, 1)), 3.0, synth.rng(70 + seed))
        tab = _numpy_sad_table(cur, ref, bw, bh, p)
        res = oracle.fsbm_frame(cur, ref, bw, bh, p, oracle.Params(lam=0))
        W = 2 * p + 1
        uu, vv = np.meshgrid(np.arange(-p, p + 1), np.arange(-p, p + 1))
        l1 = (np.abs(uu) + np.abs(vv)).ravel()
        ras = np.arange(W * W)
        for r in range(tab.shape[0]):
            for c in range(tab.shape[1]):
                s = tab[r, c].ravel()
                order = np.lexsort((ras, l1, s))
                best = order[0]
                assert int(res["mv_x"][r, c]) == int(uu.ravel()[best])
                assert int(res["mv_y"][r, c]) == int(vv.ravel()[best])
                assert int(res["sad"][r, c]) == int(s[best])


def pin_brute_fsbm():
    for i, (cur, ref, bw, bh, p) in enumerate(_tiny_cases()):
        lam = [0, 1, 4, 32][i % 4]
        got = oracle.fsbm_frame(cur, ref, bw, bh, p, oracle.Params(lam=lam))
        want = brute.fsbm(brute.as_lists(cur), brute.as_lists(ref), bw, bh, p, lam)
        _same(got, want, f"fsbm case {i}")


def _prev_for(cur, bw, bh, p, seed):
    by, bx = cur.shape[0] // bh, cur.shape[1] // bw
    g = synth.rng(seed)
    return g.integers(-p, p + 1, size=(by, bx, 2)).astype(np.int16)


def pin_brute_pbm():
    for i, (cur, ref, bw, bh, p) in enumerate(_tiny_cases()):
        lam = [0, 1, 4, 32][(i + 1) % 4]
        prev = None if i % 3 == 0 else _prev_for(cur, bw, bh, p, 900 + i)
        got = oracle.pbm_frame(cur, ref, bw, bh, p, oracle.Params(lam=lam), prev_field=prev)
        pv = None if prev is None else {(r, c): (int(prev[r, c, 0]), int(prev[r, c, 1]))
                                        for r in range(prev.shape[0]) for c in range(prev.shape[1])}
        want = brute.predictive(brute.as_lists(cur), brute.as_lists(ref), bw, bh, p, lam, prev=pv)
        _same(got, want, f"pbm case {i}")


def pin_brute_acbm():
    for i, (cur, ref, bw, bh, p) in enumerate(_tiny_cases()):
        lam = [0, 1, 4, 32][(i + 2) % 4]
        nm = bw * bh
        # thresholds that make all three outcomes occur on these inputs
        prm = oracle.Params(lam=lam, qp=lam, alpha=[0, 3, 40, 1000][i % 4] * nm // 16,
                            beta=[0, 1, 2, 8][(i // 4) % 4], gamma_num=[0, 1, 1, 3][(i // 2) % 4],
                            gamma_den=[1, 4, 2, 4][(i // 2) % 4])
        prev = None if i % 2 == 0 else _prev_for(cur, bw, bh, p, 950 + i)
        got = oracle.acbm_frame(cur, ref, bw, bh, p, prm, prev_field=prev)
        pv = None if prev is None else {(r, c): (int(prev[r, c, 0]), int(prev[r, c, 1]))
                                        for r in range(prev.shape[0]) for c in range(prev.shape[1])}
        want = brute.predictive(brute.as_lists(cur), brute.as_lists(ref), bw, bh, p, lam, prev=pv,
                                acbm=(prm.alpha, prm.beta, prm.qp, prm.gamma_num, prm.gamma_den))
        _same(got, want, f"acbm case {i}")


def pin_planted_recovery():
    """The paper's own check (Section 3.1): plant known motion in noise-free
    frames and count true vectors.  A block provably recovers its planted
    vector t when t is valid and, for every other valid m,
    SAD(m) + 2*lambda > SAD(t) + lambda*R(t - pred) (here SAD(t) = 0)."""
    wl = synth.planted_blocks(noise_sigma=0.0)
    cur, ref = wl.frames[1], wl.frames[0]
    tab = _numpy_sad_table(cur, ref, 16, 16, 7)
    t = wl.truth[0]
    for lam in (0, 2, 6):
        res = oracle.fsbm_frame(cur, ref, 16, 16, 7, oracle.Params(lam=lam))
        checked = 0
        for r in range(t.shape[0]):
            for c in range(t.shape[1]):
                dx, dy = int(t[r, c, 0]), int(t[r, c, 1])
                s = tab[r, c].astype(np.int64).copy()
                if s[dy + 7, dx + 7] != 0:
                    continue
                s[dy + 7, dx + 7] = 1 << 40
                # worst case over predictors: R(t - pred) <= 2*se_bits(2p)
                if s.min() + 2 * lam > lam * 2 * oracle.se_bits(14):
                    assert (int(res["mv_x"][r, c]), int(res["mv_y"][r, c])) == (dx, dy)
                    checked += 1
        assert checked > 40, checked
    # and a global shift over a sequence (Fig. 3 style): nine known vectors
    base = synth.texture(96, 128, 1.5, synth.rng(31))
    shifts = [(1, 0), (0, 2), (-3, 1), (2, -2), (0, 0), (-1, -3), (4, 4), (-4, 0), (3, -1)]
    for (dx, dy) in shifts:
        nxt = np.roll(base, (-dy, -dx), (0, 1))
        res = oracle.fsbm_frame(nxt, base, 16, 16, 4, oracle.Params(lam=0))
        by, bx = res.shape
        for r in range(by):
            for c in range(bx):
                x0, y0 = c * 16, r * 16
                # blocks whose source does not wrap around the roll
                if 0 <= x0 + dx and x0 + dx + 16 <= 128 and 0 <= y0 + dy and y0 + dy + 16 <= 96:
                    assert int(res["sad"][r, c]) == 0
                    assert (int(res["mv_x"][r, c]), int(res["mv_y"][r, c])) == (dx, dy)


def _acbm_inputs():
    wl = synth.planted_blocks(h=96, w=128, p=5, seeds=(41, 42, 43))
    return wl.frames[1], wl.frames[0]


def pin_fsbm_bounds_acbm():
    """J_FSBM <= J_ACBM: with lambda = 0 the full search's SAD never exceeds
    ACBM's; with lambda > 0, inside one ACBM run, the window minimum of J under
    that run's predictor bounds the block's J, with equality on critical
    blocks."""
    cur, ref = _acbm_inputs()
    for prm in (oracle.Params(lam=0, qp=0), oracle.Params(lam=0, qp=4, alpha=300, beta=2)):
        a = oracle.acbm_frame(cur, ref, 16, 16, 5, prm)
        f = oracle.fsbm_frame(cur, ref, 16, 16, 5, prm)
        assert (f["sad"] <= a["sad"]).all()
    lam = 4
    prm = oracle.Params(lam=lam, qp=4, alpha=200, beta=1)
    a = oracle.acbm_frame(cur, ref, 16, 16, 5, prm)
    tab = _numpy_sad_table(cur, ref, 16, 16, 5).astype(np.int64)
    by, bx = a.shape
    field = {(r, c): (int(a["mv_x"][r, c]), int(a["mv_y"][r, c])) for r in range(by) for c in range(bx)}
    modes = set()
    for r in range(by):
        for c in range(bx):
            px, py = brute.predictor(field, r, c, bx)
            best = None
            for v in range(-5, 6):
                for u in range(-5, 6):
                    s = tab[r, c, v + 5, u + 5]
                    if s == 0xFFFFFFFF:
                        continue
                    j = s + lam * (oracle.se_bits(u - px) + oracle.se_bits(v - py))
                    best = j if best is None else min(best, j)
            assert best <= int(a["j"][r, c])
            if int(a["mode"][r, c]) == 3:
                assert best == int(a["j"][r, c])
            modes.add(int(a["mode"][r, c]))
    assert 3 in modes and (1 in modes or 2 in modes), modes


def pin_acbm_reduces_to_fsbm():
    """alpha = beta = gamma = 0 makes both tests fail on every block, so ACBM
    is FSBM (same vectors, SAD, J, R); only the candidate count differs by the
    PBM overhead."""
    cur, ref = _acbm_inputs()
    for lam in (0, 3):
        prm = oracle.Params(lam=lam, qp=5, alpha=0, beta=0, gamma_num=0, gamma_den=1)
        a = oracle.acbm_frame(cur, ref, 16, 16, 5, prm)
        f = oracle.fsbm_frame(cur, ref, 16, 16, 5, prm)
        for k in ("mv_x", "mv_y", "sad", "j", "rate_bits"):
            assert np.array_equal(a[k], f[k]), k
        assert (a["mode"] == 3).all()
        assert (a["cands"] > f["cands"]).all()


def pin_acbm_reduces_to_pbm():
    """gamma = 0 and alpha > 2*255*N*M make the first test hold on every block
    (Section 3.2: the thresholds can avoid the full search everywhere), so
    ACBM is PBM."""
    cur, ref = _acbm_inputs()
    prev = _prev_for(cur, 16, 16, 5, 77)
    for lam in (0, 5):
        prm = oracle.Params(lam=lam, qp=0, alpha=2 * 255 * 256 + 1, beta=0, gamma_num=0,
                            gamma_den=1)
        a = oracle.acbm_frame(cur, ref, 16, 16, 5, prm, prev_field=prev)
        b = oracle.pbm_frame(cur, ref, 16, 16, 5, prm, prev_field=prev)
        for k in ("mv_x", "mv_y", "sad", "j", "rate_bits", "cands", "intra_x"):
            assert np.array_equal(a[k], b[k]), k
        assert (a["mode"] == 1).all() and (b["mode"] == 4).all()


def pin_pbm_properties():
    """PBM evaluates at most 14 predictors plus an 8-neighbour ring, and its
    result is never more expensive than the zero vector under the same
    predictor."""
    cur, ref = _acbm_inputs()
    lam = 2
    res = oracle.pbm_frame(cur, ref, 16, 16, 5, oracle.Params(lam=lam))
    by, bx = res.shape
    field = {(r, c): (int(res["mv_x"][r, c]), int(res["mv_y"][r, c])) for r in range(by) for c in range(bx)}
    for r in range(by):
        for c in range(bx):
            assert 1 <= int(res["cands"][r, c]) <= 22
            px, py = brute.predictor(field, r, c, bx)
            g = oracle.geom(cur, 16, 16, 5)
            j0 = oracle.sad(cur, ref, g, r, c, 0, 0) + lam * (oracle.se_bits(-px) + oracle.se_bits(-py))
            assert int(res["j"][r, c]) <= j0


def pin_sequence_chaining():
    """A sequence feeds each pair's field to the next pair as its temporal
    neighbourhood; the first pair sees a zero field."""
    wl = synth.cif_scene(nframes=3)
    frames = [f[:96, :128].copy() for f in wl.frames]
    prm = oracle.Params(lam=8, qp=8)
    seq = oracle.sequence(frames, 16, 16, 6, prm, oracle.ACBM)
    a1 = oracle.acbm_frame(frames[1], frames[0], 16, 16, 6, prm, prev_field=None)
    a2 = oracle.acbm_frame(frames[2], frames[1], 16, 16, 6, prm, prev_field=oracle.field_of(a1))
    assert np.array_equal(seq[0], a1) and np.array_equal(seq[1], a2)
    f = oracle.sequence(frames, 16, 16, 6, prm, oracle.FSBM)
    assert np.array_equal(f[1], oracle.fsbm_frame(frames[2], frames[1], 16, 16, 6, prm))


def pin_sad_deviation():
    """SAD_deviation (Section 3.1) against the numpy table: zero for a flat
    window, and the sum of (SAD - SAD_min) otherwise."""
    cur = synth.texture(48, 48, 1.5, synth.rng(81))
    ref = synth.texture(48, 48, 1.5, synth.rng(82))
    tab = _numpy_sad_table(cur, ref, 16, 16, 4)
    for (r, c) in [(0, 0), (1, 1), (2, 1)]:
        s = tab[r, c][tab[r, c] != 0xFFFFFFFF].astype(np.int64)
        dev, mn = oracle.sad_deviation(cur, ref, 16, 16, 4, r, c)
        assert mn == int(s.min()) and dev == int((s - s.min()).sum())
    flat = np.full((48, 48), 9, np.uint8)
    assert oracle.sad_deviation(flat, flat, 16, 16, 4, 1, 1) == (0, 0)


def pin_strict_inequalities():
    """Both ACBM tests are strict (Section 3.2).  With p = 0 the only
    candidate is (0, 0), so SAD_PBM is known exactly and each test can be put
    on its boundary: equality must not accept the PBM result."""
    nm = 256
    # first test: flat block (Intra_SAD = 0) against a flat reference 3 levels
    # away, SAD_PBM = 768; alpha = 768, beta = 0 sits on the boundary
    cur = np.full((16, 16), 100, np.uint8)
    ref = np.full((16, 16), 103, np.uint8)
    for alpha, mode in ((768, 3), (769, 1)):
        res = oracle.acbm_frame(cur, ref, 16, 16, 0, oracle.Params(lam=0, qp=0, alpha=alpha, beta=0))
        assert int(res["sad"][0, 0]) == 768 and int(res["intra_x"][0, 0]) == 0
        assert int(res["mode"][0, 0]) == mode, (alpha, int(res["mode"][0, 0]))
    # with beta: alpha + beta * Qp^2 = 700 + 2 * 36 = 772 > 768 accepts, 764 < 768 does not
    for qp, mode in ((6, 1), (4, 3)):
        res = oracle.acbm_frame(cur, ref, 16, 16, 0, oracle.Params(lam=0, qp=qp, alpha=700, beta=2))
        assert int(res["mode"][0, 0]) == mode
    # second test: half-black / half-white block, Intra_SAD = 127.5 * 256,
    # SAD_PBM = 8160 makes 4 * SAD_PBM equal to Intra_SAD (gamma = 1/4)
    cur = np.zeros((16, 16), np.uint8)
    cur[:, 8:] = 255
    for extra, mode in ((0, 3), (-1, 2)):
        ref = cur.copy()
        low = ref[:, :8].reshape(-1)
        low[:96] = 64
        low[96:] = 63
        if extra:
            low[0] = 63
        ref[:, :8] = low.reshape(16, 8)
        res = oracle.acbm_frame(cur, ref, 16, 16, 0, oracle.Params(lam=0, qp=0))
        assert int(res["intra_x"][0, 0]) == nm * nm * 255 // 2
        assert int(res["sad"][0, 0]) == 8160 + extra
        assert int(res["mode"][0, 0]) == mode, (extra, int(res["mode"][0, 0]))


ALL_PINS = [pin_strict_inequalities, 
    pin_se_codewords, pin_se_closed_form, pin_paper_counts, pin_valid_counts,
    pin_sad_table_numpy, pin_sad_planted_zero, pin_intra_exact, pin_median_rules,
    pin_fsbm_lambda0_global_min, pin_brute_fsbm, pin_brute_pbm, pin_brute_acbm,
    pin_planted_recovery, pin_fsbm_bounds_acbm, pin_acbm_reduces_to_fsbm,
    pin_acbm_reduces_to_pbm, pin_pbm_properties, pin_sequence_chaining, pin_sad_deviation,
]


def run_all(lib_path: str | None = None) -> list:
    """Run every pin (optionally on another build of the oracle); return the
    names of the pins that failed."""
    import contextlib
    failed = []
    ctx = oracle.using_library(lib_path) if lib_path else contextlib.nullcontext()
    with ctx:
        for pin in ALL_PINS:
            try:
                pin()
            except AssertionError:
                failed.append(pin.__name__)
    return failed




def pin_block_matches_raster():
    """The single-block entry point reproduces every block of whole raster
    runs when handed the final vectors of the blocks before it."""
    cur, ref = _acbm_inputs()
    prev = _prev_for(cur, 16, 16, 5, 91)
    prm = oracle.Params(lam=3, qp=3, alpha=150, beta=1)
    for algo, run in ((oracle.FSBM, lambda: oracle.fsbm_frame(cur, ref, 16, 16, 5, prm)),
                      (oracle.PBM, lambda: oracle.pbm_frame(cur, ref, 16, 16, 5, prm, prev)),
                      (oracle.ACBM, lambda: oracle.acbm_frame(cur, ref, 16, 16, 5, prm, prev))):
        res = run()
        by, bx = res.shape
        for r in range(by):
            for c in range(bx):
                one = oracle.block(cur, ref, 16, 16, 5, prm, algo, res["mv_x"], res["mv_y"], r, c,
                                   prev_field=None if algo == oracle.FSBM else prev)
                assert one == res[r, c], (algo, r, c)


ALL_PINS.append(pin_block_matches_raster)


# ----------------------------------------------------------------------------
# half-pel precision
# ----------------------------------------------------------------------------
def _half_frame_from(ref, U, V):
    """The frame whose every pixel is ref's half-pel sample at (2x + U, 2y + V)
    (brute force's sampler), ref's own pixel where that sample would leave
    the frame."""
    h, w = ref.shape
    rows = brute.as_lists(ref)
    out = ref.copy()
    for y in range(h):
        for x in range(w):
            X, Y = 2 * x + U, 2 * y + V
            if 0 <= X // 2 and X // 2 + (X & 1) < w and 0 <= Y // 2 and Y // 2 + (Y & 1) < h:
                out[y, x] = brute.half_sample(rows, X, Y)
    return out


def pin_half_sample_values():
    """Hand-worked H.263 half-pel samples (rounding half up), and the brute
    force's sampler on the same values."""
    with open(golden("half_pel_samples.txt")) as f:
        rows = [l.split("#")[0].split() for l in f if l.strip() and not l.startswith("#")]
    for kind, A, B, C, D, want in rows:
        A, B, C, D, want = int(A), int(B), int(C), int(D), int(want)
        ref = np.array([[A, B, 0], [C, D, 0], [0, 0, 0]], np.uint8)
        g = oracle.geom(ref, 1, 1, 0)
        X, Y = {"h": (1, 0), "v": (0, 1), "d": (1, 1)}[kind]
        assert oracle.ref_half(ref, g, X, Y) == want, (kind, A, B, C, D)
        assert brute.half_sample(brute.as_lists(ref), X, Y) == want


def pin_half_sample_brute():
    """Every half-pel sample of a small frame equals the brute force's, and
    even coordinates are the integer pixels themselves."""
    ref = _noise(7, 9, 611)
    g = oracle.geom(ref, 1, 1, 0)
    rows = brute.as_lists(ref)
    for Y in range(0, 2 * 7 - 1):
        for X in range(0, 2 * 9 - 1):
            assert oracle.ref_half(ref, g, X, Y) == brute.half_sample(rows, X, Y), (X, Y)
            if X % 2 == 0 and Y % 2 == 0:
                assert oracle.ref_half(ref, g, X, Y) == int(ref[Y // 2, X // 2])


def pin_half_valid_and_sad():
    """Half-pel validity and SAD against brute force over whole windows
    (negative and odd displacements at every border included); on the even
    grid they reduce to the integer validity and SAD."""
    for (h, w, bw, bh, p, seed) in [(12, 16, 4, 4, 2, 621), (16, 12, 8, 4, 3, 622)]:
        cur, ref = _noise(h, w, seed), _noise(h, w, seed + 1)
        g = oracle.geom(cur, bw, bh, p)
        cl, rl = brute.as_lists(cur), brute.as_lists(ref)
        for r in range(h // bh):
            for c in range(w // bw):
                x0, y0 = c * bw, r * bh
                for V in range(-2 * p - 1, 2 * p + 2):
                    for U in range(-2 * p - 1, 2 * p + 2):
                        ok = brute.half_valid(w, h, bw, bh, p, x0, y0, U, V)
                        assert oracle.is_valid_half(g, r, c, U, V) == ok, (r, c, U, V)
                        if U % 2 == 0 and V % 2 == 0:
                            assert ok == oracle.is_valid(g, r, c, U // 2, V // 2)
                        if ok:
                            s = oracle.sad_half(cur, ref, g, r, c, U, V)
                            assert s == brute.half_sad(cl, rl, x0, y0, bw, bh, U, V), (r, c, U, V)
                            if U % 2 == 0 and V % 2 == 0:
                                assert s == oracle.sad(cur, ref, g, r, c, U // 2, V // 2)


def _half_cases():
    return [cs for i, cs in enumerate(_tiny_cases()) if i % 3 == 0]


def pin_brute_half():
    """FSBM, PBM and ACBM with half-pel precision against the brute force on
    tiny frames of every kind (with temporal fields in half-pel units)."""
    for i, (cur, ref, bw, bh, p) in enumerate(_half_cases()):
        lam = [0, 1, 4, 32][i % 4]
        cl, rl = brute.as_lists(cur), brute.as_lists(ref)
        got = oracle.fsbm_frame(cur, ref, bw, bh, p, oracle.Params(lam=lam, subpel=1))
        _same(got, brute.fsbm(cl, rl, bw, bh, p, lam, half=True), f"half fsbm case {i}")
        prev = None
        if i % 2:
            prev = _prev_for(cur, bw, bh, 2 * p, 970 + i)
        pv = None if prev is None else {(r, c): (int(prev[r, c, 0]), int(prev[r, c, 1]))
                                        for r in range(prev.shape[0]) for c in range(prev.shape[1])}
        got = oracle.pbm_frame(cur, ref, bw, bh, p, oracle.Params(lam=lam, subpel=1),
                               prev_field=prev)
        _same(got, brute.predictive(cl, rl, bw, bh, p, lam, prev=pv, half=True),
              f"half pbm case {i}")
        nm = bw * bh
        prm = oracle.Params(lam=lam, qp=lam, alpha=[0, 3, 40, 1000][i % 4] * nm // 16,
                            beta=[0, 1, 2, 8][(i // 4) % 4], gamma_num=1,
                            gamma_den=[1, 4, 2, 4][(i // 2) % 4], subpel=1)
        got = oracle.acbm_frame(cur, ref, bw, bh, p, prm, prev_field=prev)
        want = brute.predictive(cl, rl, bw, bh, p, lam, prev=pv, half=True,
                                acbm=(prm.alpha, prm.beta, prm.qp, prm.gamma_num, prm.gamma_den))
        _same(got, want, f"half acbm case {i}")


def pin_half_table1_count():
    """Table 1 / Section 4: full search at p = 15 evaluates 969 positions per
    interior macroblock with half-pel precision (961 integer + 8 half-pel)."""
    kv = read_kv("paper_counts.txt")
    p, want = int(kv["p"]), int(kv["fsbm_positions_p15_halfpel"])
    ref = synth.texture(96, 96, 1.5, synth.rng(631))
    cur = synth.add_noise(np.roll(ref, (1, -1), (0, 1)), 1.0, synth.rng(632))
    res = oracle.fsbm_frame(cur, ref, 16, 16, p, oracle.Params(lam=2, subpel=1))
    inner = res[1:5, 1:5]  # blocks with the whole +-15 window inside the frame
    assert (inner["cands"] == want).all(), inner["cands"]


def pin_half_planted():
    """Planted half-pel motion (the Section 3.1 method on the half grid):
    the current frame is the reference sampled at a known half-pel offset by
    the brute force's sampler, so the planted vector has SAD 0 and FSBM with
    lambda = 0 must return it on every block where it is valid.  And on the
    even grid the half-pel search starts from the integer one: its SAD is
    never above the integer FSBM's, and an even result is twice that vector."""
    ref = synth.texture(48, 64, 1.5, synth.rng(641))
    for (U, V) in [(3, -1), (-2, 1), (1, 1), (0, -3)]:
        cur = _half_frame_from(ref, U, V)
        g = oracle.geom(cur, 16, 16, 3)
        half = oracle.fsbm_frame(cur, ref, 16, 16, 3, oracle.Params(lam=0, subpel=1))
        full = oracle.fsbm_frame(cur, ref, 16, 16, 3, oracle.Params(lam=0))
        by, bx = half.shape
        checked = 0
        for r in range(by):
            for c in range(bx):
                assert int(half["sad"][r, c]) <= int(full["sad"][r, c])
                hx, hy = int(half["mv_x"][r, c]), int(half["mv_y"][r, c])
                if hx % 2 == 0 and hy % 2 == 0:
                    assert (hx // 2, hy // 2) == (int(full["mv_x"][r, c]), int(full["mv_y"][r, c]))
                x0, y0 = c * 16, r * 16
                # the planted samples cover the block only away from the borders
                if not (1 <= x0 and x0 + 17 <= 64 and 1 <= y0 and y0 + 17 <= 48):
                    continue
                if oracle.is_valid_half(g, r, c, U, V):
                    assert (hx, hy, int(half["sad"][r, c])) == (U, V, 0), (U, V, r, c)
                    checked += 1
        assert checked >= 2, (U, V)


ALL_PINS += [pin_half_sample_values, pin_half_sample_brute, pin_half_valid_and_sad,
             pin_brute_half, pin_half_table1_count, pin_half_planted]


def _hostile_prev(cur, bw, bh, p, s, seed):
    """A previous field in which most blocks carry a vector that is not a
    valid candidate: beyond +-s*p, beyond a signed byte, at the int16 limits,
    and values that equal a small valid vector modulo 256."""
    by, bx = cur.shape[0] // bh, cur.shape[1] // bw
    special = [(256, 1), (200, 0), (-200, 3), (128, 0), (-129, -1), (-32768, 0), (32767, 1),
               (0, -32768), (s * p + 1, 0), (0, -(s * p + 1)), (2 * s * p + 1, 1), (-253, 2),
               (259, -1), (1, 258)]
    g = synth.rng(seed)
    prev = g.integers(-s * p, s * p + 1, size=(by, bx, 2)).astype(np.int16)
    for r in range(by):
        for c in range(bx):
            if g.random() < 0.7:
                prev[r, c] = special[int(g.integers(0, len(special)))]
    return prev


def pin_brute_hostile_prev():
    """Section 2.2's predictor set takes the previous field's vectors as
    candidates; one that is not a valid candidate is dropped (not clamped,
    not wrapped).  PBM and ACBM with such fields, at integer and half-pel
    precision, against the brute force."""
    for i, (cur, ref, bw, bh, p) in enumerate(_tiny_cases()):
        if i % 2:
            continue
        subpel = (i // 2) % 2
        s = 2 if subpel else 1
        lam = [0, 1, 4, 32][(i // 2) % 4]
        prev = _hostile_prev(cur, bw, bh, p, s, 1200 + i)
        pv = {(r, c): (int(prev[r, c, 0]), int(prev[r, c, 1]))
              for r in range(prev.shape[0]) for c in range(prev.shape[1])}
        cl, rl = brute.as_lists(cur), brute.as_lists(ref)
        got = oracle.pbm_frame(cur, ref, bw, bh, p, oracle.Params(lam=lam, subpel=subpel),
                               prev_field=prev)
        _same(got, brute.predictive(cl, rl, bw, bh, p, lam, prev=pv, half=bool(subpel)),
              f"hostile pbm case {i}")
        nm = bw * bh
        prm = oracle.Params(lam=lam, qp=lam, alpha=[0, 3, 40, 1000][i % 4] * nm // 16,
                            beta=[0, 1, 2, 8][(i // 4) % 4], gamma_num=1,
                            gamma_den=[1, 4, 2, 4][(i // 2) % 4], subpel=subpel)
        got = oracle.acbm_frame(cur, ref, bw, bh, p, prm, prev_field=prev)
        want = brute.predictive(cl, rl, bw, bh, p, lam, prev=pv, half=bool(subpel),
                                acbm=(prm.alpha, prm.beta, prm.qp, prm.gamma_num, prm.gamma_den))
        _same(got, want, f"hostile acbm case {i}")


ALL_PINS.append(pin_brute_hostile_prev)


if __name__ == "__main__":
    import sys
    bad = run_all(sys.argv[1] if len(sys.argv) > 1 else None)
    print(" ".join(bad) if bad else "all pins hold")
    sys.exit(1 if bad else 0)
