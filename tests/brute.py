"""Brute-force restatement of the ACBM definitions in pure Python.

Written separately from the C oracle (no shared code, no shared tables) and
meant only for tiny frames.  Frames are lists of rows of ints.  It checks the
oracle on inputs small enough to enumerate, with the same readings of the
paper: candidates wholly inside the reference frame, median-of-three
predictor with the usual picture-edge substitutions, signed Exp-Golomb rate,
ties broken by J, then |u|+|v|, then window raster order.
"""
from __future__ import annotations


def codeword_se(k: int) -> str:
    """Signed Exp-Golomb codeword of k as a bit string."""
    code = 2 * k - 1 if k > 0 else -2 * k
    tail = bin(code + 1)[2:]
    return "0" * (len(tail) - 1) + tail


def decode_se(bits: str, at: int) -> tuple[int, int]:
    """Decode one signed Exp-Golomb codeword starting at bit `at`."""
    zeros = 0
    while bits[at + zeros] == "0":
        zeros += 1
    val = int(bits[at + zeros: at + 2 * zeros + 1], 2) - 1
    k = (val + 1) // 2 if val % 2 == 1 else -(val // 2)
    return k, at + 2 * zeros + 1


def rate(du: int, dv: int) -> int:
    return len(codeword_se(du)) + len(codeword_se(dv))


def candidates(width, height, bw, bh, p, x0, y0):
    """Valid displacements of the block at (x0, y0) in window raster order."""
    out = []
    for v in range(-p, p + 1):
        for u in range(-p, p + 1):
            if 0 <= x0 + u and x0 + u + bw <= width and 0 <= y0 + v and y0 + v + bh <= height:
                out.append((u, v))
    return out


def sad(cur, ref, x0, y0, bw, bh, u, v) -> int:
    total = 0
    for yy in range(y0, y0 + bh):
        row_c, row_r = cur[yy], ref[yy + v]
        for xx in range(x0, x0 + bw):
            d = row_c[xx] - row_r[xx + u]
            total += d if d >= 0 else -d
    return total


def intra_x(cur, x0, y0, bw, bh) -> int:
    pix = [cur[yy][xx] for yy in range(y0, y0 + bh) for xx in range(x0, x0 + bw)]
    s, n = sum(pix), len(pix)
    return sum(abs(n * q - s) for q in pix)


def predictor(field, r, c, bx):
    left = field[(r, c - 1)] if c > 0 else (0, 0)
    if r == 0:
        top = right = left
    else:
        top = field[(r - 1, c)]
        right = field[(r - 1, c + 1)] if c + 1 < bx else (0, 0)
    return (sorted([left[0], top[0], right[0]])[1], sorted([left[1], top[1], right[1]])[1])


def _key(s, u, v, pred, lam, p):
    R = rate(u - pred[0], v - pred[1])
    return (s + lam * R, abs(u) + abs(v), (v + p) * (2 * p + 1) + (u + p)), R


def _pick(cur, ref, x0, y0, bw, bh, cands, pred, lam, p):
    best = None
    for (u, v) in cands:
        s = sad(cur, ref, x0, y0, bw, bh, u, v)
        k, R = _key(s, u, v, pred, lam, p)
        if best is None or k < best[0]:
            best = (k, u, v, s, R)
    k, u, v, s, R = best
    return {"mv_x": u, "mv_y": v, "sad": s, "j": k[0], "rate_bits": R}


def _grid(cur, bw, bh):
    return len(cur[0]) // bw, len(cur) // bh


def fsbm(cur, ref, bw, bh, p, lam):
    width, height = len(cur[0]), len(cur)
    bx, by = _grid(cur, bw, bh)
    field, out = {}, {}
    for r in range(by):
        for c in range(bx):
            x0, y0 = c * bw, r * bh
            cands = candidates(width, height, bw, bh, p, x0, y0)
            res = _pick(cur, ref, x0, y0, bw, bh, cands, predictor(field, r, c, bx), lam, p)
            res.update(cands=len(cands), mode=0, intra_x=intra_x(cur, x0, y0, bw, bh))
            out[(r, c)] = res
            field[(r, c)] = (res["mv_x"], res["mv_y"])
    return out


def _pbm(cur, ref, bw, bh, p, lam, field, prev, r, c, pred):
    width, height = len(cur[0]), len(cur)
    bx, by = _grid(cur, bw, bh)
    x0, y0 = c * bw, r * bh
    valid = set(candidates(width, height, bw, bh, p, x0, y0))
    raw = [(0, 0)]
    for (dr, dc) in ((0, -1), (-1, -1), (-1, 0), (-1, 1)):
        if (r + dr, c + dc) in field:
            raw.append(field[(r + dr, c + dc)])
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            if 0 <= r + dr < by and 0 <= c + dc < bx:
                raw.append(prev[(r + dr, c + dc)] if prev is not None else (0, 0))
    pset = []
    for mv in raw:
        if mv in valid and mv not in pset:
            pset.append(mv)
    first = _pick(cur, ref, x0, y0, bw, bh, pset, pred, lam, p)
    ring = []
    for dv in (-1, 0, 1):
        for du in (-1, 0, 1):
            mv = (first["mv_x"] + du, first["mv_y"] + dv)
            if (du, dv) != (0, 0) and mv in valid and mv not in pset and mv not in ring:
                ring.append(mv)
    res = _pick(cur, ref, x0, y0, bw, bh, pset + ring, pred, lam, p)
    return res, len(pset) + len(ring)


def predictive(cur, ref, bw, bh, p, lam, prev=None, acbm=None):
    """PBM (acbm None) or ACBM (acbm = (alpha, beta, qp, gamma_num, gamma_den))."""
    width, height = len(cur[0]), len(cur)
    bx, by = _grid(cur, bw, bh)
    field, out = {}, {}
    nm = bw * bh
    for r in range(by):
        for c in range(bx):
            x0, y0 = c * bw, r * bh
            pred = predictor(field, r, c, bx)
            ix = intra_x(cur, x0, y0, bw, bh)
            res, n = _pbm(cur, ref, bw, bh, p, lam, field, prev, r, c, pred)
            mode = 4
            if acbm is not None:
                alpha, beta, qp, gn, gd = acbm
                # Intra_SAD = ix / nm exactly; compare with fractions cleared
                if ix + nm * res["sad"] < nm * (alpha + beta * qp * qp):
                    mode = 1
                elif gd * nm * res["sad"] < gn * ix:
                    mode = 2
                else:
                    mode = 3
                    cands = candidates(width, height, bw, bh, p, x0, y0)
                    res = _pick(cur, ref, x0, y0, bw, bh, cands, pred, lam, p)
                    n += len(cands)
            res.update(cands=n, mode=mode, intra_x=ix)
            out[(r, c)] = res
            field[(r, c)] = (res["mv_x"], res["mv_y"])
    return out


def as_lists(a):
    return [list(map(int, row)) for row in a]
