"""Brute-force restatement of the ACBM definitions in pure Python.

Written separately from the C oracle (no shared code, no shared tables) and
meant only for tiny frames.  Frames are lists of rows of ints.  It checks the
oracle on inputs small enough to enumerate, with the same readings of the
paper: candidates wholly inside the reference frame, median-of-three
predictor with the usual picture-edge substitutions, signed Exp-Golomb rate,
ties broken by J, then |u|+|v|, then window raster order.  Half-pel
precision samples the reference with H.263's bilinear interpolation.
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


def half_sample(ref, X, Y) -> int:
    """Reference value at half-pel coordinates (X, Y): H.263's bilinear rule,
    averages rounded half up (the diagonal: sum of four plus 2, over 4)."""
    x, fx = divmod(X, 2)
    y, fy = divmod(Y, 2)
    assert x >= 0 and y >= 0, "outside the frame"
    a = ref[y][x]
    if fx == 0 and fy == 0:
        return a
    if fy == 0:
        return (a + ref[y][x + 1] + 1) // 2
    if fx == 0:
        return (a + ref[y + 1][x] + 1) // 2
    return (a + ref[y][x + 1] + ref[y + 1][x] + ref[y + 1][x + 1] + 2) // 4


def half_valid(width, height, bw, bh, p, x0, y0, U, V) -> bool:
    """A half-pel displacement is valid when |U|, |V| <= 2p and every
    reference pixel any block pixel interpolates from is inside the frame."""
    if abs(U) > 2 * p or abs(V) > 2 * p:
        return False
    for j in range(bh):
        for i in range(bw):
            x, fx = divmod(2 * (x0 + i) + U, 2)
            y, fy = divmod(2 * (y0 + j) + V, 2)
            for xx in (x, x + fx):
                for yy in (y, y + fy):
                    if not (0 <= xx < width and 0 <= yy < height):
                        return False
    return True


def half_sad(cur, ref, x0, y0, bw, bh, U, V) -> int:
    total = 0
    for yy in range(y0, y0 + bh):
        for xx in range(x0, x0 + bw):
            d = cur[yy][xx] - half_sample(ref, 2 * xx + U, 2 * yy + V)
            total += d if d >= 0 else -d
    return total


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
    """p here is the window half-size in the units of u and v (2p for
    half-pel vectors)."""
    R = rate(u - pred[0], v - pred[1])
    return (s + lam * R, abs(u) + abs(v), (v + p) * (2 * p + 1) + (u + p)), R


def _pick(cur, ref, x0, y0, bw, bh, cands, pred, lam, p, half=False):
    """Cheapest of `cands` (integer vectors, or half-pel ones with half)."""
    best = None
    for (u, v) in cands:
        s = half_sad(cur, ref, x0, y0, bw, bh, u, v) if half else sad(cur, ref, x0, y0, bw, bh, u, v)
        k, R = _key(s, u, v, pred, lam, 2 * p if half else p)
        if best is None or k < best[0]:
            best = (k, u, v, s, R)
    k, u, v, s, R = best
    return {"mv_x": u, "mv_y": v, "sad": s, "j": k[0], "rate_bits": R}


def _full(cur, ref, x0, y0, bw, bh, p, pred, lam, half):
    """Full search of one block: the valid integer window; with half, then
    the valid half-pel 8-neighbours of the integer winner.  Returns the
    result and the number of positions evaluated."""
    width, height = len(cur[0]), len(cur)
    ints = candidates(width, height, bw, bh, p, x0, y0)
    if not half:
        return _pick(cur, ref, x0, y0, bw, bh, ints, pred, lam, p), len(ints)
    evens = [(2 * u, 2 * v) for (u, v) in ints]
    first = _pick(cur, ref, x0, y0, bw, bh, evens, pred, lam, p, half=True)
    ring = []
    for dv in (-1, 0, 1):
        for du in (-1, 0, 1):
            mv = (first["mv_x"] + du, first["mv_y"] + dv)
            if (du, dv) != (0, 0) and half_valid(width, height, bw, bh, p, x0, y0, *mv):
                ring.append(mv)
    return _pick(cur, ref, x0, y0, bw, bh, evens + ring, pred, lam, p, half=True), \
        len(evens) + len(ring)


def _grid(cur, bw, bh):
    return len(cur[0]) // bw, len(cur) // bh


def fsbm(cur, ref, bw, bh, p, lam, half=False):
    bx, by = _grid(cur, bw, bh)
    field, out = {}, {}
    for r in range(by):
        for c in range(bx):
            x0, y0 = c * bw, r * bh
            res, n = _full(cur, ref, x0, y0, bw, bh, p, predictor(field, r, c, bx), lam, half)
            res.update(cands=n, mode=0, intra_x=intra_x(cur, x0, y0, bw, bh))
            out[(r, c)] = res
            field[(r, c)] = (res["mv_x"], res["mv_y"])
    return out


def _pbm(cur, ref, bw, bh, p, lam, field, prev, r, c, pred, half=False):
    width, height = len(cur[0]), len(cur)
    bx, by = _grid(cur, bw, bh)
    x0, y0 = c * bw, r * bh
    if half:
        valid = {(U, V) for V in range(-2 * p, 2 * p + 1) for U in range(-2 * p, 2 * p + 1)
                 if half_valid(width, height, bw, bh, p, x0, y0, U, V)}
    else:
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
    first = _pick(cur, ref, x0, y0, bw, bh, pset, pred, lam, p, half)
    ring = []
    for dv in (-1, 0, 1):
        for du in (-1, 0, 1):
            mv = (first["mv_x"] + du, first["mv_y"] + dv)
            if (du, dv) != (0, 0) and mv in valid and mv not in pset and mv not in ring:
                ring.append(mv)
    res = _pick(cur, ref, x0, y0, bw, bh, pset + ring, pred, lam, p, half)
    return res, len(pset) + len(ring)


def predictive(cur, ref, bw, bh, p, lam, prev=None, acbm=None, half=False):
    """PBM (acbm None) or ACBM (acbm = (alpha, beta, qp, gamma_num, gamma_den));
    with half, every vector is in half-pel units and the refinement ring is
    one half-pel step."""
    bx, by = _grid(cur, bw, bh)
    field, out = {}, {}
    nm = bw * bh
    for r in range(by):
        for c in range(bx):
            x0, y0 = c * bw, r * bh
            pred = predictor(field, r, c, bx)
            ix = intra_x(cur, x0, y0, bw, bh)
            res, n = _pbm(cur, ref, bw, bh, p, lam, field, prev, r, c, pred, half)
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
                    res, nf = _full(cur, ref, x0, y0, bw, bh, p, pred, lam, half)
                    n += nf
            res.update(cands=n, mode=mode, intra_x=ix)
            out[(r, c)] = res
            field[(r, c)] = (res["mv_x"], res["mv_y"])
    return out


def as_lists(a):
    return [list(map(int, row)) for row in a]
