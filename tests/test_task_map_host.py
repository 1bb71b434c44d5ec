"""The window searches' lane -> task map, on the host: for every search range
p <= 127 and every row blocking R the kernels are built for, the map that
puts the tasks holding padding candidates on the highest lanes (task_of in
the device header) is a bijection onto quads x row groups, every task it
calls interior holds only candidates with |u|, |v| <= p, and the exact
multiply-high division it uses agrees with integer division.  The same
arithmetic as the device code, written out in Python; the GPU test of the
real kernels at every R is tests/test_gpu_task_map.py."""


def window(p, R):
    u_lo = -4 * ((p + 3) // 4)
    quads = (p - u_lo + 1 + 3) // 4
    groups = (2 * p + 1 + R - 1) // R
    return u_lo, quads, groups


def task_of(p, R, t):
    u_lo, quads, groups = window(p, R)
    q_lo = 1 if u_lo < -p else 0
    q_hi = 1 if u_lo + 4 * quads - 1 > p else 0
    g_hi = 1 if groups * R > 2 * p + 1 else 0
    iq = quads - q_lo - q_hi
    imagic = (((1 << 32) + iq - 1) // iq) & 0xFFFFFFFF if iq > 1 else 0
    interior = iq * (groups - g_hi)
    if t < interior:
        g = t if iq == 1 else (t * imagic) >> 32
        assert g == t // iq
        return q_lo + (t - g * iq), g, False
    e = t - interior
    ncol = q_lo + q_hi
    if e < ncol * groups:
        c = (e & 1) if ncol == 2 else 0
        gi = (e >> 1) if ncol == 2 else e
        return (0 if (c == 0 and q_lo) else quads - 1), gi, True
    return q_lo + (e - ncol * groups), groups - 1, True


def test_task_map_every_p_and_r():
    for p in range(128):
        for R in (1, 2, 3, 4, 5, 6, 8, 11, 16):
            u_lo, quads, groups = window(p, R)
            seen = set()
            for t in range(quads * groups):
                q, gi, edge = task_of(p, R, t)
                assert 0 <= q < quads and 0 <= gi < groups, (p, R, t)
                seen.add((q, gi))
                if not edge:
                    us = [u_lo + 4 * q + i for i in range(4)]
                    vs = [-p + R * gi + r for r in range(R)]
                    assert all(abs(u) <= p for u in us) and all(abs(v) <= p for v in vs), (p, R, t)
            assert len(seen) == quads * groups, (p, R)
