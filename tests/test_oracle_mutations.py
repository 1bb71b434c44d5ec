"""Plant plausible mistakes in the CPU oracle and require the pins to catch
each one.

Each mutation is a textual edit of ``oracle/acbm_oracle.c`` (a dropped term,
a wrong sign, a flipped comparison, a transposed operand, a wrong neighbour).
The edited copy is compiled into a temporary library and the whole pin suite
runs on it in a child process (a mutation may also crash; that counts as
caught).  The real oracle is never modified.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "acbm_oracle.c")

MUTATIONS = [
    ("sad_no_abs", "int b = ref[(y0 + j + v) * g->pitch + (x0 + i + u)];\n            s += (uint32_t)abs(a - b);",
     "int b = ref[(y0 + j + v) * g->pitch + (x0 + i + u)];\n            s += (uint32_t)(a - b);"),
    ("sad_sign_u", "ref[(y0 + j + v) * g->pitch + (x0 + i + u)]",
     "ref[(y0 + j + v) * g->pitch + (x0 + i - u)]"),
    ("sad_swap_uv", ": oracle_sad(g, cur, ref, r, c, u, v);",
     ": (oracle_is_valid(g, r, c, v, u) ? oracle_sad(g, cur, ref, r, c, v, u) : 0);"),
    ("se_len_plus", "return 2 * n - 1;", "return 2 * n + 1;"),
    ("se_zero_map", "(k > 0) ? (uint64_t)(2 * k - 1)", "(k >= 0) ? (uint64_t)(2 * k - 1)"),
    ("rate_drops_y", "(oracle_se_bits((int64_t)u - px) + oracle_se_bits((int64_t)v - py))",
     "(oracle_se_bits((int64_t)u - px) + oracle_se_bits((int64_t)v))"),
    ("valid_edge", "x0 + u + (long)g->block_w > (long)g->width",
     "x0 + u + (long)g->block_w >= (long)g->width"),
    ("valid_no_p", "if (u < -p || u > p || v < -p || v > p) return 0;", ""),
    ("median_min", "return v[1];", "return v[0];"),
    ("median_row0", "        bxv = ax; byv = ay;\n        cx = ax;  cy = ay;",
     "        bxv = 0; byv = 0;\n        cx = 0;  cy = 0;"),
    ("median_lastcol", "if (c == bx - 1) {", "if (c == bx) {"),
    ("intra_no_scale", "int64_t d = nm * (int64_t)cur", "int64_t d = (int64_t)cur"),
    ("j_drops_rate", "e.j = (uint64_t)e.sad + (uint64_t)prm->lambda * e.rate;",
     "e.j = (uint64_t)e.sad;"),
    ("tie_l1_flip", "if (a->l1 != b->l1) return a->l1 < b->l1;",
     "if (a->l1 != b->l1) return a->l1 > b->l1;"),
    ("tie_raster_flip", "return a->raster < b->raster;", "return a->raster > b->raster;"),
    ("pbm_tr_is_tl", "sdc[4] = {-1, -1, 0, 1};", "sdc[4] = {-1, -1, 0, -1};"),
    ("pbm_temporal_colocated_only", "for (int dr = -1; dr <= 1; dr++) {\n        for (int dc = -1; dc <= 1; dc++) {\n            int rr = r + dr, cc = c + dc;\n            if (rr < 0 || rr >= by",
     "for (int dr = 0; dr <= 0; dr++) {\n        for (int dc = 0; dc <= 0; dc++) {\n            int rr = r + dr, cc = c + dc;\n            if (rr < 0 || rr >= by"),
    ("pbm_no_ring", "if (du == 0 && dv == 0) continue;\n            int u = b0.u", "continue;\n            int u = b0.u"),
    ("c1_le", "int c1 = (u128)intra + nm * sad_p < nm * t1;",
     "int c1 = (u128)intra + nm * sad_p <= nm * t1;"),
    ("c1_qp_linear", "(u128)prm->beta * prm->qp * prm->qp", "(u128)prm->beta * prm->qp"),
    ("c2_gamma_swapped", "(u128)prm->gamma_den * nm * sad_p < (u128)prm->gamma_num * intra",
     "(u128)prm->gamma_num * nm * sad_p < (u128)prm->gamma_den * intra"),
    ("c1_before_c2", "    if (c1) return 1;\n    if (c2) return 2;", "    if (c2) return 2;\n    if (c1) return 1;"),
    ("critical_zero_pred", "uint32_t n = full_search(g, prm, cur, ref, r, c, px, py, &fs);",
     "uint32_t n = full_search(g, prm, cur, ref, r, c, 0, 0, &fs);"),
    ("critical_count", "store(o, &fs, cands + n, 3, intra);", "store(o, &fs, n, 3, intra);"),
    # half-pel precision
    ("half_h_no_round", "(A + ref[y * g->pitch + x + 1] + 1) / 2", "(A + ref[y * g->pitch + x + 1]) / 2"),
    ("half_v_no_round", "(A + ref[(y + 1) * g->pitch + x] + 1) / 2",
     "(A + ref[(y + 1) * g->pitch + x]) / 2"),
    ("half_diag_round", "ref[(y + 1) * g->pitch + x + 1] + 2) / 4", "ref[(y + 1) * g->pitch + x + 1] + 1) / 4"),
    ("half_diag_as_h", "if (fx && !fy) return", "if (fx) return"),
    ("half_v_uses_right", "(A + ref[(y + 1) * g->pitch + x] + 1) / 2",
     "(A + ref[y * g->pitch + x + 1] + 1) / 2"),
    ("half_floor_truncates", "return X >= 0 ? X / 2 : -((-X + 1) / 2);", "return X / 2;"),
    ("half_valid_no_extra", "+ (U & 1 ? 1 : 0);", ";"),
    ("half_valid_no_window", "if (U < -p2 || U > p2 || V < -p2 || V > p2) return 0;", ""),
    ("half_sad_sign", "oracle_ref_half(g, ref, 2 * (x0 + i) + U, 2 * (y0 + j) + V)",
     "oracle_ref_half(g, ref, 2 * (x0 + i) - U, 2 * (y0 + j) + V)"),
    ("fsbm_no_half_step", "if (prm->subpel) {\n        int cu", "if (0) {\n        int cu"),
    ("fsbm_half_around_origin", "int cu = best->u, cv = best->v;", "int cu = 0, cv = 0;"),
    ("fsbm_int_grid_unscaled", "evaluate(g, prm, cur, ref, r, c, s * u, s * v, px, py)",
     "evaluate(g, prm, cur, ref, r, c, u, v, px, py)"),
    ("pbm_ring_integer_step", "int u = b0.u + du, v = b0.v + dv;",
     "int u = b0.u + units(prm) * du, v = b0.v + units(prm) * dv;"),
    ("pbm_integer_validity", "if (!valid_in_units(g, prm, r, c, pu[k], pv[k])) continue;",
     "if (!oracle_is_valid(g, r, c, pu[k], pv[k])) continue;"),
    ("half_rate_integer_units", "e.rate = (uint32_t)(oracle_se_bits((int64_t)u - px) + oracle_se_bits((int64_t)v - py));",
     "e.rate = (uint32_t)(oracle_se_bits(((int64_t)u - px) / units(prm)) + oracle_se_bits(((int64_t)v - py) / units(prm)));"),
    ("prev_wraps_to_byte", "pu[np] = prev_field ? prev_field[2 * (rr * bx + cc) + 0] : 0;\n            pv[np] = prev_field ? prev_field[2 * (rr * bx + cc) + 1] : 0;",
     "pu[np] = prev_field ? (int8_t)prev_field[2 * (rr * bx + cc) + 0] : 0;\n            pv[np] = prev_field ? (int8_t)prev_field[2 * (rr * bx + cc) + 1] : 0;"),
    ("seq_field_transposed", "prev[2 * b + 0] = (int16_t)o[b].mv_x;\n            prev[2 * b + 1] = (int16_t)o[b].mv_y;",
     "prev[2 * b + 0] = (int16_t)o[b].mv_y;\n            prev[2 * b + 1] = (int16_t)o[b].mv_x;"),
]


def _run_mutation(tmp, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation {name}: anchor not found exactly once"
    mpath = os.path.join(tmp, f"{name}.c")
    with open(mpath, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(tmp, f"lib_{name}.so")
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-I", os.path.dirname(SRC),
                    mpath, "-o", lib], check=True, capture_output=True)
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([ROOT, os.path.join(ROOT, "tests")]))
    p = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "pins.py"), lib],
                       env=env, capture_output=True, text=True, timeout=300)
    return name, p.returncode, (p.stdout + p.stderr)[-400:]


def test_every_mutation_is_caught():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=6) as ex:
            results = list(ex.map(lambda m: _run_mutation(tmp, *m), MUTATIONS))
    survivors = [(n, out) for (n, rc, out) in results if rc == 0]
    assert not survivors, f"mutations not caught by any pin: {survivors}"


def test_unmutated_oracle_passes_in_child():
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([ROOT, os.path.join(ROOT, "tests")]))
    p = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "pins.py")], env=env,
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout + p.stderr
