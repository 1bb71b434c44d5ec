"""The autotuner's cache (ACBM_TUNE_CACHE): a process that tunes a shape
appends its plan to the file, and a second process takes the plan from there
without timing anything (no window-search launch).  8x8 blocks on an even
grid tune the tiled search, which the cache marks as such."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROG = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_0710_4819_amd import acbm
torch.cuda.init()
acbm.profile_enable(True)
acbm.profile_reset()
R, ms = acbm.autotune(int(sys.argv[2]), int(sys.argv[2]), 16, 352, 288)
torch.cuda.synchronize()
_, n = acbm.profile_read("search")
print(json.dumps({"R": R, "ms": ms, "search_launches": n}), flush=True)
"""


def _run(cache, block):
    env = dict(os.environ, ACBM_TUNE_CACHE=str(cache))
    p = subprocess.run([sys.executable, "-c", PROG, ROOT, str(block)], env=env,
                       capture_output=True, text=True, timeout=100)
    assert p.returncode == 0, p.stderr[-2000:]
    return json.loads(p.stdout.strip().splitlines()[-1])


@pytest.mark.parametrize("block", [16, 8])
def test_second_process_reuses_the_tuned_plan(tmp_path, block):
    cache = tmp_path / "tune.jsonl"
    print(f"first process: tunes CIF {block}x{block} p=16", flush=True)
    first = _run(cache, block)
    assert first["search_launches"] > 0 and first["R"] in (1, 2, 3, 4, 5, 6, 8, 11, 16)
    lines = [json.loads(l) for l in cache.read_text().splitlines() if l.strip()]
    assert lines and lines[-1]["R"] == first["R"] and lines[-1]["N"] == block
    assert lines[-1]["p"] == 16 and lines[-1]["arch"].startswith("gfx950")
    assert lines[-1].get("tile", 1) == (2 if block == 8 else 1)  # CIF 8x8: a 44x36 grid
    print("second process: reads the cache", flush=True)
    second = _run(cache, block)
    assert second["search_launches"] == 0, "the second process timed plans again"
    assert second["R"] == first["R"]
    assert abs(second["ms"] - first["ms"]) < 1e-5
