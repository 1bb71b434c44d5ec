"""Every row blocking R against every kind of window edge: the window-search
kernels hand the tasks that hold padding candidates (a first quad below -p,
a last quad beyond +p, a last row group beyond +p) to the highest lanes, and
skip masking elsewhere for blocks whose whole window is valid.  The SAD table
and the tiled 8x8 FSBM search are compared with the oracle for p with each
combination of those edges, at each R the kernels are built for (ACBM_R
forces it; it is read at every call)."""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_0710_4819_amd import acbm, synth

from test_gpu_parity import dev, oparams, same, say

pytestmark = pytest.mark.gpu

# p % 4 == 0: no padding quad at -p; p % 4 == 3: none beyond +p either
P_VALUES = (1, 2, 3, 4, 5, 7, 8, 13, 16, 33)


def _frames(h, w, seed):
    ref = synth.texture(h, w, 2.0, synth.rng(seed))
    cur = synth.add_noise(np.roll(ref, (1, -2), (0, 1)), 2.0, synth.rng(seed + 1))
    return cur, ref


@pytest.fixture
def forced_rows():
    old = os.environ.get("ACBM_R")
    yield
    if old is None:
        os.environ.pop("ACBM_R", None)
    else:
        os.environ["ACBM_R"] = old


@pytest.mark.parametrize("p", P_VALUES)
def test_table_every_rows(p, forced_rows):
    cur, ref = _frames(80, 96, 700 + p)  # 16x16: 6 x 5 blocks, interior and border
    want = oracle.sad_table(cur, ref, 16, 16, p)
    for R in (1, 2, 3, 4, 5, 6, 8, 11, 16):
        os.environ["ACBM_R"] = str(R)
        say(f"task map: table 96x80 16x16 p={p} R={R}")
        try:
            got = acbm.table_to_numpy(acbm.sad_table(dev(cur), dev(ref), 16, 16, p))
        except acbm.AcbmError as e:
            assert e.status == acbm.E_UNSUPPORTED, e  # this R's plan does not fit
            continue
        torch.cuda.synchronize()
        assert np.array_equal(got, want), f"p={p} R={R}: {np.count_nonzero(got != want)} differ"


@pytest.mark.parametrize("p", P_VALUES)
def test_tiled_fsbm_every_rows(p, forced_rows):
    cur, ref = _frames(64, 80, 760 + p)  # 8x8: 10 x 8 blocks, 20 tiles
    prm = acbm.Params(lam=8, qp=8)
    want = oracle.fsbm_frame(cur, ref, 8, 8, p, oparams(prm))
    for R in (1, 2, 3, 4, 5, 6):
        os.environ["ACBM_R"] = str(R)
        say(f"task map: tiled fsbm 80x64 8x8 p={p} R={R}")
        try:
            got = acbm.to_numpy(acbm.fsbm_frame(dev(cur), dev(ref), 8, 8, p, prm))
        except acbm.AcbmError as e:
            assert e.status == acbm.E_UNSUPPORTED, e
            continue
        same(got, want, f"tiled fsbm p={p} R={R}")
