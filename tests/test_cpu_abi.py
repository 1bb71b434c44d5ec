"""The C ABI of libacbm on the CPU: the library loads, exports every function
include/acbm.h declares, and rejects bad arguments before touching a device
(argument checks run before any HIP call, so no GPU is needed)."""
import ctypes as C

import pytest

from paper_0710_4819_amd import acbm

FAKE = 0x1000  # a non-null, aligned "device pointer" that is never dereferenced


def test_library_loads_and_exports_every_declared_function():
    L = acbm.lib()
    names = acbm.declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, f"declared in acbm.h but not exported: {missing}"
    assert L.acbm_version().decode() == "0.1.0"


def test_strerror_covers_every_status():
    L = acbm.lib()
    for s in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert L.acbm_strerror(s).decode() not in ("", "unknown status")
    assert L.acbm_strerror(-99).decode() == "unknown status"


def _g(**kw):
    d = dict(width=176, height=144, pitch=176, block_w=16, block_h=16, p=7)
    d.update(kw)
    return acbm.Geom(d["width"], d["height"], d["pitch"], d["block_w"], d["block_h"], d["p"])


@pytest.mark.parametrize("kw,status", [
    (dict(width=0), acbm.E_INVAL),
    (dict(block_w=0), acbm.E_INVAL),
    (dict(pitch=100), acbm.E_INVAL),
    (dict(width=170, pitch=176), acbm.E_SHAPE),
    (dict(height=150), acbm.E_SHAPE),
    (dict(p=128), acbm.E_SHAPE),
    (dict(block_w=4, width=176), acbm.E_UNSUPPORTED),
    (dict(block_h=32, height=160), acbm.E_UNSUPPORTED),
    (dict(pitch=178), acbm.E_UNSUPPORTED),
])
def test_geometry_errors(kw, status):
    L = acbm.lib()
    g = _g(**kw)
    n = C.c_size_t()
    assert L.acbm_workspace_size(acbm.OP_FSBM, C.byref(g), 1, C.byref(n)) == status
    assert L.acbm_sad_table(C.byref(g), FAKE, FAKE, FAKE, None) == status
    assert L.acbm_last_error().decode() != ""


def test_argument_errors():
    L = acbm.lib()
    g = _g()
    prm = acbm.Params(lam=4, qp=4).c()
    n = C.c_size_t()
    assert L.acbm_workspace_size(acbm.OP_FSBM, None, 1, C.byref(n)) == acbm.E_INVAL
    assert L.acbm_workspace_size(acbm.OP_FSBM, C.byref(g), 0, C.byref(n)) == acbm.E_INVAL
    assert L.acbm_workspace_size(99, C.byref(g), 1, C.byref(n)) == acbm.E_INVAL
    # null and misaligned frames
    assert L.acbm_fsbm_frame(C.byref(g), C.byref(prm), None, FAKE, FAKE, FAKE, 1 << 20, None) == acbm.E_INVAL
    assert L.acbm_fsbm_frame(C.byref(g), C.byref(prm), FAKE + 1, FAKE, FAKE, FAKE, 1 << 20, None) == acbm.E_UNSUPPORTED
    assert L.acbm_acbm_frame(C.byref(g), C.byref(prm), FAKE, FAKE, None, None, FAKE, 1 << 20, None) == acbm.E_INVAL
    # gamma_den = 0
    bad = acbm.Params(lam=4, gamma_den=0).c()
    assert L.acbm_acbm_frame(C.byref(g), C.byref(bad), FAKE, FAKE, None, FAKE, FAKE, 1 << 20, None) == acbm.E_INVAL
    # lambda so large that J = SAD + lambda*R would not fit 32 bits
    huge = acbm.Params(lam=1 << 28).c()
    assert L.acbm_fsbm_frame(C.byref(g), C.byref(huge), FAKE, FAKE, FAKE, FAKE, 1 << 20, None) == acbm.E_RANGE


def test_workspace_sizes():
    g = _g(width=1920, height=1088, pitch=1920, p=32)
    f1 = acbm.workspace_size(acbm.OP_FSBM, g, 1)
    f59 = acbm.workspace_size(acbm.OP_FSBM, g, 59)
    assert f1 >= 8160 * 128 + 8160 * 65 * 65 * 2 and f59 > 50 * f1
    assert acbm.workspace_size(acbm.OP_SAD_TABLE, g, 1) == 0
    a1 = acbm.workspace_size(acbm.OP_ACBM, g, 1)
    assert 8160 * 4 <= a1 < 1 << 20


def test_batch_argument_errors():
    L = acbm.lib()
    n = C.c_size_t()
    ptrs = (C.c_void_p * 1)(FAKE)
    job = acbm.Job(_g(), acbm.Params(lam=4).c(), acbm.ALGO_FSBM, 1, ptrs, FAKE)
    jobs = (acbm.Job * 1)(job)
    assert L.acbm_batch_workspace_size(jobs, 1, C.byref(n)) == acbm.E_INVAL  # one frame
    job.nframes = 2
    job.algo = 7
    jobs = (acbm.Job * 1)(job)
    assert L.acbm_batch_workspace_size(jobs, 1, C.byref(n)) == acbm.E_INVAL
    job.algo = acbm.ALGO_ACBM
    ptrs2 = (C.c_void_p * 2)(FAKE, FAKE)
    job.frames = ptrs2
    jobs = (acbm.Job * 1)(job)
    assert L.acbm_batch_workspace_size(jobs, 1, C.byref(n)) == acbm.OK and n.value > 0
    assert L.acbm_batch(jobs, 1, FAKE, 16, None) == acbm.E_NOMEM
    st = C.c_int()
    assert L.acbm_batch_status(jobs, 1, None, n.value, None, C.byref(st)) == acbm.E_INVAL
    assert L.acbm_batch_status(jobs, 1, FAKE, n.value, None, None) == acbm.E_INVAL
    assert L.acbm_batch_status(jobs, 1, FAKE, 16, None, C.byref(st)) == acbm.E_NOMEM


def test_batch_workspace_grows_with_walker_groups():
    """PBM/ACBM jobs of one block size and precision share one walker
    group: the batch workspace holds every job's vector words plus one
    header and row order per group, so adding a job of another block size
    adds a header."""
    L = acbm.lib()
    ptrs = (C.c_void_p * 3)(FAKE, FAKE, FAKE)

    def size(*shapes):
        jobs = (acbm.Job * len(shapes))(*[
            acbm.Job(_g(block_w=bw, block_h=bh), acbm.Params(lam=4).c(), acbm.ALGO_ACBM, 3, ptrs,
                     FAKE) for bw, bh in shapes])
        n = C.c_size_t()
        assert L.acbm_batch_workspace_size(jobs, len(shapes), C.byref(n)) == acbm.OK
        return n.value

    one, two_same, two_diff = size((16, 16)), size((16, 16), (16, 16)), size((16, 16), (8, 8))
    assert two_same > one and two_diff > two_same


def test_default_params_scale_with_block_size():
    """acbm_default_params: Section 4's alpha, beta, gamma at 16x16, alpha and
    beta scaled by N*M/256 for other sizes, computed by the C library."""
    assert acbm.default_params(16, 16, 8) == acbm.Params(8, 8, 1000, 8, 1, 4)
    assert acbm.default_params(8, 8, 8) == acbm.Params(8, 8, 250, 2, 1, 4)
    assert acbm.default_params(16, 8, 8, qp=5) == acbm.Params(8, 5, 500, 4, 1, 4)
    assert acbm.default_params(16, 16, 2, subpel=1).subpel == 1
    L = acbm.lib()
    assert L.acbm_default_params(16, 16, 8, 8, 0, None) == acbm.E_INVAL
    c = acbm.CParams()
    assert L.acbm_default_params(0, 16, 8, 8, 0, C.byref(c)) == acbm.E_INVAL


def test_stats_and_precision_argument_errors():
    """acbm_sad_stats and the half-pel parameter are checked before any
    device call: bad geometry or pointers, subpel other than 0/1, half-pel
    with p > 63, and more block rows than the resolve gives threads."""
    L = acbm.lib()
    g = _g()
    assert L.acbm_sad_stats(C.byref(g), FAKE, FAKE, None, None) == acbm.E_INVAL
    assert L.acbm_sad_stats(C.byref(g), None, FAKE, FAKE, None) == acbm.E_INVAL
    assert L.acbm_sad_stats(C.byref(_g(height=150)), FAKE, FAKE, FAKE, None) == acbm.E_SHAPE
    bad = acbm.Params(lam=4, subpel=2).c()
    assert L.acbm_fsbm_frame(C.byref(g), C.byref(bad), FAKE, FAKE, FAKE, FAKE, 1 << 20, None) == acbm.E_INVAL
    wide = _g(width=192, height=192, pitch=192, p=64)
    hp = acbm.Params(lam=4, subpel=1).c()
    assert L.acbm_fsbm_frame(C.byref(wide), C.byref(hp), FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == acbm.E_RANGE
    assert L.acbm_acbm_frame(C.byref(wide), C.byref(hp), FAKE, FAKE, None, FAKE, FAKE, 1 << 30, None) == acbm.E_RANGE
    tall = _g(width=8, height=8 * 1025, pitch=8, block_w=8, block_h=8, p=2)
    assert L.acbm_fsbm_frame(C.byref(tall), C.byref(acbm.Params(lam=1).c()), FAKE, FAKE, FAKE, FAKE,
                             1 << 30, None) == acbm.E_UNSUPPORTED
    assert L.acbm_last_error().decode() != ""
