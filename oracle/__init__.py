"""CPU oracle for adaptive cost block matching -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper around ``liboracle_acbm.so`` (plain C, see
``acbm_oracle.c``).  Only the test suite, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package; the GPU library and
its Python binding never do, and nothing here imports them.

Frames are 2-D ``numpy.uint8`` arrays ``[height, pitch]``; the logical width
is passed separately (default: the array width), so a pitch wider than the
frame can be exercised.  Results come back as a numpy structured array with
fields ``mv_x, mv_y, sad, j, rate_bits, cands, mode, intra_x`` shaped
``[by, bx]``.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_acbm.so")

FSBM, PBM, ACBM = 0, 1, 2
MODE_FSBM, MODE_PBM_C1, MODE_PBM_C2, MODE_CRITICAL, MODE_PBM = 0, 1, 2, 3, 4


class _Geom(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("pitch", C.c_uint32),
                ("block_w", C.c_uint32), ("block_h", C.c_uint32), ("p", C.c_uint32)]


class _Params(C.Structure):
    _fields_ = [("lambda_", C.c_uint32), ("qp", C.c_uint32), ("alpha", C.c_uint32),
                ("beta", C.c_uint32), ("gamma_num", C.c_uint32), ("gamma_den", C.c_uint32),
                ("subpel", C.c_uint32)]


@dataclass(frozen=True)
class Params:
    """Lagrange multiplier, quantiser and the ACBM thresholds.

    The paper's tuned values for 16x16 macroblocks are alpha = 1000,
    beta = 8, gamma = 1/4 (Section 4).  subpel = 1: half-pel precision, all
    vectors in half-pel units.
    """
    lam: int = 0
    qp: int = 0
    alpha: int = 1000
    beta: int = 8
    gamma_num: int = 1
    gamma_den: int = 4
    subpel: int = 0

    def _c(self) -> _Params:
        return _Params(self.lam, self.qp, self.alpha, self.beta, self.gamma_num, self.gamma_den,
                       self.subpel)


_lib = None


def _bind(lib):
    """Declare the C signatures on a loaded oracle library."""
    P = C.POINTER
    u8p, i16p = P(C.c_uint8), P(C.c_int16)
    lib.oracle_result_layout.argtypes = [P(C.c_uint32)]
    lib.oracle_check_geom.argtypes = [P(_Geom)]
    lib.oracle_se_bits.argtypes = [C.c_int64]
    lib.oracle_is_valid.argtypes = [P(_Geom), C.c_int, C.c_int, C.c_int, C.c_int]
    lib.oracle_sad.argtypes = [P(_Geom), u8p, u8p, C.c_int, C.c_int, C.c_int, C.c_int]
    lib.oracle_sad.restype = C.c_uint32
    lib.oracle_intra_x.argtypes = [P(_Geom), u8p, C.c_int, C.c_int]
    lib.oracle_intra_x.restype = C.c_uint64
    lib.oracle_median_pred.argtypes = [P(C.c_int32), P(C.c_int32), C.c_int, C.c_int,
                                       C.c_int, P(C.c_int), P(C.c_int)]
    lib.oracle_sad_table.argtypes = [P(_Geom), u8p, u8p, P(C.c_uint32)]
    lib.oracle_intra_table.argtypes = [P(_Geom), u8p, P(C.c_uint64)]
    lib.oracle_fsbm_frame.argtypes = [P(_Geom), P(_Params), u8p, u8p, C.c_void_p]
    lib.oracle_pbm_frame.argtypes = [P(_Geom), P(_Params), u8p, u8p, i16p, C.c_void_p]
    lib.oracle_acbm_frame.argtypes = [P(_Geom), P(_Params), u8p, u8p, i16p, C.c_void_p]
    lib.oracle_sequence.argtypes = [P(_Geom), P(_Params), C.c_int, P(u8p), C.c_uint32,
                                    C.c_void_p]
    lib.oracle_block.argtypes = [P(_Geom), P(_Params), C.c_int, u8p, u8p, i16p, P(C.c_int32),
                                 P(C.c_int32), C.c_int, C.c_int, C.c_void_p]
    lib.oracle_sad_deviation.argtypes = [P(_Geom), u8p, u8p, C.c_int, C.c_int,
                                         P(C.c_uint64), P(C.c_uint32)]
    lib.oracle_ref_half.argtypes = [P(_Geom), u8p, C.c_long, C.c_long]
    lib.oracle_is_valid_half.argtypes = [P(_Geom), C.c_int, C.c_int, C.c_int, C.c_int]
    lib.oracle_sad_half.argtypes = [P(_Geom), u8p, u8p, C.c_int, C.c_int, C.c_int, C.c_int]
    lib.oracle_sad_half.restype = C.c_uint32
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = _bind(C.CDLL(_LIB_PATH))
    return _lib


@contextlib.contextmanager
def using_library(path: str):
    """Temporarily route every call of this module to another build of the
    oracle (the mutation tests compile deliberately broken copies)."""
    global _lib
    saved = _load()
    _lib = _bind(C.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def result_dtype() -> np.dtype:
    lib = _load()
    lay = (C.c_uint32 * 9)()
    lib.oracle_result_layout(lay)
    names = ["mv_x", "mv_y", "sad", "j", "rate_bits", "cands", "mode", "intra_x"]
    formats = ["<i4", "<i4", "<u4", "<u8", "<u4", "<u4", "<u4", "<u8"]
    return np.dtype({"names": names, "formats": formats, "offsets": list(lay[:8]),
                     "itemsize": lay[8]})


def _u8p(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _frame(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype != np.uint8 or a.ndim != 2:
        raise ValueError("frames are 2-D uint8 arrays")
    return np.ascontiguousarray(a)


def geom(frame: np.ndarray, block_w: int, block_h: int, p: int, width: int | None = None) -> _Geom:
    h, pitch = frame.shape
    return _Geom(pitch if width is None else width, h, pitch, block_w, block_h, p)


def _check(rc: int):
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (status {rc})")


def check_geom(width, height, pitch, block_w, block_h, p) -> int:
    return _load().oracle_check_geom(C.byref(_Geom(width, height, pitch, block_w, block_h, p)))


def se_bits(k: int) -> int:
    return _load().oracle_se_bits(int(k))


def is_valid(g: _Geom, r: int, c: int, u: int, v: int) -> bool:
    return bool(_load().oracle_is_valid(C.byref(g), r, c, u, v))


def sad(cur, ref, g: _Geom, r, c, u, v) -> int:
    cur, ref = _frame(cur), _frame(ref)
    return int(_load().oracle_sad(C.byref(g), _u8p(cur), _u8p(ref), r, c, u, v))


def ref_half(ref, g: _Geom, X: int, Y: int) -> int:
    ref = _frame(ref)
    return int(_load().oracle_ref_half(C.byref(g), _u8p(ref), X, Y))


def is_valid_half(g: _Geom, r: int, c: int, U: int, V: int) -> bool:
    return bool(_load().oracle_is_valid_half(C.byref(g), r, c, U, V))


def sad_half(cur, ref, g: _Geom, r, c, U, V) -> int:
    cur, ref = _frame(cur), _frame(ref)
    return int(_load().oracle_sad_half(C.byref(g), _u8p(cur), _u8p(ref), r, c, U, V))


def intra_x(cur, g: _Geom, r, c) -> int:
    cur = _frame(cur)
    return int(_load().oracle_intra_x(C.byref(g), _u8p(cur), r, c))


def median_pred(field_x: np.ndarray, field_y: np.ndarray, r: int, c: int) -> tuple[int, int]:
    fx = np.ascontiguousarray(field_x, dtype=np.int32)
    fy = np.ascontiguousarray(field_y, dtype=np.int32)
    px, py = C.c_int(), C.c_int()
    _load().oracle_median_pred(fx.ctypes.data_as(C.POINTER(C.c_int32)),
                               fy.ctypes.data_as(C.POINTER(C.c_int32)),
                               fx.shape[1], r, c, C.byref(px), C.byref(py))
    return px.value, py.value


def _blocks(g: _Geom) -> tuple[int, int]:
    return g.height // g.block_h, g.width // g.block_w


def sad_table(cur, ref, block_w, block_h, p, width=None) -> np.ndarray:
    cur, ref = _frame(cur), _frame(ref)
    g = geom(cur, block_w, block_h, p, width)
    _check(_load().oracle_check_geom(C.byref(g)))
    by, bx = _blocks(g)
    w = 2 * p + 1
    out = np.empty((by, bx, w, w), dtype=np.uint32)
    _check(_load().oracle_sad_table(C.byref(g), _u8p(cur), _u8p(ref),
                                    out.ctypes.data_as(C.POINTER(C.c_uint32))))
    return out


def intra_table(cur, block_w, block_h, width=None) -> np.ndarray:
    cur = _frame(cur)
    g = geom(cur, block_w, block_h, 0, width)
    _check(_load().oracle_check_geom(C.byref(g)))
    by, bx = _blocks(g)
    out = np.empty((by, bx), dtype=np.uint64)
    _check(_load().oracle_intra_table(C.byref(g), _u8p(cur),
                                      out.ctypes.data_as(C.POINTER(C.c_uint64))))
    return out


def _field_ptr(prev_field):
    if prev_field is None:
        return None, None
    pf = np.ascontiguousarray(prev_field, dtype=np.int16)
    return pf, pf.ctypes.data_as(C.POINTER(C.c_int16))


def fsbm_frame(cur, ref, block_w, block_h, p, params: Params, width=None) -> np.ndarray:
    cur, ref = _frame(cur), _frame(ref)
    g = geom(cur, block_w, block_h, p, width)
    _check(_load().oracle_check_geom(C.byref(g)))
    out = np.zeros(_blocks(g), dtype=result_dtype())
    _check(_load().oracle_fsbm_frame(C.byref(g), C.byref(params._c()), _u8p(cur), _u8p(ref),
                                     out.ctypes.data))
    return out


def pbm_frame(cur, ref, block_w, block_h, p, params: Params, prev_field=None, width=None):
    cur, ref = _frame(cur), _frame(ref)
    g = geom(cur, block_w, block_h, p, width)
    _check(_load().oracle_check_geom(C.byref(g)))
    out = np.zeros(_blocks(g), dtype=result_dtype())
    keep, pfp = _field_ptr(prev_field)
    _check(_load().oracle_pbm_frame(C.byref(g), C.byref(params._c()), _u8p(cur), _u8p(ref),
                                    pfp, out.ctypes.data))
    return out


def acbm_frame(cur, ref, block_w, block_h, p, params: Params, prev_field=None, width=None):
    cur, ref = _frame(cur), _frame(ref)
    g = geom(cur, block_w, block_h, p, width)
    _check(_load().oracle_check_geom(C.byref(g)))
    out = np.zeros(_blocks(g), dtype=result_dtype())
    keep, pfp = _field_ptr(prev_field)
    _check(_load().oracle_acbm_frame(C.byref(g), C.byref(params._c()), _u8p(cur), _u8p(ref),
                                     pfp, out.ctypes.data))
    return out


def sequence(frames, block_w, block_h, p, params: Params, algo: int, width=None) -> np.ndarray:
    """Run a whole sequence; returns ``[nframes-1, by, bx]`` results."""
    frames = [_frame(f) for f in frames]
    g = geom(frames[0], block_w, block_h, p, width)
    _check(_load().oracle_check_geom(C.byref(g)))
    by, bx = _blocks(g)
    arr = (C.POINTER(C.c_uint8) * len(frames))(*[_u8p(f) for f in frames])
    out = np.zeros((len(frames) - 1, by, bx), dtype=result_dtype())
    _check(_load().oracle_sequence(C.byref(g), C.byref(params._c()), algo, arr, len(frames),
                                   out.ctypes.data))
    return out


def block(cur, ref, block_w, block_h, p, params: Params, algo: int, field_x, field_y, r, c,
          prev_field=None, width=None) -> np.ndarray:
    """One block's result given the final vectors of the blocks before it
    (field_x/field_y, [by, bx]) and the previous field."""
    cur, ref = _frame(cur), _frame(ref)
    g = geom(cur, block_w, block_h, p, width)
    fx = np.ascontiguousarray(field_x, dtype=np.int32)
    fy = np.ascontiguousarray(field_y, dtype=np.int32)
    keep, pfp = _field_ptr(prev_field)
    out = np.zeros((), dtype=result_dtype())
    _check(_load().oracle_block(C.byref(g), C.byref(params._c()), algo, _u8p(cur), _u8p(ref), pfp,
                                fx.ctypes.data_as(C.POINTER(C.c_int32)),
                                fy.ctypes.data_as(C.POINTER(C.c_int32)), r, c, out.ctypes.data))
    return out


def sad_deviation(cur, ref, block_w, block_h, p, r, c, width=None) -> tuple[int, int]:
    cur, ref = _frame(cur), _frame(ref)
    g = geom(cur, block_w, block_h, p, width)
    dev, mn = C.c_uint64(), C.c_uint32()
    _check(_load().oracle_sad_deviation(C.byref(g), _u8p(cur), _u8p(ref), r, c,
                                        C.byref(dev), C.byref(mn)))
    return int(dev.value), int(mn.value)


def field_of(results: np.ndarray) -> np.ndarray:
    """(x, y) int16 pairs per block, the layout the predictive runs take as
    their previous field."""
    f = np.empty(results.shape + (2,), dtype=np.int16)
    f[..., 0] = results["mv_x"]
    f[..., 1] = results["mv_y"]
    return f
