"""Python binding of libacbm (ctypes).

Argument marshalling only: every step of the motion search runs in the HIP
library ``libacbm.so``; PyTorch supplies device memory and the stream.  The
library is loaded on first use and a missing build raises ``RuntimeError``
(there is no fallback).

Frames are 2-D ``torch.uint8`` CUDA tensors ``[height, pitch]`` (the logical
width defaults to the tensor width).  Result fields are returned as a
``[by, bx, 32]`` uint8 tensor in the C layout of ``acbm_block_result``;
``to_numpy`` turns it into a structured numpy array with fields
``mv_x, mv_y, sad, j, rate_bits, cands, mode, intra_x``.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# ACBM_LIB names another build of the library (the walker phase-profiling
# build, libacbm_phases.so); the default is the in-tree libacbm.so.
LIB_PATH = os.environ.get("ACBM_LIB") or os.path.join(HERE, "libacbm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "acbm.h")

OK, E_INVAL, E_SHAPE, E_RANGE, E_NOMEM, E_DEVICE, E_BUSY, E_UNSUPPORTED, E_TIMEOUT = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
ALGO_FSBM, ALGO_PBM, ALGO_ACBM = 0, 1, 2
MODE_FSBM, MODE_PBM_C1, MODE_PBM_C2, MODE_CRITICAL, MODE_PBM = 0, 1, 2, 3, 4
OP_SAD_TABLE, OP_FSBM, OP_PBM, OP_ACBM = 0, 1, 2, 3

RESULT_DTYPE = np.dtype({
    "names": ["mv_x", "mv_y", "sad", "j", "rate_bits", "cands", "mode", "intra_x"],
    "formats": ["<i2", "<i2", "<u4", "<u4", "<u4", "<u4", "<u4", "<u8"],
    "offsets": [0, 2, 4, 8, 12, 16, 20, 24],
    "itemsize": 32,
})

STATS_DTYPE = np.dtype({
    "names": ["sad_min", "valid", "sad_deviation", "intra_x"],
    "formats": ["<u4", "<u4", "<u8", "<u8"],
    "offsets": [0, 4, 8, 16],
    "itemsize": 32,
})


class Geom(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("pitch", C.c_uint32),
                ("block_w", C.c_uint32), ("block_h", C.c_uint32), ("p", C.c_uint32)]


class CParams(C.Structure):
    _fields_ = [("lambda_", C.c_uint32), ("qp", C.c_uint32), ("alpha", C.c_uint32),
                ("beta", C.c_uint32), ("gamma_num", C.c_uint32), ("gamma_den", C.c_uint32),
                ("subpel", C.c_uint32)]


class ServeCfg(C.Structure):
    _fields_ = [("pool_bytes", C.c_size_t), ("max_streams", C.c_uint32),
                ("max_inflight", C.c_uint32), ("queue_depth", C.c_uint32),
                ("lanes", C.c_uint32), ("pinned_bytes", C.c_size_t)]


class ServeStats(C.Structure):
    _fields_ = [("completed", C.c_uint64), ("rejected", C.c_uint64), ("p50_us", C.c_double),
                ("p99_us", C.c_double), ("mean_us", C.c_double), ("throughput_rps", C.c_double),
                ("device_busy_frac", C.c_double), ("device_busy_ms", C.c_double),
                ("passes", C.c_uint64), ("mean_batch", C.c_double)]


class Job(C.Structure):
    _fields_ = [("geom", Geom), ("params", CParams), ("algo", C.c_uint32),
                ("nframes", C.c_uint32), ("frames", C.POINTER(C.c_void_p)),
                ("out", C.c_void_p)]


@dataclass(frozen=True)
class Params:
    """lambda, Qp and the ACBM thresholds; gamma = gamma_num / gamma_den;
    subpel = 1 for half-pel precision (vectors in half-pel units)."""
    lam: int = 0
    qp: int = 0
    alpha: int = 1000
    beta: int = 8
    gamma_num: int = 1
    gamma_den: int = 4
    subpel: int = 0

    def c(self) -> CParams:
        return CParams(self.lam, self.qp, self.alpha, self.beta, self.gamma_num, self.gamma_den,
                       self.subpel)


def default_params(block_w: int, block_h: int, lam: int, qp: int | None = None,
                   subpel: int = 0) -> Params:
    """The paper's thresholds for this block size, from the library
    (acbm_default_params: alpha = 1000, beta = 8, gamma = 1/4 at 16x16,
    alpha and beta scaled by N*M/256 otherwise).  qp defaults to lambda."""
    c = CParams()
    _check(lib().acbm_default_params(block_w, block_h, lam, lam if qp is None else qp, subpel,
                                     C.byref(c)))
    return Params(lam=c.lambda_, qp=c.qp, alpha=c.alpha, beta=c.beta, gamma_num=c.gamma_num,
                  gamma_den=c.gamma_den, subpel=c.subpel)


class AcbmError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"libacbm status {status}: {detail}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P, vp, sz = C.POINTER, C.c_void_p, C.c_size_t
        L.acbm_version.restype = C.c_char_p
        L.acbm_strerror.restype = C.c_char_p
        L.acbm_strerror.argtypes = [C.c_int]
        L.acbm_last_error.restype = C.c_char_p
        L.acbm_workspace_size.argtypes = [C.c_int, P(Geom), C.c_uint32, P(sz)]
        L.acbm_workspace_status.argtypes = [vp, sz, vp, P(C.c_int)]
        L.acbm_sad_table.argtypes = [P(Geom), vp, vp, vp, vp]
        L.acbm_sad_stats.argtypes = [P(Geom), vp, vp, vp, vp]
        L.acbm_fsbm_frame.argtypes = [P(Geom), P(CParams), vp, vp, vp, vp, sz, vp]
        L.acbm_pbm_frame.argtypes = [P(Geom), P(CParams), vp, vp, vp, vp, vp, sz, vp]
        L.acbm_acbm_frame.argtypes = [P(Geom), P(CParams), vp, vp, vp, vp, vp, sz, vp]
        L.acbm_acbm_frame_noalloc.argtypes = [P(Geom), P(CParams), vp, vp, vp, vp, vp, vp]
        L.acbm_batch_workspace_size.argtypes = [P(Job), sz, P(sz)]
        L.acbm_batch.argtypes = [P(Job), sz, vp, sz, vp]
        L.acbm_batch_status.argtypes = [P(Job), sz, vp, sz, vp, P(C.c_int)]
        L.acbm_batch_graph_create.argtypes = [P(Job), sz, vp, sz, P(vp)]
        L.acbm_batch_graph_launch.argtypes = [vp, vp]
        L.acbm_batch_graph_destroy.argtypes = [vp]
        L.acbm_autotune.argtypes = [P(Geom), P(C.c_uint32), P(C.c_float), vp]
        L.acbm_serve.argtypes = [P(ServeCfg), P(vp)]
        L.acbm_serve_submit.argtypes = [vp, C.c_uint32, vp, P(Geom), P(CParams), C.c_uint32,
                                        P(C.c_uint64)]
        L.acbm_serve_wait.argtypes = [vp, C.c_uint64, vp, C.c_int64]
        L.acbm_serve_stats.argtypes = [vp, P(ServeStats)]
        L.acbm_serve_stats_get.argtypes = [vp, P(ServeStats)]
        L.acbm_default_params.argtypes = [C.c_uint32] * 5 + [P(CParams)]
        L.acbm_serve_close.argtypes = [vp]
        L.acbm_profile_enable.argtypes = [C.c_int]
        L.acbm_profile_read.argtypes = [C.c_char_p, P(C.c_double), P(C.c_uint64)]
        _lib = L
    return _lib


def declared_functions() -> list[str]:
    """Names of the functions include/acbm.h declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(acbm_[a-z_]+)\s*\(", src)))


def _check(rc: int):
    if rc != OK:
        raise AcbmError(rc, lib().acbm_last_error().decode())


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def geom(frame: torch.Tensor, block_w: int, block_h: int, p: int, width: int | None = None) -> Geom:
    if frame.dtype != torch.uint8 or frame.dim() != 2:
        raise ValueError("frames are 2-D uint8 tensors")
    if frame.stride(1) != 1:
        raise ValueError("frame rows must be contiguous")
    h = frame.shape[0]
    pitch = frame.stride(0)
    return Geom(frame.shape[1] if width is None else width, h, pitch, block_w, block_h, p)


def workspace_size(op: int, g: Geom, npairs: int = 1) -> int:
    n = C.c_size_t()
    _check(lib().acbm_workspace_size(op, C.byref(g), npairs, C.byref(n)))
    return n.value


def workspace(op: int, g: Geom, device, npairs: int = 1) -> torch.Tensor:
    return torch.empty(max(256, workspace_size(op, g, npairs)), dtype=torch.uint8, device=device)


def workspace_status(ws: torch.Tensor, stream=None) -> int:
    st = C.c_int()
    _check(lib().acbm_workspace_status(ws.data_ptr(), ws.numel(), _stream(stream), C.byref(st)))
    return st.value


def _blocks(g: Geom) -> tuple[int, int]:
    return g.height // g.block_h, g.width // g.block_w


def sad_table(cur, ref, block_w, block_h, p, width=None, stream=None) -> torch.Tensor:
    """u32 SAD table [by, bx, 2p+1, 2p+1] (returned as int32 storage)."""
    g = geom(cur, block_w, block_h, p, width)
    by, bx = _blocks(g)
    W = 2 * p + 1
    out = torch.empty((by, bx, W, W), dtype=torch.int32, device=cur.device)
    _check(lib().acbm_sad_table(C.byref(g), cur.data_ptr(), ref.data_ptr(), out.data_ptr(),
                                _stream(stream)))
    return out


def sad_stats(cur, ref, block_w, block_h, p, width=None, stream=None) -> torch.Tensor:
    """Per-block SAD_min, valid count, SAD_deviation and IntraX
    (acbm_block_stats records, [by, bx, 32] bytes; see stats_to_numpy)."""
    g = geom(cur, block_w, block_h, p, width)
    by, bx = _blocks(g)
    out = torch.empty((by, bx, 32), dtype=torch.uint8, device=cur.device)
    _check(lib().acbm_sad_stats(C.byref(g), cur.data_ptr(), ref.data_ptr(), out.data_ptr(),
                                _stream(stream)))
    return out


def _results(g: Geom, device, npairs: int | None = None) -> torch.Tensor:
    by, bx = _blocks(g)
    shape = (by, bx, 32) if npairs is None else (npairs, by, bx, 32)
    return torch.empty(shape, dtype=torch.uint8, device=device)


def fsbm_frame(cur, ref, block_w, block_h, p, params: Params, width=None, ws=None,
               stream=None) -> torch.Tensor:
    g = geom(cur, block_w, block_h, p, width)
    ws = ws if ws is not None else workspace(OP_FSBM, g, cur.device)
    out = _results(g, cur.device)
    _check(lib().acbm_fsbm_frame(C.byref(g), C.byref(params.c()), cur.data_ptr(), ref.data_ptr(),
                                 out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return out


def _predictive(fn, op, cur, ref, block_w, block_h, p, params, prev_field, width, ws, stream):
    g = geom(cur, block_w, block_h, p, width)
    ws = ws if ws is not None else workspace(op, g, cur.device)
    out = _results(g, cur.device)
    if prev_field is not None:
        by, bx = _blocks(g)
        if prev_field.dtype != torch.int16 or tuple(prev_field.shape) != (by, bx, 2):
            raise ValueError("prev_field must be an int16 [by, bx, 2] tensor")
        prev_field = prev_field.contiguous()
    _check(fn(C.byref(g), C.byref(params.c()), cur.data_ptr(), ref.data_ptr(), _ptr(prev_field),
              out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)))
    return out


def pbm_frame(cur, ref, block_w, block_h, p, params: Params, prev_field=None, width=None,
              ws=None, stream=None) -> torch.Tensor:
    return _predictive(lib().acbm_pbm_frame, OP_PBM, cur, ref, block_w, block_h, p, params,
                       prev_field, width, ws, stream)


def acbm_frame(cur, ref, block_w, block_h, p, params: Params, prev_field=None, width=None,
               ws=None, stream=None) -> torch.Tensor:
    return _predictive(lib().acbm_acbm_frame, OP_ACBM, cur, ref, block_w, block_h, p, params,
                       prev_field, width, ws, stream)


def acbm_frame_noalloc(cur, ref, block_w, block_h, p, params: Params, prev_field=None,
                       width=None, status: torch.Tensor | None = None,
                       stream=None) -> torch.Tensor:
    """ACBM for one pair through acbm_acbm_frame_noalloc (the library's own
    fixed scratch, no workspace).  status: optional int32 device tensor of
    one element that receives the run status (0 = every block finished)."""
    g = geom(cur, block_w, block_h, p, width)
    out = _results(g, cur.device)
    if prev_field is not None:
        by, bx = _blocks(g)
        if prev_field.dtype != torch.int16 or tuple(prev_field.shape) != (by, bx, 2):
            raise ValueError("prev_field must be an int16 [by, bx, 2] tensor")
        prev_field = prev_field.contiguous()
    _check(lib().acbm_acbm_frame_noalloc(C.byref(g), C.byref(params.c()), cur.data_ptr(),
                                         ref.data_ptr(), _ptr(prev_field), out.data_ptr(),
                                         _ptr(status), _stream(stream)))
    return out


class Batch:
    """A set of sequences run by one acbm_batch call.  Keeps the ctypes job
    table, the device frames and the result tensors alive."""

    def __init__(self, device):
        self.device = device
        self.jobs = []
        self._keep = []
        self.outs = []

    def add(self, frames: list, block_w: int, block_h: int, p: int, params: Params, algo: int,
            width=None) -> torch.Tensor:
        g = geom(frames[0], block_w, block_h, p, width)
        ptrs = (C.c_void_p * len(frames))(*[f.data_ptr() for f in frames])
        out = _results(g, self.device, npairs=len(frames) - 1)
        self.jobs.append(Job(g, params.c(), algo, len(frames), ptrs, out.data_ptr()))
        self._keep.append((frames, ptrs))
        self.outs.append(out)
        return out

    def table(self):
        return (Job * len(self.jobs))(*self.jobs)

    def workspace_size(self) -> int:
        n = C.c_size_t()
        _check(lib().acbm_batch_workspace_size(self.table(), len(self.jobs), C.byref(n)))
        return n.value

    def run(self, ws: torch.Tensor | None = None, stream=None) -> list:
        ws = ws if ws is not None else torch.empty(max(256, self.workspace_size()),
                                                   dtype=torch.uint8, device=self.device)
        self.ws = ws
        _check(lib().acbm_batch(self.table(), len(self.jobs), ws.data_ptr(), ws.numel(),
                                _stream(stream)))
        return self.outs

    def status(self, ws: torch.Tensor | None = None, stream=None) -> int:
        """Device-detected status of the last run on `ws` (default: the
        workspace of the last run): 0, or ACBM_E_TIMEOUT."""
        ws = ws if ws is not None else self.ws
        st = C.c_int()
        _check(lib().acbm_batch_status(self.table(), len(self.jobs), ws.data_ptr(), ws.numel(),
                                       _stream(stream), C.byref(st)))
        return st.value


class BatchGraph:
    """A Batch recorded once as a HIP graph (acbm_batch_graph_create); each
    launch() replays the whole batch with one graph launch.  Keeps the batch
    (frames, outputs, job table) and the workspace alive."""

    def __init__(self, batch: "Batch", ws: torch.Tensor | None = None):
        self.batch = batch
        self.ws = ws if ws is not None else torch.empty(max(256, batch.workspace_size()),
                                                        dtype=torch.uint8, device=batch.device)
        self.table = batch.table()
        self.h = C.c_void_p()
        _check(lib().acbm_batch_graph_create(self.table, len(batch.jobs), self.ws.data_ptr(),
                                             self.ws.numel(), C.byref(self.h)))

    def launch(self, stream=None) -> list:
        _check(lib().acbm_batch_graph_launch(self.h, _stream(stream)))
        return self.batch.outs

    def close(self):
        if self.h:
            _check(lib().acbm_batch_graph_destroy(self.h))
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(block_w: int, block_h: int, p: int, width: int, height: int, pitch: int | None = None,
             stream=None) -> tuple[int, float]:
    """Times the window-search plans of (block_w, block_h, p) on a synthetic
    frame pair of this size and makes the fastest the process-wide plan.
    Returns (rows per lane R, ms per pair)."""
    g = Geom(width, height, width if pitch is None else pitch, block_w, block_h, p)
    r = C.c_uint32()
    ms = C.c_float()
    _check(lib().acbm_autotune(C.byref(g), C.byref(r), C.byref(ms), _stream(stream)))
    return r.value, ms.value


class Server:
    """Frame-pair motion estimation requests over device-resident streams,
    served by continuous batching (acbm_serve).  Frames are host numpy arrays
    [height, pitch] uint8."""

    def __init__(self, pool_bytes=4 << 30, max_streams=32, max_inflight=64, queue_depth=256,
                 lanes=0, pinned_bytes=0):
        self.h = C.c_void_p()
        cfg = ServeCfg(pool_bytes, max_streams, max_inflight, queue_depth, lanes, pinned_bytes)
        _check(lib().acbm_serve(C.byref(cfg), C.byref(self.h)))
        self.geoms = {}

    def submit(self, stream_id: int, frame: np.ndarray, block_w: int, block_h: int, p: int,
               params: Params, algo: int, width: int | None = None) -> int:
        frame = np.ascontiguousarray(frame, dtype=np.uint8)
        g = Geom(frame.shape[1] if width is None else width, frame.shape[0], frame.shape[1],
                 block_w, block_h, p)
        t = C.c_uint64()
        rc = lib().acbm_serve_submit(self.h, stream_id, frame.ctypes.data, C.byref(g),
                                     C.byref(params.c()), algo, C.byref(t))
        _check(rc)
        self.geoms[t.value] = g
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1) -> np.ndarray | None:
        """Results of a ticket as a structured array [by, bx] (None for a
        stream's first frame, which only becomes its reference)."""
        g = self.geoms.pop(ticket)
        by, bx = g.height // g.block_h, g.width // g.block_w
        out = np.zeros((by, bx), dtype=RESULT_DTYPE)
        out["mode"] = 0xFFFFFFFF
        _check(lib().acbm_serve_wait(self.h, ticket, out.ctypes.data, timeout_us))
        return None if (out["mode"] == 0xFFFFFFFF).all() else out

    def stats(self) -> dict:
        st = ServeStats()
        _check(lib().acbm_serve_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServeStats._fields_}

    def close(self):
        if self.h:
            _check(lib().acbm_serve_close(self.h))
            self.h = C.c_void_p()


def profile_enable(on: bool):
    _check(lib().acbm_profile_enable(1 if on else 0))


def profile_reset():
    _check(lib().acbm_profile_reset())


def profile_read(kernel: str) -> tuple[float, int]:
    """(summed device ms, launches) of one kernel since the last reset."""
    ms, n = C.c_double(), C.c_uint64()
    _check(lib().acbm_profile_read(kernel.encode(), C.byref(ms), C.byref(n)))
    return ms.value, n.value


PHASE_NAMES = ("blocks", "critical_blocks", "dependency_wait", "phase_a", "phase_b", "phase_c",
               "critical_search", "row_setup")


def phase_profile_read(reset: bool = False) -> dict | None:
    """Walker phase totals (the profiling build only, else None): block
    counts and summed s_memrealtime ticks (100 MHz) per phase."""
    L = lib()
    if not hasattr(L, "acbm_phase_profile_read"):
        return None
    out = (C.c_uint64 * 8)()
    _check(L.acbm_phase_profile_read(out, 1 if reset else 0))
    return dict(zip(PHASE_NAMES, list(out)))


def to_numpy(res: torch.Tensor) -> np.ndarray:
    a = res.detach().cpu().contiguous().numpy()
    return a.view(RESULT_DTYPE).reshape(a.shape[:-1])


def table_to_numpy(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def stats_to_numpy(st: torch.Tensor) -> np.ndarray:
    a = st.detach().cpu().contiguous().numpy()
    return a.view(STATS_DTYPE).reshape(a.shape[:-1])
