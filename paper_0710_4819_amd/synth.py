"""Seeded synthetic luma sequences for the motion-estimation workloads.

The paper's experiments use standard QCIF/CIF test sequences (Section 4) that
are not available here; these generators stand in for them with the same
frame sizes and controlled motion.  This module holds no part of the motion
estimation arithmetic: it only makes frames (and, where the motion is known by
construction, the true vector of each block) from numpy's PCG64 generator.
Both the GPU library's tests and the CPU oracle's tests consume these bytes.

Building blocks
  * texture: uniform u8 noise, then a separable Gaussian blur with Q16
    fixed-point taps (radius ceil(3 sigma), reflected border), rounded half up;
  * additive noise: round-half-up N(0, sigma^2) samples, clipped to [0, 255];
  * motion: integer shifts only.  Vector convention: if the pixel at x in frame
    t shows what was at x + d in frame t-1, the true vector of that content is d.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NO_TRUTH = 0x7FFF  # marker for blocks that do not lie wholly in one moving layer


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _taps_q16(sigma: float) -> np.ndarray:
    radius = int(math.ceil(3.0 * sigma))
    x = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-(x * x) / (2.0 * sigma * sigma))
    w /= w.sum()
    q = np.floor(w * 65536.0 + 0.5).astype(np.int64)
    q[radius] += 65536 - int(q.sum())  # taps sum to exactly 1.0 in Q16
    return q


def _blur_axis(img: np.ndarray, taps: np.ndarray, axis: int) -> np.ndarray:
    r = len(taps) // 2
    pad = [(0, 0), (0, 0)]
    pad[axis] = (r, r)
    src = np.pad(img.astype(np.int64), pad, mode="reflect")
    acc = np.zeros(img.shape, dtype=np.int64)
    n = img.shape[axis]
    for k, w in enumerate(taps):
        sl = [slice(None), slice(None)]
        sl[axis] = slice(k, k + n)
        acc += w * src[tuple(sl)]
    return np.clip((acc + 32768) >> 16, 0, 255).astype(np.uint8)


def blur(img: np.ndarray, sigma: float) -> np.ndarray:
    taps = _taps_q16(sigma)
    return _blur_axis(_blur_axis(img, taps, 1), taps, 0)


def texture(h: int, w: int, sigma: float, g: np.random.Generator) -> np.ndarray:
    return blur(g.integers(0, 256, size=(h, w), dtype=np.int64).astype(np.uint8), sigma)


def add_noise(img: np.ndarray, sigma: float, g: np.random.Generator) -> np.ndarray:
    if sigma <= 0:
        return img.copy()
    n = np.floor(g.normal(0.0, sigma, size=img.shape) + 0.5).astype(np.int64)
    return np.clip(img.astype(np.int64) + n, 0, 255).astype(np.uint8)


@dataclass
class Workload:
    """Frames of one sequence plus what the method needs to run on them."""
    name: str
    frames: list            # list of [H, W] uint8 arrays
    block_w: int
    block_h: int
    p: int
    lam: int
    qp: int
    truth: np.ndarray | None = None   # [pairs, by, bx, 2] int16 (x, y) or NO_TRUTH
    meta: dict = field(default_factory=dict)

    @property
    def height(self) -> int:
        return self.frames[0].shape[0]

    @property
    def width(self) -> int:
        return self.frames[0].shape[1]


# --------------------------------------------------------------------------
# Per-block planted shifts (QCIF 176x144, 16x16, p = 7)
# --------------------------------------------------------------------------
def planted_blocks(h=144, w=176, block=16, p=7, noise_sigma=2.0, blur_sigma=1.5,
                   seeds=(1001, 1002, 1003), lam=4, qp=4) -> Workload:
    """Frame t-1 is blurred noise; frame t gives every block its own integer
    shift (dx, dy) in [-p, p]^2: f_t(x, y) = f_{t-1}(clamp(x + dx), clamp(y + dy)),
    plus N(0, noise_sigma^2).  noise_sigma = 0 gives the noise-free twin."""
    f0 = texture(h, w, blur_sigma, rng(seeds[0]))
    by, bx = h // block, w // block
    mv = rng(seeds[1]).integers(-p, p + 1, size=(by, bx, 2), dtype=np.int64)
    dx = np.repeat(np.repeat(mv[..., 0], block, 0), block, 1)
    dy = np.repeat(np.repeat(mv[..., 1], block, 0), block, 1)
    ys = np.clip(np.arange(h)[:, None] + dy, 0, h - 1)
    xs = np.clip(np.arange(w)[None, :] + dx, 0, w - 1)
    f1 = f0[ys, xs]
    f1 = add_noise(f1, noise_sigma, rng(seeds[2]))
    truth = mv.astype(np.int16)[None]
    return Workload("planted_qcif", [f0, f1], block, block, p, lam, qp, truth,
                    {"noise_sigma": noise_sigma})


# --------------------------------------------------------------------------
# Fig. 3 setup: one original frame, nine known global vectors
# --------------------------------------------------------------------------
def global_motion(h=288, w=352, block=16, p=16, nframes=10, max_shift=8, noise_sigma=2.0,
                  seed=6000) -> Workload:
    """Section 3.1's experimental setup (Fig. 3): a ten-frame sequence made
    from one original picture by nine known global vectors.

    The original is a canvas larger than the frame whose local texture
    strength varies smoothly: a fine texture (sigma 1.2) and a very smooth one
    (sigma 8) are mixed with a weight field that is itself blurred noise
    (sigma 24), so blocks range from flat to highly textured.  Frame k is the
    canvas cropped at the cumulative offset o_k, so frame k shows at x what
    frame k-1 showed at x + (o_k - o_{k-1}): every block of pair k has the
    true vector d_k = o_k - o_{k-1}, drawn uniformly from
    [-max_shift, max_shift]^2.  Each frame then gets N(0, noise_sigma^2)."""
    g = rng(seed)
    d = g.integers(-max_shift, max_shift + 1, size=(nframes - 1, 2), dtype=np.int64)
    off = np.vstack([np.zeros((1, 2), np.int64), np.cumsum(d, axis=0)])
    lo = off.min(axis=0)
    span = off.max(axis=0) - lo
    ch, cw = h + int(span[1]), w + int(span[0])
    fine = texture(ch, cw, 1.2, rng(seed + 1)).astype(np.int64)
    smooth = texture(ch, cw, 8.0, rng(seed + 2)).astype(np.int64)
    wgt = blur(rng(seed + 3).integers(0, 256, size=(ch, cw), dtype=np.int64).astype(np.uint8),
               24.0).astype(np.int64)
    # stretch the weight field to the full 0..256 range (integer arithmetic)
    wmin, wmax = int(wgt.min()), int(wgt.max())
    wq = (wgt - wmin) * 256 // max(1, wmax - wmin)
    canvas = ((wq * fine + (256 - wq) * smooth + 128) >> 8).astype(np.uint8)
    frames = []
    for k in range(nframes):
        ox, oy = int(off[k, 0] - lo[0]), int(off[k, 1] - lo[1])
        f = canvas[oy:oy + h, ox:ox + w]
        frames.append(add_noise(f, noise_sigma, rng(seed + 100 + k)))
    by, bx = h // block, w // block
    truth = np.empty((nframes - 1, by, bx, 2), np.int16)
    truth[..., 0] = d[:, 0, None, None]
    truth[..., 1] = d[:, 1, None, None]
    return Workload("global_motion_fig3", frames, block, block, p, 0, 0, truth,
                    {"shifts": d.tolist(), "noise_sigma": noise_sigma})


# --------------------------------------------------------------------------
# Panned background plus bouncing textured rectangles
# --------------------------------------------------------------------------
def moving_scene(h: int, w: int, nframes: int, n_obj: int, size_range, vel_max: int,
                 pan_max: int, seed: int, noise_sigma=2.0, blur_sigma=1.5):
    """Returns (frames, truth).  The background canvas pans by a fixed integer
    velocity with max(|vx|, |vy|) in [1, pan_max]; n_obj rectangles with their
    own textures move with integer velocities in [-vel_max, vel_max]^2 and
    bounce off the frame edges; objects are painted in a fixed order.  Truth
    is emitted for blocks that lie wholly in one layer."""
    g_pan = rng(seed + 2)
    while True:
        pan = g_pan.integers(-pan_max, pan_max + 1, size=2)
        if max(abs(int(pan[0])), abs(int(pan[1]))) >= 1:
            break
    pvx, pvy = int(pan[0]), int(pan[1])
    ch = h + abs(pvy) * nframes + 2
    cw = w + abs(pvx) * nframes + 2
    canvas = texture(ch, cw, blur_sigma, rng(seed + 1))
    oy0 = 1 + (abs(pvy) * nframes if pvy < 0 else 0)
    ox0 = 1 + (abs(pvx) * nframes if pvx < 0 else 0)

    objs = []
    for k in range(n_obj):
        g = rng(seed + 10 + k)
        ow = int(g.integers(size_range[0], size_range[1] + 1))
        oh = int(g.integers(size_range[0], size_range[1] + 1))
        ow, oh = min(ow, w), min(oh, h)
        tex = texture(oh, ow, blur_sigma, g)
        x = int(g.integers(0, w - ow + 1))
        y = int(g.integers(0, h - oh + 1))
        vx = int(g.integers(-vel_max, vel_max + 1))
        vy = int(g.integers(-vel_max, vel_max + 1))
        objs.append([tex, x, y, vx, vy])

    frames, layers, positions = [], [], []
    for t in range(nframes):
        if t > 0:
            for o in objs:
                tex, x, y, vx, vy = o
                oh, ow = tex.shape
                if not 0 <= x + vx <= w - ow:
                    vx = -vx
                if not 0 <= y + vy <= h - oh:
                    vy = -vy
                nx = min(max(x + vx, 0), w - ow)
                ny = min(max(y + vy, 0), h - oh)
                o[1], o[2], o[3], o[4] = nx, ny, vx, vy
        by0, bx0 = oy0 + pvy * t, ox0 + pvx * t
        img = canvas[by0:by0 + h, bx0:bx0 + w].copy()
        lay = np.zeros((h, w), dtype=np.int16)
        pos = []
        for k, o in enumerate(objs):
            tex, x, y = o[0], o[1], o[2]
            oh, ow = tex.shape
            img[y:y + oh, x:x + ow] = tex
            lay[y:y + oh, x:x + ow] = k + 1
            pos.append((x, y))
        img = add_noise(img, noise_sigma, rng(seed + 100 + t))
        frames.append(img)
        layers.append(lay)
        positions.append(pos)
    return frames, layers, positions, (pvx, pvy)


def _truth_fields(layers, positions, pan, block_w, block_h):
    h, w = layers[0].shape
    by, bx = h // block_h, w // block_w
    out = np.full((len(layers) - 1, by, bx, 2), NO_TRUTH, dtype=np.int16)
    for t in range(1, len(layers)):
        lay = layers[t].reshape(by, block_h, bx, block_w).transpose(0, 2, 1, 3).reshape(by, bx, -1)
        first = lay[..., 0]
        uniform = (lay == first[..., None]).all(axis=-1)
        for r in range(by):
            for c in range(bx):
                if not uniform[r, c]:
                    continue
                k = int(first[r, c])
                if k == 0:
                    d = pan
                else:
                    (x1, y1), (x0, y0) = positions[t][k - 1], positions[t - 1][k - 1]
                    d = (x0 - x1, y0 - y1)
                out[t - 1, r, c] = d
    return out


def cif_scene(nframes=30, lam=8, seed=2000, with_truth=False) -> Workload:
    """CIF 352x288, 16x16 blocks, p = 16: pan of 1-3 px/frame, 4 rectangles of
    32-96 px with velocities in [-8, 8]^2, sigma = 2 noise."""
    frames, layers, pos, pan = moving_scene(288, 352, nframes, 4, (32, 96), 8, 3, seed)
    truth = _truth_fields(layers, pos, pan, 16, 16) if with_truth else None
    return Workload("cif_scene", frames, 16, 16, 16, lam, lam, truth, {"pan": pan})


def qcif_scene(kind: str, nframes=30, seed=7000) -> Workload:
    """QCIF 176x144, 16x16 blocks, p = 15 (Section 4's setting) in two
    characters that stand in for the paper's test sequences: "smooth" (soft
    texture, sigma 3, slow motion: 2 objects, |v| <= 2, pan 1) and
    "textured" (fine texture, sigma 1, fast motion: 5 objects, |v| <= 8,
    pan up to 4).  Noise sigma 2."""
    if kind == "smooth":
        frames, _, _, _ = moving_scene(144, 176, nframes, 2, (32, 64), 2, 1, seed, blur_sigma=3.0)
    elif kind == "textured":
        frames, _, _, _ = moving_scene(144, 176, nframes, 5, (24, 64), 8, 4, seed + 500,
                                       blur_sigma=1.0)
    else:
        raise ValueError(f"unknown kind {kind}")
    return Workload(f"qcif_{kind}", frames, 16, 16, 15, 0, 0, None, {"kind": kind})


def hd_scene(nframes=60, lam=8, seed=3000, with_truth=False) -> Workload:
    """1920x1088, 16x16 blocks, p = 32: pan of 1-3 px/frame, 16 rectangles of
    64-256 px with velocities in [-24, 24]^2 (relative motion stays within p),
    sigma = 2 noise."""
    frames, layers, pos, pan = moving_scene(1088, 1920, nframes, 16, (64, 256), 24, 3, seed)
    truth = _truth_fields(layers, pos, pan, 16, 16) if with_truth else None
    return Workload("hd_scene_1920x1088", frames, 16, 16, 32, lam, lam, truth, {"pan": pan})


# --------------------------------------------------------------------------
# Mixed batch: 64 sequences of 8 frames
# --------------------------------------------------------------------------
BATCH_RES = [(176, 144), (352, 288), (1280, 720), (1920, 1088)]
BATCH_P = [7, 16, 32]
BATCH_BLOCK = [16, 8]


def batch_spec(s: int) -> dict:
    w, h = BATCH_RES[s % 4]
    return {"width": w, "height": h, "p": BATCH_P[(s // 4) % 3], "block": BATCH_BLOCK[(s // 12) % 2]}


def batch_sequence(s: int, nframes=8, lam=8, seed_base=4000) -> Workload:
    spec = batch_spec(s)
    w, h, bsz = spec["width"], spec["height"], spec["block"]
    nobj = max(2, (w * h) // (1920 * 1088 // 16))
    frames, _, _, _ = moving_scene(h, w, nframes, nobj, (max(16, w // 16), max(32, w // 8)),
                                   min(spec["p"] - 3, 24), 3, seed_base + 1000 * s)
    return Workload(f"batch{s}", frames, bsz, bsz, spec["p"], lam, lam, None, spec)


# --------------------------------------------------------------------------
# Served streams
# --------------------------------------------------------------------------
SERVE_RES = [(640, 480), (1280, 720), (1920, 1088), (3840, 2160)]
SERVE_P = [16, 32, 64]


def serve_streams(n_streams=32, seed=5100) -> list:
    """Per stream: resolution and p drawn uniformly from the served mix."""
    out = []
    for s in range(n_streams):
        g = rng(seed + s)
        w, h = SERVE_RES[int(g.integers(0, len(SERVE_RES)))]
        p = SERVE_P[int(g.integers(0, len(SERVE_P)))]
        out.append({"stream": s, "width": w, "height": h, "p": p, "seed": seed + s})
    return out


def serve_arrivals(rate_hz: float, n: int, n_streams: int, seed=5001):
    """Poisson arrivals: exponential gaps at rate_hz; each request names a
    stream uniformly at random.  Returns (times_s, stream_ids)."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate_hz, size=n)
    return np.cumsum(gaps), g.integers(0, n_streams, size=n)


def stream_frames(spec: dict, nframes: int) -> list:
    frames, _, _, _ = moving_scene(spec["height"], spec["width"], nframes, 4,
                                   (spec["width"] // 16, spec["width"] // 6),
                                   min(spec["p"] - 3, 24), 3, spec["seed"] * 7)
    return frames
