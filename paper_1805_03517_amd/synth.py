"""Seeded synthetic image pairs shaped like the paper's benchmark workloads.

The paper evaluates on KITTI 2015 and MPI Sintel (Sec. 4.2, 4.3), neither of
which is available here; these generators stand in for them with the same
image shapes and comparable displacement statistics.  Every generator is a
pure function of its integer seed (numpy PCG64) and returns uint8 arrays in
[H][W] (gray) or [H][W][3] (RGB) layout.

This module holds only image synthesis.  It contains none of the matching
method's arithmetic (no gray conversion, pyramid, descriptor, cost or search):
both the CPU oracle and the HIP path consume its output unchanged.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

__all__ = [
    "noise_texture", "translated_pair", "config0", "config1", "config2",
    "config3_stream", "config3_requests", "config4_batch", "SERVE_SIZES",
]


def _rescale(a: np.ndarray) -> np.ndarray:
    lo, hi = float(a.min()), float(a.max())
    return (a - lo) * (255.0 / max(hi - lo, 1e-9))


def _to_u8(a: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(a), 0, 255).astype(np.uint8)


def noise_texture(rng: np.random.Generator, h: int, w: int, sigma: float = 1.5) -> np.ndarray:
    """Gaussian-blurred white noise min-max rescaled to 0..255 (float64)."""
    return _rescale(ndimage.gaussian_filter(rng.standard_normal((h, w)), sigma, mode="reflect"))


def translated_pair(rng: np.random.Generator, w: int, h: int, d=(5, -3),
                    rect=(32, 24), rect_d=(-7, 4), noise_sd: float = 2.0,
                    pad: int = 32, sigma: float = 1.5):
    """Noise texture, frame 2 = frame 1 moved by integer ``d`` = (dx, dy).

    A ``rect`` = (rw, rh) block of frame-1 content moves by ``rect_d`` instead
    and is pasted over frame 2.  Frame 2 gets N(0, noise_sd) noise; both frames
    are rounded and clipped to uint8.  Returns (img1, img2, meta).
    """
    dx, dy = int(d[0]), int(d[1])
    pad = max(pad, abs(dx) + 1, abs(dy) + 1)
    tex = noise_texture(rng, h + 2 * pad, w + 2 * pad, sigma)
    i1 = tex[pad:pad + h, pad:pad + w]
    # I2(x, y) = I1(x - dx, y - dy) = tex(y - dy + pad, x - dx + pad)
    i2 = tex[pad - dy:pad - dy + h, pad - dx:pad - dx + w].copy()
    rw, rh = int(rect[0]), int(rect[1])
    rdx, rdy = int(rect_d[0]), int(rect_d[1])
    rect_xy = None
    if rw > 0 and rh > 0 and rw + abs(rdx) < w and rh + abs(rdy) < h:
        x0 = int(rng.integers(max(0, -rdx), w - rw - max(0, rdx) + 1))
        y0 = int(rng.integers(max(0, -rdy), h - rh - max(0, rdy) + 1))
        i2[y0 + rdy:y0 + rdy + rh, x0 + rdx:x0 + rdx + rw] = i1[y0:y0 + rh, x0:x0 + rw]
        rect_xy = (x0, y0)
    i2 = i2 + rng.normal(0.0, noise_sd, size=i2.shape)
    meta = {"d": (dx, dy), "rect": (rw, rh), "rect_d": (rdx, rdy), "rect_xy": rect_xy}
    return _to_u8(i1), _to_u8(i2), meta


def config0(seed: int = 0):
    """128x96 gray pair: texture moved by (+5,-3), a 32x24 block by (-7,+4)."""
    rng = np.random.default_rng(seed)
    return translated_pair(rng, 128, 96, d=(5, -3), rect=(32, 24), rect_d=(-7, 4))


def _road_texture(rng: np.random.Generator, h: int, w: int) -> np.ndarray:
    """Procedural road-scene RGB texture (float64 0..255): multi-scale blurred
    noise, a sky/road vertical gradient and random flat rectangles."""
    out = np.empty((h, w, 3))
    yy = np.linspace(0.0, 1.0, h)[:, None]
    for c in range(3):
        base = (0.55 * noise_texture(rng, h, w, 1.2) + 0.30 * noise_texture(rng, h, w, 4.0)
                + 0.15 * noise_texture(rng, h, w, 12.0))
        base = base + 60.0 * (yy - 0.5) * (1.0 if c == 2 else -0.6)
        out[..., c] = base
    for _ in range(80):
        rw = min(int(rng.integers(8, 90)), max(1, w - 1))
        rh = min(int(rng.integers(6, 60)), max(1, h - 1))
        x0 = int(rng.integers(0, max(1, w - rw)))
        y0 = int(rng.integers(0, max(1, h - rh)))
        col = rng.uniform(0, 255, size=3)
        alpha = rng.uniform(0.35, 0.8)
        out[y0:y0 + rh, x0:x0 + rw, :] = (1 - alpha) * out[y0:y0 + rh, x0:x0 + rw, :] + alpha * col
    for c in range(3):
        out[..., c] = ndimage.gaussian_filter(out[..., c], 0.7, mode="reflect")
    return np.clip(out, 0, 255)


def _warp_rgb(img: np.ndarray, sx: np.ndarray, sy: np.ndarray) -> np.ndarray:
    """Bilinear sample img (HxWx3 float) at source coordinates (sx, sy)."""
    out = np.empty(sx.shape + (3,))
    for c in range(3):
        out[..., c] = ndimage.map_coordinates(img[..., c], [sy, sx], order=1, mode="nearest")
    return out


def _kitti_like(rng: np.random.Generator, w: int, h: int, max_flow: float = 150.0,
                n_boxes: int = 4, occl: float = 0.20, noise_sd: float = 2.0):
    tex = _road_texture(rng, h, w)
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    alpha = max_flow / np.hypot(cx, cy)   # |u| = alpha * |p - c| peaks at the corners
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    # frame 2 point q comes from frame 1 point c + (q - c) / (1 + alpha)
    i2 = _warp_rgb(tex, cx + (xs - cx) / (1.0 + alpha), cy + (ys - cy) / (1.0 + alpha))
    i1 = tex.copy()
    # independently translating textured boxes, about `occl` of the area in total
    area_each = occl * w * h / n_boxes
    boxes = []
    for _ in range(n_boxes):
        aspect = rng.uniform(0.8, 2.0)
        bh = int(min(h - 2, max(8, np.sqrt(area_each / aspect))))
        bw = int(min(w - 2, max(8, area_each / bh)))
        t = rng.integers(-40, 41, size=2)
        x0 = int(rng.integers(max(0, -t[0]), w - bw - max(0, t[0]) + 1))
        y0 = int(rng.integers(max(0, -t[1]), h - bh - max(0, t[1]) + 1))
        btex = _road_texture(rng, bh, bw) if bw * bh > 0 else None
        i1[y0:y0 + bh, x0:x0 + bw] = btex
        i2[y0 + t[1]:y0 + t[1] + bh, x0 + t[0]:x0 + t[0] + bw] = btex
        boxes.append((x0, y0, bw, bh, int(t[0]), int(t[1])))
    i1 = i1 + rng.normal(0.0, noise_sd, size=i1.shape)
    i2 = i2 + rng.normal(0.0, noise_sd, size=i2.shape)
    meta = {"alpha": float(alpha), "centre": (cx, cy), "boxes": boxes}
    return _to_u8(i1), _to_u8(i2), meta


def config1(seed: int = 1, w: int = 1242, h: int = 375):
    """KITTI-shaped RGB pair: planar expansion about the image centre with
    |flow| up to 150 px, four translating boxes (~20% occlusion), N(0,2)."""
    return _kitti_like(np.random.default_rng(seed), w, h)


def _sintel_like(rng: np.random.Generator, w: int, h: int, n_bumps: int = 6,
                 peak: float = 60.0, n_layers: int = 3, noise_sd: float = 3.0):
    tex = _road_texture(rng, h, w)
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    ux = np.zeros((h, w))
    uy = np.zeros((h, w))
    for _ in range(n_bumps):
        c = rng.uniform([0, 0], [w, h])
        s = rng.uniform(40.0, 120.0)
        ang = rng.uniform(0, 2 * np.pi)
        g = np.exp(-((xs - c[0]) ** 2 + (ys - c[1]) ** 2) / (2 * s * s))
        ux += peak * np.cos(ang) * g
        uy += peak * np.sin(ang) * g
    m = np.hypot(ux, uy).max()
    if m > peak:
        ux *= peak / m
        uy *= peak / m
    i1 = tex.copy()
    i2 = _warp_rgb(tex, xs - ux, ys - uy)
    # elliptical layers with independent affine motion, drawn far to near
    depth = rng.permutation(n_layers)
    for li in np.argsort(depth):
        a = rng.uniform(40, 160)
        b = rng.uniform(30, 110)
        c = rng.uniform([a, b], [w - a, h - b])
        lt = _road_texture(rng, h, w)
        th = rng.uniform(-0.08, 0.08)
        sc = rng.uniform(0.95, 1.05)
        A = sc * np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        t = rng.uniform(-30, 30, size=2)
        inside1 = ((xs - c[0]) / a) ** 2 + ((ys - c[1]) / b) ** 2 <= 1.0
        i1[inside1] = lt[inside1]
        # frame 2: q = c + A (p - c) + t  =>  p = c + A^-1 (q - c - t)
        Ai = np.linalg.inv(A)
        qx, qy = xs - c[0] - t[0], ys - c[1] - t[1]
        px = c[0] + Ai[0, 0] * qx + Ai[0, 1] * qy
        py = c[1] + Ai[1, 0] * qx + Ai[1, 1] * qy
        inside2 = ((px - c[0]) / a) ** 2 + ((py - c[1]) / b) ** 2 <= 1.0
        warped = _warp_rgb(lt, px, py)
        i2[inside2] = warped[inside2]
    g1, g2 = rng.uniform(0.9, 1.1, size=2)
    i1 = g1 * i1 + rng.normal(0.0, noise_sd, size=i1.shape)
    i2 = g2 * i2 + rng.normal(0.0, noise_sd, size=i2.shape)
    return _to_u8(i1), _to_u8(i2), {"gains": (float(g1), float(g2))}


def config2(seed: int = 2, w: int = 1024, h: int = 436):
    """Sintel-shaped RGB pair: six Gaussian-bump displacement fields (peak
    60 px), three elliptical affine layers by depth, gain 0.9..1.1, N(0,3)."""
    return _sintel_like(np.random.default_rng(seed), w, h)


SERVE_SIZES = ((320, 240), (640, 480), (1024, 436), (1242, 375))


def config3_stream(seed: int = 3, n: int = 256, rate_hz: float = 100.0):
    """Served stream: n requests with Poisson arrivals at ``rate_hz``; sizes
    uniform over SERVE_SIZES, each pair KITTI- or Sintel-like by coin flip.

    Returns a list of dicts {arrival_s, img1, img2, size, kind}.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
    reqs = []
    for i in range(n):
        w, h = SERVE_SIZES[int(rng.integers(0, len(SERVE_SIZES)))]
        kind = "kitti" if rng.integers(0, 2) == 0 else "sintel"
        sub = np.random.default_rng([seed, i])
        if kind == "kitti":
            i1, i2, _ = _kitti_like(sub, w, h)
        else:
            i1, i2, _ = _sintel_like(sub, w, h)
        reqs.append({"arrival_s": float(t[i]), "img1": i1, "img2": i2, "size": (w, h), "kind": kind})
    return reqs


def config4_batch(seed: int = 4, n: int = 4096, lo: int = 96, hi: int = 256):
    """n uneven gray pairs, sides uniform on [lo, hi], c0-style motion with a
    random integer translation in [-24, 24]^2 (block moved independently)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        w = int(rng.integers(lo, hi + 1))
        h = int(rng.integers(lo, hi + 1))
        d = rng.integers(-24, 25, size=2)
        rd = rng.integers(-24, 25, size=2)
        sub = np.random.default_rng([seed, i])
        i1, i2, meta = translated_pair(sub, w, h, d=tuple(int(v) for v in d), rect=(32, 24),
                                       rect_d=tuple(int(v) for v in rd))
        out.append((i1, i2, meta))
    return out


def config3_requests(seed: int = 3, n: int = 256, per_kind: int = 2):
    """Served-stream workload drawn like ``config3_stream`` but over a pool of
    ``per_kind`` distinct pairs per (size, generator) so it builds quickly.

    Returns (requests, pool): requests is a list of dicts {size, kind, pool_key,
    unit_gap} (unit_gap = Exp(1) inter-arrival gap, scaled by 1/rate by the
    caller); pool maps (w, h, kind, k) -> (img1, img2).
    """
    rng = np.random.default_rng(seed)
    pool = {}
    for (w, h) in SERVE_SIZES:
        for kind in ("kitti", "sintel"):
            for k in range(per_kind):
                sub = np.random.default_rng([seed, w, h, 0 if kind == "kitti" else 1, k])
                gen = _kitti_like if kind == "kitti" else _sintel_like
                i1, i2, _ = gen(sub, w, h)
                pool[(w, h, kind, k)] = (i1, i2)
    reqs = []
    for _ in range(n):
        w, h = SERVE_SIZES[int(rng.integers(0, len(SERVE_SIZES)))]
        kind = "kitti" if rng.integers(0, 2) == 0 else "sintel"
        k = int(rng.integers(0, per_kind))
        reqs.append({"size": (w, h), "kind": kind, "pool_key": (w, h, kind, k),
                     "unit_gap": float(rng.exponential(1.0))})
    return reqs, pool
