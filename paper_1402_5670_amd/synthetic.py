"""Seeded synthetic inputs: piecewise-constant "cartoon" images and volumes
plus Gaussian noise, the model class the paper's analysis is built on
(Section 1: cartoon-like functions).  They stand in for the paper's natural
test images and videos, which are not used.

This module holds input generation only and none of the transform's
arithmetic; both the HIP path's tests/benchmarks and the FP64 oracle's tests
draw their inputs from here.

Recipe (numpy PCG64 via default_rng(seed)):
  2D: background ~ U[0,1]; n ~ U{8..16} shapes painted in order; each shape
      is an ellipse (p = 1/2; centre ~ U over the image, semi-axes
      ~ U[m/32, m/4] with m = min(H, W), angle ~ U[0, pi)) or a star-shaped
      polygon (3..8 vertices at sorted U[0, 2 pi) angles, radii r*U[0.5, 1],
      r ~ U[m/16, m/4]); intensity ~ U[0,1]; membership is tested at pixel
      centres, so images are exactly piecewise constant.
  3D: background ~ U[0,1]; n ~ U{10..20} ellipsoids, centre ~ U over the
      volume, semi-axes ~ U[m/32, m/4], rotation = Q of a QR factorisation
      of a standard normal 3x3 matrix; intensity ~ U[0,1].
  noise: default_rng([seed, 1]).standard_normal(shape) * sigma (not clipped).
"""
import numpy as np


def _inside_polygon(px, py, vx, vy):
    """Even-odd rule for points (px, py) against the closed polygon (vx, vy)."""
    inside = np.zeros(px.shape, dtype=bool)
    n = len(vx)
    for a in range(n):
        b = (a + 1) % n
        x1, y1, x2, y2 = vx[a], vy[a], vx[b], vy[b]
        crosses = (y1 > py) != (y2 > py)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = x1 + (py - y1) * (x2 - x1) / (y2 - y1)
        inside ^= crosses & (px < xint)
    return inside


def cartoon2d_shapes(H, W, seed):
    """Draw the background level and the shape list of one cartoon image.

    Each shape is ("ellipse", value, cx, cy, a, b, theta) or
    ("polygon", value, vx, vy) with vertices in pixel coordinates."""
    rng = np.random.default_rng(seed)
    background = rng.uniform(0.0, 1.0)
    m = float(min(H, W))
    shapes = []
    for _ in range(int(rng.integers(8, 17))):
        val = rng.uniform(0.0, 1.0)
        if rng.uniform() < 0.5:
            cy, cx = rng.uniform(0, H), rng.uniform(0, W)
            a, b = rng.uniform(m / 32, m / 4, size=2)
            th = rng.uniform(0.0, np.pi)
            shapes.append(("ellipse", val, cx, cy, a, b, th))
        else:
            cy, cx = rng.uniform(0, H), rng.uniform(0, W)
            nv = int(rng.integers(3, 9))
            ang = np.sort(rng.uniform(0.0, 2 * np.pi, size=nv))
            r = rng.uniform(m / 16, m / 4)
            rad = r * rng.uniform(0.5, 1.0, size=nv)
            shapes.append(("polygon", val, cx + rad * np.cos(ang), cy + rad * np.sin(ang)))
    return background, shapes


def cartoon2d(H, W, seed):
    background, shapes = cartoon2d_shapes(H, W, seed)
    img = np.full((H, W), background)
    yy, xx = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    for sh in shapes:
        if sh[0] == "ellipse":
            _, val, cx, cy, a, b, th = sh
            dx, dy = xx - cx, yy - cy
            u = dx * np.cos(th) + dy * np.sin(th)
            v = -dx * np.sin(th) + dy * np.cos(th)
            mask = (u / a) ** 2 + (v / b) ** 2 <= 1.0
        else:
            _, val, vx, vy = sh
            mask = _inside_polygon(xx, yy, vx, vy)
        img[mask] = val
    return img


SHAPE_RECORD = 24   # floats per shape in shape_table


def shape_table(H, W, seeds, max_shapes=16):
    """Pack the shapes of several images for a rasterizer:
    float32 [n_images][1 + max_shapes * SHAPE_RECORD] with
    [0] = background; per shape: type (0 none, 1 ellipse, 2 polygon), value,
    ellipse: cx, cy, a, b, cos(theta), sin(theta);
    polygon: n, then up to 8 (x, y) vertex pairs from offset 3."""
    out = np.zeros((len(seeds), 1 + max_shapes * SHAPE_RECORD), dtype=np.float32)
    for n, seed in enumerate(seeds):
        bg, shapes = cartoon2d_shapes(H, W, seed)
        out[n, 0] = bg
        for k, sh in enumerate(shapes[:max_shapes]):
            rec = out[n, 1 + k * SHAPE_RECORD:1 + (k + 1) * SHAPE_RECORD]
            if sh[0] == "ellipse":
                _, val, cx, cy, a, b, th = sh
                rec[:8] = (1, val, cx, cy, a, b, np.cos(th), np.sin(th))
            else:
                _, val, vx, vy = sh
                rec[0], rec[1], rec[2] = 2, val, len(vx)
                for v in range(len(vx)):
                    rec[3 + 2 * v] = vx[v]
                    rec[4 + 2 * v] = vy[v]
    return out


def cartoon3d(D, H, W, seed):
    rng = np.random.default_rng(seed)
    vol = np.full((D, H, W), rng.uniform(0.0, 1.0))
    zz, yy, xx = np.meshgrid(np.arange(D) + 0.5, np.arange(H) + 0.5, np.arange(W) + 0.5,
                             indexing="ij")
    m = float(min(D, H, W))
    for _ in range(int(rng.integers(10, 21))):
        val = rng.uniform(0.0, 1.0)
        c = rng.uniform([0, 0, 0], [D, H, W])
        ax = rng.uniform(m / 32, m / 4, size=3)
        q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        rel = np.stack([zz - c[0], yy - c[1], xx - c[2]], axis=-1) @ q
        mask = np.sum((rel / ax) ** 2, axis=-1) <= 1.0
        vol[mask] = val
    return vol


def moving_ellipses_video(T, H, W, seed):
    """T frames of H x W (a [T][H][W] volume): background U[0,1] and 6-12
    ellipses of intensity U[0,1] that translate at constant velocity and
    rotate at a constant rate over the frames (painter's order, membership at
    pixel centres), a synthetic stand-in for video data."""
    rng = np.random.default_rng(seed)
    vol = np.full((T, H, W), rng.uniform(0.0, 1.0))
    yy, xx = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    m = float(min(H, W))
    for _ in range(int(rng.integers(6, 13))):
        val = rng.uniform(0.0, 1.0)
        c0 = rng.uniform([0, 0], [H, W])
        vel = rng.uniform(-0.5, 0.5, size=2)            # pixels per frame
        a, b = rng.uniform(m / 24, m / 5, size=2)
        th0, om = rng.uniform(0.0, np.pi), rng.uniform(-0.02, 0.02)
        for t in range(T):
            cy, cx = c0 + vel * t
            th = th0 + om * t
            u = (xx - cx) * np.cos(th) + (yy - cy) * np.sin(th)
            v = -(xx - cx) * np.sin(th) + (yy - cy) * np.cos(th)
            mask = (u / a) ** 2 + (v / b) ** 2 <= 1.0
            vol[t][mask] = val
    return vol


def noise(shape, seed, sigma):
    return np.random.default_rng([seed, 1]).standard_normal(shape) * sigma


def noisy_cartoon2d(H, W, seed, sigma):
    clean = cartoon2d(H, W, seed)
    return clean, clean + noise((H, W), seed, sigma)


def noisy_cartoon3d(D, H, W, seed, sigma):
    clean = cartoon3d(D, H, W, seed)
    return clean, clean + noise((D, H, W), seed, sigma)


# Workload recipes ----------------------------------------------------------

def batch_sigmas(n):
    """Noise levels (20, 30, 40)/255 cycled over a batch."""
    return np.array([(20.0, 30.0, 40.0)[b % 3] / 255.0 for b in range(n)])


def uneven_sizes(n=64, seed=4000, choices=(256, 384, 512, 1024)):
    """Image sizes drawn uniformly from the given square sizes."""
    idx = np.random.default_rng(seed).integers(0, len(choices), n)
    return [int(choices[i]) for i in idx]


# Occlusion masks (1 = known sample, 0 = missing) -----------------------------
# The paper's inpainting masks (random 80 %, squares 28 %, text 25 %; random
# 80 % and cubes 5 % for video) are drawn here from seeded generators:
#   random:  default_rng([seed, 3]).random(shape) >= occlusion
#   squares: axis-aligned squares, side ~ U{m/32 .. m/8}, top-left corner ~ U
#            over the grid (clipped at the border), added until at least the
#            target fraction is covered (cubes in 3D likewise)
#   strokes: text-like strokes, each a 2-4 segment polyline of width
#            ~ U{max(2, m/256) .. max(3, m/128)} pixels and segment length
#            ~ U[m/64, m/16], drawn until the target fraction is covered

def random_mask(shape, seed, occlusion=0.8):
    return (np.random.default_rng([seed, 3]).random(shape) >= occlusion).astype(np.uint8)


def squares_mask(shape, seed, occlusion=0.28):
    rng = np.random.default_rng([seed, 4])
    shape = tuple(int(s) for s in shape)
    m = min(shape)
    miss = np.zeros(shape, dtype=bool)
    total = miss.size
    while miss.sum() < occlusion * total:
        side = int(rng.integers(max(1, m // 32), max(2, m // 8) + 1))
        corner = [int(rng.integers(0, s)) for s in shape]
        miss[tuple(slice(c, min(c + side, s)) for c, s in zip(corner, shape))] = True
    return (~miss).astype(np.uint8)


def strokes_mask(H, W, seed, occlusion=0.25):
    rng = np.random.default_rng([seed, 5])
    m = min(H, W)
    miss = np.zeros((H, W), dtype=bool)
    while miss.sum() < occlusion * H * W:
        width = float(rng.integers(max(2, m // 256), max(3, m // 128) + 1))
        p = rng.uniform([0, 0], [H, W])
        for _ in range(int(rng.integers(2, 5))):
            ang = rng.uniform(0.0, 2 * np.pi)
            q = p + rng.uniform(m / 64, m / 16) * np.array([np.sin(ang), np.cos(ang)])
            r = width / 2 + 1
            y0, y1 = int(max(0, min(p[0], q[0]) - r)), int(min(H, max(p[0], q[0]) + r + 1))
            x0, x1 = int(max(0, min(p[1], q[1]) - r)), int(min(W, max(p[1], q[1]) + r + 1))
            if y1 > y0 and x1 > x0:
                yy, xx = np.meshgrid(np.arange(y0, y1) + 0.5, np.arange(x0, x1) + 0.5, indexing="ij")
                d = q - p
                tt = np.clip(((yy - p[0]) * d[0] + (xx - p[1]) * d[1]) / max(d @ d, 1e-12), 0, 1)
                dist2 = (yy - p[0] - tt * d[0]) ** 2 + (xx - p[1] - tt * d[1]) ** 2
                miss[y0:y1, x0:x1] |= dist2 <= (width / 2) ** 2
            p = q
    return (~miss).astype(np.uint8)


def inpainting_case(H, W, seed, kind):
    """(clean cartoon image, mask) for one of the paper's mask types."""
    clean = cartoon2d(H, W, seed)
    if kind == "random":
        mask = random_mask((H, W), seed)
    elif kind == "squares":
        mask = squares_mask((H, W), seed)
    elif kind == "text":
        mask = strokes_mask(H, W, seed)
    else:
        raise ValueError(kind)
    return clean, mask


def _draw_segment(img, p, q, width):
    """Set the pixels whose centre lies within width/2 of segment pq."""
    H, W = img.shape
    r = width / 2 + 1
    y0, y1 = int(max(0, min(p[0], q[0]) - r)), int(min(H, max(p[0], q[0]) + r + 1))
    x0, x1 = int(max(0, min(p[1], q[1]) - r)), int(min(W, max(p[1], q[1]) + r + 1))
    if y1 <= y0 or x1 <= x0:
        return
    yy, xx = np.meshgrid(np.arange(y0, y1) + 0.5, np.arange(x0, x1) + 0.5, indexing="ij")
    d = q - p
    tt = np.clip(((yy - p[0]) * d[0] + (xx - p[1]) * d[1]) / max(d @ d, 1e-12), 0, 1)
    dist2 = (yy - p[0] - tt * d[0]) ** 2 + (xx - p[1] - tt * d[1]) ** 2
    img[y0:y1, x0:x1] |= dist2 <= (width / 2) ** 2


def points_and_curves(H, W, seed):
    """Binary test pair for image decomposition: (curves f0, points f1).

    default_rng([seed, 6]): f0 holds U{4..8} cubic Bezier curves (control
    points U over the image, 64 segments each, width U[m/256, m/128] with a
    floor of 1.5 pixels, m = min(H, W)); f1 holds U{30..60} disks of radius
    U[m/256, m/128] (floor 1.5 pixels) at uniform centres."""
    rng = np.random.default_rng([seed, 6])
    m = min(H, W)
    curves = np.zeros((H, W), dtype=bool)
    for _ in range(int(rng.integers(4, 9))):
        ctl = rng.uniform([0, 0], [H, W], size=(4, 2))
        width = max(1.5, rng.uniform(m / 256, m / 128))
        s = np.linspace(0.0, 1.0, 65)[:, None]
        pts = ((1 - s) ** 3 * ctl[0] + 3 * (1 - s) ** 2 * s * ctl[1] + 3 * (1 - s) * s ** 2 * ctl[2]
               + s ** 3 * ctl[3])
        for a in range(64):
            _draw_segment(curves, pts[a], pts[a + 1], width)
    points = np.zeros((H, W), dtype=bool)
    yy, xx = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    for _ in range(int(rng.integers(30, 61))):
        c = rng.uniform([0, 0], [H, W])
        rad = max(1.5, rng.uniform(m / 256, m / 128))
        y0, y1 = int(max(0, c[0] - rad - 1)), int(min(H, c[0] + rad + 2))
        x0, x1 = int(max(0, c[1] - rad - 1)), int(min(W, c[1] + rad + 2))
        sub = (yy[y0:y1, x0:x1] - c[0]) ** 2 + (xx[y0:y1, x0:x1] - c[1]) ** 2 <= rad ** 2
        points[y0:y1, x0:x1] |= sub
    return curves.astype(np.float64), points.astype(np.float64)
