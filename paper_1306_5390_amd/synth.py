"""Seeded synthetic grey images with salt-and-pepper noise.

The paper measures on natural grey images from a segmentation benchmark at
5-20% salt-and-pepper density (Section 3, Tables 1-2).  Those images are not
available here; these seeded images stand in for them.  They have the
structure such images have for this method -- flat regions with edges, a slow
gradient and fine texture -- and salt (255) and pepper (0) noise at a chosen
density.

This module only draws inputs.  It holds none of the method's arithmetic and
is shared by the tests, the benchmark and the smoke check.

Clean image recipe (every choice fixed here, all draws from one
numpy.random.Generator(PCG64(seed)) in this order):
  1. background level ~ U[20, 235];
  2. 8 convex polygons, painted in order: centre uniform in the image, radius
     U[0.1, 0.4] * min(H, W), 3-8 vertices at sorted uniform angles, level
     ~ U[20, 235];
  3. a linear gradient, uniform direction, 40 grey levels peak to peak,
     zero mean over the image;
  4. i.i.d. Gaussian texture N(0, 6^2), drawn in blocks of 256 rows;
  5. round half to even, clip to [0, 255].
Noise: each pixel independently draws u ~ U[0, 1) (float64, blocks of 256
rows, its own Generator seeded with seed + 1_000_003); u < rho/2 -> 0 (pepper),
rho/2 <= u < rho -> 255 (salt).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_BLOCK_ROWS = 256
_NOISE_SEED_OFFSET = 1_000_003


def _polygon(rng: np.random.Generator, h: int, w: int):
    cy = rng.uniform(0.0, h)
    cx = rng.uniform(0.0, w)
    rad = rng.uniform(0.1, 0.4) * min(h, w)
    nv = int(rng.integers(3, 9))
    ang = np.sort(rng.uniform(0.0, 2.0 * math.pi, size=nv))
    level = float(rng.uniform(20.0, 235.0))
    vy = cy + rad * np.sin(ang)
    vx = cx + rad * np.cos(ang)
    return vy, vx, level


def _row_span(vy: np.ndarray, vx: np.ndarray, y: float):
    """Column interval [x0, x1] where the horizontal line at y crosses the
    convex polygon, or None."""
    xs = []
    n = len(vy)
    for e in range(n):
        y0, x0 = vy[e], vx[e]
        y1, x1 = vy[(e + 1) % n], vx[(e + 1) % n]
        if (y0 <= y < y1) or (y1 <= y < y0):
            t = (y - y0) / (y1 - y0)
            xs.append(x0 + t * (x1 - x0))
    if len(xs) < 2:
        return None
    return min(xs), max(xs)


def clean_image(h: int, w: int, seed: int) -> np.ndarray:
    """Piecewise-constant regions + gradient + texture, uint8 [h, w]."""
    if h < 0 or w < 0:
        raise ValueError("negative image size")
    rng = np.random.Generator(np.random.PCG64(seed))
    base = np.empty((h, w), dtype=np.float32)
    base.fill(float(rng.uniform(20.0, 235.0)))
    polys = [_polygon(rng, h, w) for _ in range(8)]
    theta = rng.uniform(0.0, 2.0 * math.pi)
    if h == 0 or w == 0:
        return np.zeros((h, w), dtype=np.uint8)
    for vy, vx, level in polys:
        ylo = max(0, int(math.floor(vy.min())))
        yhi = min(h - 1, int(math.ceil(vy.max())))
        for y in range(ylo, yhi + 1):
            span = _row_span(vy, vx, y + 0.5)
            if span is None:
                continue
            x0 = max(0, int(math.ceil(span[0] - 0.5)))
            x1 = min(w - 1, int(math.floor(span[1] - 0.5)))
            if x1 >= x0:
                base[y, x0:x1 + 1] = level
    # gradient: 40 levels peak to peak, zero mean over the rectangle
    ct, st = math.cos(theta), math.sin(theta)
    corners = [0.0, ct * (w - 1), st * (h - 1), ct * (w - 1) + st * (h - 1)]
    pmin, pmax = min(corners), max(corners)
    span = pmax - pmin if pmax > pmin else 1.0
    xs = (ct * np.arange(w, dtype=np.float64))
    out = np.empty((h, w), dtype=np.uint8)
    for y0 in range(0, h, _BLOCK_ROWS):
        y1 = min(h, y0 + _BLOCK_ROWS)
        ys = st * np.arange(y0, y1, dtype=np.float64)
        proj = ys[:, None] + xs[None, :]
        grad = 40.0 * ((proj - pmin) / span - 0.5)
        tex = rng.standard_normal(size=(y1 - y0, w)) * 6.0
        v = base[y0:y1].astype(np.float64) + grad + tex
        out[y0:y1] = np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return out


def add_salt_pepper(img: np.ndarray, density: float, seed: int) -> np.ndarray:
    """Independent per-pixel salt-and-pepper noise at the given density."""
    if not (0.0 <= density <= 1.0):
        raise ValueError("density must be in [0, 1]")
    rng = np.random.Generator(np.random.PCG64(seed + _NOISE_SEED_OFFSET))
    out = np.array(img, dtype=np.uint8, copy=True)
    h = out.shape[0]
    for y0 in range(0, h, _BLOCK_ROWS):
        y1 = min(h, y0 + _BLOCK_ROWS)
        u = rng.random(size=(y1 - y0, out.shape[1]))
        blk = out[y0:y1]
        blk[u < density * 0.5] = 0
        blk[(u >= density * 0.5) & (u < density)] = 255
    return out


def noise_thresholds(density: float) -> tuple:
    """(t_pepper, t_salt) of the counter-based salt-and-pepper noise for a
    density in [0, 1]: a pixel whose 32-bit draw u is below t_pepper becomes
    pepper, below t_salt salt.  Integer thresholds, so that every
    implementation takes the same decision."""
    if not (0.0 <= density <= 1.0):
        raise ValueError("density must be in [0, 1]")
    t_salt = min(int(round(density * 2.0 ** 32)), 2 ** 32 - 1)
    return t_salt // 2, t_salt


def noisy_image(h: int, w: int, density: float, seed: int) -> np.ndarray:
    return add_salt_pepper(clean_image(h, w, seed), density, seed)


# ---------------------------------------------------------------------------
# Workload descriptions.  Sizes, densities and parameter draws of the
# measured configurations.
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class ImageSpec:
    rows: int
    cols: int
    density: float
    alpha: int
    beta: int
    k: int
    seed: int

    def image(self) -> np.ndarray:
        return noisy_image(self.rows, self.cols, self.density, self.seed)


def single_481x321() -> ImageSpec:
    """One 481x321 image (the segmentation-benchmark frame size), 10% noise,
    alpha=20, beta=1, k=10."""
    return ImageSpec(321, 481, 0.10, 20, 1, 10, 1)


def sweep_2048() -> list[ImageSpec]:
    """One 2048x2048 image at 30% noise, alpha in {10,20,40} x beta in {1,2},
    k=32 (the same image for all six parameter pairs)."""
    return [ImageSpec(2048, 2048, 0.30, a, b, 32, 2)
            for b in (1, 2) for a in (10, 20, 40)]


def large_single(side: int) -> ImageSpec:
    """8192^2 (seed 3) or 16384^2 (seed 4), 50% noise, alpha=20, beta=2, k=32."""
    seed = {8192: 3, 16384: 4}.get(side, 3)
    return ImageSpec(side, side, 0.50, 20, 2, 32, seed)


def _log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_512(n: int = 512, seed: int = 5) -> list[ImageSpec]:
    """n images, each side log-uniform in [128, 4096] (non-square), density
    U[5%, 60%], alpha ~ U{10..40}, beta ~ U{1,2}, k=32; image i seeded with
    seed*10^6 + i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        h = _log_uniform_int(rng, 128, 4096)
        w = _log_uniform_int(rng, 128, 4096)
        rho = float(rng.uniform(0.05, 0.60))
        a = int(rng.integers(10, 41))
        b = int(rng.integers(1, 3))
        out.append(ImageSpec(h, w, rho, a, b, 32, seed * 1_000_000 + i))
    return out


def serve_pool(n: int = 256, seed: int = 6, side_lo: int = 256,
               side_hi: int = 8192) -> list[ImageSpec]:
    """Request pool: sides log-uniform in [side_lo, side_hi], density
    U[5%, 50%], alpha=20, beta ~ U{1,2}, k=16."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n):
        h = _log_uniform_int(rng, side_lo, side_hi)
        w = _log_uniform_int(rng, side_lo, side_hi)
        rho = float(rng.uniform(0.05, 0.50))
        b = int(rng.integers(1, 3))
        out.append(ImageSpec(h, w, rho, 20, b, 16, seed * 1_000_000 + i))
    return out


def poisson_arrivals(rate: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: cumulative exponential gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def _image_of(spec: "ImageSpec") -> np.ndarray:
    return spec.image()


def generate_many(specs, workers: int = 8) -> list:
    """Images of many specs, generated in `workers` fresh interpreter
    processes (spawned, never forked, so the caller may already hold GPU
    state); results in the order of `specs`."""
    import multiprocessing as mp
    specs = list(specs)
    if workers <= 1 or len(specs) <= 1:
        return [s.image() for s in specs]
    order = sorted(range(len(specs)), key=lambda i: -specs[i].rows * specs[i].cols)
    # close() and join() let the workers exit on their own; leaving the
    # with-block alone would terminate() them with SIGTERM, which a
    # profiler's signal handler in each worker reports as an abort
    with mp.get_context("spawn").Pool(min(workers, len(specs))) as pool:
        res = pool.map(_image_of, [specs[i] for i in order], chunksize=1)
        pool.close()
        pool.join()
    out = [None] * len(specs)
    for i, r in zip(order, res):
        out[i] = r
    return out
