"""Seeded synthetic inputs for dictionary learning, shared by the HIP path and the oracle.

This module only draws inputs.  It holds none of the method's arithmetic
(no sparse coding, no atom update, no error), so both sides of every parity
test receive identical bytes from here and nothing else in common.

Workloads (the paper's image experiments, Sec. 4.2-4.4, use 8x8 blocks of
normalised images; those images are not available, so piecewise-smooth
synthetic images stand in for them, with the same patch shapes):

* ``recovery_problem``: the dictionary-recovery setting of Sec. 4.1
  (random unit-norm dictionary, s-sparse Gaussian combinations, white noise).
* ``image_patches``: patches of synthetic images that sum random star-shaped
  polygons filled with linear gradients, min-max scaled to [0, 1], plus
  Gaussian texture noise; each patch is made zero-mean.
* ``initial_dictionary``: n distinct random signals, normalised (the paper
  initialises with a random selection of data vectors, Sec. 4.1).

Layouts: signals ``Y`` are ``[m][p]`` (one signal per row), dictionaries
``D`` are ``[n][p]`` (one atom per row), both float32 unless stated.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "recovery_problem",
    "synthetic_images",
    "image_patches",
    "initial_dictionary",
    "workload",
    "batched_problems",
    "mlp_params",
    "unpack_mlp",
    "WORKLOADS",
]


@dataclass
class Workload:
    """One dictionary-learning problem instance."""

    name: str
    p: int
    n: int
    s: int
    m: int
    iters: int
    group_sizes: tuple
    Y: np.ndarray  # [m][p] float32
    D0: np.ndarray  # [n][p] float32, unit-norm rows
    extra: dict = field(default_factory=dict)


def _unit_rows(A: np.ndarray) -> np.ndarray:
    nrm = np.sqrt((A.astype(np.float64) ** 2).sum(axis=1, keepdims=True))
    nrm[nrm == 0] = 1.0
    return (A / nrm).astype(np.float32)


def recovery_problem(p: int, n: int, s: int, m: int, noise_std: float, seed: int,
                     snr_db: float | None = None):
    """Random unit-norm dictionary and s-sparse noisy signals (Sec. 4.1 setting).

    Returns ``(Y [m][p] f32, D_true [n][p] f32, idx_true [m][s] i32,
    val_true [m][s] f32)``.  Each signal combines ``s`` distinct atoms at
    uniform random positions with N(0,1) weights.  Noise is N(0, noise_std^2),
    or, when ``snr_db`` is given, white noise scaled so that
    10 log10(||DX||^2 / ||N||^2) equals it over the whole set.
    """
    rng = np.random.default_rng(seed)
    D_true = _unit_rows(rng.standard_normal((n, p)))
    idx = np.empty((m, s), dtype=np.int32)
    for i in range(m):
        idx[i] = rng.choice(n, size=s, replace=False)
    val = rng.standard_normal((m, s)).astype(np.float32)
    clean = np.einsum("ms,msp->mp", val.astype(np.float64),
                      D_true[idx].astype(np.float64))
    noise = rng.standard_normal((m, p))
    if snr_db is not None:
        if math.isinf(snr_db):
            noise = np.zeros_like(noise)
        else:
            scale = math.sqrt((clean ** 2).sum() / (noise ** 2).sum() / 10 ** (snr_db / 10))
            noise = noise * scale
    else:
        noise = noise * noise_std
    Y = (clean + noise).astype(np.float32)
    return Y, D_true, idx, val


def _polygon_mask(xs: np.ndarray, ys: np.ndarray, vx: np.ndarray, vy: np.ndarray) -> np.ndarray:
    """Even-odd point-in-polygon test at the given pixel centres."""
    inside = np.zeros(xs.shape, dtype=bool)
    k = len(vx)
    for a in range(k):
        b = (a + 1) % k
        x0, y0, x1, y1 = vx[a], vy[a], vx[b], vy[b]
        crosses = (y0 > ys) != (y1 > ys)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = x0 + (ys - y0) * (x1 - x0) / (y1 - y0)
        inside ^= crosses & (xs < xint)
    return inside


def synthetic_images(count: int, size: int, seed: int) -> np.ndarray:
    """``count`` piecewise-smooth images of ``size x size`` pixels, float64.

    Each image sums 6-12 star-shaped polygons (3-8 vertices, radii
    U(24, 192) scaled by size/512, sorted uniform angles, uniform centre);
    each polygon is filled with a linear-gradient field
    a + b (x - cx) + c (y - cy), a ~ U(-1, 1), b, c ~ N(0, (2/size)^2).
    The sum is min-max scaled to [0, 1] and N(0, 0.02^2) noise is added
    (no clipping).
    """
    rng = np.random.default_rng(seed)
    scale = size / 512.0
    yy, xx = np.mgrid[0:size, 0:size].astype(np.float64) + 0.5
    out = np.empty((count, size, size), dtype=np.float64)
    for b in range(count):
        img = np.zeros((size, size), dtype=np.float64)
        npoly = int(rng.integers(6, 13))
        for _ in range(npoly):
            nv = int(rng.integers(3, 9))
            cx, cy = rng.uniform(0, size, size=2)
            radii = rng.uniform(24 * scale, 192 * scale, size=nv)
            ang = np.sort(rng.uniform(0, 2 * math.pi, size=nv))
            vx = cx + radii * np.cos(ang)
            vy = cy + radii * np.sin(ang)
            a = rng.uniform(-1, 1)
            gb, gc = rng.normal(0, 2.0 / size, size=2)
            x0 = max(int(math.floor(vx.min())), 0)
            x1 = min(int(math.ceil(vx.max())) + 1, size)
            y0 = max(int(math.floor(vy.min())), 0)
            y1 = min(int(math.ceil(vy.max())) + 1, size)
            if x0 >= x1 or y0 >= y1:
                continue
            sx = xx[y0:y1, x0:x1]
            sy = yy[y0:y1, x0:x1]
            mask = _polygon_mask(sx, sy, vx, vy)
            field_ = a + gb * (sx - cx) + gc * (sy - cy)
            img[y0:y1, x0:x1] += np.where(mask, field_, 0.0)
        lo, hi = img.min(), img.max()
        img = (img - lo) / (hi - lo) if hi > lo else np.zeros_like(img)
        img += rng.normal(0, 0.02, size=img.shape)
        out[b] = img
    return out


def image_patches(images: np.ndarray, patch: int, m: int, seed: int) -> np.ndarray:
    """``m`` random ``patch x patch`` blocks, flattened row-major, zero-mean, float32."""
    rng = np.random.default_rng(seed)
    count, H, W = images.shape
    b = rng.integers(0, count, size=m)
    r = rng.integers(0, H - patch + 1, size=m)
    c = rng.integers(0, W - patch + 1, size=m)
    off = np.arange(patch)
    rows = r[:, None, None] + off[None, :, None]
    cols = c[:, None, None] + off[None, None, :]
    P = images[b[:, None, None], rows, cols].reshape(m, patch * patch)
    P = P - P.mean(axis=1, keepdims=True)
    return P.astype(np.float32)


def initial_dictionary(Y: np.ndarray, n: int, seed: int) -> np.ndarray:
    """n distinct random signals of ``Y``, normalised to unit norm (zero rows skipped)."""
    rng = np.random.default_rng(seed)
    m = Y.shape[0]
    nrm = np.sqrt((Y.astype(np.float64) ** 2).sum(axis=1))
    order = rng.permutation(m)
    chosen = [i for i in order if nrm[i] > 0][:n]
    if len(chosen) < n:
        raise ValueError("not enough nonzero signals to draw the initial dictionary")
    return _unit_rows(Y[np.array(chosen)])


# Workload recipes, named by what they are.  Sizes follow the paper's image
# experiments (8x8 and 16x16 patches, n in the paper's 128-512 sweep or
# above, s in its 4-12 range) and its recovery experiment.
WORKLOADS = {
    "recovery_p16_n32_s3_m1024": dict(p=16, n=32, s=3, m=1024, iters=10, group_sizes=(32,), seed=101),
    "patches_p64_n256_s6_m16384": dict(p=64, n=256, s=6, m=16384, iters=50, group_sizes=(256, 16),
                                       seed=202, images=8, image_size=512),
    "patches_p256_n1024_s12_m65536": dict(p=256, n=1024, s=12, m=65536, iters=30, group_sizes=(1024,),
                                          seed=303, images=16, image_size=512),
    "patches_p64_n256_s6_m262144": dict(p=64, n=256, s=6, m=262144, iters=40, group_sizes=(256,),
                                        seed=404, images=32, image_size=512),
}


def workload(name: str, m: int | None = None) -> Workload:
    """Build a named workload; ``m`` optionally overrides the number of signals."""
    cfg = dict(WORKLOADS[name])
    seed = cfg.pop("seed")
    mm = cfg["m"] if m is None else m
    if name.startswith("recovery"):
        Y, D_true, idx, val = recovery_problem(cfg["p"], cfg["n"], cfg["s"], mm, 0.01, seed)
        D0 = initial_dictionary(Y, cfg["n"], seed + 1)
        extra = dict(D_true=D_true, idx_true=idx, val_true=val)
    else:
        patch = int(round(math.sqrt(cfg["p"])))
        imgs = synthetic_images(cfg["images"], cfg["image_size"], seed)
        Y = image_patches(imgs, patch, mm, seed + 7)
        D0 = initial_dictionary(Y, cfg["n"], seed + 1)
        extra = {}
    return Workload(name=name, p=cfg["p"], n=cfg["n"], s=cfg["s"], m=mm, iters=cfg["iters"],
                    group_sizes=tuple(cfg["group_sizes"]), Y=Y, D0=D0, extra=extra)


def mlp_params(sizes, seed):
    """Initial weights of the proposal network, packed [W1 b1 W2 b2 W3 b3]
    (W_l of shape [out][in], row-major), float32: He-normal weights
    N(0, 2 / fan_in), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        parts.append((rng.standard_normal((fan_out, fan_in)) * math.sqrt(2.0 / fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def unpack_mlp(vec, sizes):
    """Split a packed parameter vector into [(W, b), ...]."""
    out, off = [], 0
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        W = vec[off:off + fan_in * fan_out].reshape(fan_out, fan_in)
        off += fan_in * fan_out
        b = vec[off:off + fan_out]
        off += fan_out
        out.append((W, b))
    return out


def batched_problems(count: int, seed: int, m_scale: float = 1.0):
    """Uneven independent problems: p in {16,36,64,144,256}, n = 2p or 4p,
    s ~ U{3..16} (capped at p), m log-uniform in [2048, 65536] (times m_scale).

    Each problem draws patches from 4 synthetic 512x512 images of its own (the
    generator and image size of the other patch workloads).  Returns a
    list of dicts with keys p, n, s, m, Y, D0.
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        p = int(rng.choice([16, 36, 64, 144, 256]))
        n = p * int(rng.choice([2, 4]))
        s = min(int(rng.integers(3, 17)), p)
        m = int(round(math.exp(rng.uniform(math.log(2048), math.log(65536)))))
        m = max(int(round(m * m_scale)), n)
        imgs = synthetic_images(4, 512, seed * 1000 + b)
        Y = image_patches(imgs, int(round(math.sqrt(p))), m, seed * 1000 + b + 1)
        D0 = initial_dictionary(Y, n, seed * 1000 + b + 2)
        out.append(dict(p=p, n=n, s=s, m=m, Y=Y, D0=D0))
    return out
