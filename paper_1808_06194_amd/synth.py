"""Seeded synthetic inputs: image pairs, control-point lists, request streams.

This module is shared by the test oracle and the GPU path and therefore holds
none of the matching method's arithmetic (no gradients, no CFOG, no SSD): it
only draws images, shifts and point lists.

The paper's datasets (Table I: ten multimodal pairs of 512^2 to 1074x1080 px;
Table IV: a Sentinel-1 / Sentinel-2 pair of about 30k^2 px) are not available,
so seeded stand-ins of the same character are generated instead:

* reference image A = sum of Gaussian blobs + axis-aligned rectangles + white
  noise (structure at several scales, flat regions, sharp edges);
* sensed image B = |sin(3 A)| times multiplicative Gamma speckle (shape 4,
  mean 1), i.e. a non-linear, non-monotonic intensity mapping plus SAR-like
  speckle, shifted by a seeded integer (dx, dy).

B is cut from the same canvas as A so that B(y, x) = f(A)(y - dy, x - dx)
exactly; the expected match offset of a control point is therefore +(dx, dy).
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np


@dataclasses.dataclass(frozen=True)
class PairSpec:
    """Recipe of one synthetic pair."""
    H: int
    W: int
    n_blobs: int
    blob_sigma: tuple  # (lo, hi) in px
    n_rects: int
    s_max: int  # |shift| bound per axis
    noise_std: float = 0.02
    speckle_shape: float = 4.0


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(k) for k in key]))


def make_canvas(spec: PairSpec, rng: np.random.Generator) -> np.ndarray:
    """Blob + rectangle + noise canvas of size (H + 2 s_max) x (W + 2 s_max), fp64."""
    Hc, Wc = spec.H + 2 * spec.s_max, spec.W + 2 * spec.s_max
    A = np.zeros((Hc, Wc), np.float64)
    lo, hi = spec.blob_sigma
    cy = rng.uniform(0, Hc, spec.n_blobs)
    cx = rng.uniform(0, Wc, spec.n_blobs)
    sg = rng.uniform(lo, hi, spec.n_blobs)
    amp = rng.uniform(0.0, 1.0, spec.n_blobs)
    for i in range(spec.n_blobs):
        R = int(np.ceil(4.0 * sg[i]))
        y0, y1 = max(0, int(cy[i]) - R), min(Hc, int(cy[i]) + R + 1)
        x0, x1 = max(0, int(cx[i]) - R), min(Wc, int(cx[i]) + R + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        ey = np.exp(-((np.arange(y0, y1) - cy[i]) ** 2) / (2 * sg[i] ** 2))
        ex = np.exp(-((np.arange(x0, x1) - cx[i]) ** 2) / (2 * sg[i] ** 2))
        A[y0:y1, x0:x1] += amp[i] * np.outer(ey, ex)
    # rectangles: value v added on [y0, y0+h) x [x0, x0+w) (clipped to the
    # canvas), accumulated as +-v corner impulses and two cumulative sums so
    # that the cost does not grow with the rectangle areas
    side_hi = max(8, spec.W // 4)
    corners = np.zeros((Hc + 1, Wc + 1), np.float64)
    for _ in range(spec.n_rects):
        h = int(rng.integers(8, side_hi + 1))
        w = int(rng.integers(8, side_hi + 1))
        y0 = int(rng.integers(0, Hc))
        x0 = int(rng.integers(0, Wc))
        v = rng.uniform(0.0, 1.0)
        y1, x1 = min(Hc, y0 + h), min(Wc, x0 + w)
        corners[y0, x0] += v
        corners[y0, x1] -= v
        corners[y1, x0] -= v
        corners[y1, x1] += v
    A += np.cumsum(np.cumsum(corners, axis=0), axis=1)[:Hc, :Wc]
    A += rng.normal(0.0, spec.noise_std, A.shape)
    return A


def make_pair(spec: PairSpec, seed: tuple, shift=None):
    """Return (A, B, (dx, dy)) as C-contiguous fp32 arrays of shape (H, W).

    ``shift`` overrides the seeded shift draw (it must lie in [-s_max, s_max]).
    """
    rng = _rng(*seed)
    canvas = make_canvas(spec, rng)
    s = spec.s_max
    if shift is None:
        dx, dy = (int(v) for v in rng.integers(-s, s + 1, 2))
    else:
        dx, dy = (int(v) for v in shift)
        if max(abs(dx), abs(dy)) > s:
            raise ValueError("shift exceeds s_max")
    speckle = rng.gamma(spec.speckle_shape, 1.0 / spec.speckle_shape, canvas.shape)
    Bc = np.abs(np.sin(3.0 * canvas)) * speckle
    H, W = spec.H, spec.W
    A = canvas[s:s + H, s:s + W]
    B = Bc[s - dy:s - dy + H, s - dx:s - dx + W]
    return (np.ascontiguousarray(A, np.float32), np.ascontiguousarray(B, np.float32), (dx, dy))


def grid_cps(H: int, W: int, N: int, r: int, n_side: int) -> np.ndarray:
    """n_side x n_side control points on a regular grid whose template and search
    windows all lie inside an H x W image (margin h + r + 1, h = N // 2).

    Returns int32 array (n, 4) of (x, y, bx, by) with bx = x, by = y.
    """
    h = N // 2
    M = h + r + 1
    xs = [M + int(round(i * (W - 1 - 2 * M) / max(1, n_side - 1))) for i in range(n_side)]
    ys = [M + int(round(i * (H - 1 - 2 * M) / max(1, n_side - 1))) for i in range(n_side)]
    out = np.array([(x, y, x, y) for y in ys for x in xs], np.int32)
    return out.reshape(-1, 4)


def random_cps(rng: np.random.Generator, H: int, W: int, N: int, r: int, n: int) -> np.ndarray:
    """n control points uniform over the positions whose windows fit (same margin rule)."""
    h = N // 2
    M = h + r + 1
    x = rng.integers(M, W - M, n)
    y = rng.integers(M, H - M, n)
    return np.stack([x, y, x, y], axis=1).astype(np.int32)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ---------------------------------------------------------------- workloads
#
# Workload recipes (sizes follow the stand-in plan for the paper's data):
#   plain_256   : one 256^2 pair, 40 blobs sigma 3-15, 20 rects, |shift| <= 8,
#                 25 CPs on a 5x5 grid, template 48, radius 10.
#   plain_2048  : one 2048^2 pair, 800 blobs sigma 3-40, 300 rects,
#                 |shift| <= 20, 400 CPs on a 20x20 grid, template 100, radius 20.
#   batch_64    : 64 pairs with sides from {512,1024,2048,4096}, templates even
#                 in [40,120], radii in [5,30], 50-600 CPs per pair.
#   precision_4096 : one 4096^2 pair, 10,000 random CPs, template 128, radius 32.

PLAIN_256 = dict(spec=PairSpec(256, 256, 40, (3.0, 15.0), 20, 8), N=48, r=10, grid=5, seed=(0, 0))
PLAIN_2048 = dict(spec=PairSpec(2048, 2048, 800, (3.0, 40.0), 300, 20), N=100, r=20, grid=20, seed=(1, 0))


def plain_workload(w: dict, shift=None):
    """(A, B, shift, cps, N, r) for a plain single-pair workload dict."""
    A, B, s = make_pair(w["spec"], w["seed"], shift)
    cps = grid_cps(w["spec"].H, w["spec"].W, w["N"], w["r"], w["grid"])
    return A, B, s, cps, w["N"], w["r"]


def area_scaled_spec(side: int, s_max: int, base=(256, 40, 20), sigma=(3.0, 15.0)) -> PairSpec:
    """Pair spec with blob/rectangle counts scaled by area from a base density."""
    b, nb, nr = base
    f = (side * side) / float(b * b)
    return PairSpec(side, side, max(1, int(round(nb * f))), sigma, max(1, int(round(nr * f))), s_max)


def _batch_pair(args):
    spec, seed, j = args
    return make_pair(spec, (seed, j))


def batch_draws(n_pairs: int = 64, sides=(512, 1024, 2048, 4096), seed: int = 2, max_cps: int = 600,
                min_cps: int = 50, speckle_shape: float = 4.0):
    """Per-pair draws of the heterogeneous batch: (side, N, r, n_cps, spec)."""
    meta = _rng(seed, 999)
    draws = []
    for j in range(n_pairs):
        side = int(meta.choice(sides))
        N = 2 * int(meta.integers(20, 61))
        r = int(meta.integers(5, 31))
        n = int(meta.integers(min_cps, max_cps + 1))
        spec = dataclasses.replace(area_scaled_spec(side, min(8, r)), speckle_shape=speckle_shape)
        draws.append((side, N, r, n, spec))
    return draws


def batch_pair(draws, j: int, seed: int = 2):
    """Pair j of a batch drawn by batch_draws: dict (A, B, shift, cps, N, r)."""
    side, N, r, n, spec = draws[j]
    A, B, s = make_pair(spec, (seed, j))
    cps = random_cps(_rng(seed, j, 1), side, side, N, r, n)
    return dict(A=A, B=B, shift=s, cps=cps, N=N, r=r)


def batch_workload(n_pairs: int = 64, sides=(512, 1024, 2048, 4096), seed: int = 2,
                   max_cps: int = 600, min_cps: int = 50, pool_map=map, speckle_shape: float = 4.0):
    """Heterogeneous batch: list of dicts (A, B, shift, cps, N, r) per pair.
    `pool_map` may be a process pool's map (each pair has its own seed)."""
    draws = batch_draws(n_pairs, sides, seed, max_cps, min_cps, speckle_shape)
    imgs = list(pool_map(_batch_pair, [(d[4], seed, j) for j, d in enumerate(draws)]))
    out = []
    for j, ((side, N, r, n, _), (A, B, s)) in enumerate(zip(draws, imgs)):
        cps = random_cps(_rng(seed, j, 1), side, side, N, r, n)
        out.append(dict(A=A, B=B, shift=s, cps=cps, N=N, r=r))
    return out


# ---------------------------------------------------------------- serving
#
# Serving recipe: 32 resident pairs, 8 each of 1024^2, 2048^2, 4096^2 and
# 8192^2 (densities area-scaled from plain_256, |shift| <= 8, seeds (4, j));
# requests arrive as a Poisson process; each names a pair uniformly and asks
# for 1-500 control points at uniform valid positions with template side
# 2 * U{20..64} and radius U{5..32}.

SERVE_SIDES = (1024,) * 8 + (2048,) * 8 + (4096,) * 8 + (8192,) * 8


def serve_pair(j: int, sides=SERVE_SIDES):
    """(A, B, shift) of serving pair j."""
    return make_pair(area_scaled_spec(sides[j], 8), (4, j))


def serve_requests(n: int, rate: float, sides=SERVE_SIDES, seed: int = 999, max_cps: int = 500):
    """n requests with Poisson arrivals of `rate` per second: list of dicts
    (t arrival offset in s, pair, cps (k, 4) int32, N, r)."""
    rng = _rng(4, seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    out = []
    for i in range(n):
        p = int(rng.integers(0, len(sides)))
        N = 2 * int(rng.integers(20, 65))
        r = int(rng.integers(5, 33))
        k = int(rng.integers(1, max_cps + 1))
        cps = random_cps(rng, sides[p], sides[p], N, r, k)
        out.append(dict(t=float(t[i]), pair=p, cps=cps, N=N, r=r))
    return out


def reject_points(rng: np.random.Generator, n: int, n_bad: int, side: float = 2048.0, noise: float = 0.4,
                  curve: float = 3.0):
    """n matched point pairs (src, dst), float32 (n, 2): dst = src + a smooth
    quadratic warp (amplitude `curve` px) + a constant shift + Gaussian noise,
    with n_bad of them displaced by up to 40 px (gross outliers)."""
    P = rng.uniform(0, side, (n, 2))
    u, v = (P[:, 0] - side / 2) / (side / 2), (P[:, 1] - side / 2) / (side / 2)
    Q = P + np.stack([curve * u * v + 5.0, -curve * u * u * v + 2.0], 1) + rng.normal(0, noise, (n, 2))
    bad = rng.choice(n, n_bad, replace=False)
    Q[bad] += rng.uniform(-40, 40, (n_bad, 2))
    return P.astype(np.float32), Q.astype(np.float32)
