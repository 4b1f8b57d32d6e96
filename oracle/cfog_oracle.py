"""FP64 CPU oracle for CFOG extraction and SSD template matching.

TEST INFRASTRUCTURE ONLY.  This module is the independent reference the HIP
path is checked against: only the test suite, the smoke entry point and the
benchmark's CPU baseline may import it.  It shares no code with the GPU library and must never
be used to produce a product result.

What it computes (Ye et al., "Fast and Robust Matching for Multimodal Remote
Sensing Image Registration"):

* CFOG (Section III-F): oriented gradient channels from the horizontal and
  vertical gradients of the image (Eq. 2, filters [-1, 0, 1]; scheme 1 of the
  same section as an option), convolved with a
  3-D "Gaussian-like" kernel: a 2-D Gaussian of std sigma in X and Y and a
  [1, 2, 1] kernel along the orientation (Z) axis.  Defaults sigma = 0.8 and
  m = 9 (Section V-C, Table II).
* SSD similarity (Section III-G, Eq. 3) of the template window of a control
  point in D1 against the translated window in D2, and the matching function
  (Eq. 4): the translation minimising it.  The oracle evaluates Eq. 3 directly
  by brute force; the frequency-domain form (Eqs. 5-6 and 8-9: energies plus a
  3-D FFT correlation) is provided separately as a cross-check.

Readings taken where the paper is silent (each is listed in the design notes):
  * scheme 2 of Section III-F (Eq. 2) with theta_k = k pi / m, k = 0..m-1;
  * x = column, y = row; central differences without a 1/2 factor; image
    borders replicated (clamp-to-edge) for the gradient and the Gaussian;
  * Gaussian radius R = int(4 sigma + 0.5), weights normalised to sum 1;
  * Z kernel [1, 2, 1] / 4 applied circularly over the m orientations
    (orientation is periodic over [0, 180) degrees);
  * template top-left corner = control point - floor(N / 2); search radius r
    means offsets d in [-r, r]^2; the returned offset d is the position of the
    best window in D2 relative to the search centre (d = -v of Eq. 3);
  * ties are broken towards the smallest row-major index (dy first, then dx);
  * no per-pixel normalisation of the CFOG vector.

Beyond the hot path (the first extension of the method):
  * the correlation objective of Eq. 7 (maximise the template / window
    correlation instead of minimising the SSD), evaluated by brute force;
  * sub-pixel refinement of the best offset.  The paper fits a quadratic
    polynomial around the integer match (Section V-B) without giving the
    formula; the reading taken here is a separable three-point parabola along
    x and along y through the best offset and its axis neighbours.

  * block-based Harris feature point detection in the reference image
    (Section IV): the image is divided into n x n cells, a 60 x 60 chip
    centred on each cell is read, and the k pixels with the largest Harris
    response in the chip become feature points.  The paper does not give the
    Harris details; the readings taken are: chip centre of cell (i, j) at
    (floor((2j+1) W / 2n), floor((2i+1) H / 2n)), chip rows and columns
    [centre - 30, centre + 30) clipped to the image, gradients by [-1, 0, 1]
    with the chip's borders replicated, the structure tensor smoothed by a
    normalised Gaussian (sigma 1, radius int(4 sigma + 0.5), chip borders
    replicated), R = det - kappa trace^2 with kappa = 0.04, and the k largest R
    with ties to the smallest row-major index in the chip.

  * iterative outlier rejection (Section IV): fit a cubic polynomial mapping
    from the points in A to their matches in B by least squares, remove the
    point with the largest residual, and repeat until the RMSE falls below a
    threshold (3.5 pixels in Table V).  Readings: coordinates normalised by
    the bounding box of the input points (centre and half-extent per axis)
    before forming the ten monomials; residual = Euclidean distance between
    the mapped point and its match; RMSE = sqrt(mean residual^2); ties in the
    largest residual go to the smaller index; the loop also stops when ten
    points (the model's size) remain.

  * pixel-wise HOG (FHOG, Section III-C): at every pixel, the histogram of a
    block of 2 x 2 cells centred on it, 9 unsigned orientation bins, each
    gradient spread over the neighbouring cells and bins by trilinear
    interpolation, the 36 values normalised by their L2 norm.  Readings: the
    orientation bins and their linear interpolation are those of scheme 1
    (centres k pi / 9); cells of c = 4 pixels, the block spans offsets
    [-c, c] around the pixel with cell centres at +-c/2; the spatial weight of
    a gradient at offset d for the cell centred at o is max(0, 1 - |d - o| / c)
    per axis (bilinear), zero outside the block; borders replicated; channel
    index (2 a + b) 9 + k for cell column a, cell row b, bin k; normalisation
    v / sqrt(|v|^2 + 1e-12).

Parity pins live in tests/test_oracle_pins.py.  No CFOG value, surface or
offset is printed in the paper, so agreement with the authors' own code is
"parity unpinned"; every function here is pinned by closed forms, invariants,
library routines or brute force instead.
"""
from __future__ import annotations

import numpy as np

STATUS_OK = 0
STATUS_OUT_OF_BOUNDS = 1
STATUS_NONFINITE = 2


# ----------------------------------------------------------------- CFOG (III-F)

def gradients(img: np.ndarray):
    """gx, gy by the 1-D filters [-1, 0, 1] and its transpose (Section III-F,
    text after Eq. 2), borders replicated.  x = column, y = row (Fig. 4)."""
    I = np.asarray(img, np.float64)
    P = np.pad(I, 1, mode="edge")
    gx = P[1:-1, 2:] - P[1:-1, :-2]
    gy = P[2:, 1:-1] - P[:-2, 1:-1]
    return gx, gy


def orientations(m: int) -> np.ndarray:
    """Quantised orientations theta_k = k * pi / m in [0, 180) degrees."""
    return np.arange(m, dtype=np.float64) * np.pi / m


def oriented_channels(gx: np.ndarray, gy: np.ndarray, m: int) -> np.ndarray:
    """Eq. 2: g_theta = abs(cos(theta) gx + sin(theta) gy), one channel per
    quantised orientation.  Returns (m, H, W)."""
    th = orientations(m)
    return np.abs(np.cos(th)[:, None, None] * gx[None] + np.sin(th)[:, None, None] * gy[None])


def oriented_channels_scheme1(gx: np.ndarray, gy: np.ndarray, m: int) -> np.ndarray:
    """Scheme 1 of Section III-F: the gradient orientation, taken modulo 180
    degrees, falls between two of the m orientation bins (centres k pi / m);
    the gradient magnitude is split between them with weights falling
    linearly with the distance to each bin (reading of "inversely related to
    the distance"), circularly over the m bins."""
    mag = np.hypot(gx, gy)
    phi = np.mod(np.arctan2(gy, gx), np.pi)
    b = phi * (m / np.pi)
    b = np.where(b >= m, b - m, b)
    k0 = np.floor(b).astype(np.int64)
    f = b - k0
    k0 = np.mod(k0, m)
    k1 = np.mod(k0 + 1, m)
    G = np.zeros((m,) + gx.shape, np.float64)
    rows, cols = np.indices(gx.shape)
    np.add.at(G, (k0, rows, cols), mag * (1.0 - f))
    np.add.at(G, (k1, rows, cols), mag * f)
    return G


def gaussian_weights(sigma: float, radius: int | None = None) -> np.ndarray:
    """Normalised 1-D Gaussian of std sigma on [-R, R], R = int(4 sigma + 0.5)."""
    R = int(4.0 * sigma + 0.5) if radius is None or radius < 0 else int(radius)
    j = np.arange(-R, R + 1, dtype=np.float64)
    w = np.exp(-(j * j) / (2.0 * sigma * sigma))
    return w / w.sum()


def _conv1d_edge(a: np.ndarray, w: np.ndarray, axis: int) -> np.ndarray:
    """Correlate along one axis with a symmetric kernel, clamp-to-edge borders,
    written as a plain sum of shifted copies."""
    R = (len(w) - 1) // 2
    pad = [(0, 0)] * a.ndim
    pad[axis] = (R, R)
    P = np.pad(a, pad, mode="edge")
    n = a.shape[axis]
    out = np.zeros_like(a, dtype=np.float64)
    for t in range(2 * R + 1):
        sl = [slice(None)] * a.ndim
        sl[axis] = slice(t, t + n)
        out += w[t] * P[tuple(sl)]
    return out


def smooth_xy(G: np.ndarray, sigma: float, radius: int | None = None) -> np.ndarray:
    """2-D Gaussian in X then Y on every channel (Section III-F)."""
    w = gaussian_weights(sigma, radius)
    return _conv1d_edge(_conv1d_edge(G, w, axis=G.ndim - 1), w, axis=G.ndim - 2)


def smooth_z(G: np.ndarray) -> np.ndarray:
    """[1, 2, 1] / 4 along the orientation axis (axis 0), circular over m."""
    return 0.25 * np.roll(G, 1, axis=0) + 0.5 * G + 0.25 * np.roll(G, -1, axis=0)


def cfog(img: np.ndarray, m: int = 9, sigma: float = 0.8, radius: int | None = None,
         scheme: int = 2) -> np.ndarray:
    """CFOG volume D, shape (m, H, W), fp64 (Section III-F, Fig. 9 chain:
    gradients -> oriented channels (scheme 2: Eq. 2; scheme 1: binned
    orientation) -> 3-D Gaussian-like convolution)."""
    gx, gy = gradients(img)
    G = oriented_channels(gx, gy, m) if scheme == 2 else oriented_channels_scheme1(gx, gy, m)
    return smooth_z(smooth_xy(G, sigma, radius))


# ------------------------------------------------------- energies (Eq. 5 terms)

def sat(Q: np.ndarray) -> np.ndarray:
    """Summed-area table S(y, x) = sum_{y' < y, x' < x} Q, shape (H+1, W+1), fp64."""
    Q = np.asarray(Q, np.float64)
    S = np.zeros((Q.shape[0] + 1, Q.shape[1] + 1), np.float64)
    S[1:, 1:] = Q.cumsum(axis=0).cumsum(axis=1)
    return S


def box_sum(S: np.ndarray, y0: int, x0: int, h: int, w: int) -> float:
    """Sum of Q over rows [y0, y0+h) and columns [x0, x0+w) from its SAT."""
    return S[y0 + h, x0 + w] - S[y0, x0 + w] - S[y0 + h, x0] + S[y0, x0]


# ---------------------------------------------------------- SSD (Eqs. 3 and 4)

def window_ok(cp, N: int, r: int, hA: int, wA: int, hB: int, wB: int) -> bool:
    """Template box inside A and search box inside B."""
    x, y, bx, by = (int(v) for v in cp)
    h = N // 2
    ta = (y - h >= 0) and (x - h >= 0) and (y - h + N <= hA) and (x - h + N <= wA)
    tb = (by - h - r >= 0) and (bx - h - r >= 0) and (by - h + N + r <= hB) and (bx - h + N + r <= wB)
    return ta and tb


def ssd_surface_direct(D1: np.ndarray, D2: np.ndarray, cp, N: int, r: int) -> np.ndarray:
    """Eq. 3 by brute force: S(d) = sum_{c,i,j} (D1 template - D2 window at d)^2
    for every d = (dx, dy) in [-r, r]^2.  Returns (2r+1, 2r+1), index [dy+r, dx+r]."""
    x, y, bx, by = (int(v) for v in cp)
    h = N // 2
    T = D1[:, y - h:y - h + N, x - h:x - h + N]
    out = np.empty((2 * r + 1, 2 * r + 1), np.float64)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            Sw = D2[:, by - h + dy:by - h + dy + N, bx - h + dx:bx - h + dx + N]
            out[dy + r, dx + r] = np.sum((T - Sw) ** 2)
    return out


def correlation_surface_direct(D1: np.ndarray, D2: np.ndarray, cp, N: int, r: int) -> np.ndarray:
    """Eq. 7 objective by brute force, as a cost to minimise:
    J(d) = - sum_{c,i,j} D1 template * D2 window at d, index [dy+r, dx+r]."""
    x, y, bx, by = (int(v) for v in cp)
    h = N // 2
    T = D1[:, y - h:y - h + N, x - h:x - h + N]
    out = np.empty((2 * r + 1, 2 * r + 1), np.float64)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            Sw = D2[:, by - h + dy:by - h + dy + N, bx - h + dx:bx - h + dx + N]
            out[dy + r, dx + r] = -np.sum(T * Sw)
    return out


def parabola_vertex(a: float, b: float, c: float) -> float:
    """Abscissa, relative to the middle sample, of the vertex of the parabola
    through (-1, a), (0, b), (1, c); 0 when the three samples are not convex
    (b is not below their chord)."""
    den = a - 2.0 * b + c
    if not den > 0.0:
        return 0.0
    return 0.5 * (a - c) / den


def subpixel(surface: np.ndarray, dx: int, dy: int):
    """Sub-pixel refinement of the integer best offset (dx, dy) of a cost
    surface: per axis, the parabola through the best value and its two axis
    neighbours; an axis whose neighbour falls outside the surface keeps its
    integer value.  Returns (fdx, fdy) as floats."""
    r = (surface.shape[0] - 1) // 2
    ix, iy = dx + r, dy + r
    K = 2 * r + 1
    fx, fy = float(dx), float(dy)
    if 0 < ix < K - 1:
        fx += parabola_vertex(surface[iy, ix - 1], surface[iy, ix], surface[iy, ix + 1])
    if 0 < iy < K - 1:
        fy += parabola_vertex(surface[iy - 1, ix], surface[iy, ix], surface[iy + 1, ix])
    return fx, fy


def argmin_lex(surface: np.ndarray):
    """Eq. 4 with ties broken to the smallest row-major index.  Returns
    (dx, dy, best, second) where second = min over all other offsets."""
    K = surface.size
    r = (surface.shape[0] - 1) // 2
    flat = surface.reshape(-1)
    i = int(np.argmin(flat))  # numpy returns the first occurrence of the minimum
    best = float(flat[i])
    second = float(np.min(np.delete(flat, i))) if K > 1 else float("inf")
    dy, dx = divmod(i, 2 * r + 1)
    return dx - r, dy - r, best, second


def match(D1: np.ndarray, D2: np.ndarray, cps, N: int, r: int, surfaces: bool = False,
          objective: str = "ssd", subpix: bool = False):
    """Match every control point by brute force: objective "ssd" minimises
    Eq. 3 (Eq. 4), "corr" maximises the correlation of Eq. 7 (as the cost
    -C).

    Returns dict with int arrays dx, dy, status and float arrays best, second
    (NaN for out-of-bounds points), optionally surfaces (n, 2r+1, 2r+1) and,
    with subpix, the refined offsets fdx, fdy (NaN when not ok)."""
    cps = np.asarray(cps).reshape(-1, 4)
    n = len(cps)
    res = dict(dx=np.zeros(n, np.int32), dy=np.zeros(n, np.int32),
               best=np.full(n, np.nan), second=np.full(n, np.nan),
               status=np.zeros(n, np.int32))
    if surfaces:
        res["surfaces"] = np.full((n, 2 * r + 1, 2 * r + 1), np.nan)
    if subpix:
        res["fdx"], res["fdy"] = np.full(n, np.nan), np.full(n, np.nan)
    cost = {"ssd": ssd_surface_direct, "corr": correlation_surface_direct}[objective]
    _, hA, wA = D1.shape
    _, hB, wB = D2.shape
    for k, cp in enumerate(cps):
        if not window_ok(cp, N, r, hA, wA, hB, wB):
            res["status"][k] = STATUS_OUT_OF_BOUNDS
            continue
        S = cost(D1, D2, cp, N, r)
        if not np.all(np.isfinite(S)):
            res["status"][k] = STATUS_NONFINITE
            continue
        dx, dy, b, s = argmin_lex(S)
        res["dx"][k], res["dy"][k], res["best"][k], res["second"][k] = dx, dy, b, s
        if surfaces:
            res["surfaces"][k] = S
        if subpix:
            res["fdx"][k], res["fdy"][k] = subpixel(S, dx, dy)
    return res


# ------------------------------------- cross-check form (Eqs. 5-6 and 8-9)

def template_and_window(D1, D2, cp, N, r):
    x, y, bx, by = (int(v) for v in cp)
    h = N // 2
    T = D1[:, y - h:y - h + N, x - h:x - h + N]
    Sw = D2[:, by - h - r:by - h + N + r, bx - h - r:bx - h + N + r]
    return T, Sw


def correlation_3dfft(T: np.ndarray, Sw: np.ndarray, P: int) -> np.ndarray:
    """Eq. 9 evaluated at zero orientation shift: the 3-D FFT (orientation, y, x)
    of the zero-padded template and search window, product with the conjugate,
    3-D inverse, slice vz = 0, crop to the (2r+1)^2 valid translations.

    C(u) = sum_{c, q} T_c(q) Sw_c(q + u) for u in [0, 2r]^2."""
    m, N, _ = T.shape
    Ws = Sw.shape[1]
    if P < Ws:
        raise ValueError("FFT size must cover the search window")
    Tp = np.zeros((m, P, P))
    Sp = np.zeros((m, P, P))
    Tp[:, :N, :N] = T
    Sp[:, :Ws, :Ws] = Sw
    X = np.conj(np.fft.fftn(Tp)) * np.fft.fftn(Sp)
    C3 = np.fft.ifftn(X).real
    K = Ws - N + 1
    return C3[0, :K, :K]


def ssd_surface_fft(D1, D2, cp, N, r, P: int | None = None, SAT1=None, SAT2=None) -> np.ndarray:
    """Eq. 5: S(d) = E1 + E2(d) - 2 C(d) with C from the 3-D FFT correlation and
    the energies from FP64 summed-area tables of sum_c D_c^2."""
    x, y, bx, by = (int(v) for v in cp)
    h = N // 2
    T, Sw = template_and_window(D1, D2, cp, N, r)
    Ws = N + 2 * r
    C = correlation_3dfft(T, Sw, Ws if P is None else P)
    if SAT1 is None:
        SAT1 = sat(np.sum(D1 * D1, axis=0))
    if SAT2 is None:
        SAT2 = sat(np.sum(D2 * D2, axis=0))
    E1 = box_sum(SAT1, y - h, x - h, N, N)
    out = np.empty((2 * r + 1, 2 * r + 1))
    for uy in range(2 * r + 1):
        for ux in range(2 * r + 1):
            E2 = box_sum(SAT2, by - h - r + uy, bx - h - r + ux, N, N)
            out[uy, ux] = E1 + E2 - 2.0 * C[uy, ux]
    return out


def match_fft(D1, D2, cps, N, r, P=None, surfaces=False):
    """Cross-check matcher: same outputs as ``match`` via Eqs. 5 and 9."""
    cps = np.asarray(cps).reshape(-1, 4)
    n = len(cps)
    res = dict(dx=np.zeros(n, np.int32), dy=np.zeros(n, np.int32),
               best=np.full(n, np.nan), second=np.full(n, np.nan),
               status=np.zeros(n, np.int32))
    if surfaces:
        res["surfaces"] = np.full((n, 2 * r + 1, 2 * r + 1), np.nan)
    SAT1 = sat(np.sum(D1 * D1, axis=0))
    SAT2 = sat(np.sum(D2 * D2, axis=0))
    _, hA, wA = D1.shape
    _, hB, wB = D2.shape
    for k, cp in enumerate(cps):
        if not window_ok(cp, N, r, hA, wA, hB, wB):
            res["status"][k] = STATUS_OUT_OF_BOUNDS
            continue
        S = ssd_surface_fft(D1, D2, cp, N, r, P, SAT1, SAT2)
        dx, dy, b, s = argmin_lex(S)
        res["dx"][k], res["dy"][k], res["best"][k], res["second"][k] = dx, dy, b, s
        if surfaces:
            res["surfaces"][k] = S
    return res


def energies(D1, D2, cp, N, r):
    """(E1, E2 surface) for one control point, by direct summation."""
    T, Sw = template_and_window(D1, D2, cp, N, r)
    E1 = float(np.sum(T * T))
    Q2 = np.sum(Sw * Sw, axis=0)
    E2 = np.empty((2 * r + 1, 2 * r + 1))
    for uy in range(2 * r + 1):
        for ux in range(2 * r + 1):
            E2[uy, ux] = Q2[uy:uy + N, ux:ux + N].sum()
    return E1, E2


# --------------------------------------------- feature points (Section IV)

def harris_response(chip: np.ndarray, sigma: float = 1.0, kappa: float = 0.04) -> np.ndarray:
    """Harris response R = det(M) - kappa trace(M)^2 of every pixel of a chip,
    M the Gaussian-weighted structure tensor of the [-1, 0, 1] gradients (chip
    borders replicated)."""
    gx, gy = gradients(chip)
    w = gaussian_weights(sigma)
    smooth = lambda a: _conv1d_edge(_conv1d_edge(a, w, 1), w, 0)  # noqa: E731
    a, b, c = smooth(gx * gx), smooth(gx * gy), smooth(gy * gy)
    return a * c - b * b - kappa * (a + c) ** 2


def harris_chip_origin(H: int, W: int, n: int, i: int, j: int, chip: int = 60):
    """Top-left (y0, x0) and size (h, w) of the chip of cell (i, j), clipped."""
    cy = ((2 * i + 1) * H) // (2 * n)
    cx = ((2 * j + 1) * W) // (2 * n)
    y0, x0 = max(0, cy - chip // 2), max(0, cx - chip // 2)
    y1, x1 = min(H, cy - chip // 2 + chip), min(W, cx - chip // 2 + chip)
    return y0, x0, y1 - y0, x1 - x0


def harris_grid(img: np.ndarray, n: int, k: int, chip: int = 60, sigma: float = 1.0, kappa: float = 0.04):
    """Feature points of Section IV: for each of the n x n cells (row-major),
    the k pixels of its chip with the largest Harris response, in decreasing
    response (ties: smaller row-major index in the chip first).  Returns
    (points (n*n*k, 2) int (x, y) in image coordinates, responses (n*n*k,))."""
    I = np.asarray(img, np.float64)
    H, W = I.shape
    pts, vals = [], []
    for i in range(n):
        for j in range(n):
            y0, x0, h, w = harris_chip_origin(H, W, n, i, j, chip)
            R = harris_response(I[y0:y0 + h, x0:x0 + w], sigma, kappa).reshape(-1)
            order = np.lexsort((np.arange(R.size), -R))[:k]  # by -R, then by index
            for q in order:
                yy, xx = divmod(int(q), w)
                pts.append((x0 + xx, y0 + yy))
                vals.append(R[q])
    return np.array(pts, np.int64).reshape(-1, 2), np.array(vals)


# --------------------------------------------- outlier rejection (Section IV)

def cubic_terms(u: np.ndarray, v: np.ndarray) -> np.ndarray:
    """The ten monomials of a bivariate cubic, (n, 10):
    1, u, v, u^2, u v, v^2, u^3, u^2 v, u v^2, v^3."""
    return np.stack([np.ones_like(u), u, v, u * u, u * v, v * v, u ** 3, u * u * v, u * v * v, v ** 3], axis=1)


def normalise_points(src: np.ndarray):
    """(centre, half-extent) per axis of the bounding box of the points; a
    degenerate extent becomes 1."""
    lo, hi = src.min(axis=0), src.max(axis=0)
    c = 0.5 * (lo + hi)
    s = 0.5 * (hi - lo)
    s[s <= 0] = 1.0
    return c, s


def reject_outliers(src, dst, threshold: float = 3.5):
    """Iterative rejection with a cubic polynomial model (Section IV).
    src, dst: (n, 2) point coordinates (x, y) in A and their matches in B.
    Returns (keep (n,) bool, coefficients (10, 2) in normalised coordinates,
    rmse of the last fit, number of points removed)."""
    P = np.asarray(src, np.float64)
    Q = np.asarray(dst, np.float64)
    n = len(P)
    if n < 10:
        raise ValueError("a cubic model needs at least 10 points")
    c, s = normalise_points(P)
    Tm = cubic_terms((P[:, 0] - c[0]) / s[0], (P[:, 1] - c[1]) / s[1])
    keep = np.ones(n, bool)
    removed = 0
    while True:
        idx = np.flatnonzero(keep)
        coef, *_ = np.linalg.lstsq(Tm[idx], Q[idx], rcond=None)
        res = np.sqrt(np.sum((Tm[idx] @ coef - Q[idx]) ** 2, axis=1))
        rmse = float(np.sqrt(np.mean(res ** 2)))
        if rmse < threshold or len(idx) <= 10:
            return keep, coef, rmse, removed
        keep[idx[int(np.argmax(res))]] = False  # argmax: the first of equal maxima
        removed += 1


# ------------------------------------------------- pixel-wise HOG (III-C)

FHOG_EPS = 1e-12


def fhog_cell_kernel(c: int, o: float) -> np.ndarray:
    """Spatial weights of the cell centred at offset o for block offsets
    d = -c .. c: max(0, 1 - |d - o| / c)."""
    d = np.arange(-c, c + 1, dtype=np.float64)
    return np.maximum(0.0, 1.0 - np.abs(d - o) / c)


def fhog(img: np.ndarray, c: int = 4, bins: int = 9) -> np.ndarray:
    """Pixel-wise HOG volume, shape (4 bins, H, W), fp64."""
    gx, gy = gradients(img)
    G = oriented_channels_scheme1(gx, gy, bins)
    kern = [fhog_cell_kernel(c, -c / 2.0), fhog_cell_kernel(c, c / 2.0)]
    out = np.empty((4 * bins,) + G.shape[1:], np.float64)
    for a in range(2):          # cell column (x offset -c/2, +c/2)
        Hx = np.stack([_conv1d_edge(G[k], kern[a], 1) for k in range(bins)])
        for b in range(2):      # cell row (y offset -c/2, +c/2)
            out[(2 * a + b) * bins:(2 * a + b + 1) * bins] = np.stack(
                [_conv1d_edge(Hx[k], kern[b], 0) for k in range(bins)])
    return out / np.sqrt(np.sum(out * out, axis=0) + FHOG_EPS)
