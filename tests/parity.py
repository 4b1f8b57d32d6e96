"""Parity rules shared by the GPU tests (GPU result vs FP64 oracle).

Tolerances follow from FP32 arithmetic on the GPU against the FP64 oracle:
  * CFOG volume: max |D_gpu - D_ora| <= 1e-5 * max |D_ora| per volume
    (FP32 rounding of ~60 operations per value, relative ~1e-6).
  * SSD surface: |S_gpu(d) - S_ora(d)| <= 1e-4 * (E1 + E2(d)) element-wise.
    S = E1 + E2 - 2C cancels, so the error is measured against the energies
    that the FP32 correlation C ~ sqrt(E1 E2) carries.
  * Offsets: the GPU offset d_g must equal the oracle's d_o, unless it is a
    near-tie that FP32 cannot resolve:
        S_ora(d_g) - S_ora(d_o) <= 1e-4 * (2 E1 + E2(d_g) + E2(d_o))
    (each of the two surface values may be off by its own bound).  Such cases
    are counted and reported, never silently dropped.
"""
import numpy as np

import oracle as O

SURF_TOL = 1e-4
VOL_TOL = 1e-5

U_BF16 = 2.0 ** -8   # unit roundoff of round-to-nearest bfloat16 (8 significant bits)
U_F32 = 2.0 ** -24   # unit roundoff of fp32


def bf16_tol(N: int, r: int, m: int = 9) -> float:
    """Worst-case bound on |S_bf16(d) - S(d)| / (E1 + E2(d)) for the BF16
    MFMA direct path (template side N, radius r, m channels):
      * T and S rounded to bf16 (relative error <= u each), products exact in
        fp32: |T~ S~ - T S| <= (2u + u^2) |T S|;
      * fp32 accumulation along at most L additions per output:
        gamma_L (1 + u)^2 sum |T S|, gamma_L = L u32 / (1 - L u32);
      * sum |T S| <= sqrt(E1 E2) <= (E1 + E2) / 2 (Cauchy-Schwarz, then the
        arithmetic-geometric mean), and S = E1 + E2 - 2C doubles the
        correlation error;
      * the final rounding of S (at most 2 (E1 + E2)) to fp32: 2 u32.
    L follows the kernel's accumulation: each wave adds m channels x
    ceil((N + 2r) / 8) search rows x ceil(N / 32) column chunks of MFMAs into
    one accumulator, each MFMA adding 32 products (counted as 32 sequential
    additions), then the 8 wave partials are added."""
    Ws = N + 2 * r
    L = m * (-(-Ws // 8)) * (-(-N // 32)) * 32 + 8
    gamma = L * U_F32 / (1.0 - L * U_F32)
    return (2 * U_BF16 + U_BF16 ** 2) + gamma * (1 + U_BF16) ** 2 + 2 * U_F32


def check_volume(vol_gpu: np.ndarray, vol_ora: np.ndarray, tol: float = VOL_TOL) -> float:
    err = float(np.max(np.abs(vol_gpu.astype(np.float64) - vol_ora)))
    scale = float(np.max(np.abs(vol_ora)))
    assert err <= tol * max(scale, 1e-30), (err, scale)
    return err / max(scale, 1e-30)


def check_point(k, gpu, ora_surface, E1, E2, r, surf_gpu=None, stats=None, tol=SURF_TOL):
    """Check control point k: gpu is a dict of numpy arrays (dx, dy, best,
    second, status); ora_surface (2r+1, 2r+1) fp64; E2 (2r+1, 2r+1).  tol is
    the surface bound relative to E1 + E2 (1e-4 for FP32 paths)."""
    SURF_TOL = tol
    K = 2 * r + 1
    assert int(gpu["status"][k]) == O.STATUS_OK, (k, int(gpu["status"][k]))
    dxo, dyo, bo, so = O.argmin_lex(ora_surface)
    dxg, dyg = int(gpu["dx"][k]), int(gpu["dy"][k])
    bound = SURF_TOL * (E1 + E2)
    if surf_gpu is not None:
        d = np.abs(surf_gpu.astype(np.float64) - ora_surface)
        worst = float(np.max(d / bound))
        assert worst <= 1.0, (k, worst)
        if stats is not None:
            stats["max_norm_err"] = max(stats.get("max_norm_err", 0.0), float(np.max(d / (E1 + E2))))
        # the reported best/second must be the surface's own extremes
        flat = surf_gpu.reshape(-1)
        i = int(np.argmin(flat))
        assert (i % K - r, i // K - r) == (dxg, dyg), (k, i, dxg, dyg)
        assert flat[i] == np.float32(gpu["best"][k])
    if (dxg, dyg) != (dxo, dyo):
        sg = ora_surface[dyg + r, dxg + r]
        allow = SURF_TOL * (2 * E1 + E2[dyg + r, dxg + r] + E2[dyo + r, dxo + r])
        assert sg - bo <= allow, (k, (dxg, dyg), (dxo, dyo), sg - bo, allow)
        if stats is not None:
            stats["excused"] = stats.get("excused", 0) + 1
    elif stats is not None:
        stats["exact"] = stats.get("exact", 0) + 1
    # best/second values within the surface bound
    assert abs(float(gpu["best"][k]) - ora_surface[dyg + r, dxg + r]) <= bound[dyg + r, dxg + r]
    if np.isinf(so):  # r = 0: a single candidate has no runner-up
        assert np.isinf(float(gpu["second"][k])) and float(gpu["second"][k]) > 0
    else:
        second_bound = SURF_TOL * (2 * E1 + 2 * np.max(E2))
        assert abs(float(gpu["second"][k]) - so) <= second_bound


def cfog_window(img: np.ndarray, y0: int, x0: int, h: int, w: int, m: int = 9, sigma: float = 0.8):
    """Oracle CFOG on the rows [y0, y0+h) x cols [x0, x0+w) of img, computed
    from a crop with a margin of R+1 pixels (values identical to the
    full-image oracle: CFOG at a pixel only reads its (2R+3)^2 neighbourhood,
    and the crop keeps the image's own borders where it reaches them)."""
    R = int(4 * sigma + 0.5)
    M = R + 1
    H, W = img.shape
    ya, xa = max(0, y0 - M), max(0, x0 - M)
    yb, xb = min(H, y0 + h + M), min(W, x0 + w + M)
    D = O.cfog(img[ya:yb, xa:xb].astype(np.float64), m=m, sigma=sigma)
    return D[:, y0 - ya:y0 - ya + h, x0 - xa:x0 - xa + w]


def oracle_point(A, B, cp, N, r, m=9, sigma=0.8):
    """Oracle surface, E1 and E2 of one control point computed on local crops."""
    x, y, bx, by = (int(v) for v in cp)
    h = N // 2
    T = cfog_window(A, y - h, x - h, N, N, m, sigma)
    Sw = cfog_window(B, by - h - r, bx - h - r, N + 2 * r, N + 2 * r, m, sigma)
    # the oracle's direct SSD on a volume holding just the two windows
    D1 = T
    D2 = Sw
    cp_local = (h, h, h + r, h + r)
    S = O.ssd_surface_direct(D1, D2, cp_local, N, r)
    E1, E2 = O.energies(D1, D2, cp_local, N, r)
    return S, E1, E2


def oracle_point_fft(A, B, cp, N, r, m=9, sigma=0.8):
    """As oracle_point, with the surface from the oracle's FP64 FFT form
    (Eqs. 5, 8-9; pinned to the direct form to 1e-10 by the oracle pins),
    which makes full-size checks of every point affordable on the host."""
    x, y, bx, by = (int(v) for v in cp)
    h = N // 2
    T = cfog_window(A, y - h, x - h, N, N, m, sigma)
    Sw = cfog_window(B, by - h - r, bx - h - r, N + 2 * r, N + 2 * r, m, sigma)
    loc = (h, h, h + r, h + r)
    S = O.ssd_surface_fft(T, Sw, loc, N, r)
    E1, E2 = O.energies(T, Sw, loc, N, r)
    return S, E1, E2
