"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test below would fail under a plausible mistake in the oracle:
  gradient filter / border rule ........ hand gradient fixture, ramp borders
  orientation angles, abs, Eq. 2 ....... ramp closed form
  Gaussian radius / normalisation ...... scipy.ndimage library pin
  circular [1,2,1] along Z ............. mirror invariant, channel-sum invariant
  SSD window indexing, offset sign ..... hand SSD fixture, exact known shift,
                                         pure-Python brute force
  tie rule ............................. constant image, hand fixture
  FFT form (Eqs. 5-6, 8-9) ............. direct SSD, naive DFT, per-channel sum
  summed-area tables ................... direct box sums
"""
import json
import os

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle as O
from paper_1808_06194_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------------ CFOG pins

def test_hand_gradient_fixture():
    g = _gold("hand_gradient_3x3.json")
    gx, gy = O.gradients(np.array(g["image"], np.float64))
    assert np.array_equal(gx, np.array(g["gx"], np.float64))
    assert np.array_equal(gy, np.array(g["gy"], np.float64))


def test_orientations_are_k_pi_over_m():
    th = O.orientations(9)
    assert np.allclose(np.degrees(th), [0, 20, 40, 60, 80, 100, 120, 140, 160], atol=1e-12)


@pytest.mark.parametrize("alpha,beta", [(0.5, 0.25), (-0.75, 0.125), (1.0, 0.0), (0.0, -2.0)])
def test_linear_ramp_closed_form(alpha, beta):
    """I = alpha x + beta y.  Interior: gx = 2 alpha, gy = 2 beta exactly, a
    normalised Gaussian keeps constants, so D_k = g_{k-1}/4 + g_k/2 + g_{k+1}/4
    (indices mod m) with g_k = |2 alpha cos(k pi/m) + 2 beta sin(k pi/m)|."""
    H, W, m = 24, 28, 9
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    D = O.cfog(alpha * x + beta * y, m=m, sigma=0.8)
    k = np.arange(m)
    g = np.abs(2 * alpha * np.cos(k * np.pi / m) + 2 * beta * np.sin(k * np.pi / m))
    expect = 0.25 * g[(k - 1) % m] + 0.5 * g + 0.25 * g[(k + 1) % m]
    inner = D[:, 4:H - 4, 4:W - 4]
    assert np.max(np.abs(inner - expect[:, None, None])) < 1e-13


def test_ramp_border_column_is_one_sided():
    """Column 0 of a horizontal ramp sees gx = alpha (one-sided difference
    under edge replication); the XY Gaussian then mixes it with the interior
    value 2 alpha as scipy's 'nearest' filter does."""
    alpha, m = 0.5, 9
    H, W = 20, 20
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    gx, gy = O.gradients(alpha * x)
    assert np.all(gx[:, 0] == alpha) and np.all(gx[:, -1] == alpha)
    assert np.all(gx[:, 1:-1] == 2 * alpha) and np.all(gy == 0)
    G = np.abs(np.cos(np.arange(m) * np.pi / m))[:, None, None] * gx[None]
    ref = np.stack([ndi.gaussian_filter(c, 0.8, mode="nearest", truncate=4.0) for c in G])
    ref = 0.25 * np.roll(ref, 1, 0) + 0.5 * ref + 0.25 * np.roll(ref, -1, 0)
    assert np.max(np.abs(O.cfog(alpha * x, m=m) - ref)) < 1e-13


@pytest.mark.parametrize("sigma", [0.5, 0.8, 1.3, 2.0])
def test_xy_gaussian_matches_scipy(sigma):
    rng = np.random.default_rng(5)
    G = rng.random((3, 17, 23))
    ref = np.stack([ndi.gaussian_filter(c, sigma, mode="nearest", truncate=4.0) for c in G])
    assert np.max(np.abs(O.smooth_xy(G, sigma) - ref)) < 1e-14


def test_gaussian_radius_at_default_sigma():
    w = O.gaussian_weights(0.8)
    assert len(w) == 7 and abs(w.sum() - 1) < 1e-15
    # scipy.ndimage's own 1-D kernel of the same sigma/truncation
    impulse = np.zeros(15)
    impulse[7] = 1.0
    ref = ndi.gaussian_filter1d(impulse, 0.8, mode="constant", truncate=4.0)
    assert np.max(np.abs(ref[4:11] - w)) < 1e-16 and np.all(ref[:4] == 0)


@pytest.mark.parametrize("m", [9, 8, 6])
def test_mirror_invariant(m):
    """Mirroring the image in x maps orientation theta_k to pi - theta_k, i.e.
    channel k to channel (m - k) mod m; this holds only with a circular Z kernel."""
    rng = np.random.default_rng(11)
    I = rng.random((19, 21))
    D = O.cfog(I, m=m)
    Df = O.cfog(I[:, ::-1], m=m)
    k = np.arange(m)
    assert np.max(np.abs(Df - D[(m - k) % m][:, :, ::-1])) < 1e-13


def test_inversion_invariant_is_exact():
    """abs() in Eq. 2 folds [180, 360) onto [0, 180): CFOG(-I) == CFOG(I)."""
    rng = np.random.default_rng(3)
    I = rng.random((16, 18))
    assert np.array_equal(O.cfog(-I), O.cfog(I))


def test_z_smoothing_preserves_channel_sum():
    rng = np.random.default_rng(4)
    G = rng.random((9, 7, 8))
    assert np.max(np.abs(O.smooth_z(G).sum(0) - G.sum(0))) < 1e-13


def test_constant_image_gives_zero_volume_and_tie_rule():
    D = O.cfog(np.full((40, 40), 3.25), m=9)
    assert np.array_equal(D, np.zeros_like(D))
    res = O.match(D, D, [[20, 20, 20, 20]], N=8, r=3, surfaces=True)
    assert np.all(res["surfaces"] == 0)
    # every offset ties; the smallest row-major index (dy, then dx) wins
    assert (res["dx"][0], res["dy"][0]) == (-3, -3)
    assert res["best"][0] == 0 and res["second"][0] == 0


# ------------------------------------------------------------------- SSD pins

def test_hand_ssd_fixture():
    g = _gold("hand_ssd_m1_n1_r1.json")
    D1 = np.array(g["D1"], np.float64)[None]
    D2 = np.array(g["D2"], np.float64)[None]
    S = O.ssd_surface_direct(D1, D2, g["cp"], g["N"], g["r"])
    assert np.array_equal(S, np.array(g["surface_dy_major"], np.float64))
    res = O.match(D1, D2, [g["cp"]], g["N"], g["r"])
    assert (res["dx"][0], res["dy"][0]) == (g["best_dx"], g["best_dy"])
    assert res["best"][0] == g["best"] and res["second"][0] == g["second"]


def _python_loop_ssd(D1, D2, cp, N, r):
    x, y, bx, by = cp
    h = N // 2
    m = len(D1)
    out = [[0.0] * (2 * r + 1) for _ in range(2 * r + 1)]
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            s = 0.0
            for c in range(m):
                for i in range(N):
                    for j in range(N):
                        a = D1[c][y - h + i][x - h + j]
                        b = D2[c][by - h + i + dy][bx - h + j + dx]
                        s += (a - b) * (a - b)
            out[dy + r][dx + r] = s
    return np.array(out)


@pytest.mark.parametrize("N,r,m", [(3, 1, 2), (4, 2, 3), (5, 2, 1)])
def test_direct_ssd_against_python_loops(N, r, m):
    rng = np.random.default_rng(N * 100 + r)
    D1 = rng.random((m, 12, 13))
    D2 = rng.random((m, 11, 14))
    cp = (6, 5, 7, 5)
    ref = _python_loop_ssd(D1.tolist(), D2.tolist(), cp, N, r)
    assert np.max(np.abs(O.ssd_surface_direct(D1, D2, cp, N, r) - ref)) < 1e-12


def _shifted_pair(H, W, s, seed):
    """Two crops of one random canvas: B(y, x) = A(y - dy, x - dx)."""
    rng = np.random.default_rng(seed)
    smax = max(abs(s[0]), abs(s[1]))
    C = ndi.gaussian_filter(rng.random((H + 2 * smax, W + 2 * smax)), 1.5)
    A = C[smax:smax + H, smax:smax + W]
    B = C[smax - s[1]:smax - s[1] + H, smax - s[0]:smax - s[0] + W]
    return A, B


@pytest.mark.parametrize("shift", [(3, -2), (-4, 4), (0, 0), (1, 3)])
def test_exact_known_shift_recovered(shift):
    """Windows at least 4 px inside both images see bit-identical CFOG
    neighbourhoods, so S(shift) == 0 exactly and the argmin is the shift."""
    A, B = _shifted_pair(48, 52, shift, seed=7)
    D1, D2 = O.cfog(A), O.cfog(B)
    cps = [[20, 22, 20, 22], [26, 25, 26, 25]]
    res = O.match(D1, D2, cps, N=10, r=5)
    assert np.all(res["dx"] == shift[0]) and np.all(res["dy"] == shift[1])
    assert np.all(res["best"] == 0.0) and np.all(res["second"] > 0)


def test_inverted_shift_recovered():
    """Intensity inversion (B = -shift(A)) is invisible to CFOG."""
    A, B = _shifted_pair(48, 48, (2, -3), seed=8)
    res = O.match(O.cfog(A), O.cfog(-B), [[24, 24, 24, 24]], N=12, r=4)
    assert (res["dx"][0], res["dy"][0]) == (2, -3) and res["best"][0] == 0.0


def test_out_of_bounds_status():
    D = np.zeros((1, 20, 20))
    res = O.match(D, D, [[2, 10, 10, 10], [10, 10, 16, 10], [10, 10, 10, 10]], N=6, r=2)
    assert list(res["status"]) == [O.STATUS_OUT_OF_BOUNDS, O.STATUS_OUT_OF_BOUNDS, O.STATUS_OK]


def _box_pixels_valid(x0, y0, n, h_img, w_img):
    """Every pixel of the n x n box with top-left (x0, y0) is an index of an
    h_img x w_img image (written as a loop over the box's pixels)."""
    for yy in range(y0, y0 + n):
        for xx in range(x0, x0 + n):
            if not (0 <= yy < h_img and 0 <= xx < w_img):
                return False
    return True


@pytest.mark.parametrize("N", [1, 2, 5, 6])
@pytest.mark.parametrize("r", [0, 1, 3])
def test_window_rule_against_pixel_enumeration(N, r):
    """Section III-G, Eq. 3: the template box (side N, top-left p - N//2)
    must lie in A and the search box (side N + 2r) in B.  window_ok against
    enumerating the boxes' pixels at every position, even and odd N, A and B of
    different sizes: pins both the left/top and the right/bottom edges."""
    hA, wA, hB, wB = 9, 11, 13, 12
    h = N // 2
    for y in range(-3, 14):
        for x in range(-3, 16):
            for by, bx in ((6, 6), (y, x), (x, y)):
                want = (_box_pixels_valid(x - h, y - h, N, hA, wA)
                        and _box_pixels_valid(bx - h - r, by - h - r, N + 2 * r, hB, wB))
                assert O.window_ok((x, y, bx, by), N, r, hA, wA, hB, wB) == want, (x, y, bx, by)


def _ssd_loop(D1, D2, cp, N, r):
    """Eq. 3 as explicit loops with every index checked (numpy would wrap a
    negative index or silently shorten a slice)."""
    x, y, bx, by = cp
    h = N // 2
    m, hA, wA = D1.shape
    _, hB, wB = D2.shape
    K = 2 * r + 1
    out = np.zeros((K, K))
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            acc = 0.0
            for c in range(m):
                for i in range(N):
                    for j in range(N):
                        ya, xa = y - h + i, x - h + j
                        yb, xb = by - h + i + dy, bx - h + j + dx
                        assert 0 <= ya < hA and 0 <= xa < wA and 0 <= yb < hB and 0 <= xb < wB
                        acc += (D1[c, ya, xa] - D2[c, yb, xb]) ** 2
            out[dy + r, dx + r] = acc
    return out


@pytest.mark.parametrize("N", [3, 4])
def test_flush_right_and_bottom_windows(N):
    """A template flush against A's right and bottom edges, and a search box
    flush against B's, are inside and matched over every offset (the surface
    equals the index-checked loop, so the last row and column are read); one
    pixel further is out of bounds.  Even and odd N."""
    rng = np.random.default_rng(40 + N)
    r = 2
    D1 = rng.random((2, 10, 12))   # A: 10 x 12
    D2 = rng.random((2, 13, 11))   # B: 13 x 11
    h = N // 2
    xr, yb = 12 - N + h, 10 - N + h            # template flush right / bottom in A
    sxr, syb = 11 - N - r + h, 13 - N - r + h  # search box flush right / bottom in B
    cases = [((xr, yb, 5, 6), True), ((xr + 1, yb, 5, 6), False), ((xr, yb + 1, 5, 6), False),
             ((5, 5, sxr, syb), True), ((5, 5, sxr + 1, syb), False), ((5, 5, sxr, syb + 1), False),
             ((h, h, h + r, h + r), True), ((h - 1, h, h + r, h + r), False), ((h, h, h + r - 1, h + r), False)]
    res = O.match(D1, D2, [c for c, _ in cases], N, r, surfaces=True)
    for k, (cp, inside) in enumerate(cases):
        assert res["status"][k] == (O.STATUS_OK if inside else O.STATUS_OUT_OF_BOUNDS), cp
        if inside:
            np.testing.assert_allclose(res["surfaces"][k], _ssd_loop(D1, D2, cp, N, r), rtol=1e-13)
        else:
            assert np.all(np.isnan(res["surfaces"][k]))


# ------------------------------------------------------- FFT cross-check pins

@pytest.mark.parametrize("m", [1, 3, 9])
@pytest.mark.parametrize("N,r", [(1, 1), (4, 2), (7, 3), (8, 1)])
def test_fft_form_equals_direct(m, N, r):
    rng = np.random.default_rng(m * 31 + N * 7 + r)
    D1 = rng.random((m, 24, 26))
    D2 = rng.random((m, 27, 22))
    h = N // 2
    cp = (h + r + 3, h + r + 2, h + r + 4, h + r + 5)
    Sd = O.ssd_surface_direct(D1, D2, cp, N, r)
    E1, E2 = O.energies(D1, D2, cp, N, r)
    for P in (N + 2 * r, N + 2 * r + 3, 32):
        Sf = O.ssd_surface_fft(D1, D2, cp, N, r, P=P)
        assert np.max(np.abs(Sf - Sd) / (E1 + E2)) < 1e-10


def test_3dfft_correlation_equals_naive_dft_at_P12():
    rng = np.random.default_rng(12)
    m, N, r, P = 3, 5, 2, 12
    T = rng.random((m, N, N))
    Sw = rng.random((m, N + 2 * r, N + 2 * r))
    Tp = np.zeros((m, P, P)); Tp[:, :N, :N] = T
    Sp = np.zeros((m, P, P)); Sp[:, :N + 2 * r, :N + 2 * r] = Sw

    def dft_mat(n, sign):
        k = np.arange(n)
        return np.exp(sign * 2j * np.pi * np.outer(k, k) / n)

    Fz, Fp = dft_mat(m, -1), dft_mat(P, -1)
    Iz, Ip = dft_mat(m, +1) / m, dft_mat(P, +1) / P

    def f3(a, Mz, My):
        return np.einsum("az,by,cx,zyx->abc", Mz, My, My, a)

    C = f3(np.conj(f3(Tp, Fz, Fp)) * f3(Sp, Fz, Fp), Iz, Ip).real
    assert np.max(np.abs(C[0, :2 * r + 1, :2 * r + 1] - O.correlation_3dfft(T, Sw, P))) < 1e-12


def test_vz0_slice_is_sum_of_channel_correlations():
    """Parseval along the orientation axis: the zero-shift slice of the 3-D
    correlation equals the sum over channels of plain 2-D correlations."""
    rng = np.random.default_rng(13)
    m, N, r = 9, 6, 3
    T = rng.random((m, N, N))
    Sw = rng.random((m, N + 2 * r, N + 2 * r))
    C = O.correlation_3dfft(T, Sw, 16)
    ref = np.zeros((2 * r + 1, 2 * r + 1))
    for uy in range(2 * r + 1):
        for ux in range(2 * r + 1):
            ref[uy, ux] = np.sum(T * Sw[:, uy:uy + N, ux:ux + N])
    assert np.max(np.abs(C - ref)) < 1e-11


def test_match_fft_agrees_with_direct_on_synthetic_pair():
    w = dict(synth.PLAIN_256)
    spec = synth.PairSpec(96, 96, 12, (3.0, 8.0), 6, 4)
    A, B, s = synth.make_pair(spec, (90, 1))
    D1, D2 = O.cfog(A), O.cfog(B)
    cps = synth.grid_cps(96, 96, 16, 4, 3)
    a = O.match(D1, D2, cps, 16, 4, surfaces=True)
    b = O.match_fft(D1, D2, cps, 16, 4, surfaces=True)
    assert np.array_equal(a["dx"], b["dx"]) and np.array_equal(a["dy"], b["dy"])
    assert np.max(np.abs(a["surfaces"] - b["surfaces"])) < 1e-9 * np.max(a["surfaces"])
    del w


# ------------------------------------------------------------------ SAT pins

def test_sat_box_sums_equal_direct_sums():
    rng = np.random.default_rng(21)
    Q = rng.random((23, 31)) * 1e3
    S = O.sat(Q)
    assert S.shape == (24, 32) and np.all(S[0] == 0) and np.all(S[:, 0] == 0)
    for (y0, x0, h, w) in [(0, 0, 23, 31), (3, 4, 5, 6), (22, 30, 1, 1), (10, 0, 13, 31)]:
        assert abs(O.box_sum(S, y0, x0, h, w) - Q[y0:y0 + h, x0:x0 + w].sum()) < 1e-9


def test_energy_terms_match_sat():
    rng = np.random.default_rng(22)
    D1, D2 = rng.random((3, 20, 20)), rng.random((3, 20, 20))
    cp, N, r = (9, 9, 10, 10), 6, 2
    E1, E2 = O.energies(D1, D2, cp, N, r)
    S1, S2 = O.sat((D1 ** 2).sum(0)), O.sat((D2 ** 2).sum(0))
    assert abs(E1 - O.box_sum(S1, 6, 6, 6, 6)) < 1e-12
    assert abs(E2[0, 0] - O.box_sum(S2, 5, 5, 6, 6)) < 1e-12


# ------------------------------------------------------- generator sanity

def test_generator_is_seeded_and_shift_consistent():
    spec = synth.PairSpec(64, 64, 10, (3.0, 6.0), 5, 6)
    A1, B1, s1 = synth.make_pair(spec, (1, 2))
    A2, B2, s2 = synth.make_pair(spec, (1, 2))
    assert np.array_equal(A1, A2) and np.array_equal(B1, B2) and s1 == s2
    assert A1.dtype == np.float32 and A1.flags.c_contiguous
    cps = synth.grid_cps(64, 64, 12, 4, 3)
    h = 6
    assert cps[:, 0].min() - h - 4 >= 0 and cps[:, 0].max() - h + 12 + 4 <= 64


def test_paper_workload_recovers_most_shifts():
    """Sanity (not parity): on the 256^2 stand-in pair with mild speckle
    (Gamma shape 100) CFOG recovers the seeded shift within the paper's 1.5 px
    correctness criterion (Section V-B) for most control points.  The default
    speckle (shape 4) is much harsher; its recovery rate is only reported."""
    import dataclasses
    spec = dataclasses.replace(synth.PLAIN_256["spec"], speckle_shape=100.0)
    A, B, s = synth.make_pair(spec, synth.PLAIN_256["seed"])
    cps = synth.grid_cps(256, 256, 48, 10, 5)
    res = O.match_fft(O.cfog(A), O.cfog(B), cps, 48, 10)
    ok = np.hypot(res["dx"] - s[0], res["dy"] - s[1]) <= 1.5
    assert ok.mean() >= 0.6


# -------------------------------------- Eq. 7 objective, sub-pixel refinement

def _python_loop_corr(D1, D2, cp, N, r):
    x, y, bx, by = cp
    h = N // 2
    m = len(D1)
    out = [[0.0] * (2 * r + 1) for _ in range(2 * r + 1)]
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            acc = 0.0
            for c in range(m):
                for i in range(N):
                    for j in range(N):
                        acc += float(D1[c][y - h + i][x - h + j]) * float(D2[c][by - h + dy + i][bx - h + dx + j])
            out[dy + r][dx + r] = -acc
    return np.array(out)


@pytest.mark.parametrize("N,r,m", [(3, 1, 2), (4, 2, 1), (5, 2, 3)])
def test_correlation_objective_against_python_loops(N, r, m):
    rng = np.random.default_rng(N * 10 + r)
    D1 = rng.normal(size=(m, 12, 12))
    D2 = rng.normal(size=(m, 12, 12))
    cp = (6, 6, 6, 5)
    J = O.correlation_surface_direct(D1, D2, cp, N, r)
    np.testing.assert_allclose(J, _python_loop_corr(D1.tolist(), D2.tolist(), cp, N, r), rtol=0, atol=1e-12)


def test_correlation_objective_is_ssd_without_energies():
    """Eq. 5 rearranged: -C(d) = (S(d) - E1 - E2(d)) / 2, from the SSD oracle
    and the energies (a different formula for every term)."""
    A, B, _ = synth.make_pair(synth.PairSpec(64, 64, 12, (3.0, 8.0), 6, 4), (9, 1))
    D1, D2 = O.cfog(A.astype(np.float64)), O.cfog(B.astype(np.float64))
    cp, N, r = (30, 31, 32, 30), 20, 5
    S = O.ssd_surface_direct(D1, D2, cp, N, r)
    E1, E2 = O.energies(D1, D2, cp, N, r)
    J = O.correlation_surface_direct(D1, D2, cp, N, r)
    np.testing.assert_allclose(J, 0.5 * (S - E1 - E2), rtol=1e-12, atol=1e-9 * E1)


@pytest.mark.parametrize("t0,alpha,beta", [(0.0, 1.0, 0.0), (0.3, 2.5, -1.0), (-0.45, 0.1, 7.0), (0.49, 3.0, 2.0)])
def test_parabola_vertex_is_exact_for_quadratics(t0, alpha, beta):
    q = lambda t: alpha * (t - t0) ** 2 + beta  # noqa: E731
    assert O.parabola_vertex(q(-1), q(0), q(1)) == pytest.approx(t0, abs=1e-12)


def test_parabola_vertex_without_a_minimum_is_zero():
    assert O.parabola_vertex(1.0, 1.0, 1.0) == 0.0   # flat
    assert O.parabola_vertex(0.0, 1.0, 0.0) == 0.0   # a maximum
    assert O.parabola_vertex(2.0, 1.0, 0.0) == 0.0   # a straight line


@pytest.mark.parametrize("x0,y0", [(0.3, -1.2), (-2.49, 1.5001), (1.0, 0.0), (2.2, -2.4)])
def test_subpixel_recovers_a_sampled_quadratic_bowl(x0, y0):
    r = 3
    d = np.arange(-r, r + 1)
    S = 2.0 * (d[None, :] - x0) ** 2 + 0.5 * (d[:, None] - y0) ** 2 + 3.0
    dx, dy, _, _ = O.argmin_lex(S)
    assert (dx, dy) == (int(np.floor(x0 + 0.5)), int(np.floor(y0 + 0.5)))
    fx, fy = O.subpixel(S, dx, dy)
    assert fx == pytest.approx(x0, abs=1e-12) and fy == pytest.approx(y0, abs=1e-12)


def test_subpixel_keeps_integer_offsets_at_the_border():
    r = 2
    d = np.arange(-r, r + 1)
    S = (d[None, :] + 2.4) ** 2 + (d[:, None] - 0.25) ** 2   # x minimum beyond -r
    dx, dy, _, _ = O.argmin_lex(S)
    assert dx == -r
    fx, fy = O.subpixel(S, dx, dy)
    assert fx == -r and fy == pytest.approx(0.25, abs=1e-12)


def test_match_with_correlation_objective_and_subpixel():
    rng = np.random.default_rng(3)
    D1, D2 = rng.random((2, 30, 30)), rng.random((2, 30, 30))
    cps = [(12, 12, 13, 12), (15, 14, 15, 15), (1, 1, 1, 1)]
    res = O.match(D1, D2, cps, 8, 3, surfaces=True, objective="corr", subpix=True)
    assert list(res["status"]) == [0, 0, O.STATUS_OUT_OF_BOUNDS]
    for k in range(2):
        J = O.correlation_surface_direct(D1, D2, cps[k], 8, 3)
        dx, dy, b, s = O.argmin_lex(J)
        assert (res["dx"][k], res["dy"][k], res["best"][k]) == (dx, dy, b)
        assert (res["fdx"][k], res["fdy"][k]) == O.subpixel(J, dx, dy)
    assert np.isnan(res["fdx"][2])


# ------------------------------------------ block-based Harris (Section IV)

def _python_loop_harris(chip, sigma=1.0, kappa=0.04):
    h, w = len(chip), len(chip[0])
    cl = lambda v, n: min(max(v, 0), n - 1)  # noqa: E731
    gx = [[chip[y][cl(x + 1, w)] - chip[y][cl(x - 1, w)] for x in range(w)] for y in range(h)]
    gy = [[chip[cl(y + 1, h)][x] - chip[cl(y - 1, h)][x] for x in range(w)] for y in range(h)]
    R = int(4 * sigma + 0.5)
    wt = [np.exp(-j * j / (2 * sigma * sigma)) for j in range(-R, R + 1)]
    tot = sum(wt)
    wt = [v / tot for v in wt]

    def smooth(a):
        t = [[sum(wt[j + R] * a[y][cl(x + j, w)] for j in range(-R, R + 1)) for x in range(w)] for y in range(h)]
        return [[sum(wt[j + R] * t[cl(y + j, h)][x] for j in range(-R, R + 1)) for x in range(w)] for y in range(h)]
    A = smooth([[gx[y][x] * gx[y][x] for x in range(w)] for y in range(h)])
    B = smooth([[gx[y][x] * gy[y][x] for x in range(w)] for y in range(h)])
    C = smooth([[gy[y][x] * gy[y][x] for x in range(w)] for y in range(h)])
    return np.array([[A[y][x] * C[y][x] - B[y][x] ** 2 - kappa * (A[y][x] + C[y][x]) ** 2
                      for x in range(w)] for y in range(h)])


def test_harris_response_against_python_loops():
    chip = np.random.default_rng(4).random((9, 11))
    np.testing.assert_allclose(O.harris_response(chip), _python_loop_harris(chip.tolist()), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("alpha,beta", [(0.5, 0.25), (-1.0, 2.0), (0.0, 1.5)])
def test_harris_of_a_ramp_is_the_closed_form(alpha, beta):
    """I = alpha x + beta y: gradients (2 alpha, 2 beta) everywhere off the
    border, so M is rank one (det = 0) and R = -kappa (4 alpha^2 + 4 beta^2)^2
    wherever the smoothing window avoids the border rows and columns."""
    y, x = np.mgrid[0:30, 0:30].astype(np.float64)
    R = O.harris_response(alpha * x + beta * y)
    want = -0.04 * (4 * alpha ** 2 + 4 * beta ** 2) ** 2
    np.testing.assert_allclose(R[5:-5, 5:-5], want, rtol=1e-12, atol=1e-12)


def test_harris_is_transpose_symmetric():
    chip = np.random.default_rng(5).random((20, 20))
    np.testing.assert_allclose(O.harris_response(chip.T), O.harris_response(chip).T, rtol=1e-13, atol=1e-15)


def test_harris_constant_image_selects_first_pixels():
    pts, vals = O.harris_grid(np.full((120, 120), 3.0), 2, 3)
    assert np.all(vals == 0.0)
    # cell (0, 0): chip centred at (30, 30) -> top-left (0, 0); ties: first three pixels
    assert [tuple(p) for p in pts[:3]] == [(0, 0), (1, 0), (2, 0)]
    y0, x0, h, w = O.harris_chip_origin(120, 120, 2, 1, 1)
    assert (y0, x0, h, w) == (60, 60, 60, 60)


def test_harris_finds_the_corners_of_a_square():
    img = np.zeros((60, 60))
    img[20:40, 20:40] = 1.0
    pts, vals = O.harris_grid(img, 1, 4)
    for x, y in pts:
        # each of the four strongest responses sits within a pixel of a corner
        assert min(abs(x - cx) + abs(y - cy) for cx, cy in [(19.5, 19.5), (39.5, 19.5), (19.5, 39.5), (39.5, 39.5)]) <= 1.0
    assert len({(int(x) // 30, int(y) // 30) for x, y in pts}) == 4  # one per corner


def test_harris_grid_chip_clipping_and_order():
    img = np.random.default_rng(6).random((100, 130))
    pts, vals = O.harris_grid(img, 3, 5, chip=60)
    assert pts.shape == (45, 2)
    for c in range(9):
        v = vals[5 * c:5 * c + 5]
        assert np.all(np.diff(v) <= 0)
        i, j = divmod(c, 3)
        y0, x0, h, w = O.harris_chip_origin(100, 130, 3, i, j)
        assert h <= 60 and w <= 60 and y0 >= 0 and x0 >= 0 and y0 + h <= 100 and x0 + w <= 130
        R = O.harris_response(img[y0:y0 + h, x0:x0 + w])
        assert vals[5 * c] == R.max()
        for (x, y), val in zip(pts[5 * c:5 * c + 5], v):
            assert R[y - y0, x - x0] == val


# ------------------------------------------- outlier rejection (Section IV)

def _cubic_map(P, C):
    """Apply a cubic (10, 2) given in pixel coordinates of the normalised
    frame built from P itself."""
    c, s = O.normalise_points(P)
    return O.cubic_terms((P[:, 0] - c[0]) / s[0], (P[:, 1] - c[1]) / s[1]) @ C


def _gauss_solve(A, b):
    """Least squares by hand: normal equations and Gaussian elimination with
    partial pivoting, in plain Python."""
    n = len(A[0])
    M = [[sum(A[k][i] * A[k][j] for k in range(len(A))) for j in range(n)] +
         [sum(A[k][i] * b[k] for k in range(len(A)))] for i in range(n)]
    for col in range(n):
        piv = max(range(col, n), key=lambda r: abs(M[r][col]))
        M[col], M[piv] = M[piv], M[col]
        for r in range(col + 1, n):
            f = M[r][col] / M[col][col]
            for cc in range(col, n + 1):
                M[r][cc] -= f * M[col][cc]
    x = [0.0] * n
    for r in range(n - 1, -1, -1):
        x[r] = (M[r][n] - sum(M[r][cc] * x[cc] for cc in range(r + 1, n))) / M[r][r]
    return x


def test_cubic_fit_against_hand_normal_equations():
    rng = np.random.default_rng(8)
    P = rng.uniform(0, 500, (40, 2))
    Q = P + rng.normal(0, 2.0, (40, 2))
    keep, coef, rmse, removed = O.reject_outliers(P, Q, threshold=1e9)  # no removal: one fit
    assert removed == 0 and keep.all()
    c, s = O.normalise_points(P)
    T = O.cubic_terms((P[:, 0] - c[0]) / s[0], (P[:, 1] - c[1]) / s[1]).tolist()
    for axis in range(2):
        np.testing.assert_allclose(coef[:, axis], _gauss_solve(T, Q[:, axis].tolist()), rtol=1e-8, atol=1e-8)


def test_exact_cubic_map_is_recovered_without_removal():
    rng = np.random.default_rng(9)
    P = rng.uniform(100, 900, (60, 2))
    C = rng.normal(0, 3.0, (10, 2))
    C[1, 0] += 400.0  # mostly x -> x', y -> y'
    C[2, 1] += 400.0
    Q = _cubic_map(P, C)
    keep, coef, rmse, removed = O.reject_outliers(P, Q)
    assert removed == 0 and keep.all() and rmse < 1e-9
    np.testing.assert_allclose(coef, C, rtol=1e-9, atol=1e-8)


def test_gross_outliers_are_removed_first():
    rng = np.random.default_rng(10)
    P = rng.uniform(0, 1000, (80, 2))
    C = np.zeros((10, 2))
    C[0] = [500.0, 500.0]
    C[1, 0], C[2, 1] = 500.0, 500.0     # identity in pixel units
    C[3, 0], C[5, 1] = 2.0, -1.5         # mild curvature
    Q = _cubic_map(P, C) + rng.normal(0, 0.5, (80, 2))
    bad = [3, 17, 42, 77]
    Q[bad] += np.array([[40.0, -25.0], [-30.0, 60.0], [55.0, 10.0], [-20.0, -45.0]])
    keep, coef, rmse, removed = O.reject_outliers(P, Q, threshold=1.0)
    assert set(np.flatnonzero(~keep)) == set(bad) and removed == 4
    assert 0.3 < rmse < 1.0


def test_rejection_stops_at_ten_points_and_needs_ten():
    rng = np.random.default_rng(11)
    P = rng.uniform(0, 100, (12, 2))
    Q = rng.uniform(0, 100, (12, 2))   # no model fits: removal continues to ten points
    keep, coef, rmse, removed = O.reject_outliers(P, Q, threshold=0.0)
    assert keep.sum() == 10 and removed == 2 and rmse < 1e-6  # ten points are interpolated
    with pytest.raises(ValueError):
        O.reject_outliers(P[:9], Q[:9])


# ---------------------------------------------- CFOG scheme 1 (Section III-F)

def test_scheme1_on_and_between_bins():
    m = 9
    th = np.arange(m) * np.pi / m
    # a gradient exactly at bin 4's orientation goes entirely to bin 4
    gx, gy = np.array([[2.0 * np.cos(th[4])]]), np.array([[2.0 * np.sin(th[4])]])
    G = O.oriented_channels_scheme1(gx, gy, m)[:, 0, 0]
    np.testing.assert_allclose(G, np.eye(m)[4] * 2.0, atol=1e-12)
    # halfway between bins 8 and 0 (170 degrees): half to each, circularly
    a = np.pi * (m - 0.5) / m
    G = O.oriented_channels_scheme1(np.array([[np.cos(a)]]), np.array([[np.sin(a)]]), m)[:, 0, 0]
    want = np.zeros(m)
    want[8] = want[0] = 0.5
    np.testing.assert_allclose(G, want, atol=1e-12)


def test_scheme1_channels_sum_to_the_magnitude_and_ignore_sign():
    rng = np.random.default_rng(12)
    gx, gy = rng.normal(size=(2, 20, 20))
    G = O.oriented_channels_scheme1(gx, gy, 7)
    np.testing.assert_allclose(G.sum(axis=0), np.hypot(gx, gy), rtol=1e-12)
    assert np.all(G >= 0) and np.all((G > 0).sum(axis=0) <= 2)
    np.testing.assert_allclose(O.oriented_channels_scheme1(-gx, -gy, 7), G, rtol=1e-12, atol=1e-15)


def test_scheme1_against_python_loops():
    rng = np.random.default_rng(13)
    gx, gy, m = rng.normal(size=(6, 5)), rng.normal(size=(6, 5)), 6
    G = O.oriented_channels_scheme1(gx, gy, m)
    for y in range(6):
        for x in range(5):
            phi = np.arctan2(gy[y, x], gx[y, x]) % np.pi
            mag = (gx[y, x] ** 2 + gy[y, x] ** 2) ** 0.5
            for k in range(m):
                d = abs(phi - k * np.pi / m)
                d = min(d, np.pi - d)  # circular distance over [0, pi)
                assert G[k, y, x] == pytest.approx(mag * max(0.0, 1.0 - d * m / np.pi), abs=1e-12)


def test_scheme1_mirror_invariant():
    img = np.random.default_rng(14).random((24, 30))
    m = 8
    D = O.cfog(img, m=m, scheme=1)
    Df = O.cfog(img[:, ::-1], m=m, scheme=1)
    for k in range(m):
        np.testing.assert_allclose(Df[(m - k) % m], D[k][:, ::-1], rtol=1e-12, atol=1e-13)


# ------------------------------------------------- pixel-wise HOG (III-C)

def _python_loop_fhog(img, c=4, bins=9):
    """The histogram of the definition, pixel by pixel: every gradient q of
    the block around p adds |g| x (orientation weight) x (bilinear weight of
    each cell); then the 36 values are L2-normalised."""
    H, W = len(img), len(img[0])
    cl = lambda v, n: min(max(v, 0), n - 1)  # noqa: E731
    out = np.zeros((4 * bins, H, W))
    for py in range(H):
        for px in range(W):
            v = np.zeros(4 * bins)
            for dy in range(-c, c + 1):
                for dx in range(-c, c + 1):
                    y, x = cl(py + dy, H), cl(px + dx, W)
                    gx = img[y][cl(x + 1, W)] - img[y][cl(x - 1, W)]
                    gy = img[cl(y + 1, H)][x] - img[cl(y - 1, H)][x]
                    mag = (gx * gx + gy * gy) ** 0.5
                    phi = np.arctan2(gy, gx) % np.pi
                    for a, ox in enumerate((-c / 2, c / 2)):
                        wx = max(0.0, 1.0 - abs(dx - ox) / c)
                        for b, oy in enumerate((-c / 2, c / 2)):
                            wy = max(0.0, 1.0 - abs(dy - oy) / c)
                            for k in range(bins):
                                d = abs(phi - k * np.pi / bins)
                                d = min(d, np.pi - d)
                                wo = max(0.0, 1.0 - d * bins / np.pi)
                                v[(2 * a + b) * bins + k] += mag * wo * wx * wy
            out[:, py, px] = v / np.sqrt(np.sum(v * v) + O.FHOG_EPS)
    return out


def test_fhog_against_python_loops():
    img = np.random.default_rng(15).random((7, 9))
    np.testing.assert_allclose(O.fhog(img, c=2), _python_loop_fhog(img.tolist(), c=2), rtol=1e-10, atol=1e-12)


def test_fhog_unit_norm_zero_on_flat_and_invariances():
    img = np.random.default_rng(16).random((20, 24))
    F = O.fhog(img)
    np.testing.assert_allclose(np.sqrt(np.sum(F * F, axis=0)), 1.0, rtol=1e-9)
    assert np.all(O.fhog(np.full((12, 12), 2.0)) == 0.0)
    np.testing.assert_allclose(O.fhog(3.0 * img), F, rtol=1e-9, atol=1e-12)   # contrast
    np.testing.assert_allclose(O.fhog(-img), F, rtol=1e-12, atol=1e-14)        # intensity inversion


def test_fhog_vertical_edge_fills_bin_zero_only():
    img = np.zeros((16, 16))
    img[:, 8:] = 1.0                                  # horizontal gradient only: orientation 0
    F = O.fhog(img)
    mask = np.ones(36, bool)
    mask[[0, 9, 18, 27]] = False                      # bin 0 of each cell
    assert np.all(F[mask] == 0.0)
    assert np.all(F[~mask][:, :, 4:12].sum(axis=0) > 0)


def test_fhog_cell_kernels():
    np.testing.assert_allclose(O.fhog_cell_kernel(4, -2.0), [0.5, 0.75, 1.0, 0.75, 0.5, 0.25, 0.0, 0.0, 0.0])
    np.testing.assert_allclose(O.fhog_cell_kernel(4, 2.0), O.fhog_cell_kernel(4, -2.0)[::-1])
