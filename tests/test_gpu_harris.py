"""GPU tests of the block-based Harris feature points (Section IV) against
the FP64 oracle.

Parity rule: the FP32 response at every selected point is within
1e-4 * max|R| of the chip's oracle response (rounding of ~40 FP32 operations on
products of gradients); a selected point equals the oracle's of the same rank
or is an excused near-tie: the oracle responses of the GPU's k points, sorted,
match the oracle's top k within twice that bound.

Every case prints its name, sizes and seed before touching the GPU."""
import numpy as np
import pytest

import oracle as O
from paper_1808_06194_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def cf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1808_06194_amd import cfog
    cfog.load()
    return cfog


def _run(cf, img, n, k, chip=60, sigma=1.0):
    cps, resp = cf.harris_grid(torch.from_numpy(np.ascontiguousarray(img, np.float32)).cuda(), n, k, chip, sigma)
    torch.cuda.synchronize()
    return cps.cpu().numpy(), resp.cpu().numpy()


def _check(img, n, k, chip, cps, resp, sigma=1.0):
    I = np.asarray(img, np.float32).astype(np.float64)
    H, W = I.shape
    pts_o, vals_o = O.harris_grid(I, n, k, chip, sigma)
    exact = excused = 0
    for c in range(n * n):
        i, j = divmod(c, n)
        y0, x0, h, w = O.harris_chip_origin(H, W, n, i, j, chip)
        R = O.harris_response(I[y0:y0 + h, x0:x0 + w], sigma)
        tol = TOL * float(np.max(np.abs(R)))
        g = cps[c * k:(c + 1) * k]
        assert np.all(g[:, 0] == g[:, 2]) and np.all(g[:, 1] == g[:, 3])
        assert len({(int(x), int(y)) for x, y, _, _ in g}) == k, "duplicate points"
        rg = []
        for q, (x, y, _, _) in enumerate(g):
            assert x0 <= x < x0 + w and y0 <= y < y0 + h, (c, q, x, y)
            ro = R[y - y0, x - x0]
            assert abs(float(resp[c * k + q]) - ro) <= tol, (c, q, float(resp[c * k + q]), ro, tol)
            rg.append(ro)
            if (x, y) == tuple(pts_o[c * k + q]):
                exact += 1
            else:
                excused += 1
        np.testing.assert_allclose(np.sort(rg)[::-1], vals_o[c * k:(c + 1) * k], rtol=0, atol=2 * tol)
    return exact, excused


@pytest.mark.parametrize("H,W,n,k,chip,seed", [
    (256, 256, 4, 5, 60, 1), (200, 333, 3, 8, 60, 2), (50, 70, 1, 6, 60, 3), (160, 160, 5, 3, 16, 4),
    (300, 300, 2, 64, 64, 5), (97, 131, 6, 2, 60, 6)])
def test_harris_grid_against_oracle(cf, H, W, n, k, chip, seed):
    _say(f"harris {H}x{W} n={n} k={k} chip={chip} seed={seed}")
    A, _, _ = synth.make_pair(synth.PairSpec(H, W, max(4, H * W // 1500), (3.0, 15.0), max(2, H * W // 3000), 4),
                              (70, seed))
    cps, resp = _run(cf, A, n, k, chip)
    exact, excused = _check(A, n, k, chip, cps, resp)
    _say("exact", exact, "excused near-ties", excused)


def test_harris_constant_image_takes_the_first_pixels(cf):
    _say("harris constant 120x120 n=2 k=3")
    cps, resp = _run(cf, np.full((120, 120), 3.0), 2, 3)
    assert np.all(resp == 0.0)
    pts_o, _ = O.harris_grid(np.full((120, 120), 3.0), 2, 3)
    assert np.array_equal(cps[:, :2], pts_o)


def test_harris_square_corners(cf):
    _say("harris square corners 60x60 n=1 k=4")
    img = np.zeros((60, 60), np.float32)
    img[20:40, 20:40] = 1.0
    cps, resp = _run(cf, img, 1, 4)
    pts_o, _ = O.harris_grid(img, 1, 4)
    assert {tuple(p) for p in cps[:, :2]} == {tuple(p) for p in pts_o}


def test_harris_rejects_bad_arguments(cf):
    _say("harris argument checks")
    img = torch.zeros((40, 40), device="cuda")
    with pytest.raises(cf.CfogError) as e:
        cf.harris_grid(img, 2, 65)
    assert e.value.code == cf.CFOG_EINVAL
    with pytest.raises(cf.CfogError) as e:
        cf.harris_grid(img, 1, 4, chip=65)
    assert e.value.code == cf.CFOG_EINVAL
    with pytest.raises(cf.CfogError) as e:
        cf.harris_grid(img, 40, 2, chip=1)  # 1-pixel chips cannot hold 2 points
    assert e.value.code == cf.CFOG_EINVAL
    with pytest.raises(cf.CfogError) as e:
        cf.harris_grid(img, 1, 1, sigma=2.5)  # radius 10 > 8
    assert e.value.code == cf.CFOG_EUNSUPPORTED


def test_harris_points_feed_the_matcher(cf):
    """The registration flow of Section IV: feature points in A, matched in B
    around the same positions (a sanity run: statuses and shift recovery on a
    pair with mild speckle)."""
    _say("harris -> match, 512^2, n=5 k=2, template 48 radius 10, seed (71, 0)")
    spec = synth.PairSpec(512, 512, 160, (3.0, 15.0), 80, 8, speckle_shape=100.0)
    A, B, s = synth.make_pair(spec, (71, 0), shift=(3, -2))
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    cps, _ = cf.harris_grid(dA, 5, 2)
    vA, sA = cf.cfog_extract(dA)
    vB, sB = cf.cfog_extract(dB)
    job = cf.Job(vA, sA, vB, sB, cps, 48, 10)
    cf.match_batch([job])
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in cf.results(job.out).items()}
    ok = res["status"] == 0
    assert ok.sum() >= 20
    rec = np.mean((res["dx"][ok] == 3) & (res["dy"][ok] == -2))
    _say("points", len(ok), "ok", int(ok.sum()), "recovered", float(rec))
    assert rec >= 0.6
