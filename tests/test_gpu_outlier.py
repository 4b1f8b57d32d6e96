"""GPU tests of the iterative cubic-polynomial outlier rejection (Section IV)
against the FP64 oracle: the GPU (FP64 normal equations formed once and
downdated per removed point, Cholesky) removes exactly the oracle's points
(least squares by QR on the kept points); the final model and RMSE agree to
1e-6 relative (the two solvers differ only in rounding).  Sets of up to 8192
points are held in LDS, larger ones are read from global memory (n = 9000).

Every case prints its name, sizes and seed before touching the GPU."""
import numpy as np
import pytest

import oracle as O
from paper_1808_06194_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def cf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1808_06194_amd import cfog
    cfog.load()
    return cfog


def _points(seed, n, n_bad, noise=0.4, curve=3.0):
    rng = np.random.default_rng(np.random.SeedSequence([80, seed]))
    P = rng.uniform(0, 2048, (n, 2))
    u, v = (P[:, 0] - 1024) / 1024, (P[:, 1] - 1024) / 1024
    Q = P + np.stack([curve * u * v + 5.0, -curve * u * u * v + 2.0], 1) + rng.normal(0, noise, (n, 2))
    bad = rng.choice(n, n_bad, replace=False)
    Q[bad] += rng.uniform(-40, 40, (n_bad, 2))
    return P.astype(np.float32), Q.astype(np.float32), set(int(b) for b in bad)


def _compare(cf, P, Q, thr):
    keep_g, res = cf.reject_outliers(torch.from_numpy(P).cuda(), torch.from_numpy(Q).cuda(), thr)
    keep_o, coef_o, rmse_o, removed_o = O.reject_outliers(P.astype(np.float64), Q.astype(np.float64), thr)
    assert res["status"] == 0
    assert np.array_equal(keep_g.cpu().numpy().astype(bool), keep_o)
    assert res["removed"] == removed_o and res["n_kept"] == int(keep_o.sum())
    c, s = O.normalise_points(P.astype(np.float64))
    np.testing.assert_allclose(res["centre"], c, rtol=1e-12)
    np.testing.assert_allclose(res["half_extent"], s, rtol=1e-12)
    np.testing.assert_allclose(res["coef"], coef_o, rtol=1e-6, atol=1e-6 * np.max(np.abs(coef_o)))
    assert abs(res["rmse"] - rmse_o) <= 1e-6 * max(rmse_o, 1e-3)
    return keep_o, res


@pytest.mark.parametrize("n,n_bad,thr,seed", [(200, 12, 1.0, 1), (900, 60, 3.5, 2), (37, 5, 1.0, 3),
                                              (3000, 150, 1.0, 4), (8192, 200, 1.0, 5), (9000, 120, 1.0, 6)])
def test_rejection_matches_oracle(cf, n, n_bad, thr, seed):
    _say(f"reject n={n} outliers={n_bad} threshold={thr} seed={seed}")
    P, Q, bad = _points(seed, n, n_bad)
    keep, res = _compare(cf, P, Q, thr)
    removed = set(np.flatnonzero(~keep).tolist())
    _say("removed", len(removed), "of which injected", len(removed & bad), "rmse", res["rmse"])


def test_rejection_stops_at_ten_points(cf):
    _say("reject: no model fits, stops at ten points")
    rng = np.random.default_rng(81)
    P = rng.uniform(0, 100, (25, 2)).astype(np.float32)
    Q = rng.uniform(0, 100, (25, 2)).astype(np.float32)
    keep, res = _compare(cf, P, Q, 0.0)
    assert keep.sum() == 10 and res["removed"] == 15


def test_rejection_of_coincident_points_is_singular(cf):
    _say("reject: coincident points (normalised coordinates all zero)")
    P = np.full((30, 2), 7.0, np.float32)
    keep, res = cf.reject_outliers(torch.from_numpy(P).cuda(), torch.from_numpy(P + 1).cuda(), 1.0)
    assert res["status"] == 1 and np.all(np.isnan(res["coef"]))


def test_rejection_rejects_bad_arguments(cf):
    _say("reject: argument checks")
    P = torch.zeros((9, 2), device="cuda")
    with pytest.raises(cf.CfogError):
        cf.reject_outliers(P, P)


def test_rejection_after_harris_and_subpixel_matching(cf):
    """Section IV's chain: Harris points in A, matched with sub-pixel
    refinement, then outlier rejection (threshold 3.5 as in Table V)."""
    _say("harris -> match (subpix) -> reject, 1024^2, n=12 k=3, template 60 radius 12, seed (82, 0)")
    spec = synth.PairSpec(1024, 1024, 600, (3.0, 15.0), 300, 8, speckle_shape=100.0)
    A, B, s = synth.make_pair(spec, (82, 0), shift=(4, -3))
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    cps, _ = cf.harris_grid(dA, 12, 3)
    vA, sA = cf.cfog_extract(dA)
    vB, sB = cf.cfog_extract(dB)
    sub = torch.empty((cps.shape[0], 2), device="cuda")
    job = cf.Job(vA, sA, vB, sB, cps, 60, 12, subpix=sub)
    cf.match_batch([job])
    torch.cuda.synchronize()
    st = cf.results(job.out)["status"].cpu().numpy()
    ok = st == 0
    src = cps[:, :2].float().cpu().numpy()[ok]
    dst = (src + sub.cpu().numpy()[ok]).astype(np.float32)
    keep, res = _compare(cf, src.astype(np.float32), dst, 3.5)
    d = dst - src
    _say("points", int(ok.sum()), "kept", int(keep.sum()), "rmse", res["rmse"],
         "median kept offset", np.median(d[keep], axis=0).tolist())
    assert np.allclose(np.median(d[keep], axis=0), [4, -3], atol=0.5)
