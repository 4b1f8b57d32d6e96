"""GPU tests of the matching server (serving entry points of the C-ABI):
results equal direct match_batch calls bit for bit and the FP64 oracle within
the parity rules; each request's result is the same alone and in a mix of
concurrent requests; admission under a small memory budget evicts and
recomputes volumes without changing any result.

Every case prints its name, sizes and seed before touching the GPU."""
import numpy as np
import pytest

from paper_1808_06194_amd import synth
from tests import parity

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


PAIR_SHAPES = [(160, 160, 20, 10), (200, 232, 30, 14), (256, 256, 40, 20)]  # H, W, blobs, rects


def _pairs(seed):
    out = []
    for i, (H, W, nb, nr) in enumerate(PAIR_SHAPES):
        A, B, s = synth.make_pair(synth.PairSpec(H, W, nb, (3.0, 15.0), nr, 8), (seed, i))
        out.append((A, B))
    return out


def _requests(seed, pairs, n, surf_every=3, oob_every=7):
    """n requests: random pair, template side N in [16, 48] (even and odd),
    radius in [2, 10], 1-30 control points; some with surfaces, some with one
    out-of-bounds point."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 77]))
    reqs = []
    for q in range(n):
        p = int(rng.integers(0, len(pairs)))
        H, W = pairs[p][0].shape
        N = int(rng.integers(16, 49))
        r = int(rng.integers(2, 11))
        k = int(rng.integers(1, 31))
        h = N // 2
        M = h + r + 1
        cps = np.stack([rng.integers(M, W - M, k), rng.integers(M, H - M, k)], 1)
        cps = np.concatenate([cps, cps], 1).astype(np.int32)
        if q % oob_every == oob_every - 1:
            cps[0] = (1, 1, 1, 1)
        reqs.append(dict(pair=p, cps=cps, N=N, r=r, surfaces=(q % surf_every == 0)))
    return reqs


def _direct(cf, pairs, reqs, flags):
    """Reference results: each request as its own match_batch call on volumes
    extracted separately (same kernels, same FFT sizes: a fresh context, like
    the server's own, so that no FFT size tuned by another test applies)."""
    ctx = cf.Context(0)
    vols = []
    for A, B in pairs:
        vA, sA = cf.cfog_extract(torch.from_numpy(A).cuda())
        vB, sB = cf.cfog_extract(torch.from_numpy(B).cuda())
        vols.append((vA, sA, vB, sB))
    out = []
    for q in reqs:
        vA, sA, vB, sB = vols[q["pair"]]
        K = 2 * q["r"] + 1
        surf = torch.empty((len(q["cps"]), K, K), device="cuda") if q["surfaces"] else None
        job = cf.Job(vA, sA, vB, sB, torch.from_numpy(q["cps"]).cuda(), q["N"], q["r"], surfaces=surf)
        cf.match_batch([job], flags=flags | cf.NO_SPLIT, ctx=ctx)  # the server matches every point whole
        out.append((job, surf))
    torch.cuda.synchronize()
    res = [(j.out.cpu().numpy(), None if s is None else s.cpu().numpy()) for j, s in out]
    ctx.close()
    return res


def _same(a, b):
    """Bit-identical results (and surfaces, NaN positions included)."""
    assert np.array_equal(a[0], b[0])
    if a[1] is not None or b[1] is not None:
        assert np.array_equal(a[1].view(np.int32), b[1].view(np.int32))


def _server(cf, imgs, budget, **kw):
    srv = cf.Server(budget, **kw)
    for A, B in imgs:
        srv.add_pair(A, B)
    return srv


def _dev_pairs(pairs):
    out = [(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()) for A, B in pairs]
    torch.cuda.synchronize()  # the server's streams do not order after torch's
    return out


def test_server_matches_direct_and_oracle_alone_and_in_mix(cf):
    seed = 41
    _say("server: 3 pairs (160^2, 200x232, 256^2), 80 requests, 4 slots, seed", seed)
    pairs = _pairs(seed)
    imgs = _dev_pairs(pairs)
    reqs = _requests(seed, pairs, 80)
    ref = _direct(cf, pairs, reqs, cf.PATH_BATCHED_FFT)
    with _server(cf, imgs, 2 << 30, n_slots=4, max_batch_cps=240, max_batch_reqs=6) as srv:
        sample = list(range(0, 80, 8))
        alone = {}
        for i in sample:
            q = reqs[i]
            rid = srv.submit(q["pair"], q["cps"], q["N"], q["r"], surfaces=q["surfaces"])
            c = srv.wait([rid])[rid]
            assert c.status == cf.CFOG_OK and c.batch_reqs == 1
            alone[i] = (c.out, c.surfaces)
        ids = [srv.submit(q["pair"], q["cps"], q["N"], q["r"], surfaces=q["surfaces"]) for q in reqs]
        got = srv.wait(ids)
        st = srv.stats()
    _say("server stats", st)
    mixed_batches = 0
    for i, rid in enumerate(ids):
        c = got[rid]
        assert c.status == cf.CFOG_OK
        assert c.t_submit <= c.t_admit <= c.t_launch <= c.t_done
        _same((c.out, c.surfaces), ref[i])
        if i in alone:
            _same((c.out, c.surfaces), alone[i])
            mixed_batches += c.batch_reqs > 1
    assert mixed_batches > 0, "no sampled request shared a batch in the mix"
    assert st["max_in_flight"] >= 2, "batches never overlapped"
    assert st["completed"] == st["submitted"] == 90 and st["evictions"] == 0 and st["extractions"] == 3
    # the FP64 oracle on the first points of a few requests
    stats = {}
    for i in range(0, 80, 10):
        q = reqs[i]
        A, B = pairs[q["pair"]]
        res = cf.results_np(ref[i][0])
        for k in range(min(2, len(q["cps"]))):
            if int(res["status"][k]) != 0:
                assert int(res["status"][k]) == cf.CP_OUT_OF_BOUNDS and tuple(q["cps"][k]) == (1, 1, 1, 1)
                continue
            S, E1, E2 = parity.oracle_point(A, B, q["cps"][k], q["N"], q["r"])
            sg = ref[i][1][k] if ref[i][1] is not None else None
            parity.check_point(k, res, S, E1, E2, q["r"], surf_gpu=sg, stats=stats)
    _say("oracle sample", stats)


def test_server_admission_under_small_budget_evicts_and_recomputes(cf):
    seed = 42
    pairs = _pairs(seed)
    imgs = _dev_pairs(pairs)
    reqs = _requests(seed, pairs, 60, surf_every=4)
    _say("server budget gate: probing fixed staging size")
    with cf.Server(1 << 30, n_slots=2, max_batch_cps=240, max_batch_reqs=4) as probe:
        fixed = (1 << 30) - probe.stats()["arena_bytes"]
    # the largest pair: 2 x (9 x 256^2 x 4 + 257^2 x 8) bytes + extraction scratch
    big = 2 * (9 * 256 * 256 * 4 + 257 * 257 * 8) + 64 * 1024
    budget = fixed + int(1.5 * big)
    _say("server budget gate: budget", budget, "fixed", fixed, "60 requests over 3 pairs, seed", seed)
    ref = _direct(cf, pairs, reqs, cf.PATH_BATCHED_FFT)
    with _server(cf, imgs, budget, n_slots=2, max_batch_cps=240, max_batch_reqs=4) as srv:
        ids = [srv.submit(q["pair"], q["cps"], q["N"], q["r"], surfaces=q["surfaces"]) for q in reqs]
        got = srv.wait(ids)
        st = srv.stats()
    _say("server stats", st)
    for i, rid in enumerate(ids):
        assert got[rid].status == cf.CFOG_OK
        _same((got[rid].out, got[rid].surfaces), ref[i])
    assert st["evictions"] > 0 and st["blocked"] > 0 and st["extractions"] > 3
    assert st["arena_peak"] <= st["arena_bytes"] < big * 2


def test_server_mfma_path_matches_direct(cf):
    seed = 43
    _say("server MFMA path: 3 pairs, 24 requests, seed", seed)
    pairs = _pairs(seed)
    imgs = _dev_pairs(pairs)
    reqs = _requests(seed, pairs, 24)
    ref = _direct(cf, pairs, reqs, cf.PATH_MFMA_BF16)
    with _server(cf, imgs, 1 << 30, n_slots=3, max_batch_reqs=5, flags=cf.PATH_MFMA_BF16) as srv:
        ids = [srv.submit(q["pair"], q["cps"], q["N"], q["r"], surfaces=q["surfaces"]) for q in reqs]
        got = srv.wait(ids)
    for i, rid in enumerate(ids):
        assert got[rid].status == cf.CFOG_OK
        _same((got[rid].out, got[rid].surfaces), ref[i])


def test_server_rejections(cf):
    _say("server rejections")
    A = torch.zeros((64, 64), device="cuda")
    with cf.Server(1 << 30, n_slots=1, max_batch_cps=16) as srv:
        pid = srv.add_pair(A, A)
        cps = np.array([[32, 32, 32, 32]], np.int32)
        with pytest.raises(cf.CfogError) as e:
            srv.submit(pid + 1, cps, 16, 2)
        assert e.value.code == cf.CFOG_EINVAL
        with pytest.raises(cf.CfogError) as e:
            srv.submit(pid, cps, 300, 2)
        assert e.value.code == cf.CFOG_EUNSUPPORTED
        with pytest.raises(cf.CfogError) as e:
            srv.submit(pid, np.repeat(cps, 17, 0), 16, 2)
        assert e.value.code == cf.CFOG_ENOMEM
        # a constant pair: every offset ties, the first one wins
        rid = srv.submit(pid, cps, 16, 2)
        c = srv.wait([rid])[rid]
        assert c.status == cf.CFOG_OK and tuple(c.out[0, :2]) == (-2, -2)
    with cf.Server(1 << 30, n_slots=1, max_batch_cps=16) as small:
        big = torch.zeros((8192, 8192), device="cuda")
        with pytest.raises(cf.CfogError) as e:
            small.add_pair(big, big)
        assert e.value.code == cf.CFOG_ENOMEM


def test_server_points_outside_never_reach_the_device(cf):
    """Points at int32 extremes and one pixel past an edge, mixed with valid
    points in one request, give the out-of-bounds result without disturbing
    the others (equal to a direct match_batch call, whose kernels apply the
    same rule); a request with no point inside completes at once."""
    seed = 44
    _say("server: out-of-bounds and extreme points, seed", seed)
    pairs = _pairs(seed)
    imgs = _dev_pairs(pairs)
    H, W = pairs[1][0].shape  # 200 x 232
    N, r = 21, 5
    h = N // 2
    I32_MIN, I32_MAX = -2 ** 31, 2 ** 31 - 1
    good = [(60, 70, 62, 68), (W - N + h, H - N + h, W - N - r + h, H - N - r + h), (h, h, h + r, h + r)]
    bad = [(I32_MIN, 70, 60, 70), (60, I32_MAX, 60, 70), (60, 70, I32_MAX - h, 70), (60, 70, 60, I32_MIN + 1),
           (W - N + h + 1, 70, 60, 70), (60, 70, 60, H - N - r + h + 1), (I32_MAX, I32_MAX, I32_MAX, I32_MAX)]
    mixed = np.array([bad[0], good[0], bad[1], bad[2], good[1], bad[3], bad[4], good[2], bad[5], bad[6]], np.int32)
    reqs = [dict(pair=1, cps=mixed, N=N, r=r, surfaces=True), dict(pair=1, cps=mixed, N=N, r=r, surfaces=False)]
    ref = _direct(cf, pairs, reqs, cf.PATH_BATCHED_FFT)
    res = cf.results_np(ref[0][0])
    assert [int(s) for s in res["status"]] == [1, 0, 1, 1, 0, 1, 1, 0, 1, 1]
    with _server(cf, imgs, 1 << 30, n_slots=2, max_batch_cps=64, max_batch_reqs=4) as srv:
        ids = [srv.submit(q["pair"], q["cps"], q["N"], q["r"], surfaces=q["surfaces"]) for q in reqs]
        none_inside = srv.submit(1, np.array(bad, np.int32), N, r, surfaces=True)
        got = srv.wait(ids + [none_inside])
        st = srv.stats()
    for i, rid in enumerate(ids):
        assert got[rid].status == cf.CFOG_OK
        _same((got[rid].out, got[rid].surfaces), ref[i])
    c = got[none_inside]
    assert c.status == cf.CFOG_OK and c.batch_reqs == 0
    assert np.all(c.out[:, 4] == cf.CP_OUT_OF_BOUNDS) and np.all(c.out[:, :2] == 0)
    assert np.all(np.isnan(cf.results_np(c.out)["best"])) and np.all(np.isnan(c.surfaces))
    assert st["completed"] == st["submitted"] == 3
    stats = {}
    A, B = pairs[1]
    for k in np.flatnonzero(res["status"] == 0):
        S, E1, E2 = parity.oracle_point(A, B, mixed[k], N, r)
        parity.check_point(int(k), res, S, E1, E2, r, surf_gpu=ref[0][1][k], stats=stats)
    _say("oracle", stats)
