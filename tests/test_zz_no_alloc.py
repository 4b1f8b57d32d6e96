"""GPU test of match_batch_noalloc, the matching entry point that allocates
nothing (its workspace is the library's static device array): on two calls
in a row, the second with a smaller input, its results equal match_batch's on
the same inputs bit for bit (plain FFT path with channel splits, a plain
call at the largest FFT size, and the MFMA path), and a sample of points
agrees with the FP64 oracle.  Every case
prints its name before touching the GPU."""
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


def _case(cf, side, N, r, n, seed):
    spec = synth.PairSpec(side, side, max(8, side * side // 2000), (3.0, 15.0), max(4, side // 16), 6)
    A, B, _ = synth.make_pair(spec, (900, seed))
    cps = synth.random_cps(np.random.default_rng(seed), side, side, N, r, n)
    vA, sA = cf.cfog_extract(torch.from_numpy(A).cuda())
    vB, sB = cf.cfog_extract(torch.from_numpy(B).cuda())
    return A, B, cps, (vA, sA, vB, sB, torch.from_numpy(cps).cuda())


def _job(cf, vols, N, r):
    vA, sA, vB, sB, c = vols
    K = 2 * r + 1
    return cf.Job(vA, sA, vB, sB, c, N, r, out=torch.empty((len(c), 6), dtype=torch.int32, device="cuda"),
                  surfaces=torch.empty((len(c), K, K), device="cuda"))


def test_noalloc_equals_match_batch_on_two_calls(cf):
    assert cf.load().cfog_noalloc_scratch_bytes() == 48 << 20
    # first call: 300 points, N = 100, r = 20 (P = 144, split last round);
    # second call, smaller: 24 points, N = 48, r = 10 (P = 72); then a call
    # with N = 128, r = 32 (P = 192, the largest FFT size) and
    # one on the MFMA path
    cases = [("plain", 512, 100, 20, 300, 1, cf.PATH_PLAIN_FFT), ("plain", 256, 48, 10, 24, 2, cf.PATH_PLAIN_FFT),
             ("plain", 320, 128, 32, 40, 3, cf.PATH_PLAIN_FFT), ("mfma", 256, 48, 10, 16, 4, cf.PATH_MFMA_BF16)]
    for name, side, N, r, n, seed, flags in cases:
        _say(f"noalloc vs match_batch: {name}, {side}^2, N={N}, r={r}, {n} points, seed {seed}")
        A, B, cps, vols = _case(cf, side, N, r, n, seed)
        ref = _job(cf, vols, N, r)
        cf.match_batch([ref], flags=flags)
        torch.cuda.synchronize()
        got = _job(cf, vols, N, r)
        got.out.fill_(-7)
        got.surfaces.fill_(float("nan"))
        torch.cuda.synchronize()
        cf.match_batch_noalloc([got], flags=flags)
        torch.cuda.synchronize()
        assert torch.equal(got.out, ref.out), name
        assert torch.equal(got.surfaces.view(torch.int32), ref.surfaces.view(torch.int32)), name
        res = {k: v.cpu().numpy() for k, v in cf.results(got.out).items()}
        assert np.all(res["status"] == 0)
        surf = got.surfaces.cpu().numpy()
        tol = parity.bf16_tol(N, r) if flags == cf.PATH_MFMA_BF16 else parity.SURF_TOL
        stats = {}
        for k in range(0, n, max(1, n // 3)):
            S, E1, E2 = parity.oracle_point(A, B, cps[k], N, r)
            parity.check_point(k, res, S, E1, E2, r, surf[k], stats, tol=tol)
        _say("oracle sample", stats)


def test_noalloc_refuses_paths_that_stage_or_time(cf):
    _say("noalloc: refused flags")
    A, B, cps, vols = _case(cf, 128, 16, 4, 3, 5)
    job = _job(cf, vols, 16, 4)
    for flags in (cf.PATH_BATCHED_FFT, cf.PATH_PLAIN_FFT | cf.AUTOTUNE, cf.PATH_PLAIN_FFT | cf.USE_GRAPH):
        with pytest.raises(cf.CfogError) as e:
            cf.match_batch_noalloc([job], flags=flags)
        assert e.value.code == cf.CFOG_EINVAL
