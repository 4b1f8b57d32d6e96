"""GPU tests of the pixel-wise HOG descriptor (Section III-C, FHOG built at
every pixel) against the FP64 oracle, and of matching on its 36-channel
volumes.

Parity rule for the volume: every value within 1e-5 of the oracle's (the
values are normalised, at most 1; all terms of the cell sums are
non-negative, so FP32 rounding of the ~2 (2 cell + 1) products and of the bin
position from atan2f stays near 1e-6 relative).  The SAT of the channel
energies and the matching surfaces follow the CFOG rules.

Every case prints its name, sizes and seed before touching the GPU."""
import numpy as np
import pytest

import oracle as O
from tests import parity
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _image(H, W, seed):
    A, _, _ = synth.make_pair(synth.PairSpec(H, W, max(4, H * W // 1500), (3.0, 15.0), max(2, H * W // 3000), 4),
                              (seed, 0))
    return A


@pytest.mark.parametrize("H,W,cell,seed", [(96, 130, 4, 101), (64, 64, 1, 102), (300, 257, 3, 103),
                                           (17, 65, 8, 104), (5, 3, 2, 105), (200, 190, 6, 106)])
def test_fhog_volume_and_sat_match_oracle(cf, H, W, cell, seed):
    _say(f"fhog {H}x{W} cell={cell} seed={seed}")
    A = _image(H, W, seed)
    vol, sat = cf.fhog_extract(_dev(A), cell=cell)
    torch.cuda.synchronize()
    D = O.fhog(A.astype(np.float64), c=cell)
    v = vol.cpu().numpy()
    err = float(np.max(np.abs(v.astype(np.float64) - D)))
    _say("max abs error", err)
    assert err <= 1e-5
    Q = np.sum(v.astype(np.float64) ** 2, axis=0)
    np.testing.assert_allclose(sat.cpu().numpy(), O.sat(Q), rtol=1e-12, atol=1e-9 * max(O.sat(Q)[-1, -1], 1.0))


def test_fhog_strided_image_and_no_sat(cf):
    _say("fhog 80x100 view of a 80x128 buffer, cell 4, no SAT, seed 107")
    A = _image(80, 128, 107)
    full = _dev(A)
    view = full[:, 10:110]
    vol, sat = cf.fhog_extract(view, cell=4, with_sat=False)
    torch.cuda.synchronize()
    assert sat is None
    D = O.fhog(np.ascontiguousarray(A[:, 10:110]).astype(np.float64), c=4)
    assert float(np.max(np.abs(vol.cpu().numpy().astype(np.float64) - D))) <= 1e-5


def test_fhog_flat_image_is_zero(cf):
    _say("fhog flat 40x70 cell 4")
    vol, sat = cf.fhog_extract(torch.full((40, 70), 2.5, device="cuda"), cell=4)
    torch.cuda.synchronize()
    assert torch.count_nonzero(vol).item() == 0
    assert torch.count_nonzero(sat).item() == 0


def test_fhog_rejects_bad_arguments(cf):
    _say("fhog argument checks")
    img = torch.zeros((40, 40), device="cuda")
    with pytest.raises(cf.CfogError) as e:
        cf.fhog_extract(img, cell=9)
    assert e.value.code == cf.CFOG_EUNSUPPORTED
    with pytest.raises(cf.CfogError) as e:
        cf.fhog_extract(img, cell=0)
    assert e.value.code == cf.CFOG_EINVAL


@pytest.mark.parametrize("path", ["plain", "batched", "mfma"])
def test_match_on_fhog_volumes(cf, path):
    """The matcher on 36-channel pixel-wise HOG volumes of a 256^2 pair (cell
    4), 16 CPs, template 48, radius 10, against the oracle on its own
    volumes."""
    spec = synth.PairSpec(256, 256, 40, (3.0, 15.0), 20, 8)
    A, B, _ = synth.make_pair(spec, (108, 0))
    cps = synth.grid_cps(256, 256, 48, 10, 4)
    N, r = 48, 10
    _say(f"match on fhog volumes, path {path}, 256^2, 16 CPs, template {N}, radius {r}, seed 108")
    vA, sA = cf.fhog_extract(_dev(A))
    vB, sB = cf.fhog_extract(_dev(B))
    K = 2 * r + 1
    surf = torch.empty((len(cps), K, K), device="cuda")
    job = cf.Job(vA, sA, vB, sB, torch.from_numpy(np.asarray(cps, np.int32)).cuda(), N, r, surfaces=surf)
    flags = {"plain": cf.PATH_PLAIN_FFT, "batched": cf.PATH_BATCHED_FFT, "mfma": cf.PATH_MFMA_BF16}[path]
    cf.match_batch([job], m=cf.FHOG_CHANNELS, flags=flags)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in cf.results(job.out).items()}
    D1, D2 = O.fhog(A.astype(np.float64)), O.fhog(B.astype(np.float64))
    ora = O.match(D1, D2, cps, N, r, surfaces=True)
    tol = parity.bf16_tol(N, r, m=cf.FHOG_CHANNELS) if path == "mfma" else parity.SURF_TOL
    stats = {}
    for k, cp in enumerate(cps):
        E1, E2 = O.energies(D1, D2, cp, N, r)
        parity.check_point(k, res, ora["surfaces"][k], E1, E2, r, surf_gpu=surf[k].cpu().numpy(), stats=stats,
                           tol=tol)
    _say("fhog match parity", stats)
