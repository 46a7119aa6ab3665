"""Ragged image batches on the device against the FP64 reference, through the C ABI.

Windows of every image are projected on the device (rsc_project_images) and coded
(rsc_omp_encode); the reference extracts the same windows from the same FP32
pixels and codes them.  Also: device stamping, and capture of a whole batch in a
HIP graph replayed several times.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc
from paper_1806_04374_amd import workloads as wl
from tests.parity import compare_codes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04374_amd import rsc
    rsc.lib()
    return torch.device("cuda:0")


def _images(basis, D, draws):
    imgs = [orc.synthesize_image(basis, D, d.H, d.W, d.centre, d.atom, d.angle, d.amplitude, d.noise)
            for d in draws]
    return [im.astype(np.float32) for im in imgs]


def _pack(imgs, dev):
    flat = np.concatenate([im.ravel() for im in imgs]) if imgs else np.zeros(0, np.float32)
    return torch.from_numpy(flat).to(dev)


def _setup(geom, M, R):
    from paper_1806_04374_amd import rsc
    D = wl.draw_dictionary(M, geom.B, seed=0)
    h = rsc.rsc_create(geom.N, geom.S, geom.T)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), R)
    return D, h


@pytest.mark.parametrize("geom,M,R,K", [(wl.GEOM15, 128, 64, 6), (wl.GEOM11, 32, 32, 3)])
def test_small_ragged_batch(dev, geom, M, R, K):
    from paper_1806_04374_amd import rsc
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D, h = _setup(geom, M, R)
    sizes = [(40, 57), (geom.N, geom.N), (geom.N - 1, 30), (33, 90), (64, 19)]
    draws = [wl.draw_image(i, H, W, M, 0.02, 0.05, seed=4) for i, (H, W) in enumerate(sizes)]
    imgs = _images(basis, D, draws)
    batch = rsc.ImageBatch(sizes, geom.N, dev)
    xh = rsc.rsc_project_images(h, _pack(imgs, dev), batch)
    atom, angle, coef, r2 = rsc.rsc_omp_encode(h, xh, K)
    torch.cuda.synchronize()
    patches = np.concatenate([orc.image_patches(im.astype(np.float64), geom.N) for im in imgs])
    assert patches.shape[0] == batch.P_total
    xh_ref, code = orc.encode(basis, D, R, patches, K)
    err = np.abs(xh.cpu().numpy() - xh_ref).max(axis=1) / np.maximum(np.linalg.norm(xh_ref, axis=1), 1e-30)
    assert err.max() < 2e-5
    rep = compare_codes(atom.cpu().numpy(), angle.cpu().numpy(), coef.cpu().numpy(), code)
    print(f"ragged N={geom.N}", rep, flush=True)
    assert rep.match_rate >= 0.999 and rep.coef_bad == 0, str(rep)
    h.close()


def test_device_stamping_matches_reference(dev):
    from paper_1806_04374_amd import rsc
    geom = wl.GEOM15
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D, h = _setup(geom, 128, 64)
    sizes = [(70, 45), (20, 100), (15, 15)]
    draws = [wl.draw_image(i, H, W, 128, 0.02, 0.05, seed=6) for i, (H, W) in enumerate(sizes)]
    ref = _images(basis, D, draws)
    batch = rsc.ImageBatch(sizes, geom.N, dev)
    pix = _pack([d.noise.astype(np.float32) for d in draws], dev)
    cat = lambda f, dt: torch.from_numpy(np.concatenate([f(d) for d in draws]).astype(dt)).to(dev)
    rsc.rsc_synthesize_images(h, batch, cat(lambda d: d.atom, np.int32), cat(lambda d: d.angle, np.float32),
                              cat(lambda d: d.amplitude, np.float32),
                              cat(lambda d: d.centre.reshape(-1, 2), np.int32).reshape(-1, 2).contiguous(),
                              torch.from_numpy(np.concatenate([np.full(len(d.atom), i) for i, d in enumerate(draws)])
                                               .astype(np.int32)).to(dev), pix)
    torch.cuda.synchronize()
    got = pix.cpu().numpy()
    want = np.concatenate([r.ravel() for r in ref])
    assert np.abs(got - want).max() < 1e-5 * max(1.0, np.abs(want).max())
    h.close()


def test_batch_in_hip_graph(dev):
    """project_images + encode captured once, replayed with new pixels; every replay
    equals the eager result."""
    from paper_1806_04374_amd import rsc
    geom = wl.GEOM15
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D, h = _setup(geom, 128, 64)
    sizes = [(60, 80), (31, 47), (90, 20)]
    batch = rsc.ImageBatch(sizes, geom.N, dev)
    pix = torch.zeros(batch.total_pixels, dtype=torch.float32, device=dev)
    xh = torch.empty((batch.P_total, geom.B), dtype=torch.float32, device=dev)
    outs = (torch.empty((batch.P_total, 6), dtype=torch.int32, device=dev),
            torch.empty((batch.P_total, 6), dtype=torch.int32, device=dev),
            torch.empty((batch.P_total, 6), dtype=torch.float32, device=dev),
            torch.empty((batch.P_total,), dtype=torch.float32, device=dev))

    def run(stream=None):
        rsc.rsc_project_images(h, pix, batch, xhat=xh, stream=stream)
        rsc.rsc_omp_encode(h, xh, 6, out=outs, stream=stream)

    pix.copy_(_pack(_images(basis, D, [wl.draw_image(i, H, W, 128, 0.02, 0.05, seed=7)
                                       for i, (H, W) in enumerate(sizes)]), dev))
    run()          # warm-up launches outside the capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        run(stream=s)
    torch.cuda.synchronize()
    for seed in (8, 9, 10):
        imgs = _images(basis, D, [wl.draw_image(i, H, W, 128, 0.02, 0.05, seed=seed) for i, (H, W) in enumerate(sizes)])
        pix.copy_(_pack(imgs, dev))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        replay = [o.clone() for o in outs]
        run()
        torch.cuda.synchronize()
        for a, b in zip(replay, outs):
            assert torch.equal(a, b)
    h.close()


def test_full_ragged_batch_sampled(dev):
    """All windows of the 256-image batch in one projection + one encode launch;
    20,000 sampled windows checked against the reference."""
    from paper_1806_04374_amd import rsc
    w = wl.RAGGED
    geom = w["geom"]
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D, h = _setup(geom, w["M"], w["R"])
    draws = wl.ragged_draws()
    sizes = [(d.H, d.W) for d in draws]
    batch = rsc.ImageBatch(sizes, geom.N, dev)
    print("ragged batch", batch.n, "images", batch.P_total, "windows", flush=True)
    imgs = _images(basis, D, draws)
    xh = rsc.rsc_project_images(h, _pack(imgs, dev), batch)
    atom, angle, coef, _ = rsc.rsc_omp_encode(h, xh, w["K"])
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(batch.P_total, 20000, replace=False))
    starts = np.concatenate([[0], np.cumsum(batch.patches_per_image)])
    patches = []
    for p in idx:
        i = int(np.searchsorted(starts, p, side="right") - 1)
        wp = batch.W[i] - geom.N + 1
        y, x = divmod(int(p - starts[i]), int(wp))
        patches.append(imgs[i][y:y + geom.N, x:x + geom.N].astype(np.float64))
    _, code = orc.encode(basis, D, w["R"], np.stack(patches), w["K"])
    rep = compare_codes(atom.cpu().numpy()[idx], angle.cpu().numpy()[idx], coef.cpu().numpy()[idx], code)
    print("ragged-full-sampled", rep, flush=True)
    assert rep.match_rate >= 0.999 and rep.coef_bad == 0, str(rep)
    h.close()


@pytest.mark.parametrize("geom", [wl.GEOM15, wl.GEOM11])
@pytest.mark.parametrize("sizes", [[(15, 15)], [(16, 20)], [(15, 15), (17, 17)], [(40, 15)], [(15, 300)],
                                   [(20, 33)] * 9])
def test_small_batches_with_few_blocks(dev, geom, sizes):
    """Batches of a handful of tiles (launches of fewer than 8 blocks, where the tile ranges
    per XCD group shrink to one per block, and empty ranges): every window against the
    reference's projection."""
    from paper_1806_04374_amd import rsc
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    h = rsc.rsc_create(geom.N, geom.S, geom.T)
    rng = np.random.default_rng(len(sizes) + sizes[0][1])
    imgs = [rng.standard_normal(s).astype(np.float32) for s in sizes]
    batch = rsc.ImageBatch(sizes, geom.N, dev)
    xh = rsc.rsc_project_images(h, _pack(imgs, dev), batch)
    torch.cuda.synchronize()
    patches = np.concatenate([orc.image_patches(im.astype(np.float64), geom.N) for im in imgs])
    assert patches.shape[0] == batch.P_total
    ref = orc.project(basis, patches)
    assert np.abs(xh.cpu().numpy() - ref).max() < 2e-5 * np.abs(ref).max()
    h.close()
