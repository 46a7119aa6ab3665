"""Encode server on the device: every request's codes are bit-identical alone and in
the served mix (mixed sizes, admission under a small memory budget, many steps)."""
import numpy as np
import pytest

from oracle import rsc_oracle as orc
from paper_1806_04374_amd import workloads as wl
from tests.parity import compare_codes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04374_amd import rsc
    g = wl.GEOM15
    D = wl.draw_dictionary(128, g.B, seed=0)
    h = rsc.rsc_create(g.N, g.S, g.T)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), 64)
    yield g, D, h
    h.close()


def _image(basis, D, i, side):
    centre, atom, angle, amp = wl.request_stamps(i, side, side, 128, 0.02, seed=5)
    noise = 0.05 * np.random.default_rng(i).standard_normal((side, side))
    return orc.synthesize_image(basis, D, side, side, centre, atom, angle, amp, noise).astype(np.float32)


def test_served_codes_equal_alone(setup):
    from paper_1806_04374_amd import rsc, serve
    g, D, h = setup
    basis = orc.build_basis(g.N, g.S, g.T)
    rng = np.random.default_rng(11)
    sides = list(rng.integers(10, 130, 24)) + [14, 15, 16]
    reqs = [serve.Request(i, 0.0, _image(basis, D, i, int(s)), int(s), int(s)) for i, s in enumerate(sides)]
    be = serve.DeviceBackend(h, 6, budget_bytes=4 * 40_000, step_windows=3000)
    sch = serve.Scheduler(be, budget_elems=40_000, step_windows=3000)
    serve.replay(sch, reqs, realtime=False)
    assert len(sch.finished) == len(reqs) and not sch.rejected
    assert sch.steps > 5 and sch.max_active > 1
    dev = torch.device("cuda:0")
    for r in reqs:
        if r.windows == 0:
            continue
        batch = rsc.ImageBatch([(r.H, r.W)], g.N, dev)
        xh = rsc.rsc_project_images(h, torch.from_numpy(r.pixels.ravel()).to(dev), batch)
        atom, angle, coef, _ = rsc.rsc_omp_encode(h, xh, 6)
        torch.cuda.synchronize()
        assert np.array_equal(r.codes[0], atom.cpu().numpy()), r.rid
        assert np.array_equal(r.codes[1], angle.cpu().numpy()), r.rid
        assert np.array_equal(r.codes[2], coef.cpu().numpy()), r.rid
    # served requests against the FP64 reference, >= 20,000 windows
    _against_reference(basis, D, [r for r in reqs if r.windows])


def _against_reference(basis, D, reqs, need=20000):
    n = 0
    codes, refs = [[], [], []], []
    for r in reqs:
        wins = orc.image_patches(r.pixels.astype(np.float64), basis.N)
        _, code = orc.encode(basis, D, 64, wins, 6)
        refs.append(code)
        for i in range(3):
            codes[i].append(r.codes[i])
        n += len(wins)
        if n >= need:
            break
    assert n >= need, n
    cat = lambda f: np.concatenate([getattr(c, f) for c in refs])
    ref = orc.Code(cat("atom"), cat("angle"), cat("coef"), cat("resid2"), cat("corr"), cat("gap"))
    rep = compare_codes(*(np.concatenate(c) for c in codes), ref)
    print("served-vs-reference", rep, flush=True)
    assert rep.match_rate >= 0.999 and rep.coef_bad == 0, str(rep)


def test_one_at_a_time_baseline_matches(setup):
    from paper_1806_04374_amd import serve
    g, D, h = setup
    basis = orc.build_basis(g.N, g.S, g.T)
    reqs = [serve.Request(i, 0.0, _image(basis, D, 100 + i, s), s, s)
            for i, s in enumerate([20, 33, 15, 47, 120, 130])]
    serve.encode_one_at_a_time(h, 6, reqs, realtime=False)
    _against_reference(basis, D, reqs)


def test_served_codes_annular_basis():
    """The server on a handle of the paper's annular basis (N = 11, B = 81, K = 4): codes
    bit-identical alone and in the mix, and against the FP64 reference on every window."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04374_amd import rsc, serve
    ab = orc.build_annular_basis(11)
    h = rsc.rsc_create_annular(11)
    D = wl.draw_dictionary(32, ab.B, seed=3)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), 32)
    rng = np.random.default_rng(12)
    sides = [int(s) for s in rng.integers(10, 70, 12)] + [11, 12]
    reqs = []
    for i, s in enumerate(sides):
        img = rng.standard_normal((s, s))
        # a few stamps of rotated atoms in the annular basis' own steering
        for _ in range(max(1, s * s // 200)):
            m, th, a = int(rng.integers(0, 32)), float(rng.uniform(0, 2 * np.pi)), float(rng.normal())
            patch = orc.to_pixels(ab, a * orc.steer_ragged(D[m], th, ab.Sk)).reshape(11, 11)
            if s >= 11:
                y, x = int(rng.integers(0, s - 10)), int(rng.integers(0, s - 10))
                img[y:y + 11, x:x + 11] += 3.0 * patch
        reqs.append(serve.Request(i, 0.0, img.astype(np.float32), s, s))
    be = serve.DeviceBackend(h, 4, budget_bytes=4 * 12_000, step_windows=1500)
    sch = serve.Scheduler(be, budget_elems=12_000, step_windows=1500)
    serve.replay(sch, reqs, realtime=False)
    assert len(sch.finished) == len(reqs) and not sch.rejected
    assert sch.steps > 3 and sch.max_active > 1
    dev = torch.device("cuda:0")
    codes, refs = [[], [], []], []
    for r in reqs:
        if r.windows == 0:
            continue
        batch = rsc.ImageBatch([(r.H, r.W)], 11, dev)
        xh = rsc.rsc_project_images(h, torch.from_numpy(r.pixels.ravel()).to(dev), batch)
        atom, angle, coef, _ = rsc.rsc_omp_encode(h, xh, 4)
        torch.cuda.synchronize()
        assert np.array_equal(r.codes[0], atom.cpu().numpy()), r.rid
        assert np.array_equal(r.codes[1], angle.cpu().numpy()), r.rid
        assert np.array_equal(r.codes[2], coef.cpu().numpy()), r.rid
        _, code = orc.encode(ab, D, 32, orc.image_patches(r.pixels.astype(np.float64), 11), 4)
        refs.append(code)
        for i in range(3):
            codes[i].append(r.codes[i])
    cat = lambda f: np.concatenate([getattr(c, f) for c in refs])
    ref = orc.Code(cat("atom"), cat("angle"), cat("coef"), cat("resid2"), cat("corr"), cat("gap"))
    rep = compare_codes(*(np.concatenate(c) for c in codes), ref)
    print("served annular vs reference", rep, flush=True)
    assert rep.n > 10_000 and rep.match_rate >= 0.999 and rep.coef_bad == 0, str(rep)
    h.close()
