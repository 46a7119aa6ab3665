"""Texture classifier on the device (rsc_classify, rsc_label_histogram, rsc_chi2_nearest)
against the FP64 reference, through the C ABI.

Acceptance: labels equal the reference's wherever the reference's two best classes are
separated by more than 1e-3 relative (FP32 pursuits may resolve closer calls either
way) and on >= 99% of all patches; the winning error within 1e-4 relative (plus 1e-6
of the patch energy); histograms of the same labels exactly equal (integer counts,
one rounding); nearest neighbours equal, distances within 1e-6 relative.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc
from paper_1806_04374_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04374_amd import rsc
    rsc.lib()
    return torch.device("cuda:0")


def _handles(geom, D_list, R, precs=None):
    from paper_1806_04374_amd import rsc
    hs = []
    for c, D in enumerate(D_list):
        h = rsc.rsc_create(geom.N, geom.S, geom.T, prec=(precs[c] if precs else "fp32"))
        rsc.rsc_set_dictionary(h, np.asarray(D, np.float32), R)
        hs.append(h)
    return hs


def _check_labels(label, sse, ref_label, ref_sse, X):
    P = len(ref_label)
    srt = np.sort(ref_sse, axis=1)
    margin = (srt[:, 1] - srt[:, 0]) / np.maximum(srt[:, 1], 1e-30) if ref_sse.shape[1] > 1 else np.ones(P)
    clear = margin > 1e-3
    assert np.array_equal(label[clear], ref_label[clear]), np.flatnonzero(label[clear] != ref_label[clear])[:10]
    assert np.mean(label == ref_label) >= 0.99
    same = label == ref_label
    energy = np.sum(X * X, 1)
    err = np.abs(sse[same] - ref_sse[np.arange(P), ref_label][same])
    assert np.all(err <= 1e-4 * ref_sse[np.arange(P), ref_label][same] + 1e-6 * energy[same])


@pytest.mark.parametrize("geom,C,M,R,K,P", [(wl.GEOM11, 4, 8, 16, 3, 777), (wl.GEOM15, 3, 12, 32, 1, 515)])
def test_labels_match_reference(dev, geom, C, M, R, K, P):
    from paper_1806_04374_amd import rsc
    D_list = [wl.draw_dictionary(M, geom.B, seed=50 + c).astype(np.float32).astype(np.float64) for c in range(C)]
    # patches drawn from the union of the class dictionaries, so several classes compete
    D_all = np.concatenate(D_list)
    d = wl.draw_mixtures(P, geom.N, C * M, 2, 0.05, seed=51)
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    X = orc.project(basis, orc.synthesize(basis, D_all, d.atom, d.angle, d.weight, d.noise).astype(np.float32))
    X = X.astype(np.float32).astype(np.float64)
    ref_label, ref_sse = orc.classify(D_list, R, geom.S, geom.T, X, K)
    hs = _handles(geom, D_list, R)
    label, sse = rsc.rsc_classify(hs, torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev), K)
    torch.cuda.synchronize()
    _check_labels(label.cpu().numpy(), sse.cpu().numpy().astype(np.float64), ref_label, ref_sse, X)
    for h in hs:
        h.close()


def test_separable_classes_exact_on_device(dev):
    """Classes in disjoint harmonics: every patch is coded exactly by its own class only."""
    from paper_1806_04374_amd import rsc
    from tests.test_oracle_classify import _separable
    D_list, R, X, truth = _separable(300, 7)
    hs = _handles(wl.GEOM11, D_list, R)
    label, sse = rsc.rsc_classify(hs, torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev), 2)
    torch.cuda.synchronize()
    assert np.array_equal(label.cpu().numpy(), truth)
    assert np.all(sse.cpu().numpy() < 1e-8 * np.sum(X * X, 1))
    for h in hs:
        h.close()


def test_rot90_leaves_labels_unchanged(dev):
    """Pixel patches turned by 90 degrees (exact on the grid) keep their labels and errors."""
    from paper_1806_04374_amd import rsc
    g = wl.GEOM11
    C, M, R, K = 3, 6, 32, 2
    D_list = [wl.draw_dictionary(M, g.B, seed=60 + c) for c in range(C)]
    hs = _handles(g, D_list, R)
    basis = orc.build_basis(g.N, g.S, g.T)
    d = wl.draw_mixtures(400, g.N, C * M, 2, 0.02, seed=61)
    pix = orc.synthesize(basis, np.concatenate(D_list), d.atom, d.angle, d.weight, d.noise).astype(np.float32)
    out = []
    for img in (pix, np.ascontiguousarray(np.rot90(pix, 1, axes=(1, 2)))):
        xh = rsc.rsc_project(hs[0], torch.from_numpy(img).to(dev))
        label, sse = rsc.rsc_classify(hs, xh, K)
        out.append((label.cpu().numpy(), sse.cpu().numpy()))
    (l0, s0), (l1, s1) = out
    assert np.mean(l0 == l1) >= 0.995
    same = l0 == l1
    assert np.allclose(s0[same], s1[same], rtol=1e-3, atol=1e-6)
    for h in hs:
        h.close()


def test_mixed_precision_classes(dev):
    """Class handles of different precisions (FP32, BF16, FP16) classify together."""
    from paper_1806_04374_amd import rsc
    g = wl.GEOM11
    D_list = [wl.draw_dictionary(8, g.B, seed=70 + c).astype(np.float32).astype(np.float64) for c in range(3)]
    d = wl.draw_mixtures(300, g.N, 24, 2, 0.05, seed=71)
    basis = orc.build_basis(g.N, g.S, g.T)
    X = orc.project(basis, orc.synthesize(basis, np.concatenate(D_list), d.atom, d.angle, d.weight,
                                          d.noise).astype(np.float32)).astype(np.float32).astype(np.float64)
    ref_label, ref_sse = orc.classify(D_list, 32, g.S, g.T, X, 2)
    hs = _handles(g, D_list, 32, precs=["fp32", "bf16", "fp16"])
    label, sse = rsc.rsc_classify(hs, torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev), 2)
    torch.cuda.synchronize()
    _check_labels(label.cpu().numpy(), sse.cpu().numpy().astype(np.float64), ref_label, ref_sse, X)
    for h in hs:
        h.close()


def test_histograms_exact(dev):
    from paper_1806_04374_amd import rsc
    rng = np.random.default_rng(80)
    C = 24
    sizes = [0, 1, 5, 999, 70000, 3, 0, 4096]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    label = rng.integers(0, C, offsets[-1]).astype(np.int32)
    label[rng.random(offsets[-1]) < 0.01] = C + 3          # out-of-range labels are not counted
    ref = orc.label_histogram(np.where(label < C, label, C), offsets, C + 1)[:, :C]
    hist = rsc.rsc_label_histogram(torch.from_numpy(label).to(dev), torch.from_numpy(offsets).to(dev), C)
    torch.cuda.synchronize()
    assert np.array_equal(hist.cpu().numpy(), ref.astype(np.float32))


def test_chi2_nearest_matches_reference(dev):
    from paper_1806_04374_amd import rsc
    rng = np.random.default_rng(81)
    C = 24
    for n_train, n_test in ((1, 3), (480, 700), (1000, 5)):
        train = rng.dirichlet(np.ones(C), n_train).astype(np.float32)
        test = rng.dirichlet(np.ones(C), n_test).astype(np.float32)
        train[:, 5] = 0.0                                     # empty bins on both sides
        test[:, 5] = 0.0
        if n_train > 10:
            train[7] = train[3]                               # a tie: the smaller index wins
            test[0] = train[3]
        ref_idx, ref_d = orc.nearest_chi2(train.astype(np.float64), test.astype(np.float64))
        idx, dist = rsc.rsc_chi2_nearest(torch.from_numpy(train).to(dev), torch.from_numpy(test).to(dev))
        torch.cuda.synchronize()
        assert np.array_equal(idx.cpu().numpy(), ref_idx)
        assert np.allclose(dist.cpu().numpy(), ref_d, rtol=1e-6, atol=1e-12)


def test_classifier_argument_errors(dev):
    from paper_1806_04374_amd import rsc
    g = wl.GEOM11
    h0 = rsc.rsc_create(g.N, g.S, g.T)
    rsc.rsc_set_dictionary(h0, wl.draw_dictionary(4, g.B).astype(np.float32), 8)
    h1 = rsc.rsc_create(g.N, g.S, g.T)                      # no dictionary
    h2 = rsc.rsc_create(15, 7, 7)
    rsc.rsc_set_dictionary(h2, wl.draw_dictionary(4, 105).astype(np.float32), 8)
    x = torch.zeros((10, g.B), dtype=torch.float32, device=dev)
    with pytest.raises(rsc.RscError) as e:
        rsc.rsc_classify([h0, h1], x, 1)
    assert e.value.status == rsc.RSC_E_NOT_READY
    with pytest.raises(rsc.RscError, match="geometry"):
        rsc.rsc_classify([h0, h2], x, 1)
    with pytest.raises(rsc.RscError, match="K must"):
        rsc.rsc_classify([h0], x, 9)
    with pytest.raises(rsc.RscError, match="n_train"):
        rsc.rsc_chi2_nearest(torch.zeros((0, 4), dtype=torch.float32, device=dev),
                             torch.zeros((2, 4), dtype=torch.float32, device=dev))
    for h in (h0, h1, h2):
        h.close()


def test_texture_pipeline_against_reference(dev):
    """Small band-pass texture set (4 classes, 40x40 images, test images turned by 45
    degrees): dictionaries learned by the reference (R-K-SVD, M = 12, K = 1, R = 32) are
    loaded on the device; the device's window labels, histograms and nearest neighbours
    match the reference pipeline's.  The device's own learning loop then classifies the
    test images as well as the reference does."""
    from paper_1806_04374_amd import rsc
    from paper_1806_04374_amd import texture as tx
    g = wl.GEOM15
    cfg = dict(wl.TEXTURE, C=4, freqs=(0.06, 0.2), anisotropy=0.9, bands=(0.02, 0.05))
    C, side, M, K, R = 4, 40, 12, 1, 32
    basis = orc.build_basis(g.N, g.S, g.T)
    tr = [wl.draw_texture_image(c, i, side, 0.05, 0.0, w=cfg) for c in range(C) for i in range(2)]
    te = [wl.draw_texture_image(c, 10 + i, side, 0.05, np.deg2rad(45), w=cfg) for c in range(C) for i in range(2)]
    Xtr = [orc.project(basis, orc.image_patches(im.astype(np.float32).astype(np.float64), g.N)) for im in tr]
    Xte = [orc.project(basis, orc.image_patches(im.astype(np.float32).astype(np.float64), g.N)) for im in te]
    rng = np.random.default_rng(3)
    D_ref = []
    for c in range(C):
        X = np.concatenate(Xtr[2 * c:2 * c + 2])
        X = X[rng.choice(len(X), 800, replace=False)]
        D0 = X[rng.choice(len(X), M, replace=False)]
        D, _, _ = orc.rksvd(D0 / np.linalg.norm(D0, axis=1, keepdims=True), R, g.S, g.T, X, K, 4)
        D_ref.append(D.astype(np.float32).astype(np.float64))
    off = lambda Xs: np.concatenate([[0], np.cumsum([len(x) for x in Xs])])
    lab_tr, _ = orc.classify(D_ref, R, g.S, g.T, np.concatenate(Xtr), K)
    lab_te, sse_te = orc.classify(D_ref, R, g.S, g.T, np.concatenate(Xte), K)
    H_tr = orc.label_histogram(lab_tr, off(Xtr), C)
    H_te = orc.label_histogram(lab_te, off(Xte), C)
    ref_nn, _ = orc.nearest_chi2(H_tr, H_te)
    # device, reference dictionaries
    hs = _handles(g, D_ref, R)
    proj = rsc.rsc_create(g.N, g.S, g.T)
    feats = []
    for ims in (tr, te):
        b, pix = tx.upload_batch(ims, g.N, dev)
        xh = rsc.rsc_project_images(proj, pix, b)
        label, _ = rsc.rsc_classify(hs, xh, K)
        feats.append((label, rsc.rsc_label_histogram(label, tx.window_offsets(b, dev), C), xh))
    nn, _ = rsc.rsc_chi2_nearest(feats[0][1], feats[1][1])
    torch.cuda.synchronize()
    lab_dev = feats[1][0].cpu().numpy()
    assert np.mean(lab_dev == lab_te) >= 0.99
    assert np.abs(feats[1][1].cpu().numpy() - H_te).sum(1).max() < 0.02
    assert np.array_equal(nn.cpu().numpy(), ref_nn)
    ref_acc = np.mean(np.repeat(np.arange(C), 2)[ref_nn] == np.repeat(np.arange(C), 2))
    # device learning from the same windows
    clf = tx.TextureClassifier(g.N, g.S, g.T, R, K)
    xtr = feats[0][2]
    per = (side - g.N + 1) ** 2
    wins = [xtr[2 * c * per:(2 * c + 2) * per] for c in range(C)]
    clf.learn([w.contiguous() for w in wins], M, 4)
    b, pix = tx.upload_batch(tr, g.N, dev)
    clf.fit(clf.features(rsc.rsc_project_images(proj, pix, b), tx.window_offsets(b, dev)), np.repeat(np.arange(C), 2))
    b, pix = tx.upload_batch(te, g.N, dev)
    nn_dev, _ = clf.predict(clf.features(rsc.rsc_project_images(proj, pix, b), tx.window_offsets(b, dev)))
    dev_acc = np.mean(clf.train_class[nn_dev.cpu().numpy()] == np.repeat(np.arange(C), 2))
    print("accuracy reference", ref_acc, "device-learned", dev_acc)
    assert dev_acc >= ref_acc - 0.125
    clf.close()
    proj.close()
    for h in hs:
        h.close()


def test_labels_match_reference_annular(dev):
    """Classes on the paper's annular basis (N = 11, B = 81): labels and errors against the
    reference's per-class pursuits in that basis; a grid handle among annular ones is refused."""
    from paper_1806_04374_amd import rsc
    ab = orc.build_annular_basis(11)
    C, M, R, K, P = 3, 8, 16, 2, 600
    D_list = [wl.draw_dictionary(M, ab.B, seed=70 + c).astype(np.float32).astype(np.float64) for c in range(C)]
    d = wl.draw_mixtures(P, 11, C * M, 2, 0.05, seed=71)
    X = orc.project(ab, orc.synthesize(ab, np.concatenate(D_list), d.atom, d.angle, d.weight,
                                       d.noise).astype(np.float32))
    X = X.astype(np.float32).astype(np.float64)
    ref_sse = np.stack([orc.omp(orc.augmented_dictionary_basis(ab, D, R), X, K, M).resid2 for D in D_list], 1)
    ref_label = np.argmin(ref_sse, axis=1)
    hs = []
    for D in D_list:
        h = rsc.rsc_create_annular(11)
        rsc.rsc_set_dictionary(h, np.asarray(D, np.float32), R)
        hs.append(h)
    xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    label, sse = rsc.rsc_classify(hs, xd, K)
    torch.cuda.synchronize()
    _check_labels(label.cpu().numpy(), sse.cpu().numpy().astype(np.float64), ref_label, ref_sse, X)
    g = rsc.rsc_create(11, 5, 5)
    rsc.rsc_set_dictionary(g, wl.draw_dictionary(M, g.B, seed=1).astype(np.float32), R)
    with pytest.raises(rsc.RscError) as e:
        rsc.rsc_classify([hs[0], g], xd, K)
    assert e.value.status == rsc.RSC_E_INVALID
    g.close()
    for h in hs:
        h.close()
