"""R-K-SVD dictionary update and learning loop on the device against the FP64 reference.

The update is checked on identical inputs: the reference's codes (rounded to FP32,
as the device stores them) go to both sides.  Acceptance: usage counts and reset
patches equal exactly; for every atom whose top eigenvalue is separated from the
next by more than 1e-3 relative, the new atom agrees elementwise within 1e-5 (an
atom with a near-degenerate top eigenvalue has no well-defined first singular
vector, and is compared only through its Rayleigh quotient).
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


def _fp32_code(code):
    return orc.Code(code.atom, code.angle, code.coef.astype(np.float32).astype(np.float64),
                    code.resid2.astype(np.float32).astype(np.float64), code.corr, code.gap)


def _covariances(D, R, S, T, X, code):
    """Per-atom sum of y y^T through the residual identity (independent of the update's code path)."""
    M, B = D.shape
    recon = orc.code_to_hat(D, R, S, T, code)
    C = np.zeros((M, B, B))
    for p in range(X.shape[0]):
        seen = set()
        for i in range(code.atom.shape[1]):
            m = int(code.atom[p, i])
            if m < 0 or m in seen:
                continue
            seen.add(m)
            y = orc.steer(X[p] - recon[p], -2 * np.pi * code.angle[p, i] / R, S, T) + code.coef[p, i] * D[m]
            C[m] += np.outer(y, y)
    return C


def _check_update(geom, D, R, K, X, dev, tol=1e-5, repeat=False):
    from paper_1806_04374_amd import rsc
    S, T = geom.S, geom.T
    code = _fp32_code(orc.omp(orc.augmented_dictionary(D, R, S, T), X, K, D.shape[0]))
    ref, usage_ref, reset_ref = orc.rksvd_update(D, R, S, T, X, code)
    h = rsc.rsc_create(geom.N, S, T)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), R)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to(dev)
    args = (t(X, np.float32), t(code.atom, np.int32), t(code.angle, np.int32), t(code.coef, np.float32),
            t(code.resid2, np.float32))
    d_new, usage, reset = rsc.rsc_rksvd_update(h, *args)
    if repeat:   # every sum runs in a fixed order: a second call gives the same bits
        again = rsc.rsc_rksvd_update(h, *args)[0]
        assert torch.equal(again.view(torch.int32), d_new.view(torch.int32))
    torch.cuda.synchronize()
    d_new, usage, reset = d_new.cpu().numpy().astype(np.float64), usage.cpu().numpy(), reset.cpu().numpy()
    assert np.array_equal(usage, usage_ref), (usage, usage_ref)
    assert np.array_equal(reset, reset_ref), (reset, reset_ref)
    C = _covariances(D, R, S, T, X, code)
    worst = 0.0
    for m in range(D.shape[0]):
        assert abs(np.linalg.norm(d_new[m]) - 1) < 1e-6
        if usage_ref[m] == 0:
            assert np.abs(d_new[m] - ref[m]).max() < 1e-6
            continue
        ev = np.linalg.eigvalsh(C[m])
        q = d_new[m] @ C[m] @ d_new[m]
        assert q >= ev[-1] * (1 - 1e-6), (m, q, ev[-1])      # a top eigenvector either way
        if ev[-1] - ev[-2] > 1e-3 * ev[-1]:
            err = np.abs(d_new[m] - ref[m]).max()
            worst = max(worst, err)
            assert err < tol, (m, err, (ev[-1] - ev[-2]) / ev[-1])
    h.close()
    return worst


def test_update_matches_reference_11x11(dev):
    g = wl.GEOM11
    M, R, K = 16, 32, 3
    D = wl.draw_dictionary(M, g.B, seed=21).astype(np.float32).astype(np.float64)
    basis = orc.build_basis(g.N, g.S, g.T)
    d = wl.draw_mixtures(3000, g.N, M, 3, 0.05, seed=21)
    X = orc.project(basis, orc.synthesize(basis, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32))
    X = X.astype(np.float32).astype(np.float64)
    # a perturbed dictionary, so that the update has work to do
    Dp = D + 0.2 * np.random.default_rng(22).standard_normal(D.shape)
    Dp = (Dp / np.linalg.norm(Dp, axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    print("worst atom difference", _check_update(g, Dp, R, K, X, dev))


def test_update_matches_reference_15x15(dev):
    g = wl.GEOM15
    M, R, K = 24, 64, 4
    D = wl.draw_dictionary(M, g.B, seed=23).astype(np.float32).astype(np.float64)
    basis = orc.build_basis(g.N, g.S, g.T)
    d = wl.draw_mixtures(1500, g.N, M, 3, 0.05, seed=23)
    X = orc.project(basis, orc.synthesize(basis, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32))
    X = X.astype(np.float32).astype(np.float64)
    Dp = D + 0.2 * np.random.default_rng(24).standard_normal(D.shape)
    Dp = (Dp / np.linalg.norm(Dp, axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    print("worst atom difference", _check_update(g, Dp, R, K, X, dev))


def test_update_with_more_than_four_slots(dev):
    """K = 6 takes the eight-slot kernel."""
    g = wl.GEOM11
    M, R, K = 12, 16, 6
    D = wl.draw_dictionary(M, g.B, seed=26).astype(np.float32).astype(np.float64)
    basis = orc.build_basis(g.N, g.S, g.T)
    d = wl.draw_mixtures(1500, g.N, M, 5, 0.05, seed=26)
    X = orc.project(basis, orc.synthesize(basis, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32))
    X = X.astype(np.float32).astype(np.float64)
    Dp = D + 0.2 * np.random.default_rng(27).standard_normal(D.shape)
    Dp = (Dp / np.linalg.norm(Dp, axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    print("worst atom difference", _check_update(g, Dp, R, K, X, dev))


def test_update_largest_dictionary(dev):
    """M = 256 atoms at B = 105: the residual kernel's dictionary no longer fits in LDS as
    pairs and takes the single-value layout."""
    g = wl.GEOM15
    M, R, K = 256, 32, 2
    D = wl.draw_dictionary(M, g.B, seed=28).astype(np.float32).astype(np.float64)
    basis = orc.build_basis(g.N, g.S, g.T)
    d = wl.draw_mixtures(1500, g.N, M, 2, 0.05, seed=28)
    X = orc.project(basis, orc.synthesize(basis, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32))
    X = X.astype(np.float32).astype(np.float64)
    Dp = D + 0.2 * np.random.default_rng(29).standard_normal(D.shape)
    Dp = (Dp / np.linalg.norm(Dp, axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    print("worst atom difference", _check_update(g, Dp, R, K, X, dev))


def test_update_over_many_chunks_matches_reference(dev):
    """Scale geometry (M=64, R=64, K=4) on 12,000 patches: about 750 pairs per atom,
    so every bucket spans several 256-pair chunks and the chunk partials are summed;
    a repeated call is bit-identical."""
    w = wl.SCALE
    g = w["geom"]
    basis = orc.build_basis(g.N, g.S, g.T)
    D, d = wl.scale_draw(P=12000)
    X = orc.project(basis, orc.synthesize(basis, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32))
    X = X.astype(np.float32).astype(np.float64)
    Dp = D + 0.1 * np.random.default_rng(25).standard_normal(D.shape)
    Dp = (Dp / np.linalg.norm(Dp, axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    print("worst atom difference", _check_update(g, Dp, w["R"], w["K"], X, dev, repeat=True))


@pytest.mark.parametrize("geom,M,R,K,P", [(wl.GEOM11, 16, 32, 2, 1), (wl.GEOM11, 16, 32, 2, 2),
                                          (wl.GEOM11, 16, 32, 2, 5), (wl.GEOM15, 8, 64, 3, 3)])
def test_update_tiny_inputs(dev, geom, M, R, K, P):
    """A handful of patches: every bucket is shorter than one batch of pairs, and more
    atoms go unused than there are patches to reset them to (the rest keep -1)."""
    D = wl.draw_dictionary(M, geom.B, seed=41).astype(np.float32).astype(np.float64)
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    d = wl.draw_mixtures(P, geom.N, M, 2, 0.05, seed=41)
    X = orc.project(basis, orc.synthesize(basis, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32))
    X = X.astype(np.float32).astype(np.float64)
    _check_update(geom, D, R, K, X, dev, repeat=True)


def test_unused_atoms_are_reset_on_device(dev):
    """Atoms in harmonics that no patch contains are never selected and take the
    worst-coded patches, in index order."""
    g = wl.GEOM11
    S, T, B = g.S, g.T, g.B
    rng = np.random.default_rng(10)
    D = np.zeros((4, B))
    D[0, :S] = rng.standard_normal(S)
    D[1, S:3 * S] = rng.standard_normal(2 * S)
    D[2, B - 2 * S:] = rng.standard_normal(2 * S)
    D[3, B - 4 * S:B - 2 * S] = rng.standard_normal(2 * S)
    D = (D / np.linalg.norm(D, axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    X = np.zeros((300, B))
    X[:, :3 * S] = rng.standard_normal((300, 3 * S))
    X = X.astype(np.float32).astype(np.float64)
    _check_update(g, D, 8, 1, X, dev)


def test_training_loop_recovers_toy_atoms(dev):
    """Three atoms, two grid-rotated copies per patch, noise-free: the device loop from
    a random start finds every atom up to a rotation, like the reference loop."""
    from paper_1806_04374_amd import rsc
    g = wl.GEOM11
    S, T, B, R = g.S, g.T, g.B, 32
    rng = np.random.default_rng(2)
    D_true = rng.standard_normal((3, B))
    D_true /= np.linalg.norm(D_true, axis=1, keepdims=True)
    P = 400
    a = rng.integers(0, 3, (P, 2))
    r = rng.integers(0, R, (P, 2))
    w = rng.uniform(0.5, 1.5, (P, 2)) * rng.choice([-1.0, 1.0], (P, 2))
    X = np.stack([sum(w[p, j] * orc.steer(D_true[a[p, j]], 2 * np.pi * r[p, j] / R, S, T) for j in range(2))
                  for p in range(P)]).astype(np.float32)
    D0 = np.random.default_rng(7).standard_normal((3, B))
    D0 = (D0 / np.linalg.norm(D0, axis=1, keepdims=True)).astype(np.float32)
    h = rsc.rsc_create(g.N, S, T)
    D, codes, hist = rsc.rsc_rksvd_train(h, torch.from_numpy(X).to(dev), D0, R, 2, 20)
    print("history", hist)
    for m in range(3):
        best = max(max(abs(orc.steer(D[m].astype(np.float64), 2 * np.pi * k / R, S, T) @ D_true[j])
                       for k in range(R)) for j in range(3))
        assert best > 0.9999, (m, best)
    assert hist[-1] < 1e-2 * hist[0]
    _, _, ref_hist = orc.rksvd(D0.astype(np.float64), R, S, T, X.astype(np.float64), 2, 1)
    assert abs(hist[0] - ref_hist[0]) < 1e-4 * ref_hist[0]      # same first pursuit
    h.close()


def test_one_training_iteration_matches_reference(dev):
    """Scale geometry (M=64, R=64, K=4) on 4,000 patches: one device iteration (pursuit +
    update + final pursuit) against the reference loop on the same FP32 inputs."""
    from paper_1806_04374_amd import rsc
    w = wl.SCALE
    g = w["geom"]
    basis = orc.build_basis(g.N, g.S, g.T)
    D, d = wl.scale_draw(P=4000)
    X = orc.project(basis, orc.synthesize(basis, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32))
    X = np.ascontiguousarray(X, dtype=np.float32)
    D0 = D + 0.1 * np.random.default_rng(31).standard_normal(D.shape)
    D0 = (D0 / np.linalg.norm(D0, axis=1, keepdims=True)).astype(np.float32)
    h = rsc.rsc_create(g.N, g.S, g.T)
    Dg, codes, hist = rsc.rsc_rksvd_train(h, torch.from_numpy(X).to(dev), D0, w["R"], w["K"], 1)
    Dr, code_r, hist_r = orc.rksvd(D0.astype(np.float64), w["R"], g.S, g.T, X.astype(np.float64), w["K"], 1)
    print("history device", hist, "reference", hist_r)
    assert abs(hist[0] - hist_r[0]) < 1e-4 * hist_r[0]
    assert abs(hist[1] - hist_r[1]) < 1e-3 * hist_r[1]
    cos = np.abs(np.sum(Dg.astype(np.float64) * Dr, axis=1))
    print("atom agreement min", cos.min(), "median", np.median(cos))
    assert np.median(cos) > 1 - 1e-8 and cos.min() > 0.999
    h.close()


def test_update_argument_errors(dev):
    from paper_1806_04374_amd import rsc
    h = rsc.rsc_create(11, 5, 5)
    with pytest.raises(rsc.RscError) as e:
        rsc.rsc_rksvd_workspace_size(h, 10, 2)
    assert e.value.status == rsc.RSC_E_NOT_READY
    rsc.rsc_set_dictionary(h, wl.draw_dictionary(4, 55).astype(np.float32), 8)
    z = torch.zeros((10, 55), dtype=torch.float32, device=dev)
    ia = torch.zeros((10, 9), dtype=torch.int32, device=dev)
    with pytest.raises(rsc.RscError, match="K must"):
        rsc.rsc_rksvd_update(h, z, ia, ia, torch.zeros((10, 9), dtype=torch.float32, device=dev),
                             torch.zeros(10, dtype=torch.float32, device=dev))
    h.close()


# ----------------------------------------------------------------- the paper's annular basis
@pytest.mark.parametrize("N", [11, 15])
def test_update_matches_reference_annular_basis(dev, N):
    """The update in the annular layout (harmonic k on the annuli that carry it; B = 81 at
    N = 11, 153 at N = 15, whose covariance takes 10 x 10 tiles) against the reference's
    update with that basis' steering, on the reference's codes."""
    from paper_1806_04374_amd import rsc
    ab = orc.build_annular_basis(N)
    M, R, K = 16, 32, 3
    D = wl.draw_dictionary(M, ab.B, seed=41).astype(np.float32).astype(np.float64)
    d = wl.draw_mixtures(3000, N, M, 3, 0.05, seed=41)
    X = orc.project(ab, orc.synthesize(ab, D, d.atom, d.angle, d.weight, d.noise).astype(np.float32))
    X = X.astype(np.float32).astype(np.float64)
    Dp = D + 0.2 * np.random.default_rng(42).standard_normal(D.shape)
    Dp = (Dp / np.linalg.norm(Dp, axis=1, keepdims=True)).astype(np.float32).astype(np.float64)
    code = _fp32_code(orc.omp(orc.augmented_dictionary_basis(ab, Dp, R), X, K, M))
    ref, usage_ref, reset_ref = orc.rksvd_update_basis(ab, Dp, R, X, code)
    h = rsc.rsc_create_annular(N)
    rsc.rsc_set_dictionary(h, Dp.astype(np.float32), R)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to(dev)
    d_new, usage, reset = rsc.rsc_rksvd_update(h, t(X, np.float32), t(code.atom, np.int32), t(code.angle, np.int32),
                                               t(code.coef, np.float32), t(code.resid2, np.float32))
    torch.cuda.synchronize()
    d_new, usage, reset = d_new.cpu().numpy().astype(np.float64), usage.cpu().numpy(), reset.cpu().numpy()
    h.close()
    assert np.array_equal(usage, usage_ref) and np.array_equal(reset, reset_ref)
    recon = orc.code_to_hat_basis(ab, Dp, R, code)
    worst = 0.0
    for m in range(M):
        C = np.zeros((ab.B, ab.B))
        for p in range(X.shape[0]):
            slots = np.flatnonzero(code.atom[p] == m)
            if slots.size:
                i0 = slots[0]
                y = orc.steer_ragged(X[p] - recon[p], -2 * np.pi * code.angle[p, i0] / R, ab.Sk) + code.coef[p, i0] * Dp[m]
                C += np.outer(y, y)
        assert abs(np.linalg.norm(d_new[m]) - 1) < 1e-6
        if usage_ref[m] == 0:
            continue
        ev = np.linalg.eigvalsh(C)
        assert d_new[m] @ C @ d_new[m] >= ev[-1] * (1 - 1e-6)
        if ev[-1] - ev[-2] > 1e-3 * ev[-1]:
            worst = max(worst, np.abs(d_new[m] - ref[m]).max())
    print("worst atom difference", worst)
    assert worst < 1e-5


@pytest.mark.parametrize("N", [11, 15])
def test_training_loop_recovers_toy_atoms_annular_basis(dev, N):
    """The device loop on the annular basis: three atoms, two grid-rotated copies per patch,
    noise-free, found from a random start up to a rotation, as the reference loop does."""
    from paper_1806_04374_amd import rsc
    ab = orc.build_annular_basis(N)
    R, P = 32, 400
    rng = np.random.default_rng(2)
    D_true = rng.standard_normal((3, ab.B))
    D_true /= np.linalg.norm(D_true, axis=1, keepdims=True)
    a = rng.integers(0, 3, (P, 2))
    r = rng.integers(0, R, (P, 2))
    w = rng.uniform(0.5, 1.5, (P, 2)) * rng.choice([-1.0, 1.0], (P, 2))
    X = np.stack([sum(w[p, j] * orc.steer_ragged(D_true[a[p, j]], 2 * np.pi * r[p, j] / R, ab.Sk) for j in range(2))
                  for p in range(P)]).astype(np.float32)
    D0 = np.random.default_rng(7).standard_normal((3, ab.B))
    D0 = (D0 / np.linalg.norm(D0, axis=1, keepdims=True)).astype(np.float32)
    h = rsc.rsc_create_annular(N)
    D, codes, hist = rsc.rsc_rksvd_train(h, torch.from_numpy(X).to(dev), D0, R, 2, 20)
    print("history", hist)
    for m in range(3):
        best = max(max(abs(orc.steer_ragged(D[m].astype(np.float64), 2 * np.pi * k / R, ab.Sk) @ D_true[j])
                       for k in range(R)) for j in range(3))
        assert best > 0.9999, (m, best)
    assert hist[-1] < 1e-2 * hist[0]
    _, _, ref_hist = orc.rksvd_basis(ab, D0.astype(np.float64), R, X.astype(np.float64), 2, 1)
    assert abs(hist[0] - ref_hist[0]) < 1e-4 * ref_hist[0]
    h.close()
