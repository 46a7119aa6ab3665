"""Device path against the FP64 reference, through the C ABI.

Acceptance: the selected (atom, angle) sets agree on >= 99.9% of patches,
coefficients of matched patches agree within 1e-4 relative (FP32), and the
reconstruction MSE agrees within 1e-3 relative.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc
from paper_1806_04374_amd import workloads as wl
from tests.parity import compare_codes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MATCH = 0.999
COEF_REL = 1e-4
MSE_REL = 1e-3


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04374_amd import rsc
    rsc.lib()
    return torch.device("cuda:0")


def _handle(geom, D, R, tile="auto"):
    from paper_1806_04374_amd import rsc
    h = rsc.rsc_create(geom.N, geom.S, geom.T)
    rsc.rsc_set_dictionary(h, D.astype(np.float32), R)
    rsc.rsc_set_tile(h, tile)
    return h


def _encode(h, X32, K, dev):
    from paper_1806_04374_amd import rsc
    x = torch.from_numpy(X32).to(dev)
    xh = rsc.rsc_project(h, x)
    atom, angle, coef, r2 = rsc.rsc_omp_encode(h, xh, K)
    torch.cuda.synchronize()
    return xh, atom, angle, coef, r2


def _check(label, X32, D, R, K, geom, dev, basis=None, mse=True, tile="auto"):
    """Full path parity: project + encode (+ reconstruct) against the reference."""
    from paper_1806_04374_amd import rsc
    basis = basis or orc.build_basis(geom.N, geom.S, geom.T)
    h = _handle(geom, D, R, tile)
    xh, atom, angle, coef, r2 = _encode(h, X32, K, dev)
    xh_ref, code = orc.encode(basis, D, R, X32.astype(np.float64), K)
    # projection parity (FP32 GEMM against FP64 least squares)
    err = np.abs(xh.cpu().numpy() - xh_ref).max(axis=1) / np.maximum(np.linalg.norm(xh_ref, axis=1), 1e-30)
    assert err.max() < 2e-5, (label, err.max())
    rep = compare_codes(atom.cpu().numpy(), angle.cpu().numpy(), coef.cpu().numpy(), code, COEF_REL,
                        xnorm=np.linalg.norm(xh_ref, axis=1))
    print(label, rep, flush=True)
    assert rep.match_rate >= MATCH, (label, str(rep))
    assert rep.coef_bad == 0, (label, str(rep))
    if mse:
        rec = rsc.rsc_reconstruct(h, atom, angle, coef)
        torch.cuda.synchronize()
        mse_gpu = orc.mse(basis, X32, rec.cpu().numpy().astype(np.float64))
        mse_ref = orc.mse(basis, X32, orc.reconstruct(basis, D, R, code))
        print(label, "mse", mse_gpu, mse_ref, flush=True)
        assert abs(mse_gpu - mse_ref) <= MSE_REL * mse_ref + 1e-12, label
    # reported hat residual agrees with the reference residual
    r2 = r2.cpu().numpy()
    close = np.abs(r2 - code.resid2) <= 1e-3 * code.resid2 + 1e-5 * np.einsum("ij,ij->i", xh_ref, xh_ref) + 1e-12
    assert close.mean() >= MATCH, (label, close.mean())
    h.close()
    return rep


@pytest.mark.parametrize("tile", ["16", "32"])
def test_small_plain_workload_full(dev, tile):
    """2,000 11x11 patches, M=16, K=2, R=32: two grid-rotated atoms plus N(0, 0.01^2) noise."""
    w = wl.SMALL
    geom = w["geom"]
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D, draw = wl.small_draw()
    X = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise).astype(np.float32)
    _check(f"small-t{tile}", X, D, w["R"], w["K"], geom, dev, basis, tile=tile)


@pytest.mark.parametrize("tile", ["16", "32"])
def test_scale_workload_ragged_slice(dev, tile):
    """Scale geometry (M=64, K=4, R=64) on 20,011 patches: many tiles plus a ragged tail."""
    w = wl.SCALE
    geom = w["geom"]
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D, draw = wl.scale_draw(P=20011)
    X = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise).astype(np.float32)
    _check(f"scale-20011-t{tile}", X, D, w["R"], w["K"], geom, dev, basis, tile=tile)


def test_scale_workload_full_size_sampled(dev):
    """All 1,000,000 scale patches encoded in one launch (the benchmark's launch); 20,000
    sampled patches and the last one checked against the reference."""
    from paper_1806_04374_amd import rsc
    w = wl.SCALE
    geom = w["geom"]
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D, draw = wl.scale_draw()
    X = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise).astype(np.float32)
    h = _handle(geom, D, w["R"])
    xh, atom, angle, coef, r2 = _encode(h, X, w["K"], dev)
    idx = np.sort(np.random.default_rng(0).choice(len(X) - 1, 20000, replace=False))
    idx = np.concatenate([idx, [len(X) - 1]])
    _, code = orc.encode(basis, D, w["R"], X[idx].astype(np.float64), w["K"])
    rep = compare_codes(atom.cpu().numpy()[idx], angle.cpu().numpy()[idx], coef.cpu().numpy()[idx], code)
    print("scale-full-sampled", rep, flush=True)
    assert rep.match_rate >= MATCH, str(rep)
    assert rep.coef_bad == 0, str(rep)
    h.close()


def test_large_geometry(dev):
    """15x15 geometry (S=T=7, B=105), M=128, K=6, R=64 on 3,000 patches."""
    geom = wl.GEOM15
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D = wl.draw_dictionary(128, geom.B, seed=0)
    draw = wl.draw_mixtures(3000, geom.N, 128, 6, 0.05, seed=0)
    X = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise).astype(np.float32)
    _check("geom15", X, D, 64, 6, geom, dev, basis)


@pytest.mark.parametrize("M,R,K,tile", [(20, 8, 3, "32"), (20, 8, 3, "16"), (16, 60, 2, "32"), (16, 60, 2, "16"),
                                        (5, 1, 4, "16"), (33, 100, 8, "16"), (64, 128, 1, "16"),
                                        (9, 17, 6, "16"), (200, 64, 5, "16")])
def test_uneven_shapes(dev, M, R, K, tile):
    """Atom counts off the atom tiles, angle grids off the angle tiles (60 as in the paper)."""
    geom = wl.GEOM11
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D = wl.draw_dictionary(M, geom.B, seed=3)
    draw = wl.draw_mixtures(1000, geom.N, M, 3, 0.02, seed=3)
    X = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise).astype(np.float32)
    _check(f"M{M}-R{R}-K{K}-t{tile}", X, D, R, K, geom, dev, basis, mse=K <= 4, tile=tile)


def test_edge_cases(dev):
    from paper_1806_04374_amd import rsc
    geom = wl.GEOM11
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    M, R = 16, 32
    D = wl.draw_dictionary(M, geom.B, seed=0)
    h = _handle(geom, D, R)
    # empty input is a no-op
    e = torch.empty((0, 11, 11), dtype=torch.float32, device=dev)
    xh = rsc.rsc_project(h, e)
    out = rsc.rsc_omp_encode(h, xh, 2)
    torch.cuda.synchronize()
    assert out[0].shape == (0, 2)
    # zero patches: every slot empty, zero residual
    z = torch.zeros((5, 11, 11), dtype=torch.float32, device=dev)
    atom, angle, coef, r2 = rsc.rsc_omp_encode(h, rsc.rsc_project(h, z), 3)
    torch.cuda.synchronize()
    assert (atom.cpu() == -1).all() and (angle.cpu() == -1).all() and (coef.cpu() == 0).all()
    assert (r2.cpu() == 0).all()
    # one exact grid-rotated atom: recovered, then the early stop leaves the other slots empty
    rng = np.random.default_rng(1)
    a = rng.integers(0, M, (64, 1))
    r = rng.integers(0, R, (64, 1))
    wgt = rng.uniform(0.5, 2.0, (64, 1)) * rng.choice([-1, 1], (64, 1))
    X = orc.synthesize(basis, D, a, 2 * np.pi * r / R, wgt).astype(np.float32)
    atom, angle, coef, r2 = _encode(h, X, 3, dev)[1:]
    atom, angle, coef = atom.cpu().numpy(), angle.cpu().numpy(), coef.cpu().numpy()
    assert np.array_equal(atom[:, 0], a[:, 0]) and np.array_equal(angle[:, 0], r[:, 0])
    assert np.all(atom[:, 1:] == -1)
    assert np.abs(coef[:, 0] - wgt[:, 0]).max() < 1e-4 * np.abs(wgt).max()
    # rotation-invariant content: every angle ties, the smallest angle index wins
    v = np.zeros((3, geom.B), np.float32)
    v[:, :5] = rng.standard_normal((3, 5))
    atom, angle, coef, r2 = rsc.rsc_omp_encode(h, torch.from_numpy(v).to(dev), 1)
    torch.cuda.synchronize()
    ref = orc.omp(orc.augmented_dictionary(D, R, 5, 5), v.astype(np.float64), 1, M)
    assert np.all(ref.angle[:, 0] == 0)
    assert np.all(angle.cpu().numpy()[:, 0] == 0)
    assert np.array_equal(atom.cpu().numpy()[:, 0], ref.atom[:, 0])
    h.close()


@pytest.mark.parametrize("tile", ["16", "32"])
def test_batch_position_invariance(dev, tile):
    """A patch gives bit-identical codes wherever it sits in the batch."""
    from paper_1806_04374_amd import rsc
    geom = wl.GEOM11
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D, draw = wl.scale_draw(P=4099)
    X = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise).astype(np.float32)
    h = _handle(geom, D, 64, tile)
    full = _encode(h, X, 4, dev)
    for lo, n in [(0, 1), (7, 33), (1000, 517), (4090, 9)]:
        part = _encode(h, X[lo:lo + n].copy(), 4, dev)
        for a, b in zip(full[1:], part[1:]):
            assert torch.equal(a[lo:lo + n].cpu(), b.cpu())
    h.close()


def test_rotation_equivariance_on_device(dev):
    """Rotating a patch inside the basis span by r0 grid steps shifts every angle by r0
    (eq. (3)): exactly, on every patch whose reference top-2 gap stays above 1e-6 at each
    step (a closer pair is decided by rounding)."""
    from paper_1806_04374_amd import rsc
    geom = wl.GEOM11
    M, R, K = 16, 32, 2
    D = wl.draw_dictionary(M, geom.B, seed=5)
    draw = wl.draw_mixtures(500, geom.N, M, 2, 0.0, seed=5)
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    v = np.zeros((500, geom.B))
    for i in range(2):
        v += draw.weight[:, i, None] * orc.steer(D[draw.atom[:, i]], 2 * np.pi * np.round(draw.angle[:, i] / (2 * np.pi) * R) / R, 5, 5)
    h = _handle(geom, D, R)
    base = rsc.rsc_omp_encode(h, torch.from_numpy(v.astype(np.float32)).to(dev), K)
    torch.cuda.synchronize()
    ref = orc.omp(orc.augmented_dictionary(D, R, 5, 5), v.astype(np.float32).astype(np.float64), K, M)
    clear = np.array([np.all(ref.gap[p][ref.atom[p] >= 0] >= 1e-6) for p in range(len(v))])
    assert clear.mean() > 0.95
    ok = tot = 0
    for r0 in (1, 8, 13):
        vr = orc.steer(v, 2 * np.pi * r0 / R, 5, 5).astype(np.float32)
        rot = rsc.rsc_omp_encode(h, torch.from_numpy(vr).to(dev), K)
        torch.cuda.synchronize()
        a0, g0 = base[0].cpu().numpy(), base[1].cpu().numpy()
        a1, g1 = rot[0].cpu().numpy(), rot[1].cpu().numpy()
        for p in np.flatnonzero(clear):
            tot += 1
            s0 = {(int(a), (int(g) + r0) % R) for a, g in zip(a0[p], g0[p]) if a >= 0}
            s1 = {(int(a), int(g)) for a, g in zip(a1[p], g1[p]) if a >= 0}
            ok += s0 == s1
    assert ok == tot, (ok, tot)
    h.close()


def test_synthesize_and_reconstruct_match_reference(dev):
    from paper_1806_04374_amd import rsc
    geom = wl.GEOM11
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D, draw = wl.scale_draw(P=777)
    h = _handle(geom, D, 64)
    X_ref = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise)
    X = rsc.rsc_synthesize(h, torch.from_numpy(draw.atom.astype(np.int32)).to(dev),
                           torch.from_numpy(draw.angle.astype(np.float32)).to(dev),
                           torch.from_numpy(draw.weight.astype(np.float32)).to(dev),
                           torch.from_numpy(draw.noise.astype(np.float32)).to(dev))
    torch.cuda.synchronize()
    assert np.abs(X.cpu().numpy() - X_ref).max() < 1e-5 * np.abs(X_ref).max()
    # reconstruction of given codes on a grid
    rng = np.random.default_rng(2)
    code = orc.Code(rng.integers(-1, 64, (777, 4)), rng.integers(0, 64, (777, 4)),
                    rng.standard_normal((777, 4)), np.zeros(777), np.zeros((777, 4)), np.zeros((777, 4)))
    code.angle[code.atom < 0] = -1
    code.coef[code.atom < 0] = 0
    ref = orc.reconstruct(basis, D, 64, code)
    out = rsc.rsc_reconstruct(h, torch.from_numpy(code.atom.astype(np.int32)).to(dev),
                              torch.from_numpy(code.angle.astype(np.int32)).to(dev),
                              torch.from_numpy(code.coef.astype(np.float32)).to(dev))
    torch.cuda.synchronize()
    assert np.abs(out.cpu().numpy() - ref).max() < 1e-5 * np.abs(ref).max()
    h.close()


def test_device_argument_errors(dev):
    from paper_1806_04374_amd import rsc
    geom = wl.GEOM11
    h = rsc.rsc_create(11, 5, 5)
    x = torch.zeros((4, 55), dtype=torch.float32, device=dev)
    with pytest.raises(rsc.RscError, match="no dictionary") as e:
        rsc.rsc_omp_encode(h, x, 2)
    assert e.value.status == rsc.RSC_E_NOT_READY
    bad = np.ones((4, 55), np.float32)
    with pytest.raises(rsc.RscError, match="unit norm"):
        rsc.rsc_set_dictionary(h, bad, 8)
    D = wl.draw_dictionary(4, 55)
    rsc.rsc_set_dictionary(h, D, 8)
    with pytest.raises(rsc.RscError, match="K must"):
        rsc.rsc_omp_encode(h, x, 9)
    with pytest.raises(rsc.RscError, match="R must"):
        rsc.rsc_set_dictionary(h, D, 129)
    h.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_dictionary_reload_on_one_handle(dev, prec):
    """Dictionaries of growing and shrinking size loaded one after another into the same
    handle (the tables are refilled in place when they fit, reallocated when they grow):
    each encode matches the reference for the dictionary loaded last."""
    from paper_1806_04374_amd import rsc
    geom = wl.GEOM11
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    h = rsc.rsc_create(geom.N, geom.S, geom.T, prec=prec)
    for i, (M, R, K) in enumerate([(16, 32, 2), (64, 64, 4), (8, 16, 3), (64, 64, 4)]):
        D = wl.draw_dictionary(M, geom.B, seed=40 + i)
        draw = wl.draw_mixtures(600, geom.N, M, 2, 0.02, seed=40 + i)
        X = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise).astype(np.float32)
        rsc.rsc_set_dictionary(h, D.astype(np.float32), R)
        xh, atom, angle, coef, r2 = _encode(h, X, K, dev)
        _, code = orc.encode(basis, D, R, X.astype(np.float64), K)
        rep = compare_codes(atom.cpu().numpy(), angle.cpu().numpy(), coef.cpu().numpy(), code, COEF_REL)
        assert rep.match_rate >= MATCH, (M, R, K, str(rep))
    h.close()


@pytest.mark.parametrize("geom", [wl.GEOM11, wl.GEOM15])
@pytest.mark.parametrize("P", [1, 31, 32, 33, 2000, 64 * 1024 + 7])
def test_projection_patch_arrays(dev, geom, P):
    """Patch arrays: whole 32-patch chunks and the partial last one by the register-operand
    MFMA kernel; also from a buffer that is not 16-byte aligned (another kernel) and into an
    output that is not (scalar stores)."""
    from paper_1806_04374_amd import rsc
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    h = rsc.rsc_create(geom.N, geom.S, geom.T)
    X = np.random.default_rng(P).standard_normal((P, geom.N, geom.N)).astype(np.float32)
    n = min(P, 3000)
    ref = orc.project(basis, X[:n].astype(np.float64))
    tol = 2e-5 * np.abs(ref).max()
    xh = rsc.rsc_project(h, torch.from_numpy(X).to(dev)).cpu().numpy()
    assert np.abs(xh[:n] - ref).max() < tol
    if P > n:   # the rest: the same rows through the reference at a sample of indices
        idx = np.random.default_rng(1).choice(P, 500, replace=False)
        ref_s = orc.project(basis, X[idx].astype(np.float64))
        assert np.abs(xh[idx] - ref_s).max() < 2e-5 * np.abs(ref_s).max()
    flat = torch.zeros(P * geom.N * geom.N + 1, dtype=torch.float32, device=dev)
    flat[1:] = torch.from_numpy(X.ravel()).to(dev)
    out = torch.zeros(P * geom.B + 1, dtype=torch.float32, device=dev)
    rsc.rsc_project(h, flat[1:].view(P, geom.N, geom.N), out[1:].view(P, geom.B))
    assert np.abs(out[1:].view(P, geom.B).cpu().numpy()[:n] - ref).max() < tol
    xo = torch.zeros(P * geom.B + 1, dtype=torch.float32, device=dev)
    rsc.rsc_project(h, torch.from_numpy(X).to(dev), xo[1:].view(P, geom.B))
    assert np.abs(xo[1:].view(P, geom.B).cpu().numpy()[:n] - ref).max() < tol
    h.close()


@pytest.mark.parametrize("tile", ["16", "32"])
def test_duplicate_atom_ties_go_to_smaller_index(dev, tile):
    """Atom 1 is a copy of atom 0: every column of atom 1 ties exactly with the same column
    of atom 0, so the smaller atom index must win every time.  The codes then equal, bit
    for bit, those of the dictionary without the copy (indices above 1 shifted)."""
    from paper_1806_04374_amd import rsc
    geom = wl.GEOM11
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    M, R, K = 16, 32, 2
    D = wl.draw_dictionary(M, geom.B, seed=7)
    D[1] = D[0]
    Dm = np.delete(D, 1, axis=0)
    draw = wl.draw_mixtures(3000, geom.N, M, 2, 0.02, seed=7)
    X = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise).astype(np.float32)
    h, hm = _handle(geom, D, R, tile), _handle(geom, Dm, R, tile)
    a, g, c = (t.cpu().numpy() for t in _encode(h, X, K, dev)[1:4])
    am, gm, cm = (t.cpu().numpy() for t in _encode(hm, X, K, dev)[1:4])
    assert (a == 1).sum() == 0 and (a == 0).sum() > 0
    assert np.array_equal(a, np.where(am >= 1, am + 1, am))
    assert np.array_equal(g, gm) and np.array_equal(c, cm)
    h.close()
    hm.close()


@pytest.mark.parametrize("eps,fp64", [(0.2, False), (6.3e-3, True), (1e-3, True)])
@pytest.mark.parametrize("R,tile", [(1, "16"), (2, "32")])
def test_ill_conditioned_supports(dev, eps, fp64, R, tile):
    """Two atoms eps apart: once both are selected the Gram matrix has cond ~ 1e2 (eps =
    0.2, least squares in FP32), ~ 1e5 or ~ 4e6 (re-solved in FP64, since the bound
    k ||L^{-1}||_F^2 passes 1e3).  Coefficients must match the reference's QR solve to
    1e-4 in every case; the FP64 steps are counted by rsc_precision_stats.  With R = 2 (the
    32x32 tiles) the direction n separating the two atoms is also orthogonal to the half
    turn of the first, so that after one of the pair is selected the other one is the best
    second column (as with R = 1)."""
    from paper_1806_04374_amd import rsc
    g = wl.GEOM11
    rng = np.random.default_rng(5)
    d1 = rng.standard_normal(g.B)
    d1 /= np.linalg.norm(d1)
    n = rng.standard_normal(g.B)
    for v in [d1] + [orc.steer(d1, 2 * np.pi * r / R, g.S, g.T) for r in range(1, R)]:
        v = v / np.linalg.norm(v)
        n -= (n @ v) * v
    d2 = d1 + eps * n / np.linalg.norm(n)
    d2 /= np.linalg.norm(d2)
    D = np.stack([d1, d2]).astype(np.float32).astype(np.float64)   # used as they are on both sides
    cond = np.linalg.cond(D @ D.T)
    P = 200
    w = rng.uniform(0.5, 1.5, (P, 2)) * rng.choice([-1.0, 1.0], (P, 2))
    xh = (w @ D).astype(np.float32)       # coordinates handed over directly
    h = _handle(g, D, R, tile)
    rsc.rsc_precision_stats(h, reset=True)
    atom, angle, coef, _ = rsc.rsc_omp_encode(h, torch.from_numpy(xh).to(dev), 2)
    torch.cuda.synchronize()
    stats = rsc.rsc_precision_stats(h)
    code = orc.omp(orc.augmented_dictionary(D, R, g.S, g.T), xh.astype(np.float64), 2, 2)
    rep = compare_codes(atom.cpu().numpy(), angle.cpu().numpy(), coef.cpu().numpy(), code, COEF_REL)
    print(f"cond {cond:.3g}", rep, stats, flush=True)
    assert rep.match_rate >= MATCH, str(rep)
    assert rep.coef_bad == 0, str(rep)
    if fp64:
        assert stats["fp64_solves"] >= P * MATCH, stats
    else:
        assert stats["fp64_solves"] == 0, stats
    h.close()


def test_workload_never_needs_fp64(dev):
    """On the scale workload every selected support is well conditioned (bound below 1e3):
    the FP64 fallback does not fire."""
    from paper_1806_04374_amd import rsc
    w = wl.SCALE
    geom = w["geom"]
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    D, draw = wl.scale_draw(P=50000)
    X = orc.synthesize(basis, D, draw.atom, draw.angle, draw.weight, draw.noise).astype(np.float32)
    h = _handle(geom, D, w["R"])
    rsc.rsc_precision_stats(h, reset=True)
    _encode(h, X, w["K"], dev)
    assert rsc.rsc_precision_stats(h)["fp64_solves"] == 0
    h.close()


def test_pursuit_that_runs_out_of_span_stops_cleanly(dev):
    """Atom 2 is (atom 0 + 2 atom 1) normalised and x = d0 + d1 + 1e-3 e with e orthogonal to
    the three atoms (R = 1).  The pursuit takes atom 2, then atom 0; their span holds d0 + d1,
    so the residual is 1e-3 e and every correlation of the third step is rounding noise: the
    best column is either already selected (the duplicate stop) or atom 1, which lies inside
    the span (its FP64 pivot is rounding-sized: the pivot stop).  Either way the patch ends
    with two atoms, the exact coefficients (sqrt(5)/2, 1/2) and the residual 1e-3 e, where a
    refit with atom 1 would give meaningless coefficients."""
    from paper_1806_04374_amd import rsc
    g = wl.GEOM11
    rng = np.random.default_rng(11)
    d0 = rng.standard_normal(g.B)
    d0 /= np.linalg.norm(d0)
    d1 = rng.standard_normal(g.B)
    d1 -= (d1 @ d0) * d0
    d1 /= np.linalg.norm(d1)
    d2 = (d0 + 2 * d1) / np.sqrt(5.0)
    D = np.stack([d0, d1, d2]).astype(np.float32)
    Q, _ = np.linalg.qr(D.astype(np.float64).T)
    P = 64
    E = rng.standard_normal((P, g.B))
    E -= (E @ Q) @ Q.T
    E /= np.linalg.norm(E, axis=1, keepdims=True)
    xh = (d0 + d1)[None, :] + 1e-3 * E
    h = _handle(g, D, 1, "16")
    atom, angle, coef, r2 = (t.cpu().numpy() for t in rsc.rsc_omp_encode(h, torch.from_numpy(xh.astype(np.float32)).to(dev), 3))
    h.close()
    assert np.all(atom[:, 0] == 2) and np.all(atom[:, 1] == 0) and np.all(angle[:, :2] == 0)
    assert np.all(atom[:, 2] == -1) and np.all(angle[:, 2] == -1) and np.all(coef[:, 2] == 0)
    assert np.abs(coef[:, 0] - np.sqrt(5.0) / 2).max() < 1e-4 and np.abs(coef[:, 1] - 0.5).max() < 1e-4
    assert np.abs(np.sqrt(r2) - 1e-3).max() < 2e-5
