"""Patch rotation on the device (rsc_rotate_interp, rsc_steer, rsc_synthesize_hat) against
the FP64 reference, through the C ABI.

Acceptance: nearest-neighbour rotation bit-exact (one tap of weight 1); bicubic within
1e-5 of the largest input magnitude; steering within 1e-6 relative; synthesis and the
full steering rotation within 1e-5 of the largest value.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc
from paper_1806_04374_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

THETA = np.deg2rad(100 + np.sqrt(2))     # the paper's test angle


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04374_amd import rsc
    rsc.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("mode", ["nearest", "bicubic"])
@pytest.mark.parametrize("N,P", [(11, 1037), (15, 333), (25, 17), (3, 5)])
def test_interp_matches_reference(dev, mode, N, P):
    from paper_1806_04374_amd import rsc
    X = np.random.default_rng(N).standard_normal((P, N, N)).astype(np.float32)
    for theta in (THETA, np.deg2rad(37.0), -1.3):
        plan = rsc.RotationPlan(N, theta, mode)
        out = rsc.rsc_rotate_interp(plan, torch.from_numpy(X).to(dev)).cpu().numpy()
        ref = orc.rotate_interp(X.astype(np.float64), theta, mode)
        if mode == "nearest":
            assert np.array_equal(out, ref.astype(np.float32))
        else:
            assert np.abs(out - ref).max() < 1e-5 * np.abs(X).max()
        plan.close()


@pytest.mark.parametrize("N", [5, 11, 15])
def test_interp_quarter_turn_exact(dev, N):
    """A quarter turn is np.rot90 for both modes: at 5x5 and 11x11 bicubic runs in the
    plan's sorted lane order (through the general and the fixed kernel), at 15x15 in the
    natural one; 64 + 7 patches cover whole chunks and a partial one."""
    from paper_1806_04374_amd import rsc
    X = np.random.default_rng(1).standard_normal((71, N, N)).astype(np.float32)
    for mode in ("nearest", "bicubic"):
        plan = rsc.RotationPlan(N, np.pi / 2, mode)
        out = rsc.rsc_rotate_interp(plan, torch.from_numpy(X).to(dev)).cpu().numpy()
        assert np.allclose(out, np.rot90(X, 1, axes=(1, 2)), atol=1e-6)
        plan.close()


@pytest.mark.parametrize("geom", [wl.GEOM11, wl.GEOM15])
def test_steer_synth_and_full_rotation(dev, geom):
    from paper_1806_04374_amd import rsc
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    h = rsc.rsc_create(geom.N, geom.S, geom.T)
    rng = np.random.default_rng(2)
    P = 777
    xh = rng.standard_normal((P, geom.B)).astype(np.float32)
    xd = torch.from_numpy(xh).to(dev)
    # one angle for all
    out = rsc.rsc_steer(h, xd, THETA).cpu().numpy()
    ref = orc.steer(xh.astype(np.float64), THETA, geom.S, geom.T)
    assert np.abs(out - ref).max() < 1e-6 * np.abs(ref).max()
    # per-patch angles
    th = rng.uniform(-7, 7, P).astype(np.float32)
    out = rsc.rsc_steer(h, xd, theta=torch.from_numpy(th).to(dev)).cpu().numpy()
    ref = np.stack([orc.steer(xh[p].astype(np.float64), float(th[p]), geom.S, geom.T) for p in range(P)])
    assert np.abs(out - ref).max() < 5e-6 * np.abs(ref).max()
    # synthesis
    pix = rsc.rsc_synthesize_hat(h, xd).cpu().numpy()
    ref = orc.to_pixels(basis, xh.astype(np.float64))
    assert np.abs(pix - ref).max() < 1e-5 * np.abs(ref).max()
    # full steering rotation of pixel patches: project, steer, synthesize
    X = rng.standard_normal((P, geom.N, geom.N)).astype(np.float32)
    xp = rsc.rsc_project(h, torch.from_numpy(X).to(dev))
    rot = rsc.rsc_synthesize_hat(h, rsc.rsc_steer(h, xp, THETA)).cpu().numpy()
    ref = orc.rotate_steer(basis, X.astype(np.float64), THETA)
    assert np.abs(rot - ref).max() < 1e-4 * np.abs(ref).max()
    h.close()


def test_rotation_argument_errors(dev):
    from paper_1806_04374_amd import rsc
    with pytest.raises(rsc.RscError, match="N must"):
        rsc.RotationPlan(12, 0.1)
    with pytest.raises(rsc.RscError, match="N must"):
        rsc.RotationPlan(27, 0.1)
    plan = rsc.RotationPlan(11, 0.1)
    x = torch.zeros((4, 11, 11), dtype=torch.float32, device=dev)
    with pytest.raises(rsc.RscError, match="distinct"):
        rsc.rsc_rotate_interp(plan, x, out=x)
    plan.close()


@pytest.mark.parametrize("N,S,T", [(11, 5, 2), (15, 7, 3), (9, 3, 4)])
def test_basis_only_geometries(dev, N, S, T):
    """Handles of geometries the pursuit is not compiled for (here the low-pass bases with T
    halved) project, steer and synthesize like the reference; a dictionary is refused."""
    from paper_1806_04374_amd import rsc
    basis = orc.build_basis(N, S, T)
    h = rsc.rsc_create(N, S, T)
    with pytest.raises(rsc.RscError) as e:
        rsc.rsc_set_dictionary(h, np.ones((2, h.B), np.float32), 8)
    assert e.value.status == rsc.RSC_E_UNSUPPORTED
    rng = np.random.default_rng(N + T)
    X = rng.standard_normal((301, N, N)).astype(np.float32)
    xh = rsc.rsc_project(h, torch.from_numpy(X).to(dev))
    ref = orc.project(basis, X.astype(np.float64))
    assert np.abs(xh.cpu().numpy() - ref).max() < 2e-5 * np.abs(ref).max()
    rot = rsc.rsc_synthesize_hat(h, rsc.rsc_steer(h, xh, THETA)).cpu().numpy()
    ref = orc.rotate_steer(basis, X.astype(np.float64), THETA)
    assert np.abs(rot - ref).max() < 1e-4 * np.abs(ref).max()
    h.close()


@pytest.mark.parametrize("geom", [wl.GEOM11, wl.GEOM15])
@pytest.mark.parametrize("P", [1, 63, 64, 128, 64 * 2048 + 5])
def test_steer_chunk_edges(dev, geom, P):
    """One angle for all patches: whole 64-patch chunks are streamed and the rest handled
    per coordinate; both parts, and a buffer offset by one float (not 16-byte aligned),
    agree with the reference."""
    from paper_1806_04374_amd import rsc
    h = rsc.rsc_create(geom.N, geom.S, geom.T)
    xh = np.random.default_rng(P).standard_normal((P, geom.B)).astype(np.float32)
    ref = orc.steer(xh.astype(np.float64), THETA, geom.S, geom.T)
    out = rsc.rsc_steer(h, torch.from_numpy(xh).to(dev), THETA).cpu().numpy()
    assert np.abs(out - ref).max() < 1e-6 * np.abs(ref).max()
    flat = torch.zeros(P * geom.B + 1, dtype=torch.float32, device=dev)
    flat[1:] = torch.from_numpy(xh.ravel()).to(dev)
    out = rsc.rsc_steer(h, flat[1:].view(P, geom.B), THETA).cpu().numpy()
    assert np.abs(out - ref).max() < 1e-6 * np.abs(ref).max()
    h.close()


@pytest.mark.parametrize("N", [5, 11, 15])
def test_interp_unaligned_input(dev, N):
    """A patch buffer that is not 16-byte aligned takes the scalar staging path."""
    from paper_1806_04374_amd import rsc
    P = 100
    X = np.random.default_rng(N + 7).standard_normal((P, N, N)).astype(np.float32)
    flat = torch.zeros(P * N * N + 1, dtype=torch.float32, device=dev)
    flat[1:] = torch.from_numpy(X.ravel()).to(dev)
    plan = rsc.RotationPlan(N, THETA, "bicubic")
    out = rsc.rsc_rotate_interp(plan, flat[1:].view(P, N, N)).cpu().numpy()
    ref = orc.rotate_interp(X.astype(np.float64), THETA, "bicubic")
    assert np.abs(out - ref).max() < 1e-5 * np.abs(X).max()
    plan.close()


@pytest.mark.parametrize("N,S,T,P", [(7, 2, 3, 77), (9, 3, 4, 1000), (11, 5, 5, 33), (15, 7, 7, 65),
                                     (15, 3, 5, 40), (17, 3, 3, 50)])
def test_synthesis_geometries(dev, N, S, T, P):
    """Phi x_hat for pixel counts in each lane-group size (N*N <= 64, <= 128, <= 256) and
    above 256 (the LDS kernel), with row lengths B both compiled exactly and padded."""
    from paper_1806_04374_amd import rsc
    basis = orc.build_basis(N, S, T)
    h = rsc.rsc_create(N, S, T)
    xh = np.random.default_rng(N * S + T).standard_normal((P, h.B)).astype(np.float32)
    pix = rsc.rsc_synthesize_hat(h, torch.from_numpy(xh).to(dev)).cpu().numpy()
    ref = orc.to_pixels(basis, xh.astype(np.float64))
    assert np.abs(pix - ref).max() < 1e-5 * np.abs(ref).max()
    h.close()


@pytest.mark.parametrize("geom", [wl.GEOM11, wl.GEOM15])
@pytest.mark.parametrize("P", [32, 64 * 700 + 3])
def test_synthesis_chunks_and_alignment(dev, geom, P):
    """Phi x_hat through the MFMA kernel (whole 32-patch chunks, aligned hat rows), the
    register kernel (remainder, or hat rows not 16-byte aligned), and scalar stores into an
    output that is not 16-byte aligned, all equal to the reference."""
    from paper_1806_04374_amd import rsc
    basis = orc.build_basis(geom.N, geom.S, geom.T)
    h = rsc.rsc_create(geom.N, geom.S, geom.T)
    xh = np.random.default_rng(P + geom.N).standard_normal((P, geom.B)).astype(np.float32)
    n = min(P, 2000)
    ref = orc.to_pixels(basis, xh[:n].astype(np.float64))
    tol = 1e-5 * np.abs(ref).max()
    x = torch.from_numpy(xh).to(dev)
    assert np.abs(rsc.rsc_synthesize_hat(h, x).cpu().numpy()[:n] - ref).max() < tol
    flat = torch.zeros(P * geom.B + 1, dtype=torch.float32, device=dev)
    flat[1:] = x.ravel()
    assert np.abs(rsc.rsc_synthesize_hat(h, flat[1:].view(P, geom.B)).cpu().numpy()[:n] - ref).max() < tol
    o = torch.zeros(P * geom.N * geom.N + 1, dtype=torch.float32, device=dev)
    rsc.rsc_synthesize_hat(h, x, o[1:].view(P, geom.N, geom.N))
    assert np.abs(o[1:].view(P, geom.N, geom.N).cpu().numpy()[:n] - ref).max() < tol
    if P > n:
        idx = np.random.default_rng(2).choice(P, 300, replace=False)
        ref_s = orc.to_pixels(basis, xh[idx].astype(np.float64))
        assert np.abs(rsc.rsc_synthesize_hat(h, x).cpu().numpy()[idx] - ref_s).max() < 1e-5 * np.abs(ref_s).max()
    h.close()


def test_empty_and_negative_sizes(dev):
    """P = 0 is a no-op that reads no pointer (null pointers are accepted); P < 0 and
    a non-finite common angle are refused; the binding returns empty outputs."""
    from paper_1806_04374_amd import rsc
    L = rsc.lib()
    h = rsc.rsc_create(11, 5, 5)
    plan = rsc.RotationPlan(11, THETA)
    assert L.rsc_rotate_interp(plan.ptr, None, 0, None, None) == rsc.RSC_OK
    assert L.rsc_steer(h.ptr, None, 0, None, 0.3, None, None) == rsc.RSC_OK
    assert L.rsc_synthesize_hat(h.ptr, None, 0, None, None) == rsc.RSC_OK
    assert L.rsc_rotate_interp(plan.ptr, None, -1, None, None) == rsc.RSC_E_INVALID
    assert L.rsc_steer(h.ptr, None, -1, None, 0.3, None, None) == rsc.RSC_E_INVALID
    assert L.rsc_synthesize_hat(h.ptr, None, -1, None, None) == rsc.RSC_E_INVALID
    assert L.rsc_steer(h.ptr, None, 0, None, float("nan"), None, None) == rsc.RSC_E_INVALID
    e = torch.empty((0, 11, 11), dtype=torch.float32, device=dev)
    assert rsc.rsc_rotate_interp(plan, e).shape == (0, 11, 11)
    xe = torch.empty((0, h.B), dtype=torch.float32, device=dev)
    assert rsc.rsc_steer(h, xe, THETA).shape == (0, h.B)
    assert rsc.rsc_synthesize_hat(h, xe).shape == (0, 11, 11)
    plan.close()
    h.close()


@pytest.mark.parametrize("N", [11, 15])
def test_interp_unaligned_output(dev, N):
    """An aligned input with an output that is not 16-byte aligned: whole chunks go through
    the fixed kernel and the rest through the general kernel, both storing per pixel; both
    agree with the reference."""
    from paper_1806_04374_amd import rsc
    P = 32 * 7 + 5
    X = np.random.default_rng(N + 11).standard_normal((P, N, N)).astype(np.float32)
    plan = rsc.RotationPlan(N, THETA, "bicubic")
    o = torch.zeros(P * N * N + 1, dtype=torch.float32, device=dev)
    rsc.rsc_rotate_interp(plan, torch.from_numpy(X).to(dev), o[1:].view(P, N, N))
    ref = orc.rotate_interp(X.astype(np.float64), THETA, "bicubic")
    assert np.abs(o[1:].view(P, N, N).cpu().numpy() - ref).max() < 1e-5 * np.abs(X).max()
    plan.close()


@pytest.mark.parametrize("P", [1, 31, 32, 33, 777, 32 * 2100 + 7])
def test_steer_plan_one_pass(dev, P):
    """The one-pass steering plan (Phi S_theta Phi^+ as one operator) against the reference's
    projection, steering and synthesis, and against the device's three calls; whole 32-patch
    chunks, the partial last one, and an output not 16-byte aligned."""
    from paper_1806_04374_amd import rsc
    g = wl.GEOM11
    basis = orc.build_basis(g.N, g.S, g.T)
    h = rsc.rsc_create(g.N, g.S, g.T)
    plan = rsc.RotationPlan.steer(h, THETA)
    X = np.random.default_rng(P + 3).standard_normal((P, g.N, g.N)).astype(np.float32)
    x = torch.from_numpy(X).to(dev)
    out = rsc.rsc_rotate_interp(plan, x).cpu().numpy()
    n = min(P, 2000)
    ref = orc.rotate_steer(basis, X[:n].astype(np.float64), THETA)
    assert np.abs(out[:n] - ref).max() < 1e-4 * np.abs(ref).max()
    three = rsc.rsc_synthesize_hat(h, rsc.rsc_steer(h, rsc.rsc_project(h, x), THETA)).cpu().numpy()
    assert np.abs(out - three).max() < 2e-5 * np.abs(three).max()
    o = torch.zeros(P * g.N * g.N + 1, dtype=torch.float32, device=dev)
    rsc.rsc_rotate_interp(plan, x, o[1:].view(P, g.N, g.N))
    assert np.array_equal(o[1:].view(P, g.N, g.N).cpu().numpy(), out)
    plan.close()
    h.close()


def test_steer_plan_refusals(dev):
    """Steering plans: 11x11 handles of rsc_create only, finite angles, aligned patches."""
    from paper_1806_04374_amd import rsc
    h15 = rsc.rsc_create(15, 7, 7)
    with pytest.raises(rsc.RscError) as e:
        rsc.RotationPlan.steer(h15, THETA)
    assert e.value.status == rsc.RSC_E_UNSUPPORTED
    ha = rsc.rsc_create_annular(11)
    with pytest.raises(rsc.RscError) as e:
        rsc.RotationPlan.steer(ha, THETA)
    assert e.value.status == rsc.RSC_E_UNSUPPORTED
    h = rsc.rsc_create(11, 5, 5)
    with pytest.raises(rsc.RscError, match="finite"):
        rsc.RotationPlan.steer(h, float("inf"))
    plan = rsc.RotationPlan.steer(h, THETA)
    flat = torch.zeros(10 * 121 + 1, dtype=torch.float32, device=dev)
    with pytest.raises(rsc.RscError, match="aligned"):
        rsc.rsc_rotate_interp(plan, flat[1:].view(10, 11, 11))
    plan.close()
    h.close()
    ha.close()
    h15.close()
