"""The paper's annular basis on the device (rsc_create_annular): projection, steering in
its ragged layout and synthesis against the FP64 reference, through the C ABI.

Acceptance as for the other rotation paths: projection within 2e-5 of the largest
coordinate, steering within 1e-6 relative, synthesis within 1e-5 and the full steering
rotation within 1e-4 of the largest value.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

THETA = np.deg2rad(100 + np.sqrt(2))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1806_04374_amd import rsc
    rsc.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("N,lowpass", [(11, False), (11, True), (15, False), (15, True), (9, False)])
def test_annular_rotation_path(dev, N, lowpass):
    from paper_1806_04374_amd import rsc
    b = orc.build_annular_basis(N, lowpass)
    h = rsc.rsc_create_annular(N, lowpass)
    assert h.B == b.B and h.Ts == b.Ts
    rng = np.random.default_rng(N + int(lowpass))
    P = 777
    X = rng.standard_normal((P, N, N)).astype(np.float32)
    xh = rsc.rsc_project(h, torch.from_numpy(X).to(dev))
    ref = orc.project(b, X.astype(np.float64))
    assert np.abs(xh.cpu().numpy() - ref).max() < 2e-5 * np.abs(ref).max()
    # steering: one angle (streamed chunks and the partial chunk), per-patch angles
    xr = rng.standard_normal((P, b.B)).astype(np.float32)
    xd = torch.from_numpy(xr).to(dev)
    out = rsc.rsc_steer(h, xd, THETA).cpu().numpy()
    sref = orc.steer_ragged(xr.astype(np.float64), THETA, b.Sk)
    assert np.abs(out - sref).max() < 1e-6 * np.abs(sref).max()
    th = rng.uniform(-7, 7, P).astype(np.float32)
    out = rsc.rsc_steer(h, xd, theta=torch.from_numpy(th).to(dev)).cpu().numpy()
    sref = np.stack([orc.steer_ragged(xr[p].astype(np.float64), float(th[p]), b.Sk) for p in range(P)])
    assert np.abs(out - sref).max() < 5e-6 * np.abs(sref).max()
    # synthesis and the full steering rotation
    pix = rsc.rsc_synthesize_hat(h, xd).cpu().numpy()
    pref = orc.to_pixels(b, xr.astype(np.float64))
    assert np.abs(pix - pref).max() < 1e-5 * np.abs(pref).max()
    rot = rsc.rsc_synthesize_hat(h, rsc.rsc_steer(h, xh, THETA)).cpu().numpy()
    rref = orc.rotate_steer(b, X.astype(np.float64), THETA)
    assert np.abs(rot - rref).max() < 1e-4 * np.abs(rref).max()
    # a quarter turn inside the span is exact up to FP32 rounding
    Xs = orc.to_pixels(b, rng.standard_normal((64, b.B))).astype(np.float32)
    q = rsc.rsc_synthesize_hat(h, rsc.rsc_steer(h, rsc.rsc_project(h, torch.from_numpy(Xs).to(dev)), np.pi / 2))
    assert np.abs(q.cpu().numpy() - np.rot90(Xs, 1, axes=(1, 2))).max() < 1e-4 * np.abs(Xs).max()
    h.close()


@pytest.mark.parametrize("P", [1, 63, 64, 64 * 300 + 17])
def test_annular_steering_chunk_edges_and_alignment(dev, P):
    from paper_1806_04374_amd import rsc
    b = orc.build_annular_basis(11)
    h = rsc.rsc_create_annular(11)
    xr = np.random.default_rng(P).standard_normal((P, b.B)).astype(np.float32)
    sref = orc.steer_ragged(xr.astype(np.float64), THETA, b.Sk)
    out = rsc.rsc_steer(h, torch.from_numpy(xr).to(dev), THETA).cpu().numpy()
    assert np.abs(out - sref).max() < 1e-6 * np.abs(sref).max()
    flat = torch.zeros(P * b.B + 1, dtype=torch.float32, device=dev)
    flat[1:] = torch.from_numpy(xr.ravel()).to(dev)
    out = rsc.rsc_steer(h, flat[1:].view(P, b.B), THETA).cpu().numpy()
    assert np.abs(out - sref).max() < 1e-6 * np.abs(sref).max()
    h.close()


def test_annular_refusals(dev):
    from paper_1806_04374_amd import rsc
    with pytest.raises(rsc.RscError) as e:
        rsc.rsc_create_annular(17)           # B = 204
    assert e.value.status == rsc.RSC_E_UNSUPPORTED
    h = rsc.rsc_create_annular(11)
    with pytest.raises(rsc.RscError) as e:
        rsc.rsc_set_dictionary(h, np.ones((2, h.B), np.float32) / np.sqrt(h.B), 8)
    assert e.value.status == rsc.RSC_E_UNSUPPORTED
    h.close()
