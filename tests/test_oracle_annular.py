"""Pins of the reference annular basis (eq. (5)-(7), Sec. II-D) and its steering, CPU only.

The half-circumference cut-offs reproduce the (1, 5, 8) of the paper's basis figure; the
cap keeps exactly the largest linearly independent harmonic set per annulus (checked by
matrix rank, and in closed form on the 8-pixel annulus whose pixels sit at multiples of
45 degrees); Phi^+ Phi = I; disjoint annuli give orthogonal columns; a quarter turn inside
span(Phi) equals np.rot90 (annuli are invariant under it), which a flipped steering sign
fails; the low-pass basis' columns are columns of the full one.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc


def test_half_circumference_reproduces_the_basis_figure():
    assert orc.annular_cutoffs(11, cap=False)[:3] == [1, 5, 8]


@pytest.mark.parametrize("N", [11, 15, 21])
def test_cap_is_the_largest_independent_harmonic_set(N):
    _, rho, theta = orc.disk_grid(N)
    S = N // 2
    capped, uncapped = orc.annular_cutoffs(N), orc.annular_cutoffs(N, cap=False)
    for s in range(1, S + 1):
        ring = (rho >= N * (s - 1) / (2 * S)) & (rho < N * s / (2 * S))
        T = capped[s - 1]
        assert 0 <= T <= uncapped[s - 1]
        t = np.arange(-T, T + 1)
        A = np.exp(1j * np.outer(theta[ring], t))
        A[(rho[ring] == 0)[:, None] & (t != 0)[None, :]] = 0
        assert np.linalg.matrix_rank(A) == 2 * T + 1
        if T < uncapped[s - 1]:
            t = np.arange(-T - 1, T + 2)
            A = np.exp(1j * np.outer(theta[ring], t))
            A[(rho[ring] == 0)[:, None] & (t != 0)[None, :]] = 0
            assert np.linalg.matrix_rank(A) < 2 * T + 3


def test_eight_pixel_annulus_closed_form():
    """Annulus 2 at N = 11 (1.1 <= r < 2.2) holds the 8 pixels at radius sqrt 2 and 2, at
    the multiples of 45 degrees: harmonics t and t + 8 coincide there, so t = -3..3 is the
    largest symmetric independent set (t = +-4 coincide)."""
    _, rho, theta = orc.disk_grid(11)
    ring = (rho >= 1.1) & (rho < 2.2)
    assert ring.sum() == 8
    assert np.allclose(np.sort(np.mod(np.rad2deg(theta[ring]), 360)), np.arange(0, 360, 45))
    assert orc.annular_cutoffs(11)[1] == 3


@pytest.mark.parametrize("N,lowpass", [(11, False), (11, True), (15, False), (15, True)])
def test_biorthogonal_and_disjoint(N, lowpass):
    b = orc.build_annular_basis(N, lowpass)
    assert b.B == sum(2 * t + 1 for t in b.Ts)
    assert np.abs(b.pinv @ b.phi - np.eye(b.B)).max() < 1e-12
    assert np.allclose(np.linalg.norm(b.phi, axis=0)[: b.Sk[0]], 1.0)
    # columns whose supports (annuli) differ are exactly orthogonal
    support = [frozenset(np.flatnonzero(np.abs(b.phi[:, j]) > 0)) for j in range(b.B)]
    G = b.phi.T @ b.phi
    for i in range(b.B):
        for j in range(b.B):
            if not (support[i] & support[j]):
                assert G[i, j] == 0.0
    # harmonic 0 is the annulus indicator, normalised
    _, rho, _ = orc.disk_grid(N)
    S = N // 2
    for s in range(1, S + 1):
        ring = (rho >= N * (s - 1) / (2 * S)) & (rho < N * s / (2 * S))
        assert np.allclose(b.phi[:, s - 1], ring / np.sqrt(ring.sum()))


@pytest.mark.parametrize("N,lowpass", [(11, False), (11, True), (15, False), (15, True)])
def test_quarter_turn_inside_the_span_is_exact(N, lowpass):
    b = orc.build_annular_basis(N, lowpass)
    X = orc.to_pixels(b, np.random.default_rng(N).standard_normal((3, b.B)))
    for q in (1, 2, 3):
        assert np.abs(orc.rotate_steer(b, X, q * np.pi / 2) - np.rot90(X, q, axes=(1, 2))).max() < 1e-10


def test_planted_sign_error_is_caught():
    b = orc.build_annular_basis(11)
    X = orc.to_pixels(b, np.random.default_rng(0).standard_normal((1, b.B)))
    wrong = orc.to_pixels(b, orc.steer_ragged(orc.project(b, X), -np.pi / 2, b.Sk))
    assert np.abs(wrong - np.rot90(X, 1, axes=(1, 2))).max() > 0.1


def test_steering_group_law_and_norm():
    b = orc.build_annular_basis(11)
    x = np.random.default_rng(1).standard_normal((4, b.B))
    a, c = 0.37, 1.9
    assert np.allclose(orc.steer_ragged(orc.steer_ragged(x, a, b.Sk), c, b.Sk), orc.steer_ragged(x, a + c, b.Sk),
                       atol=1e-13)
    assert np.allclose(np.linalg.norm(orc.steer_ragged(x, a, b.Sk), axis=1), np.linalg.norm(x, axis=1))


@pytest.mark.parametrize("N", [11, 15])
def test_lowpass_columns_are_columns_of_the_full_basis(N):
    full, low = orc.build_annular_basis(N), orc.build_annular_basis(N, True)
    assert low.Ts == [t // 2 for t in full.Ts]
    for j in range(low.B):
        assert np.min(np.abs(full.phi - low.phi[:, j : j + 1]).max(axis=0)) < 1e-15


@pytest.mark.parametrize("N,lowpass", [(11, False), (11, True), (15, False), (15, True), (21, False), (9, True)])
def test_library_host_basis_matches_reference(N, lowpass):
    """The library builds the annular basis with its own code (real cos/sin columns, a
    Jacobi rank test); cut-offs, Phi and its partner equal the reference's."""
    from paper_1806_04374_amd import rsc
    phi, pinv, Ts, cond = rsc.rsc_annular_basis_host(N, lowpass)
    b = orc.build_annular_basis(N, lowpass)
    assert Ts == b.Ts
    ref = np.zeros((N * N, b.B))
    ref[b.mask.ravel()] = b.phi
    assert np.abs(phi - ref).max() < 1e-13
    refp = np.zeros((b.B, N * N))
    refp[:, b.mask.ravel()] = b.pinv
    assert np.abs(pinv - refp).max() < 1e-9 * np.abs(refp).max()
    w = np.linalg.eigvalsh(b.phi.T @ b.phi)
    assert abs(cond - w[-1] / w[0]) < 1e-8 * cond
