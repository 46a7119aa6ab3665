"""Pins of the reference patch rotations (Sec. III-C, rotation speed), CPU only.

Interpolation: identity at 0, exact quarter and half turns, exact reproduction of
quadratics by the bicubic kernel where its support lies inside the patch, nearest
neighbour outputs taken from the input, the kernel's partition of unity, and a
planted wrong direction.  Steering: in-span patches turn exactly (quarter turn equal
to np.rot90, composition), and it agrees with bicubic on a smooth patch.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc


@pytest.mark.parametrize("mode", ["nearest", "bicubic"])
@pytest.mark.parametrize("N", [5, 11, 15])
def test_identity_and_quarter_turns(mode, N):
    rng = np.random.default_rng(N)
    X = rng.standard_normal((3, N, N))
    assert np.allclose(orc.rotate_interp(X, 0.0, mode), X, atol=1e-14)
    for q in (1, 2, 3):
        assert np.allclose(orc.rotate_interp(X, q * np.pi / 2, mode), np.rot90(X, q, axes=(1, 2)), atol=1e-12)


def test_planted_wrong_direction_is_caught():
    X = np.random.default_rng(1).standard_normal((1, 7, 7))
    wrong = orc.rotate_interp(X, -np.pi / 2, "bicubic")
    assert not np.allclose(wrong, np.rot90(X, 1, axes=(1, 2)))


def test_keys_kernel_partition_of_unity_and_values():
    for f in np.linspace(0, 1, 11):
        assert abs(sum(orc._keys(f - k) for k in range(-1, 3)) - 1.0) < 1e-14
    assert orc._keys(0.0) == 1.0 and orc._keys(1.0) == 0.0 and orc._keys(2.0) == 0.0
    assert abs(orc._keys(0.5) - 0.5625) < 1e-15          # (a + 2)/8 - (a + 3)/4 + 1 at a = -1/2
    assert abs(orc._keys(1.5) + 0.0625) < 1e-15          # a (27/8 - 45/4 + 12 - 4) at a = -1/2


def test_bicubic_reproduces_quadratics():
    """Keys' kernel (a = -1/2) interpolates polynomials of degree <= 2 exactly, so an
    output pixel whose 4 x 4 source neighbourhood lies inside the patch equals the
    quadratic at the turned position."""
    N = 15
    c = (N - 1) / 2
    f = lambda x, y: 1.0 + 0.3 * x - 0.7 * y + 0.05 * x * x - 0.02 * x * y + 0.04 * y * y
    rows, cols = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    X = f(cols - c, c - rows)[None]
    theta = np.deg2rad(100 + np.sqrt(2))
    out = orc.rotate_interp(X, theta, "bicubic")[0]
    cs, sn = np.cos(theta), np.sin(theta)
    checked = 0
    for i in range(N):
        for j in range(N):
            x, y = j - c, c - i
            xs, ys = cs * x + sn * y, -sn * x + cs * y
            col, row = c + xs, c - ys
            if np.floor(row) - 1 >= 0 and np.floor(row) + 2 < N and np.floor(col) - 1 >= 0 and np.floor(col) + 2 < N:
                assert abs(out[i, j] - f(xs, ys)) < 1e-12
                checked += 1
    assert checked > 60


def test_nearest_takes_input_values():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((1, 11, 11))
    out = orc.rotate_interp(X, 0.7, "nearest")[0]
    vals = set(np.round(X.ravel(), 12)) | {0.0}
    assert all(round(v, 12) in vals for v in out.ravel())


def test_steering_turns_in_span_patches_exactly():
    basis = orc.build_basis(11, 5, 5)
    rng = np.random.default_rng(3)
    X = orc.to_pixels(basis, rng.standard_normal((4, basis.B)))     # inside span(Phi)
    assert np.allclose(orc.rotate_steer(basis, X, np.pi / 2), np.rot90(X, 1, axes=(1, 2)), atol=1e-10)
    a, b = 0.4, 1.1
    twice = orc.rotate_steer(basis, orc.rotate_steer(basis, X, a), b)
    assert np.allclose(twice, orc.rotate_steer(basis, X, a + b), atol=1e-10)


@pytest.mark.parametrize("N,S,T", [(11, 5, 5), (15, 7, 7)])
def test_rotation_quality_against_the_exact_turn(N, S, T):
    """A Gaussian blob off the centre, turned by 100 + sqrt(2) degrees, against the blob
    evaluated at the turned positions (inside radius N/2 - 2): bicubic is closest;
    steering, whose only loss is the part of the patch outside span(Phi), is clearly
    better than nearest neighbour (no staircase), as in the paper's comparison."""
    basis = orc.build_basis(N, S, T)
    c = (N - 1) / 2
    rows, cols = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    x, y = cols - c, c - rows
    f = lambda x, y: np.exp(-((x - 1.5) ** 2 + (y - 0.5) ** 2) / 4.0)
    theta = np.deg2rad(100 + np.sqrt(2))
    cs, sn = np.cos(theta), np.sin(theta)
    exact = f(cs * x + sn * y, -sn * x + cs * y)
    inner = np.hypot(x, y) < N / 2 - 2
    X = f(x, y)[None]
    err = lambda z: np.linalg.norm((z - exact)[inner]) / np.linalg.norm(exact[inner])
    e_steer = err(orc.rotate_steer(basis, X * basis.mask, theta)[0])
    e_bic = err(orc.rotate_interp(X, theta, "bicubic")[0])
    e_near = err(orc.rotate_interp(X, theta, "nearest")[0])
    assert e_bic < 0.02 and e_steer < 0.1
    assert e_steer < 0.8 * e_near
