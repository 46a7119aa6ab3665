"""Seeded synthetic workload draws for rotational sparse coding.

This module only draws random numbers: dictionaries in packed hat coordinates,
which atoms sit in a patch, at which angle and with which weight, pixel noise,
image sizes and stamp positions.  It contains none of the coding method's
arithmetic (no basis, no steering, no projection, no pursuit).  Turning a draw
into pixels is done separately by the CPU reference (test side) and by the
library's own synthesis call (GPU side), so both consume the same random
numbers without sharing code.

Workload shapes follow the experiments of the paper: circular 11x11 patches
(97 pixels, Sec. III-A), 15x15 patches with about a hundred atoms (the
parameters selected for texture classification, Sec. III-B), and an angle grid
of a few tens of points (60 steering angles in Sec. III-A).

Reproducibility: every stream is a ``numpy.random.SeedSequence(seed,
spawn_key=...)`` so that any slice of patches can be drawn without drawing
the ones before it.  Stream keys: (0,) dictionary, (1, c) structure of chunk
c, (2, c) weights of chunk c, (3, c) noise of chunk c, (4,) image sizes,
(5, i) stamps of image i, (6, i) noise of image i, (7,) request arrivals,
(8,) request image sides, (9, i) stamps of request i.
Patch streams are cut in chunks of ``CHUNK`` patches.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

CHUNK = 65536


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(seed, spawn_key=tuple(key)))


@dataclasses.dataclass(frozen=True)
class Geometry:
    """Patch side N (odd), radial profiles S, largest harmonic T."""

    N: int
    S: int
    T: int

    @property
    def B(self) -> int:
        """Packed real hat dimension: S profiles times harmonics -T..T."""
        return self.S * (2 * self.T + 1)


GEOM11 = Geometry(11, 5, 5)
GEOM15 = Geometry(15, 7, 7)


def draw_dictionary(M: int, B: int, seed: int = 0) -> np.ndarray:
    """M atoms with i.i.d. N(0,1) packed hat coordinates, each scaled to unit norm.

    Returns float64 [M, B]; callers cast to float32 for the device.
    """
    d = _rng(seed, 0).standard_normal((M, B))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


@dataclasses.dataclass
class PatchDraw:
    """Random content of P patches, each a weighted sum of up to J rotated atoms plus noise.

    atom[p, i], angle[p, i] (radians, counter-clockwise) and weight[p, i] describe
    the i-th term of patch p; unused terms have weight 0.  noise is [P, N, N].
    angle_index is set when the angles are on a grid 2*pi*r/R.
    """

    atom: np.ndarray
    angle: np.ndarray
    weight: np.ndarray
    noise: np.ndarray
    angle_index: np.ndarray | None = None


def _chunks(start: int, count: int):
    """Yield (chunk id, lo, hi) intersecting [start, start+count) in CHUNK units."""
    end = start + count
    c = start // CHUNK
    while c * CHUNK < end:
        lo = max(start, c * CHUNK)
        hi = min(end, (c + 1) * CHUNK)
        yield c, lo - c * CHUNK, hi - c * CHUNK
        c += 1


def draw_pairs_on_grid(P: int, N: int, M: int, R: int, sigma: float,
                       seed: int = 0, start: int = 0, distinct: bool = True) -> PatchDraw:
    """Two (atom, grid angle) terms per patch with N(0,1) weights and N(0, sigma^2) noise.

    The two columns are drawn uniformly over the M*R (atom, angle) pairs, without
    replacement when ``distinct`` (the small plain workload).
    """
    atom = np.empty((P, 2), np.int64)
    ridx = np.empty((P, 2), np.int64)
    weight = np.empty((P, 2))
    noise = np.empty((P, N, N))
    out = 0
    for c, lo, hi in _chunks(start, P):
        n = CHUNK
        rs = _rng(seed, 1, c)
        j1 = rs.integers(0, M * R, n)
        if distinct:
            j2 = rs.integers(0, M * R - 1, n)
            j2 = j2 + (j2 >= j1)
        else:
            j2 = rs.integers(0, M * R, n)
        w = _rng(seed, 2, c).standard_normal((n, 2))
        k = hi - lo
        atom[out:out + k, 0] = (j1 % M)[lo:hi]
        atom[out:out + k, 1] = (j2 % M)[lo:hi]
        ridx[out:out + k, 0] = (j1 // M)[lo:hi]
        ridx[out:out + k, 1] = (j2 // M)[lo:hi]
        weight[out:out + k] = w[lo:hi]
        noise[out:out + k] = sigma * _rng(seed, 3, c).standard_normal((n, N, N))[lo:hi]
        out += k
    return PatchDraw(atom, 2 * np.pi * ridx / R, weight, noise, angle_index=ridx)


def draw_mixtures(P: int, N: int, M: int, J: int, sigma: float,
                  seed: int = 0, start: int = 0) -> PatchDraw:
    """1..J atoms per patch (count uniform), atoms uniform with replacement,
    continuous angles U[0, 2*pi), Laplace(0, 1) weights, N(0, sigma^2) noise."""
    atom = np.zeros((P, J), np.int64)
    angle = np.zeros((P, J))
    weight = np.zeros((P, J))
    noise = np.empty((P, N, N))
    out = 0
    for c, lo, hi in _chunks(start, P):
        n = CHUNK
        rs = _rng(seed, 1, c)
        count = rs.integers(1, J + 1, n)
        a = rs.integers(0, M, (n, J))
        th = rs.uniform(0.0, 2 * np.pi, (n, J))
        w = _rng(seed, 2, c).laplace(0.0, 1.0, (n, J))
        w = np.where(np.arange(J)[None, :] < count[:, None], w, 0.0)
        k = hi - lo
        atom[out:out + k] = a[lo:hi]
        angle[out:out + k] = th[lo:hi]
        weight[out:out + k] = w[lo:hi]
        noise[out:out + k] = sigma * _rng(seed, 3, c).standard_normal((n, N, N))[lo:hi]
        out += k
    return PatchDraw(atom, angle, weight, noise)


@dataclasses.dataclass
class ImageDraw:
    """One texture image: H x W, Poisson stamp centres (row, col), atoms, angles,
    amplitudes, and N(0, sigma^2) pixel noise [H, W]."""

    H: int
    W: int
    centre: np.ndarray
    atom: np.ndarray
    angle: np.ndarray
    amplitude: np.ndarray
    noise: np.ndarray


def draw_image_sizes(n: int, lo: int, hi: int, square: bool, seed: int = 0) -> np.ndarray:
    """[n, 2] (H, W) log-uniform on [lo, hi], rounded; H == W when ``square``."""
    rs = _rng(seed, 4)
    u = rs.uniform(math.log(lo), math.log(hi), (n, 1 if square else 2))
    s = np.rint(np.exp(u)).astype(np.int64).clip(lo, hi)
    return np.repeat(s, 2, axis=1) if square else s


def draw_image(i: int, H: int, W: int, M: int, density: float, sigma: float,
               seed: int = 0) -> ImageDraw:
    """Stamp process for image i: Poisson(density * H * W) stamps with integer centres
    uniform over the image, atom uniform over M, angle U[0, 2*pi), N(0,1) amplitude."""
    rs = _rng(seed, 5, i)
    n = rs.poisson(density * H * W)
    centre = np.stack([rs.integers(0, H, n), rs.integers(0, W, n)], axis=1)
    atom = rs.integers(0, M, n)
    angle = rs.uniform(0.0, 2 * np.pi, n)
    amplitude = rs.standard_normal(n)
    noise = sigma * _rng(seed, 6, i).standard_normal((H, W))
    return ImageDraw(H, W, centre, atom, angle, amplitude, noise)


def draw_arrivals(rate: float, duration: float, seed: int = 0) -> np.ndarray:
    """Open-loop Poisson arrival times (seconds) on [0, duration)."""
    rs = _rng(seed, 7)
    gaps = rs.exponential(1.0 / rate, int(rate * duration * 2 + 64))
    t = np.cumsum(gaps)
    return t[t < duration]


# Concrete workloads.  Small plain: 2,000 11x11 patches, 16 atoms, K=2, R=32.
# At scale: 1,000,000 11x11 patches, 64 atoms, K=4, R=64.
SMALL = dict(name="small-fp32", geom=GEOM11, P=2000, M=16, K=2, R=32, sigma=0.01)
SCALE = dict(name="scale-fp32", geom=GEOM11, P=1_000_000, M=64, K=4, R=64, sigma=0.05, J=4)
RAGGED = dict(name="ragged-images", geom=GEOM15, n_images=256, side=(64, 1024), M=128,
              K=6, R=64, density=0.02, sigma=0.05)
SERVING = dict(name="serving", geom=GEOM15, rate=200.0, duration=30.0, side=(32, 2048),
               M=128, K=6, R=64, density=0.02, sigma=0.05)


# Texture classification (Sec. III-B, "Classifier"; synthetic stand-in for the paper's
# 24-class rotated texture set): C classes of stationary band-pass Gaussian fields (six
# centre frequencies x isotropic / oriented x narrow / wide band); 128 x 128 images, 20
# upright training images and 20 test images per class at each of 8 rotations; the
# R-K-SVD parameters selected in the paper (M = 100, N = 15, K = 1), R = 64; 4,000
# training windows per image.
TEXTURE = dict(name="texture", geom=GEOM15, C=24, M=100, K=1, R=64, side=128, n_train=20, n_test=20,
               test_rot_deg=(5, 10, 15, 30, 45, 60, 75, 90), sigma=0.05, train_windows=4000, n_iter=10,
               freqs=(0.06, 0.09, 0.12, 0.16, 0.2, 0.25), anisotropy=0.9, bands=(0.02, 0.05))


def texture_params(c: int, seed: int = 0, w: dict | None = None):
    """(centre frequency in cycles/pixel, anisotropy, bandwidth, orientation) of class c:
    frequency cycles with c, every other group of six classes is oriented, the second
    half of the classes is wide-band; orientation U[0, pi)."""
    w = TEXTURE if w is None else w
    f = w["freqs"][c % len(w["freqs"])]
    aniso = w["anisotropy"] if (c // len(w["freqs"])) % 2 else 0.0
    bw = w["bands"][0] if c < w["C"] // 2 else w["bands"][1]
    return f, aniso, bw, float(_rng(seed, 14, c).uniform(0.0, np.pi))


def draw_texture_image(c: int, i: int, side: int, sigma: float, rot: float = 0.0, seed: int = 0,
                       w: dict | None = None) -> np.ndarray:
    """Image i of class c as it appears turned by rot radians (counter-clockwise): white
    noise filtered by exp(-(|f| - f_c)^2 / (2 b^2)) (1 + a cos 2(phi - theta_c - rot)) on a
    grid with 64 pixels of margin (so the periodic filtering does not wrap into the
    image), cropped, scaled to unit variance, plus N(0, sigma^2) noise.  float64 [side, side]."""
    f0, a, bw, th = texture_params(c, seed, w)
    n = side + 64
    rs = _rng(seed, 12, c, i)
    white = rs.standard_normal((n, n))
    fy = np.fft.fftfreq(n)[:, None]
    fx = np.fft.fftfreq(n)[None, :]
    fr = np.hypot(fx, fy)
    ph = np.arctan2(fy, fx)
    H = np.exp(-((fr - f0) ** 2) / (2 * bw * bw)) * (1.0 + a * np.cos(2.0 * (ph - th - rot)))
    x = np.real(np.fft.ifft2(np.fft.fft2(white) * H))[:side, :side]
    x = x / x.std()
    return x + sigma * _rng(seed, 13, c, i).standard_normal((side, side))


def small_draw(P: int | None = None, start: int = 0, seed: int = 0) -> tuple[np.ndarray, PatchDraw]:
    w = SMALL
    g = w["geom"]
    D = draw_dictionary(w["M"], g.B, seed)
    return D, draw_pairs_on_grid(w["P"] if P is None else P, g.N, w["M"], w["R"],
                                 w["sigma"], seed, start)


def scale_draw(P: int | None = None, start: int = 0, seed: int = 0) -> tuple[np.ndarray, PatchDraw]:
    w = SCALE
    g = w["geom"]
    D = draw_dictionary(w["M"], g.B, seed)
    return D, draw_mixtures(w["P"] if P is None else P, g.N, w["M"], w["J"],
                            w["sigma"], seed, start)


def ragged_draws(n_images: int | None = None, first: int = 0, seed: int = 0,
                 square: bool = False, side=None, M: int | None = None):
    """Stamp draws of the ragged image batch: sizes log-uniform on the side range (H and W
    drawn independently unless ``square``), then each image's stamp process."""
    w = RAGGED
    lo, hi = side or w["side"]
    n_all = w["n_images"] if n_images is None else first + n_images
    sizes = draw_image_sizes(n_all, lo, hi, square, seed)
    M = w["M"] if M is None else M
    return [draw_image(i, int(sizes[i, 0]), int(sizes[i, 1]), M, w["density"], w["sigma"], seed)
            for i in range(first, n_all)]


def serving_trace(duration: float | None = None, rate: float | None = None, seed: int = 0):
    """Open-loop request trace: Poisson arrival times (s) and square image sides,
    log-uniform on the serving side range."""
    w = SERVING
    t = draw_arrivals(w["rate"] if rate is None else rate, w["duration"] if duration is None else duration, seed)
    lo, hi = w["side"]
    rs = _rng(seed, 8)
    side = np.rint(np.exp(rs.uniform(math.log(lo), math.log(hi), t.size))).astype(np.int64).clip(lo, hi)
    return t, side


def request_stamps(i: int, H: int, W: int, M: int, density: float, seed: int = 0):
    """Stamp process of request i (centres, atoms, angles, amplitudes), as draw_image but
    without the pixel noise, which the serving benchmark draws on the device."""
    rs = _rng(seed, 9, i)
    n = rs.poisson(density * H * W)
    centre = np.stack([rs.integers(0, H, n), rs.integers(0, W, n)], axis=1)
    return centre, rs.integers(0, M, n), rs.uniform(0.0, 2 * np.pi, n), rs.standard_normal(n)
