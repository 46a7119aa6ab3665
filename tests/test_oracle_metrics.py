"""Pins of the reference's error measures and of its tie rule, CPU only.

* ``mse``: the matched MSE of the metric (Sec. III-A: mean over patches and disk pixels
  of the squared coding error).  Pinned by a plain enumeration of the disk with the
  integer test of the 97-pixel count (4 (x^2 + y^2) < N^2) and by closed cases.
* ``span_error``: the lower bound of Sec. III-A, the distance of a patch to span(Phi)
  on the disk.  Pinned by Pythagoras with the orthogonal complement of span(Phi) taken
  from an SVD (not from the projection the reference uses).
* The tie rule of the pursuit: exact ties go to the smallest atom, then the smallest
  angle.  Pinned on the selection helper and through the pursuit on an augmented
  dictionary with planted duplicate columns.

The planted mistakes show that plausible slips (averaging over all N^2 pixels,
counting off-disk pixels, dropping the Gram inverse, angle-first ties) fail a pin.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc


@pytest.fixture(scope="module")
def b11():
    return orc.build_basis(11, 5, 5)


@pytest.fixture(scope="module")
def b15():
    return orc.build_basis(15, 7, 7)


def _disk_pixels(N):
    c = (N - 1) // 2
    return [(i, j) for i in range(N) for j in range(N) if 4 * ((i - c) ** 2 + (j - c) ** 2) < N * N]


def _mse_by_enumeration(N, patches, recon):
    pix = _disk_pixels(N)
    tot, cnt = 0.0, 0
    for p in range(len(patches)):
        for i, j in pix:
            d = float(patches[p][i][j]) - float(recon[p][i][j])
            tot += d * d
            cnt += 1
    return tot / cnt if cnt else 0.0


def _mse_pin_error(mse_fn, basis):
    """Largest deviation of mse_fn from the enumerated and closed-form values."""
    N = basis.N
    rng = np.random.default_rng(21)
    errs = []
    X = rng.standard_normal((7, N, N))
    Y = rng.standard_normal((7, N, N))
    ref = _mse_by_enumeration(N, X, Y)
    errs.append(abs(mse_fn(basis, X, Y) - ref) / ref)
    # zero code: the mean of the squared disk pixels; the disk indicator gives exactly 1
    ind = np.zeros((1, N, N))
    for i, j in _disk_pixels(N):
        ind[0, i, j] = 1.0
    errs.append(abs(mse_fn(basis, ind, np.zeros_like(ind)) - 1.0))
    # content only off the disk: no error at all
    off = (1.0 - ind) * 3.0
    errs.append(abs(mse_fn(basis, off, np.zeros_like(off))))
    # per-patch averaging: two disk-constant patches a and b give (a^2 + b^2) / 2
    two = np.concatenate([2.0 * ind, -3.0 * ind])
    errs.append(abs(mse_fn(basis, two, np.zeros_like(two)) - 6.5))
    return max(errs)


def test_mse_equals_disk_enumeration_and_closed_cases(b11, b15):
    assert _mse_pin_error(orc.mse, b11) < 1e-12
    assert _mse_pin_error(orc.mse, b15) < 1e-12
    assert orc.mse(b11, np.zeros((0, 11, 11)), np.zeros((0, 11, 11))) == 0.0


def test_planted_mse_over_all_grid_pixels_is_caught(b11):
    def mse_grid(basis, patches, recon):
        d = np.asarray(patches, np.float64) - recon
        return float(np.mean(d * d))
    assert _mse_pin_error(mse_grid, b11) > 0.1          # 97/121 instead of 1, off-disk counted


def test_planted_mse_divided_by_grid_size_is_caught(b11):
    def mse_n2(basis, patches, recon):
        d = (np.asarray(patches, np.float64) - recon)[:, basis.mask]
        return float(np.sum(d * d) / (len(d) * basis.N ** 2))
    assert _mse_pin_error(mse_n2, b11) > 0.1


# ----------------------------------------------------------------------------- span error
def _complement(basis):
    """Orthonormal basis of the disk-pixel vectors orthogonal to span(Phi), from an SVD."""
    U, s, _ = np.linalg.svd(basis.phi, full_matrices=True)
    assert s.min() > 1e-8 * s.max()
    return U[:, basis.B:]


def _span_pin_error(span_fn, basis):
    rng = np.random.default_rng(22)
    N, mask = basis.N, basis.mask.ravel()
    Uc = _complement(basis)
    P = 6
    v = rng.standard_normal((P, basis.B))
    w = rng.standard_normal((P, Uc.shape[1])) @ Uc.T           # [P, n_pix], orthogonal to span
    X = np.zeros((P, N * N))
    X[:, mask] = v @ basis.phi.T + w
    X[:, ~mask] = rng.standard_normal((P, int((~mask).sum())))  # off-disk pixels are ignored
    X = X.reshape(P, N, N)
    expect = float(np.sum(w * w) / (P * basis.n_pix))
    e1 = abs(span_fn(basis, X) - expect) / expect
    inside = np.zeros((P, N * N))
    inside[:, mask] = v @ basis.phi.T
    e2 = abs(span_fn(basis, inside.reshape(P, N, N)))             # in the span: 0
    return max(e1, e2 / expect)


def test_span_error_is_the_distance_to_the_span(b11, b15):
    assert _span_pin_error(orc.span_error, b11) < 1e-10
    assert _span_pin_error(orc.span_error, b15) < 1e-10


def test_span_error_bounds_every_code(b11):
    """No code can beat the span: MSE of any pursuit >= span error (Sec. III-A)."""
    rng = np.random.default_rng(23)
    D = rng.standard_normal((8, b11.B))
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    X = rng.standard_normal((20, 11, 11))
    _, code = orc.encode(b11, D, 16, X, 3)
    rec = orc.reconstruct(b11, D, 16, code)
    assert orc.mse(b11, X, rec) >= orc.span_error(b11, X) * (1 - 1e-12)


def test_planted_span_error_without_gram_inverse_is_caught(b11):
    def span_no_gram(basis, patches):
        Xd = np.asarray(patches, np.float64).reshape(len(patches), -1)[:, basis.mask.ravel()]
        xhat = Xd @ basis.phi                                     # Phi^T x, no (Phi^T Phi)^{-1}
        return orc.mse(basis, patches, orc.to_pixels(basis, xhat))
    assert _span_pin_error(span_no_gram, b11) > 0.1


# ----------------------------------------------------------------------------- tie rule
def _pick_ref(absc, M):
    """The tie rule stated plainly: among the largest |c|, smallest atom, then smallest angle."""
    best = max(absc)
    tied = [(j % M, j // M) for j, v in enumerate(absc) if v == best]
    m, r = min(tied)
    return r * M + m


@pytest.mark.parametrize("ties", [
    [(1, 0), (0, 2)],            # atom first: (0, 2) beats (1, 0) although its angle is larger
    [(2, 1), (2, 3)],            # same atom: smaller angle
    [(3, 0), (1, 5), (1, 6)],
    [(0, 7)],
])
def test_tie_rule_atom_then_angle(ties):
    M, R = 4, 8
    absc = np.linspace(0.1, 0.5, M * R)
    for m, r in ties:
        absc[r * M + m] = 2.0
    j = orc._pick(absc, M)
    assert j == _pick_ref(list(absc), M)
    assert (j % M, j // M) == min(ties)


def test_tie_rule_through_the_pursuit():
    """Duplicate columns (m=1, r=0) and (m=0, r=2) of an augmented dictionary: the patch
    equal to that column is coded by (0, 2), the smaller atom."""
    rng = np.random.default_rng(24)
    M, R, B = 3, 4, 12
    Da = rng.standard_normal((M * R, B))
    Da /= np.linalg.norm(Da, axis=1, keepdims=True)
    Da[0 * M + 1] = Da[2 * M + 0]
    x = 1.5 * Da[2 * M + 0][None, :]
    code = orc.omp(Da, x, 1, M)
    assert (code.atom[0, 0], code.angle[0, 0]) == (0, 2)
    assert abs(code.coef[0, 0] - 1.5) < 1e-12


def test_planted_angle_first_tie_rule_is_caught():
    M, R = 4, 8
    absc = np.zeros(M * R)
    absc[0 * M + 1] = absc[2 * M + 0] = 1.0
    angle_first = int(np.flatnonzero(absc == absc.max())[0])     # smallest j = r M + m
    assert angle_first != _pick_ref(list(absc), M)


# ----------------------------------------------------------------------------- parity helper
def test_parity_floor_for_coefficients_tiny_against_their_patch():
    """The coefficient check of the device tests: 1e-4 relative, floored at 1e-3 of the
    largest coefficient and, when given, at 1e-2 of the patch's coordinate norm."""
    from tests.parity import compare_codes
    ref = orc.Code(np.array([[0, -1], [1, 2]]), np.array([[3, -1], [0, 5]]),
                   np.array([[8e-4, 0.0], [1.0, 0.5]]), np.zeros(2), np.zeros((2, 2)), np.zeros((2, 2)))
    atom, angle = ref.atom.copy(), ref.angle.copy()
    coef = ref.coef.copy()
    coef[0, 0] += 3e-7                                  # 3.75e-4 of itself, 2e-7 of ||x_hat|| = 1.4
    assert compare_codes(atom, angle, coef, ref).coef_bad == 1
    assert compare_codes(atom, angle, coef, ref, xnorm=np.array([1.4, 1.2])).coef_bad == 0
    coef[1, 1] += 1e-4                                  # 2e-4 relative on a coefficient of 0.5
    assert compare_codes(atom, angle, coef, ref, xnorm=np.array([1.4, 1.2])).coef_bad == 1
    coef[0, 0] += 3e-5                                  # now 2e-5 of ||x_hat||: beyond the floor
    assert compare_codes(atom, angle, coef, ref, xnorm=np.array([1.4, 1.2])).coef_bad == 2
