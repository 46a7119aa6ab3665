"""Pins of the reference pursuit on the paper's annular basis (eq. (5)-(8), Sec. II-D,
Sec. II-E step 3), CPU only.

The annular basis keeps harmonic k only on the annuli whose cut-off T_s reaches k, so its
packed coordinates are ragged: Sk[k] annuli per harmonic.  The pursuit is the same OMP over
[S_0 D, ..., S_{R-1} D] with the steering of that layout.  Pinned here:

* the factored correlation: per-harmonic complex inner products C_k followed by the angle
  DFT (eq. (8): harmonic k turns by exp(-i k theta)) equal the dense augmented dictionary's
  product, and the steering keeps its group law and norms (P4);
* the first selection is the brute-force best single column (P6); with R = 1 the pursuit
  is scikit-learn's OMP (P5); single rotated atoms are recovered exactly (P9);
* rotating a patch inside the span by r0 grid steps shifts every selected angle by r0
  (eq. (3), P10);
* planted slips of the layout (Re and Im interleaved per annulus, a harmonic off by one)
  fail the factorisation.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc


@pytest.fixture(scope="module", params=[11, 15])
def ab(request):
    return orc.build_annular_basis(request.param)


def _harmonic_blocks(Sk):
    """(k, Re slice, Im slice) of each harmonic k >= 1 in the packed layout."""
    out, off = [], Sk[0]
    for k in range(1, len(Sk)):
        n = Sk[k]
        out.append((k, slice(off, off + n), slice(off + n, off + 2 * n)))
        off += 2 * n
    return out


def _factored_correlation(Sk, d, x, R):
    """<S_r d, x> for r = 0..R-1 from C_0 = <d_0, x_0> and C_k = sum conj(d_k) x_k (complex
    coefficients Re + i Im of harmonic k), then Re(exp(i k theta) C_k) summed over k."""
    c = np.full(R, float(d[: Sk[0]] @ x[: Sk[0]]))
    th = 2 * np.pi * np.arange(R) / R
    for k, re, im in _harmonic_blocks(Sk):
        Ck = np.sum(np.conj(d[re] + 1j * d[im]) * (x[re] + 1j * x[im]))
        c += np.cos(k * th) * Ck.real - np.sin(k * th) * Ck.imag
    return c


def _dictionary(ab, M, seed):
    rng = np.random.default_rng(seed)
    D = rng.standard_normal((M, ab.B))
    return D / np.linalg.norm(D, axis=1, keepdims=True)


def test_sk_layout_sums_to_B(ab):
    assert ab.Sk[0] + 2 * sum(ab.Sk[1:]) == ab.B
    assert ab.Sk == sorted(ab.Sk, reverse=True)          # annuli drop out as k grows
    assert ab.B == (81 if ab.N == 11 else 153)


def test_p4_factored_correlation_on_ragged_layout(ab):
    M, R = 5, 24
    D = _dictionary(ab, M, 1)
    x = np.random.default_rng(2).standard_normal(ab.B)
    Da = orc.augmented_dictionary_basis(ab, D, R)
    dense = (Da @ x).reshape(R, M)
    for m in range(M):
        assert np.abs(dense[:, m] - _factored_correlation(ab.Sk, D[m], x, R)).max() < 1e-12


def test_p4_group_law_and_orthogonality(ab):
    x = np.random.default_rng(3).standard_normal((4, ab.B))
    a, b = 0.7, -2.3
    two = orc.steer_ragged(orc.steer_ragged(x, a, ab.Sk), b, ab.Sk)
    assert np.abs(two - orc.steer_ragged(x, a + b, ab.Sk)).max() < 1e-12
    assert np.abs(np.linalg.norm(orc.steer_ragged(x, a, ab.Sk), axis=1) - np.linalg.norm(x, axis=1)).max() < 1e-12
    # a full turn is the identity, and each row of the augmented dictionary has unit norm
    assert np.abs(orc.steer_ragged(x, 2 * np.pi, ab.Sk) - x).max() < 1e-12
    Da = orc.augmented_dictionary_basis(ab, _dictionary(ab, 3, 4), 16)
    assert np.abs(np.linalg.norm(Da, axis=1) - 1).max() < 1e-12


def _steer_interleaved(x, theta, Sk):
    """A plausible slip: harmonic k's coordinates read as (Re, Im) pairs per annulus instead
    of a Re block then an Im block."""
    out = np.array(x, dtype=float)
    off = Sk[0]
    for k in range(1, len(Sk)):
        n = Sk[k]
        blk = out[..., off:off + 2 * n]
        z = (blk[..., 0::2] + 1j * blk[..., 1::2]) * np.exp(-1j * k * theta)
        blk[..., 0::2], blk[..., 1::2] = z.real, z.imag
        off += 2 * n
    return out


def _steer_shifted(x, theta, Sk):
    """Another slip: block k turned as harmonic k + 1."""
    return _steer_with(x, theta, Sk, lambda k: k + 1)


def _steer_with(x, theta, Sk, harm):
    out = np.array(x, dtype=float)
    for k, re, im in _harmonic_blocks(Sk):
        z = (out[..., re] + 1j * out[..., im]) * np.exp(-1j * harm(k) * theta)
        out[..., re], out[..., im] = z.real, z.imag
    return out


@pytest.mark.parametrize("slip", [_steer_interleaved, _steer_shifted])
def test_planted_layout_slips_are_caught(ab, slip):
    M, R = 3, 8
    D = _dictionary(ab, M, 5)
    x = np.random.default_rng(6).standard_normal(ab.B)
    wrong = np.concatenate([slip(D, 2 * np.pi * r / R, ab.Sk) for r in range(R)])
    dense = (wrong @ x).reshape(R, M)
    err = max(np.abs(dense[:, m] - _factored_correlation(ab.Sk, D[m], x, R)).max() for m in range(M))
    assert err > 1e-3
    # the correct layout through the same helper passes
    right = np.concatenate([_steer_with(D, 2 * np.pi * r / R, ab.Sk, lambda k: k) for r in range(R)])
    assert np.abs((right @ x).reshape(R, M) - (orc.augmented_dictionary_basis(ab, D, R) @ x).reshape(R, M)).max() < 1e-12


def test_p6_first_step_is_brute_force_best_column(ab):
    M, R = 6, 16
    D = _dictionary(ab, M, 7)
    X = np.random.default_rng(8).standard_normal((20, ab.B))
    Da = orc.augmented_dictionary_basis(ab, D, R)
    code = orc.omp(Da, X, 1, M)
    for p in range(len(X)):
        errs = [np.sum((X[p] - Da[j] * (Da[j] @ X[p])) ** 2) for j in range(M * R)]
        j = int(np.argmin(errs))
        assert (code.atom[p, 0], code.angle[p, 0]) == (j % M, j // M)


def test_p5_single_angle_is_textbook_omp(ab):
    from sklearn.linear_model import orthogonal_mp
    M, K = 12, 3
    D = _dictionary(ab, M, 9)
    X = np.random.default_rng(10).standard_normal((15, ab.B))
    code = orc.omp(orc.augmented_dictionary_basis(ab, D, 1), X, K, M)
    ref = orthogonal_mp(D.T, X.T, n_nonzero_coefs=K).T
    for p in range(len(X)):
        mine = np.zeros(M)
        mine[code.atom[p]] = code.coef[p]
        assert set(np.flatnonzero(mine)) == set(np.flatnonzero(ref[p]))
        assert np.abs(mine - ref[p]).max() < 1e-10


def test_p9_single_rotated_atoms_recovered_exactly(ab):
    M, R = 8, 32
    D = _dictionary(ab, M, 11)
    rng = np.random.default_rng(12)
    m = rng.integers(0, M, 30)
    r = rng.integers(0, R, 30)
    w = rng.uniform(0.5, 2, 30) * rng.choice([-1, 1], 30)
    X = orc.synthesize(ab, D, m[:, None], 2 * np.pi * r[:, None] / R, w[:, None])
    xh, code = orc.encode(ab, D, R, X, 2)
    assert np.array_equal(code.atom[:, 0], m) and np.array_equal(code.angle[:, 0], r)
    assert np.abs(code.coef[:, 0] - w).max() < 1e-10
    assert np.all(code.atom[:, 1] == -1)                   # residual below tau: stop
    rec = orc.reconstruct(ab, D, R, code)
    assert np.abs(rec - X).max() < 1e-10 * np.abs(X).max()


def test_p10_equivariance_in_span(ab):
    M, R, K = 8, 32, 2
    D = _dictionary(ab, M, 13)
    X = np.random.default_rng(14).standard_normal((40, ab.N, ab.N))
    xh, base = orc.encode(ab, D, R, X, K)
    Da = orc.augmented_dictionary_basis(ab, D, R)
    for r0 in (1, 8, 13):
        xr = orc.steer_ragged(xh, 2 * np.pi * r0 / R, ab.Sk)
        rot = orc.omp(Da, xr, K, M)
        for p in range(len(X)):
            if base.gap[p][base.atom[p] >= 0].min() < 1e-9:
                continue
            s0 = {(a, (g + r0) % R) for a, g in zip(base.atom[p], base.angle[p]) if a >= 0}
            s1 = {(a, g) for a, g in zip(rot.atom[p], rot.angle[p]) if a >= 0}
            assert s0 == s1
            assert np.abs(np.sort(rot.coef[p]) - np.sort(base.coef[p])).max() < 1e-10
