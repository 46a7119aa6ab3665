"""Pins of the reference R-K-SVD update in the paper's annular basis (Fig. 2, Sec. II-C, run in
the steerable basis' coordinates as Sec. II-E does), at N = 11 (B = 81) and 15 (B = 153), CPU
only.

The update is the grid's (rksvd_update) with the annular layout's steering: harmonic k of each
annulus that carries it turned by exp(-i k theta).  Pinned here, as for the grid, by things
other than its own code: exact recovery of a single rotated atom, an independent assembly of
each atom's covariance through the residual identity x - D b = r + c S_r0 d (checked by power
iteration), invariance to rotating every patch, agreement with the grid form where the two
layouts coincide (R = 1 turns nothing), and a planted wrong upright direction.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc


@pytest.fixture(scope="module", params=[11, 15])
def ab(request):
    return orc.build_annular_basis(request.param)


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _toy(ab, P, M, K, R, seed):
    rng = np.random.default_rng(seed)
    D = _unit(rng.standard_normal((M, ab.B)))
    atoms = rng.integers(0, M, (P, K))
    angles = rng.integers(0, R, (P, K))
    w = rng.standard_normal((P, K))
    X = np.stack([sum(w[p, j] * orc.steer_ragged(D[atoms[p, j]], 2 * np.pi * angles[p, j] / R, ab.Sk)
                      for j in range(K)) for p in range(P)])
    return D, X


def _best_rotation_corr(ab, d, ref, R):
    return max(abs(orc.steer_ragged(d, 2 * np.pi * k / R, ab.Sk) @ ref) for k in range(R))


def test_single_rotated_atom_is_recovered_exactly(ab):
    """Patches c_p S_{r_p} d: one update from a random start returns d up to a grid rotation,
    and the next pursuit codes every patch exactly."""
    R = 32
    d, X = _toy(ab, 300, 1, 1, R, seed=1)
    D0 = _unit(np.random.default_rng(100).standard_normal((1, ab.B)))
    D, code, hist = orc.rksvd_basis(ab, D0, R, X, 1, 1)
    assert 1 - _best_rotation_corr(ab, D[0], d[0], R) < 1e-12
    assert hist[-1] < 1e-20 * hist[0]


def _covariance_via_residuals(ab, D, R, X, code, m):
    C = np.zeros((ab.B, ab.B))
    n = 0
    recon = orc.code_to_hat_basis(ab, D, R, code)
    for p in range(X.shape[0]):
        slots = np.flatnonzero(code.atom[p] == m)
        if slots.size == 0:
            continue
        i0 = slots[0]
        y = orc.steer_ragged(X[p] - recon[p], -2 * np.pi * code.angle[p, i0] / R, ab.Sk) + code.coef[p, i0] * D[m]
        C += np.outer(y, y)
        n += 1
    return C, n


def _power_top(C, iters=5000):
    v = np.ones(C.shape[0]) / np.sqrt(C.shape[0])
    for _ in range(iters):
        v = C @ v
        v /= np.linalg.norm(v)
    return v, float(v @ C @ v)


def test_update_is_top_eigenvector_of_independently_assembled_covariance(ab):
    R, M, K = 16, 4, 3
    D_true, X = _toy(ab, 250, M, K, R, seed=3)
    X += 0.05 * np.random.default_rng(3).standard_normal(X.shape)
    D = _unit(D_true + 0.3 * np.random.default_rng(4).standard_normal(D_true.shape))
    code = orc.omp(orc.augmented_dictionary_basis(ab, D, R), X, K, M)
    D_new, usage, reset = orc.rksvd_update_basis(ab, D, R, X, code)
    for m in range(M):
        C, n = _covariance_via_residuals(ab, D, R, X, code, m)
        assert usage[m] == n
        if n == 0:
            continue
        v, lam = _power_top(C)
        ev = np.linalg.eigvalsh(C)
        assert ev[-1] - ev[-2] > 1e-3 * ev[-1]
        assert abs(D_new[m] @ v) > 1 - 1e-9
        assert D_new[m] @ D[m] > 0                         # sign rule
    assert np.all(reset == -1)


def test_invariant_to_rotating_every_patch(ab):
    R, M, K = 16, 3, 2
    D_true, X = _toy(ab, 120, M, K, R, seed=5)
    D = _unit(D_true + 0.2 * np.random.default_rng(6).standard_normal(D_true.shape))
    code = orc.omp(orc.augmented_dictionary_basis(ab, D, R), X, K, M)
    ref, _, _ = orc.rksvd_update_basis(ab, D, R, X, code)
    r0 = 5
    Xr = orc.steer_ragged(X, 2 * np.pi * r0 / R, ab.Sk)
    code_r = orc.Code(code.atom, np.where(code.atom >= 0, (code.angle + r0) % R, -1), code.coef,
                      code.resid2, code.corr, code.gap)
    got, _, _ = orc.rksvd_update_basis(ab, D, R, Xr, code_r)
    assert np.abs(got - ref).max() < 1e-12


def test_R1_matches_the_layout_free_form(ab):
    """With R = 1 nothing is turned, so the update does not depend on the layout: it equals
    the grid routine run on the same coordinates (any S, T with S (2T + 1) = B would do;
    B = 81 = 27 x 3 is read as S = 27, T = 1, and B = 153 = 51 x 3 as S = 51, T = 1)."""
    R, M, K = 1, 5, 2
    D_true, X = _toy(ab, 200, M, K, R, seed=9)
    D = _unit(D_true + 0.2 * np.random.default_rng(10).standard_normal(D_true.shape))
    code = orc.omp(orc.augmented_dictionary_basis(ab, D, R), X, K, M)
    a, ua, ra = orc.rksvd_update_basis(ab, D, R, X, code)
    b, ub, rb = orc.rksvd_update(D, R, ab.B // 3, 1, X, code)
    assert np.abs(a - b).max() < 1e-12 and np.array_equal(ua, ub) and np.array_equal(ra, rb)


def test_planted_wrong_upright_direction_is_caught(ab, monkeypatch):
    """Turning the residuals by +r0 instead of -r0 must change the atoms."""
    R, M, K = 16, 3, 2
    D_true, X = _toy(ab, 150, M, K, R, seed=11)
    D = _unit(D_true + 0.2 * np.random.default_rng(12).standard_normal(D_true.shape))
    code = orc.omp(orc.augmented_dictionary_basis(ab, D, R), X, K, M)
    ref, _, _ = orc.rksvd_update_basis(ab, D, R, X, code)
    real = orc.steer_ragged
    monkeypatch.setattr(orc, "steer_ragged", lambda x, th, Sk: real(x, -np.asarray(th), Sk))
    wrong, _, _ = orc.rksvd_update_basis(ab, D, R, X, code)
    assert np.abs(wrong - ref).max() > 1e-3
