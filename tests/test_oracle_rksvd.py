"""Pins of the reference R-K-SVD dictionary update (Fig. 2, Sec. II-C), CPU only.

Each test fixes the update by something other than its own code: exact recovery
where the answer is known in closed form, an independent assembly of the
per-atom covariance (through the residual identity x - D b = r + c S_r0 d) checked
by power iteration, invariances, the matrix-form K-SVD update for R = 1, the
reset rule, and planted mistakes that must be caught.
"""
import numpy as np
import pytest

from oracle import rsc_oracle as orc

S, T = 5, 5
B = S * (2 * T + 1)


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _best_rotation_corr(d, ref, R):
    return max(abs(orc.steer(d, 2 * np.pi * k / R, S, T) @ ref) for k in range(R))


def _toy(P, M, K, R, seed, weights="normal"):
    rng = np.random.default_rng(seed)
    D = _unit(rng.standard_normal((M, B)))
    atoms = rng.integers(0, M, (P, K))
    angles = rng.integers(0, R, (P, K))
    if weights == "normal":
        w = rng.standard_normal((P, K))
    else:
        w = rng.uniform(0.5, 1.5, (P, K)) * rng.choice([-1.0, 1.0], (P, K))
    X = np.stack([sum(w[p, j] * orc.steer(D[atoms[p, j]], 2 * np.pi * angles[p, j] / R, S, T)
                      for j in range(K)) for p in range(P)])
    return D, X


def test_single_rotated_atom_is_recovered_exactly():
    """Patches c_p S_{r_p} d: every upright column is a multiple of d, so one update
    from a random start returns d (with the sign of the start) and the next pursuit
    codes every patch exactly."""
    R = 32
    d, X = _toy(300, 1, 1, R, seed=1)
    D0 = _unit(np.random.default_rng(100).standard_normal((1, B)))
    D, code, hist = orc.rksvd(D0, R, S, T, X, 1, 1)
    assert 1 - _best_rotation_corr(D[0], d[0], R) < 1e-12
    assert hist[-1] < 1e-20 * hist[0]


def test_three_atom_toy_is_recovered_up_to_rotation():
    """Three atoms, two rotated copies per patch, noise-free: R-K-SVD from a random start
    finds every atom up to a rotation and the coding error falls by orders of magnitude
    (not monotonically: greedy pursuit and the update without a coefficient refresh
    give no descent guarantee)."""
    R = 32
    D_true, X = _toy(400, 3, 2, R, seed=2, weights="uniform")
    D0 = _unit(np.random.default_rng(7).standard_normal((3, B)))
    D, _, hist = orc.rksvd(D0, R, S, T, X, 2, 20)
    for m in range(3):
        assert max(_best_rotation_corr(D[m], D_true[j], R) for j in range(3)) > 0.9999
    assert hist[-1] < 1e-2 * hist[0], hist


def _covariance_via_residuals(D, R, X, code, m):
    """sum of y y^T over the patches using atom m, with y = S_{-r0}(r_p) + c_{i0} d_m: the
    residual identity x_p - D b_p = r_p + c_{i0} S_{r0} d_m, r_p the pursuit's residual."""
    C = np.zeros((B, B))
    n = 0
    recon = orc.code_to_hat(D, R, S, T, code)
    for p in range(X.shape[0]):
        slots = np.flatnonzero(code.atom[p] == m)
        if slots.size == 0:
            continue
        i0 = slots[0]
        r = X[p] - recon[p]
        y = orc.steer(r, -2 * np.pi * code.angle[p, i0] / R, S, T) + code.coef[p, i0] * D[m]
        C += np.outer(y, y)
        n += 1
    return C, n


def _power_top(C, iters=5000):
    v = np.ones(C.shape[0]) / np.sqrt(C.shape[0])
    for _ in range(iters):
        v = C @ v
        v /= np.linalg.norm(v)
    return v, float(v @ C @ v)


@pytest.mark.parametrize("seed", [3, 4])
def test_update_is_top_eigenvector_of_independently_assembled_covariance(seed):
    R, M, K = 16, 4, 3
    D_true, X = _toy(250, M, K, R, seed=seed)
    X += 0.05 * np.random.default_rng(seed).standard_normal(X.shape)
    D = _unit(D_true + 0.3 * np.random.default_rng(seed + 1).standard_normal(D_true.shape))
    code = orc.omp(orc.augmented_dictionary(D, R, S, T), X, K, M)
    D_new, usage, reset = orc.rksvd_update(D, R, S, T, X, code)
    for m in range(M):
        C, n = _covariance_via_residuals(D, R, X, code, m)
        assert usage[m] == n
        if n == 0:
            continue
        v, lam = _power_top(C)
        ev = np.linalg.eigvalsh(C)
        assert ev[-1] - ev[-2] > 1e-3 * ev[-1]            # well-separated top eigenvalue
        assert abs(D_new[m] @ v) > 1 - 1e-9
        assert abs(D_new[m] @ C @ D_new[m] - lam) < 1e-9 * lam
        assert D_new[m] @ D[m] > 0                         # sign rule
    assert np.all(reset == -1)


def test_invariant_to_rotating_every_patch_scaling_and_order():
    R, M, K = 16, 3, 2
    D_true, X = _toy(120, M, K, R, seed=5)
    D = _unit(D_true + 0.2 * np.random.default_rng(6).standard_normal(D_true.shape))
    code = orc.omp(orc.augmented_dictionary(D, R, S, T), X, K, M)
    ref, _, _ = orc.rksvd_update(D, R, S, T, X, code)
    # every patch rotated by r0 steps: its code's angles shift by r0
    r0 = 5
    Xr = orc.steer(X, 2 * np.pi * r0 / R, S, T)
    code_r = orc.Code(code.atom, np.where(code.atom >= 0, (code.angle + r0) % R, -1), code.coef,
                      code.resid2, code.corr, code.gap)
    got, _, _ = orc.rksvd_update(D, R, S, T, Xr, code_r)
    assert np.abs(got - ref).max() < 1e-12
    # scaling patches and coefficients
    code_s = orc.Code(code.atom, code.angle, 3.0 * code.coef, 9.0 * code.resid2, code.corr, code.gap)
    got, _, _ = orc.rksvd_update(D, R, S, T, 3.0 * X, code_s)
    assert np.abs(got - ref).max() < 1e-12
    # patch order
    perm = np.random.default_rng(8).permutation(X.shape[0])
    code_p = orc.Code(code.atom[perm], code.angle[perm], code.coef[perm], code.resid2[perm],
                      code.corr[perm], code.gap[perm])
    got, _, _ = orc.rksvd_update(D, R, S, T, X[perm], code_p)
    assert np.abs(got - ref).max() < 1e-12


def test_R1_equals_matrix_form_ksvd_atom_update():
    """With R = 1 the update is K-SVD's atom step without the coefficient refresh:
    the first left singular vector of E_m = X_w - sum_{j != m} d_j a_j restricted to the
    patches w that use atom m (written here in matrix form)."""
    M, K = 5, 3
    rng = np.random.default_rng(9)
    D = _unit(rng.standard_normal((M, B)))
    X = rng.standard_normal((200, B))
    code = orc.omp(orc.augmented_dictionary(D, 1, S, T), X, K, M)
    D_new, _, _ = orc.rksvd_update(D, 1, S, T, X, code)
    A = np.zeros((M, X.shape[0]))                          # sparse code matrix
    for p in range(X.shape[0]):
        for i in range(K):
            if code.atom[p, i] >= 0:
                A[code.atom[p, i], p] += code.coef[p, i]
    for m in range(M):
        w = np.flatnonzero(A[m] != 0)
        if w.size == 0:
            continue
        E = X[w].T - (D.T @ A[:, w] - np.outer(D[m], A[m, w]))
        U, _, _ = np.linalg.svd(E, full_matrices=False)
        assert abs(U[:, 0] @ D_new[m]) > 1 - 1e-10


def test_unused_atoms_take_the_worst_coded_patches():
    """Atoms that live in harmonics no patch contains are never selected; they are
    reset, in index order, to the patches with the largest coding error."""
    R, K = 8, 1
    rng = np.random.default_rng(10)
    D = np.zeros((4, B))
    D[0, :S] = rng.standard_normal(S)                       # harmonic 0 only
    D[1, S:S + 2 * S] = rng.standard_normal(2 * S)          # harmonic 1 only
    D[2, B - 2 * S:] = rng.standard_normal(2 * S)           # harmonic 5 only: unused
    D[3, B - 4 * S:B - 2 * S] = rng.standard_normal(2 * S)  # harmonic 4 only: unused
    D = _unit(D)
    X = np.zeros((30, B))
    X[:, :3 * S] = rng.standard_normal((30, 3 * S))         # harmonics 0, 1 only
    code = orc.omp(orc.augmented_dictionary(D, R, S, T), X, K, 4)
    D_new, usage, reset = orc.rksvd_update(D, R, S, T, X, code)
    assert usage[2] == 0 and usage[3] == 0 and usage[0] + usage[1] == 30
    worst = sorted(range(30), key=lambda p: (-code.resid2[p], p))
    assert reset[2] == worst[0] and reset[3] == worst[1]
    assert np.allclose(D_new[2], _unit(X[worst[0]])) and np.allclose(D_new[3], _unit(X[worst[1]]))


def test_planted_wrong_upright_direction_is_caught(monkeypatch):
    """Turning residuals by +r0 instead of -r0 breaks the exact single-atom recovery."""
    R = 32
    d, X = _toy(300, 1, 1, R, seed=1)
    D0 = _unit(np.random.default_rng(100).standard_normal((1, B)))
    real = orc.steer

    def flipped(x, theta, S_, T_):
        return real(x, -theta, S_, T_) if np.ndim(theta) == 0 and theta < 0 else real(x, theta, S_, T_)
    code = orc.omp(orc.augmented_dictionary(D0, R, S, T), X, 1, 1)
    monkeypatch.setattr(orc, "steer", flipped)
    D1, _, _ = orc.rksvd_update(D0, R, S, T, X, code)
    monkeypatch.setattr(orc, "steer", real)
    code = orc.omp(orc.augmented_dictionary(D1, R, S, T), X, 1, 1)
    assert code.resid2.sum() > 1e-3 * (X * X).sum()


def test_planted_removal_of_every_use_is_caught():
    """Removing all entries of atom m from b (instead of the one at r0) changes the
    covariance whenever a patch uses m twice; the independent assembly notices."""
    R, M, K = 8, 2, 4
    D_true, X = _toy(200, M, K, R, seed=11)
    D = _unit(D_true + 0.3 * np.random.default_rng(12).standard_normal(D_true.shape))
    code = orc.omp(orc.augmented_dictionary(D, R, S, T), X, K, M)
    twice = [p for p in range(X.shape[0]) if np.sum(code.atom[p] == 0) > 1]
    assert twice, "the fixture must contain patches that use an atom twice"
    wrong = []
    for p in range(X.shape[0]):
        slots = np.flatnonzero(code.atom[p] == 0)
        if slots.size == 0:
            continue
        keep = [i for i in range(K) if code.atom[p, i] >= 0 and code.atom[p, i] != 0]
        others = sum((code.coef[p, i] * orc.steer(D[code.atom[p, i]], 2 * np.pi * code.angle[p, i] / R, S, T)
                      for i in keep), np.zeros(B))
        wrong.append(orc.steer(X[p] - others, -2 * np.pi * code.angle[p, slots[0]] / R, S, T))
    U, _, _ = np.linalg.svd(np.stack(wrong, 1), full_matrices=False)
    C, _ = _covariance_via_residuals(D, R, X, code, 0)
    v, _ = _power_top(C)
    assert abs(U[:, 0] @ v) < 1 - 1e-6


def _ray_atom(N, S, T):
    """A bar from the centre outwards (no rotational symmetry), in hat coordinates, unit norm."""
    basis = orc.build_basis(N, S, T)
    c = (N - 1) / 2
    rows, cols = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    x, y = cols - c, c - rows
    along = np.clip(x, 0, None)
    img = np.exp(-(y * y) / 2.0) * (x >= 0) * np.exp(-((along - N / 4) ** 2) / (2 * (N / 6) ** 2))
    d = orc.project(basis, img[None])[0]
    return d / np.linalg.norm(d)


def _toy_crosses(R, P, seed=40):
    d = _ray_atom(11, S, T)
    rng = np.random.default_rng(seed)
    r = rng.integers(0, R, (P, 2))
    w = rng.uniform(0.5, 1.5, (P, 2))
    X = np.stack([w[p, 0] * orc.steer(d, 2 * np.pi * r[p, 0] / R, S, T) +
                  w[p, 1] * orc.steer(d, 2 * np.pi * r[p, 1] / R, S, T) for p in range(P)])
    return d, X


def test_toy_two_rotations_of_one_atom():
    """The paper's toy experiment (Fig. toyCoding, Sec. III-A, synthetic patches): patches are
    the sum of two random rotations of one atom.  R-K-SVD with M = 1, K = 2 recovers the
    atom up to a rotation; plain K-SVD (R = 1) with M = 1, K = 1 or M = 2, K = 2 learns
    angular averages and codes far worse.  Greedy pursuit does not separate two nearby
    rotations exactly, so the R-K-SVD error is small but not zero (the paper's is not
    zero either)."""
    R, P = 32, 400
    d, X = _toy_crosses(R, P)
    energy = float(np.sum(X * X))
    D0 = _unit(np.random.default_rng(41).standard_normal((1, B)))
    D, code, hist = orc.rksvd(D0, R, S, T, X, 2, 15)
    assert _best_rotation_corr(D[0], d, R) > 0.99, _best_rotation_corr(D[0], d, R)
    assert hist[-1] < 0.05 * energy
    for M, K in ((1, 1), (2, 2)):
        D0k = _unit(np.random.default_rng(42).standard_normal((M, B)))
        Dk, _, hk = orc.rksvd(D0k, 1, S, T, X, K, 15)
        assert hk[-1] > 20 * hist[-1], (M, K, hk[-1], hist[-1])
        assert max(_best_rotation_corr(Dk[m], d, R) for m in range(M)) < 0.8
