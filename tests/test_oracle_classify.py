"""Pins of the reference texture classifier (Sec. III-B, "Classifier"), CPU only.

Closed forms of the chi^2 distance, brute force for the nearest neighbour, exact
histograms, a separable toy whose labels are known, the rotation invariance of the
per-class errors (the reason the paper codes rotationally), the reduction to one
class, and planted mistakes.
"""
import numpy as np

from oracle import rsc_oracle as orc

S, T = 5, 5
B = S * (2 * T + 1)


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _harmonic_slice(k):
    return slice(0, S) if k == 0 else slice(S + 2 * S * (k - 1), S + 2 * S * k)


def test_chi2_closed_forms():
    assert orc.chi2([1, 0], [0, 1]) == 2.0                     # disjoint supports: the maximum, 2
    assert abs(orc.chi2([0.5, 0.5], [1, 0]) - (0.25 / 1.5 + 0.25 / 0.5)) < 1e-15
    assert orc.chi2([0.2, 0.3, 0.0, 0.5], [0.2, 0.3, 0.0, 0.5]) == 0.0
    assert orc.chi2([0, 0, 1], [0, 0, 1]) == 0.0               # empty bins contribute nothing
    rng = np.random.default_rng(0)
    a, b = rng.dirichlet(np.ones(24)), rng.dirichlet(np.ones(24))
    assert orc.chi2(a, b) == orc.chi2(b, a)
    assert 0 < orc.chi2(a, b) <= 2.0
    # the written-out sum on one bin pair
    assert abs(orc.chi2([3.0], [1.0]) - 1.0) < 1e-15            # (3 - 1)^2 / 4


def test_nearest_neighbour_brute_force_and_ties():
    rng = np.random.default_rng(1)
    train = rng.dirichlet(np.ones(6), 9)
    test = rng.dirichlet(np.ones(6), 5)
    idx, dist = orc.nearest_chi2(train, test)
    for q in range(5):
        d = [sum((test[q, i] - train[j, i]) ** 2 / (test[q, i] + train[j, i]) for i in range(6)) for j in range(9)]
        assert idx[q] == int(np.argmin(d)) and abs(dist[q] - min(d)) < 1e-15
    twin = np.vstack([train[3], train[3]])
    idx, _ = orc.nearest_chi2(twin, train[3:4])
    assert idx[0] == 0                                         # tie: the smaller index


def test_label_histogram_exact():
    label = np.array([0, 2, 2, 1, 2, 0, 0])
    h = orc.label_histogram(label, np.array([0, 3, 3, 7]), 3)
    assert np.array_equal(h[0], [1 / 3, 0, 2 / 3])
    assert np.array_equal(h[1], [0, 0, 0])                     # empty group
    assert np.array_equal(h[2], [2 / 4, 1 / 4, 1 / 4])


def _separable(P, seed):
    """Three classes whose atoms live in disjoint harmonics ({0, 1}, {2, 3}, {4, 5}); a patch
    of class c is one of class c's atoms at a grid angle with a weight in [0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    R = 16
    D_list = []
    for c in range(3):
        D = np.zeros((3, B))
        for k in (2 * c, 2 * c + 1):
            D[:, _harmonic_slice(k)] = rng.standard_normal((3, _harmonic_slice(k).stop - _harmonic_slice(k).start))
        D_list.append(_unit(D))
    truth = rng.integers(0, 3, P)
    X = np.zeros((P, B))
    for p in range(P):
        D = D_list[truth[p]]
        X[p] = rng.uniform(0.5, 1.5) * orc.steer(D[rng.integers(0, 3)], 2 * np.pi * rng.integers(0, R) / R, S, T)
    return D_list, R, X, truth


def test_separable_classes_are_labelled_exactly():
    D_list, R, X, truth = _separable(60, 2)
    label, sse = orc.classify(D_list, R, S, T, X, 2)
    assert np.array_equal(label, truth)
    energy = np.sum(X * X, 1)
    assert np.all(sse[np.arange(60), truth] < 1e-20 * energy)             # coded exactly
    other = np.where(np.arange(3)[None, :] != truth[:, None], sse, np.inf).min(1)
    assert np.allclose(other, energy, rtol=1e-12)                         # nothing of it coded


def test_planted_argmax_is_caught():
    D_list, R, X, truth = _separable(60, 2)
    _, sse = orc.classify(D_list, R, S, T, X, 2)
    assert not np.array_equal(np.argmax(sse, 1), truth)


def test_errors_are_invariant_to_rotating_the_patches():
    """Rotating every patch by a grid angle inside the span leaves each class's coding
    error unchanged (the pursuit is rotation-equivariant), so the labels do not move:
    the property the paper's classifier relies on."""
    rng = np.random.default_rng(3)
    R = 32
    D_list = [_unit(rng.standard_normal((6, B))) for _ in range(4)]
    X = rng.standard_normal((80, B))
    label, sse = orc.classify(D_list, R, S, T, X, 3)
    for r0 in (5, 8, 21):
        Xr = orc.steer(X, 2 * np.pi * r0 / R, S, T)
        label_r, sse_r = orc.classify(D_list, R, S, T, Xr, 3)
        assert np.allclose(sse_r, sse, rtol=1e-9, atol=1e-12)
        assert np.array_equal(label_r, label)


def test_rotational_coding_keeps_rotated_patches_in_their_class():
    """Patches are single atoms of one of three classes at random grid rotations plus a
    little noise.  With the rotational pursuit every patch is labelled correctly; the
    same dictionaries without rotations (R = 1, plain sparse coding) mislabel many."""
    rng = np.random.default_rng(4)
    R = 32
    D_list = [_unit(rng.standard_normal((2, B))) for _ in range(3)]
    P = 90
    truth = np.repeat(np.arange(3), P // 3)
    X = np.stack([orc.steer(D_list[c][rng.integers(0, 2)], 2 * np.pi * rng.integers(0, R) / R, S, T)
                  for c in truth]) + 0.01 * rng.standard_normal((P, B))
    lab_rot, _ = orc.classify(D_list, R, S, T, X, 1)
    lab_plain, _ = orc.classify(D_list, 1, S, T, X, 1)
    assert np.mean(lab_rot == truth) == 1.0
    assert np.mean(lab_plain == truth) < 0.8


def test_one_class_reduces_to_the_pursuit():
    rng = np.random.default_rng(5)
    D = _unit(rng.standard_normal((5, B)))
    X = rng.standard_normal((20, B))
    label, sse = orc.classify([D], 8, S, T, X, 2)
    code = orc.omp(orc.augmented_dictionary(D, 8, S, T), X, 2, 5)
    assert np.all(label == 0) and np.array_equal(sse[:, 0], code.resid2)
