"""Comparison of device codes with reference codes (test helper).

A patch matches when its set of selected (atom, angle) pairs, empty slots
included, equals the reference's.  On matched patches every coefficient must
satisfy |a - a*| <= rel * max(|a*|, 1e-3 * max_i |a*_i|, 1e-2 * ||x_hat*||) (the last
term only when the patches' coordinate norms are given).

The last term: the device codes FP32 coordinates, and with unit-norm columns a
coefficient moves by up to about the coordinates' own rounding, a few 1e-7 ||x_hat||
after the FP32 projection.  A coefficient that is tiny against its patch (a patch
nearly orthogonal to everything selected) therefore cannot be held to 1e-4 of itself;
it is held to 1e-6 ||x_hat|| instead, ten times that rounding.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Report:
    n: int
    matched: int
    coef_err_max: float       # worst relative coefficient error on matched patches
    coef_err_p99: float
    coef_bad: int             # matched patches that break the coefficient tolerance
    mismatched_gap_max: float # largest reference top-2 gap among mismatched patches

    @property
    def match_rate(self) -> float:
        return self.matched / max(self.n, 1)

    def __str__(self):
        return (f"n={self.n} match={self.match_rate:.5f} coef_err_max={self.coef_err_max:.3g} "
                f"p99={self.coef_err_p99:.3g} coef_bad={self.coef_bad} "
                f"mismatch_gap_max={self.mismatched_gap_max:.3g}")


def compare_codes(atom, angle, coef, ref, rel: float = 1e-4, xnorm=None) -> Report:
    """atom/angle/coef: device results as numpy [P, K]; ref: oracle Code; xnorm: the
    reference coordinates' norms ||x_hat*|| [P], or None."""
    atom = np.asarray(atom)
    angle = np.asarray(angle)
    coef = np.asarray(coef, dtype=np.float64)
    P = atom.shape[0]
    matched = 0
    errs = []
    bad = 0
    gap_max = 0.0
    for p in range(P):
        g = {(int(a), int(r)): float(c) for a, r, c in zip(atom[p], angle[p], coef[p]) if a >= 0}
        o = {(int(a), int(r)): float(c) for a, r, c in zip(ref.atom[p], ref.angle[p], ref.coef[p]) if a >= 0}
        if set(g) != set(o) or (atom[p] < 0).sum() != (ref.atom[p] < 0).sum():
            gap = ref.gap[p][ref.atom[p] >= 0]
            gap_max = max(gap_max, float(gap.min()) if gap.size else 0.0)
            continue
        matched += 1
        if not o:
            continue
        scale = max(abs(v) for v in o.values())
        floor = 1e-3 * scale if xnorm is None else max(1e-3 * scale, 1e-2 * float(xnorm[p]))
        worst = 0.0
        for key, v in o.items():
            e = abs(g[key] - v) / max(abs(v), floor)
            worst = max(worst, e)
        errs.append(worst)
        bad += worst > rel
    errs = np.array(errs) if errs else np.zeros(1)
    return Report(P, matched, float(errs.max()), float(np.percentile(errs, 99)), int(bad), gap_max)
