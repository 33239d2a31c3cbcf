"""Quadrature rules for the oracle (test infrastructure only).

The paper gives the point counts of its triangle rules but not the points (section "Integral
evaluation"; Tables 1 and 4): K = 1, 3 or 4 for far panels and K_fine = 19, 25 or 37 for
near-singular ones.  These counts are those of Dunavant's symmetric rules (1982), so the
oracle reads them as Dunavant's rules of degree 1, 2, 3 (far) and 9, 10, 13 (fine), plus the
7-point degree-5 rule of Radon.  The 37-point rule is the fine rule of the paper's strict
setting (grid-convergence study, Table quadparams1).

A rule is returned as barycentric points b [n, 3] and weights w [n] summing to 1, so that
integral over a triangle of f ~= Area * sum_g w_g f(sum_k b_gk v_k).
"""
from __future__ import annotations

import numpy as np

# (weight, a) for the orbit (a, b, b) with b = (1 - a)/2; (weight, a, b) for the six
# permutations of (a, b, 1 - a - b); ("c", weight) for the centroid.
_S15 = np.sqrt(15.0)
_ORBITS = {
    1: [("c", 1.0)],
    3: [("s2", 1.0 / 3.0, 2.0 / 3.0)],
    4: [("c", -27.0 / 48.0), ("s2", 25.0 / 48.0, 0.6)],
    7: [("c", 9.0 / 40.0),
        ("s2", (155.0 - _S15) / 1200.0, (9.0 + 2.0 * _S15) / 21.0),
        ("s2", (155.0 + _S15) / 1200.0, (9.0 - 2.0 * _S15) / 21.0)],
    19: [("c", 0.097135796282799),
         ("s2", 0.031334700227139, 0.020634961602525),
         ("s2", 0.077827541004774, 0.125820817014127),
         ("s2", 0.079647738927210, 0.623592928761935),
         ("s2", 0.025577675658698, 0.910540973211095),
         ("s3", 0.043283539377289, 0.036838412054736, 0.221962989160766)],
    25: [("c", 0.090817990382754),
         ("s2", 0.036725957756467, 0.028844733232685),
         ("s2", 0.045321059435528, 0.781036849029926),
         ("s3", 0.072757916845420, 0.141707219414880, 0.307939838764121),
         ("s3", 0.028327242531057, 0.025003534762686, 0.246672560639903),
         ("s3", 0.009421666963733, 0.009540815400299, 0.066803251012200)],
    37: [("c", 0.052520923400802),
         ("s2", 0.011280145209330, 0.009903630120591),
         ("s2", 0.031423518362454, 0.062566729780852),
         ("s2", 0.047072502504194, 0.170957326397447),
         ("s2", 0.047363586536355, 0.541200855914337),
         ("s2", 0.031167529045794, 0.771151009607340),
         ("s2", 0.007975771465074, 0.950377217273082),
         ("s3", 0.036848402728732, 0.094853828379579, 0.268794997058761),
         ("s3", 0.017401463303822, 0.018100773278807, 0.291730066734288),
         ("s3", 0.015521786839045, 0.022233076674090, 0.126357385491669)],
}

RULE_DEGREE = {1: 1, 3: 2, 4: 3, 7: 5, 19: 9, 25: 10, 37: 13}


def triangle_rule(n_points: int):
    """Symmetric triangle rule with n_points nodes: (bary [n,3], weights [n])."""
    if n_points not in _ORBITS:
        raise ValueError(f"no {n_points}-point triangle rule (have {sorted(_ORBITS)})")
    pts, wts = [], []
    for orbit in _ORBITS[n_points]:
        kind, w = orbit[0], orbit[1]
        if kind == "c":
            perms = [(1 / 3, 1 / 3, 1 / 3)]
        elif kind == "s2":
            a = orbit[2]
            b = (1.0 - a) / 2.0
            perms = [(a, b, b), (b, a, b), (b, b, a)]
        else:
            a, b = orbit[2], orbit[3]
            c = 1.0 - a - b
            perms = [(a, b, c), (a, c, b), (b, a, c), (b, c, a), (c, a, b), (c, b, a)]
        for p in perms:
            pts.append(p)
            wts.append(w)
    w = np.asarray(wts, dtype=np.float64)
    return np.asarray(pts, dtype=np.float64), w


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [-1, 1] (numpy's library routine)."""
    return np.polynomial.legendre.leggauss(n)
