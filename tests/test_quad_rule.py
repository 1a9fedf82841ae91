"""The Gauss-Kronrod (7, 15) constants of the library's adaptive frequency
integral (read from its source, no GPU): the Gauss subset equals the 7-point
Gauss-Legendre rule (numpy.polynomial.legendre.leggauss), and the 15-point
Kronrod rule integrates every monomial up to degree 22 exactly on [-1, 1]
(the degree 3n + 1 of Kronrod's extension of an n = 7 point Gauss rule)."""
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_2305_18643_amd", "csrc",
                   "vca.hip")


def _table(name):
    txt = open(SRC).read()
    m = re.search(r"__constant__ double %s\[\d+\] = \{([^}]*)\}" % name, txt)
    return np.array([float(x) for x in m.group(1).replace("\n", " ").split(",") if x.strip()])


def test_gauss_subset_is_gauss_legendre():
    x, wk, wg = _table("kGkX"), _table("kGkW"), _table("kGW")
    gx, gw = np.polynomial.legendre.leggauss(7)
    nodes = np.sort(np.concatenate([-x[1:7:2], x[1::2]]))
    assert np.abs(nodes - np.sort(gx)).max() <= 1e-15
    w = np.concatenate([wg[:3], [wg[3]], wg[:3][::-1]])
    assert np.abs(w - gw[np.argsort(gx)]).max() <= 1e-15


def test_kronrod_rule_is_exact_to_degree_22():
    x, wk = _table("kGkX"), _table("kGkW")
    nodes = np.concatenate([-x[:7], [0.0], x[:7][::-1]])
    weights = np.concatenate([wk[:7], [wk[7]], wk[:7][::-1]])
    assert abs(weights.sum() - 2.0) <= 1e-15
    for deg in range(0, 23):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.dot(weights, nodes ** deg) - exact) <= 4e-16, deg
    # and not beyond: degree 24 is not integrated exactly
    assert abs(np.dot(weights, nodes ** 24) - 2.0 / 25) > 1e-12
