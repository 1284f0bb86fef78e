"""Pins of the two-drop problem (paper section 4.3, eq. (IE-2Surf)) in the oracle.

- the operator on a uniform translation U of both drops: the on-surface double layer of a constant is
  U/2 exactly, the other drop's exterior double layer of a constant is 0 exactly (q - q0 = 0), so
  A U = (lambda + 1) U - 2 (lambda - 1) U / 2 = 2 U for lambda = 2;
- the single layers of a uniform force g: Stokes' translating-sphere solution, (2/3) g on the own
  sphere plus the other sphere's exterior flow;
- GMRES from zero to 1e-10 at h = 1/16 takes the paper's count of iterations, within one
  (tests/golden/two_drops_table2.json, Table 2: 13).
"""
import json
import os

import numpy as np
import pytest

import workload
from oracle.rigid import RigidProblem, Sphere, gmres

HERE = os.path.dirname(os.path.abspath(__file__))
LAM = 2.0


def problem(h):
    cen, rad, surfs = workload.two_drops(h)
    prob = RigidProblem([Sphere(s, c, a, h) for s, c, a in zip(surfs, cen, rad)], h, rho=(3.0, 4.0, 5.0), sharp=True,
                        sharp_rho=3.0, a_id=LAM + 1, a_dl=-2 * (LAM - 1), completion=False)
    return prob, cen, surfs


def test_drop_operator_on_translation():
    prob, _, _ = problem(1 / 8)
    U = np.array([0.3, -0.8, 0.5])
    out = prob.matvec(np.tile(U, (prob.ntot, 1)))
    assert np.abs(out - 2 * U).max() < 1e-13


def test_single_layers_of_uniform_force():
    h = 1 / 16
    prob, cen, surfs = problem(h)
    g = np.array([0.4, 0.1, -0.7])
    u = prob.single_layers(np.tile(g, (prob.ntot, 1)))
    ex = np.zeros_like(u)
    for m, c in enumerate(cen):
        d = prob.y - c
        r = np.linalg.norm(d, axis=1)[:, None]
        gd = (d @ g)[:, None]
        out = 0.5 * (g / r + gd * d / r ** 3) + (1 / 6) * (g / r ** 3 - 3 * gd * d / r ** 5)
        own = np.zeros(prob.ntot, bool)
        own[prob.off[m]:prob.off[m + 1]] = True
        ex[own] += 2 / 3 * g
        ex[~own] += out[~own]
    err = np.abs(u - ex).max()
    print("single layers of a uniform force:", err)
    assert err < 2e-4


def test_gmres_iterations_match_table2():
    gold = json.load(open(os.path.join(HERE, "golden", "two_drops_table2.json")))
    h = 1 / 16
    prob, cen, surfs = problem(h)
    f = np.concatenate([workload.drop_force(s.x, c) for s, c in zip(surfs, cen)])
    b = -2.0 * prob.single_layers(f)
    u, it, rr = gmres(prob.matvec, b, tol=1e-10, maxit=60)
    print(f"h = 1/16: {it} iterations (paper {gold['gmres_iterations'][0]}), relres {rr:.1e}")
    assert rr <= 1e-10 and abs(it - gold["gmres_iterations"][0]) <= 1
