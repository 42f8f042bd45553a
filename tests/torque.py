"""Force, spin torque and cross product from a cell's moments and local
coefficients (shared by the angular-momentum tests): the force evaluated from
L, -sum_{|a| <= 2} (M_a/a!) L_{a+e_k}, and the torque on the cell's mass
about its centre, tau_m = -sum_{|g| <= 2} eps_mnl (M_{g+e_n}/g!) L_{g+e_l}."""
from math import factorial

import numpy as np

import oracle

SUB3 = 512
EXPS = [tuple(oracle.multi_index(g)) for g in range(20)]
IDX = {e: g for g, e in enumerate(EXPS)}
FACT = np.array([factorial(a) * factorial(b) * factorial(c) for a, b, c in EXPS], float)
EYE = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]


def _add(a, b):
    return tuple(x + y for x, y in zip(a, b))


def eval_force(M, L):
    """-sum_{|a| <= 2} (M_a/a!) L_{a+e_k}: the force evaluated from L."""
    F = np.zeros((3, M.shape[1]))
    for g, e in enumerate(EXPS):
        if sum(e) <= 2:
            for k in range(3):
                F[k] -= M[g] / FACT[g] * L[IDX[_add(e, EYE[k])]]
    return F


def spin_torque(M, L):
    """tau_m = -sum_{|g| <= 2} eps_mnl (M_{g+e_n}/g!) L_{g+e_l}."""
    tau = np.zeros((3, M.shape[1]))
    for g, e in enumerate(EXPS):
        if sum(e) > 2:
            continue
        for m, n, l, sgn in ((0, 1, 2, 1), (0, 2, 1, -1), (1, 2, 0, 1), (1, 0, 2, -1), (2, 0, 1, 1),
                             (2, 1, 0, -1)):
            tau[m] -= sgn * M[IDX[_add(e, EYE[n])]] / FACT[g] * L[IDX[_add(e, EYE[l])]]
    return tau


def cross(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])
