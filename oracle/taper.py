"""Aliasing level of the classical optimal window, epsilon(beta) (oracle check).

§4.1: the optimal window for classical gridding with kernel support beta is
the prolate spheroidal wave function; its normalised side-lobe energy is
epsilon^2 = 1 - lambda_0(alpha), alpha = beta pi / 2, lambda_0 being the
largest eigenvalue of the concentration problem.  Table 1 column 2 lists
epsilon for beta = 3 .. 15.

lambda_0 is the top eigenvalue of the sinc-kernel operator
    (K f)(x) = int_{-1}^{1} sin(alpha (x - y)) / (pi (x - y)) f(y) dy.
For beta >= 11, 1 - lambda_0 is below float64 resolution, so the operator is
discretised with Gauss-Legendre quadrature (n = 64 nodes, refined to the
working precision), restricted to even functions (psi_0 is even), and its
symmetric eigenproblem is solved in mpmath at 40 decimal digits.
"""

import mpmath as mp
import numpy as np


def _gauss_legendre_mp(n):
    x0, _ = np.polynomial.legendre.leggauss(n)
    nodes, weights = [], []
    for xi in x0:
        x = mp.mpf(xi)
        for _ in range(4):
            p = mp.legendre(n, x)
            dp = n * (x * p - mp.legendre(n - 1, x)) / (x * x - 1)
            x = x - p / dp
        p = mp.legendre(n, x)
        dp = n * (x * p - mp.legendre(n - 1, x)) / (x * x - 1)
        nodes.append(x)
        weights.append(2 / ((1 - x * x) * dp * dp))
    return nodes, weights


def classical_aliasing(beta, n=64, dps=40):
    """epsilon(beta) = sqrt(1 - lambda_0(beta pi / 2)) as a float."""
    with mp.workdps(dps):
        alpha = mp.mpf(beta) * mp.pi / 2

        def kern(d):
            return alpha / mp.pi if d == 0 else mp.sin(alpha * d) / (mp.pi * d)

        nodes, weights = _gauss_legendre_mp(n)
        pos = [(x, w) for x, w in zip(nodes, weights) if x > 0]
        m = mp.matrix(len(pos), len(pos))
        for i, (xi, wi) in enumerate(pos):
            for j, (xj, wj) in enumerate(pos):
                m[i, j] = mp.sqrt(wi * wj) * (kern(xi - xj) + kern(xi + xj))
        evals, _ = mp.eigsy(m)
        lam0 = max(evals)
        return float(mp.sqrt(1 - lam0))
