"""Prolate-spheroidal taper used as an *input* to gridding (paper §4.1, §4.2).

The classical optimal anti-aliasing window (§4.1) is the zeroth prolate
spheroidal wave function psi_0 with bandwidth parameter alpha = beta*pi/2,
where beta is the kernel support in uv pixels.  The image-domain taper is
separable, c[i, j] = a_i a_j (§4.2, the equation defining c[i,j]), with the
1-D coefficients sampled at x_i = -1/2 + i/L (§4.2, the sample points of the
effective window):

    a_i = psi_0(alpha, 2 x_i) / psi_0(alpha, 0).

psi_0 is computed here by a Nystrom discretisation of the sinc-kernel
concentration operator on [-1, 1] (Gauss-Legendre nodes, symmetric weighted
eigenproblem) and evaluated off the nodes with the Nystrom interpolant.  The
edge sample x_0 = -1/2 maps to psi_0(-1), where scipy's pro_ang1 is undefined,
which is why the generator does not use it.
"""

import numpy as np


def _sinc_kernel(c, d):
    d = np.asarray(d, dtype=np.float64)
    out = np.empty_like(d)
    small = d == 0.0
    out[small] = c / np.pi
    out[~small] = np.sin(c * d[~small]) / (np.pi * d[~small])
    return out


def pswf_psi0(beta, xs, n=64):
    """psi_0(alpha = beta*pi/2, x) normalised to psi_0(0) = 1, for x in [-1, 1]."""
    c = beta * np.pi / 2.0
    y, wq = np.polynomial.legendre.leggauss(n)
    sw = np.sqrt(wq)
    m = sw[:, None] * _sinc_kernel(c, y[:, None] - y[None, :]) * sw[None, :]
    lam, vec = np.linalg.eigh(m)
    lam0 = lam[-1]
    v = vec[:, -1] / sw
    xs = np.atleast_1d(np.asarray(xs, dtype=np.float64))
    psi = (_sinc_kernel(c, xs[:, None] - y[None, :]) @ (wq * v)) / lam0
    psi_at_0 = (_sinc_kernel(c, 0.0 - y) @ (wq * v)) / lam0
    return psi / psi_at_0


def pswf_taper_1d(L, beta):
    """1-D taper coefficients a_i, i = 0..L-1, float64."""
    x = -0.5 + np.arange(L, dtype=np.float64) / L
    return pswf_psi0(beta, 2.0 * x)


def pswf_taper_2d(L, beta):
    """2-D separable taper c[j, i] = a_j a_i as float32 [L, L] (row j <-> m, column i <-> l)."""
    a = pswf_taper_1d(L, beta)
    return np.outer(a, a).astype(np.float32)
