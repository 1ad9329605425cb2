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


# ---------------------------------------------------------------------------
# The optimal window of image domain gridding (§4.3 and Appendix A).
#
# Index units: subgrid pixel k sits at x = k (k = 0 .. L-1), the imaged field
# (the main lobe) is [0, L), the side lobes are x < 0 and x >= L.  A sample
# shifted by s uv pixels from the subgrid centre sees the effective window
#     f(x, s) = sum_k a_k sinc(x - k) exp(2 pi i (k - x) s / L)          (§4.2)
# and the cost is the side-lobe energy averaged over the allowed shifts
# |s| <= h (§4.3; Table 1 is computed with h = (L - beta + 1)/2):
#     eps^2 = a^T Rbar a,  Rbar = Qbar o Sbar  (elementwise),
#     Qbar_kl = (int_{-inf}^0 + int_L^inf) sinc(x - k) sinc(x - l) dx,
#     Sbar_kl = sinc(2 h (k - l) / L)  (the mean of exp(2 pi i (k - l) s / L) over |s| <= h).
# With a^T a = 1 the total energy is 1 (the shifted sincs are orthonormal), so
# the smallest eigenvalue of Rbar is eps^2 and its eigenvector the optimal a.
#
# Closed forms of the tail integrals (the appendix's antiderivative, with the
# standard Ci(x) = -int_x^inf cos t / t dt):
#   k != l: sinc(x-k) sinc(x-l) = (-1)^(k+l) sin^2(pi x) / (pi^2 (k-l)) [1/(x-k) - 1/(x-l)],
#           int sin^2(pi y) / y dy = G(y) = (ln|y| - Ci(2 pi |y|)) / 2, G(0) = -(gamma + ln 2 pi) / 2;
#   k == l: int sinc^2(y) dy = H(y) = -sin^2(pi y) / (pi^2 y) + Si(2 pi y) / pi,
#           so the two tails give 1 - (Si(2 pi k) + Si(2 pi (L - k))) / pi.
# ---------------------------------------------------------------------------


def shift_half_range(L, beta):
    """The shift bound of Table 1 for kernel width beta: (L - beta + 1)/2 uv pixels (§4.3)."""
    return (L - beta + 1) / 2


def _si_ci(x, dps):
    """(Si(x), Ci(x)) for x > 0: scipy in float64 (dps None), mpmath otherwise."""
    if dps is None:
        from scipy.special import sici
        s, c = sici(float(x))
        return float(s), float(c)
    return mp.si(x), mp.ci(x)


def idg_window_matrix(L, max_shift, dps=None):
    """Rbar (L x L, symmetric) for shifts |s| <= max_shift: numpy float64 when dps is None, else an
    mpmath matrix at dps digits."""
    hi = dps is not None
    ctx = mp.workdps(dps) if hi else None
    if ctx:
        ctx.__enter__()
    try:
        pi = mp.pi if hi else np.pi
        one = mp.mpf(1) if hi else 1.0
        si_tab, ci_tab = {}, {}
        for m in range(1, L + 1):
            si_tab[m], ci_tab[m] = _si_ci(2 * pi * m, dps)
        g0 = -(mp.euler + mp.log(2 * pi)) / 2 if hi else -(np.euler_gamma + np.log(2 * np.pi)) / 2

        def G(y):                   # y a nonnegative integer here
            if y == 0:
                return g0
            return ((mp.log(y) if hi else np.log(y)) - ci_tab[y]) / 2

        def si(m):
            return 0 if m == 0 else si_tab[m]

        R = mp.matrix(L, L) if hi else np.zeros((L, L))
        w = 2 * (mp.mpf(max_shift) if hi else float(max_shift)) / L
        for k in range(L):
            for l in range(L):
                if k == l:
                    q = 1 - (si(k) + si(L - k)) / pi
                    s = one
                else:
                    q = (-1) ** (k + l) / (pi * pi * (k - l)) * ((G(k) - G(l)) - (G(L - k) - G(L - l)))
                    d = (k - l) * w
                    s = (mp.sin(pi * d) / (pi * d)) if hi else np.sinc(d)
                R[k, l] = q * s
        return R
    finally:
        if ctx:
            ctx.__exit__(None, None, None)


def side_lobe_matrix_at_shift(L, s):
    """R(s) (L x L, float64): the side-lobe energy of the effective window at one position shift s (uv
    pixels) is a^T R(s) a.  R(s) = Qbar o C(s) with C_kl(s) = cos(2 pi (k - l) s / L), the phasor product
    z_k z_l^* of §4.2 without the average over shifts that gives Rbar; the mean of R(s) over |s| <= h is
    idg_window_matrix(L, h).  Qbar is taken from idg_window_matrix at zero shift range (Sbar = 1)."""
    q = idg_window_matrix(L, 0.0)
    d = np.subtract.outer(np.arange(L), np.arange(L))
    return q * np.cos(2 * np.pi * d * float(s) / L)


def side_lobe_error_at_shift(a, s):
    """The error of taper a for samples at position shift s from the subgrid centre (§4.3, the dependence
    on position): sqrt(a^T R(s) a / a^T a)."""
    a = np.asarray(a, np.float64)
    return float(np.sqrt(max(a @ side_lobe_matrix_at_shift(a.size, s) @ a / (a @ a), 0.0)))


def effective_window(a, s, x):
    """The effective window f(x, s) of §4.2 at index-unit positions x (subgrid pixel k at x = k): the sinc
    interpolation of the taper samples times the phase gradient of a sample shifted s uv pixels from the
    subgrid centre, which cancels at the sample points:
        f(x, s) = sum_k a_k sinc(x - k) exp(2 pi i (k - x) s / L)."""
    a = np.asarray(a, np.float64)
    L = a.size
    k = np.arange(L)
    x = np.atleast_1d(np.asarray(x, np.float64))
    return (np.sinc(x[:, None] - k[None, :]) * np.exp(2j * np.pi * (k[None, :] - x[:, None]) * s / L)) @ a


def idg_optimal_window(L, max_shift, dps=None):
    """(eps, a): eps = sqrt(smallest eigenvalue of Rbar), a its eigenvector (float64, a[L/2] = 1)."""
    R = idg_window_matrix(L, max_shift, dps)
    if dps is None:
        lam, vec = np.linalg.eigh(R)
        lam0, a = lam[0], vec[:, 0]
    else:
        with mp.workdps(dps):
            lam, vec = mp.eigsy(R)
            i0 = min(range(L), key=lambda i: lam[i])
            lam0 = lam[i0]
            a = np.array([float(vec[k, i0]) for k in range(L)])
    a = a / a[L // 2]
    return float(mp.sqrt(max(lam0, 0))) if dps is not None else float(np.sqrt(max(lam0, 0.0))), a


def idg_window_error(a, max_shift):
    """eps of an arbitrary taper a (float64): sqrt(a^T Rbar a / a^T a)."""
    a = np.asarray(a, np.float64)
    return float(np.sqrt(a @ idg_window_matrix(a.size, max_shift) @ a / (a @ a)))


def rms_window(a, max_shift, x):
    """The effective window's rms over the allowed shifts, at index-unit positions x (§4.2, §4.3):
    sqrt(mean_s |f(x, s)|^2) = sqrt(sum_kl a_k a_l sinc(x - k) sinc(x - l) Sbar_kl)."""
    a = np.asarray(a, np.float64)
    L = a.size
    k = np.arange(L)
    d = np.subtract.outer(k, k)
    sbar = np.sinc(d * 2 * max_shift / L)
    x = np.atleast_1d(np.asarray(x, np.float64))
    v = np.sinc(x[:, None] - k[None, :]) * a[None, :]          # [nx, L]
    return np.sqrt(np.einsum("xk,kl,xl->x", v, sbar, v))


def taper_correction(a, max_shift, N):
    """Correction for the master-grid image steps: corr[X] = L rms_window(L X / N), X = 0 .. N-1
    (image pixel X at l = (X - N/2) S / N is at index-unit position L X / N of a subgrid)."""
    L = np.asarray(a).size
    return L * rms_window(a, max_shift, L * np.arange(N) / N)
