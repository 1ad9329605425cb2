"""Direct imaging and direct prediction at the subgrid lattice (oracle checks).

These evaluate the paper's direct equations without any partitioning, shifting
or transforming, so they pin the gridding chain from outside:

* the direct imaging equation (§2, eq. imaging):
      I[i, j] = sum_k exp(+2 pi i (u_k l_i + v_k m_j + w_k n'_ij)) g_k^* y_k,
  here with the polarised gain g_k^* y_k -> A_s1^H Y_k A_s2 and the taper c;
* the discrete measurement equation (§2, eq. DME):
      y_k = sum_ij exp(-2 pi i (u_k l_i + v_k m_j + w_k n'_ij)) g_k I[i, j],
  here with g_k I -> A_s1 I A_s2^H and the taper;
* the grid's image at arbitrary (l, m): sum_{x,y} V[y][x] exp(+2 pi i (u_x l + v_y m)).
"""

import numpy as np

from .plan import C0, F


def _lattice(L, S):
    idx = (np.arange(L, dtype=np.float64) - L // 2) * (S / L)
    return idx


def grid_image_at_lattice(grid, S, L):
    """D[pol, j, i] = sum_{y,x} grid[pol, y, x] exp(+2 pi i (u_x l_i + v_y m_j)), u_x = (x - N/2)/S."""
    N = grid.shape[-1]
    lat = _lattice(L, S)
    ux = (np.arange(N, dtype=np.float64) - N // 2) / S
    ex = np.exp(2j * np.pi * np.outer(ux, lat))        # [N(x), L(i)]
    return np.stack([ex.T @ grid[pol] @ ex for pol in range(grid.shape[0])])  # rows j (y), cols i (x)


def grid_from_lattice_image(img, N, S):
    """Master grid whose image is ``img`` [4, L, L] on the lattice: V[y][x] = sum_ij I[j][i] e^{-2 pi i (u_x l_i + v_y m_j)}."""
    L = img.shape[-1]
    lat = _lattice(L, S)
    ux = (np.arange(N, dtype=np.float64) - N // 2) / S
    ex = np.exp(-2j * np.pi * np.outer(ux, lat))       # [N, L]
    return np.stack([ex @ img[pol] @ ex.T for pol in range(img.shape[0])])


def direct_image_lattice(plan, uvw, freqs, vis, aterms, taper):
    """L^2 * c[j,i] * sum over planned samples of A_s1^H Y A_s2 exp(+2 pi i (u l + v m + w n')), [4, L, L]."""
    L, S = plan.subgrid_size, plan.image_size
    lat = _lattice(L, S)
    l = lat[None, :]
    m = lat[:, None]
    nprime = np.sqrt(1.0 - l * l - m * m) - 1.0
    acc = np.zeros((L, L, 2, 2), np.complex128)
    for p in range(plan.nr_subgrids):
        sub = plan.subgrids[p]
        tc = plan.subgrid_samples(p)
        bl = sub[F["bl"]]
        lam_inv = freqs[tc[:, 1]] / C0
        u = uvw[bl, tc[:, 0], 0] * lam_inv
        v = uvw[bl, tc[:, 0], 1] * lam_inv
        w = uvw[bl, tc[:, 0], 2] * lam_inv
        y = np.asarray(vis[bl, tc[:, 0], tc[:, 1]], np.complex128).reshape(-1, 2, 2)
        a1 = np.asarray(aterms[sub[F["slot"]], sub[F["st1"]]], np.complex128).reshape(L, L, 2, 2)
        a2 = np.asarray(aterms[sub[F["slot"]], sub[F["st2"]]], np.complex128).reshape(L, L, 2, 2)
        for k in range(y.shape[0]):
            ph = np.exp(2j * np.pi * (u[k] * l + v[k] * m + w[k] * nprime))
            acc += ph[:, :, None, None] * (np.conj(np.swapaxes(a1, -1, -2)) @ y[k] @ a2)
    acc *= (L * L) * np.asarray(taper, np.float64)[:, :, None, None]
    return acc.reshape(L, L, 4).transpose(2, 0, 1)


def predict_direct_lattice(plan, uvw, freqs, img, aterms, taper):
    """Visibilities [nbl, nt, nch, 4] from a lattice image by the DME with A-terms and taper (x L^2)."""
    L, S = plan.subgrid_size, plan.image_size
    lat = _lattice(L, S)
    l = lat[None, :]
    m = lat[:, None]
    nprime = np.sqrt(1.0 - l * l - m * m) - 1.0
    out = np.zeros((plan.nr_baselines, plan.nr_timesteps, plan.nr_channels, 4), np.complex128)
    im = np.asarray(img, np.complex128).transpose(1, 2, 0).reshape(L, L, 2, 2)
    tap = np.asarray(taper, np.float64)
    for p in range(plan.nr_subgrids):
        sub = plan.subgrids[p]
        tc = plan.subgrid_samples(p)
        bl = sub[F["bl"]]
        a1 = np.asarray(aterms[sub[F["slot"]], sub[F["st1"]]], np.complex128).reshape(L, L, 2, 2)
        a2 = np.asarray(aterms[sub[F["slot"]], sub[F["st2"]]], np.complex128).reshape(L, L, 2, 2)
        b = (a1 @ im @ np.conj(np.swapaxes(a2, -1, -2))) * tap[:, :, None, None] * (L * L)
        for k in range(tc.shape[0]):
            t, c = tc[k]
            lam_inv = freqs[c] / C0
            u, v, w = uvw[bl, t] * lam_inv
            ph = np.exp(-2j * np.pi * (u * l + v * m + w * nprime))
            out[bl, t, c] = (ph[:, :, None, None] * b).sum(axis=(0, 1)).reshape(4)
    return out
