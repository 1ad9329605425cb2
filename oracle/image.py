"""Master grid <-> image (the steps around the hot path), in float64 (oracle).

Test infrastructure only: nothing in the library calls this module.

Algorithm 1 ends with the transform of the master grid to the image domain
and the division by the taper; Algorithm 2 starts from the model image
divided by the taper and transformed to the uv grid (§3.3: the subgrid
images approximate the image multiplied by the taper, so the image is the
transform of the grid divided by it).  Conventions (the readings are kept with
the design notes of the repository):

* grid G[pol][v][u] with u_u = (u - N/2) / S; image I[pol][y][x] at
  l_x = (x - N/2) S / N, m_y = (y - N/2) S / N (§2 pixel positions with N
  pixels across S), so u_u l_x = (u - N/2)(x - N/2) / N exactly;
* grid_to_image: I[y][x] = sum_{v,u} G[v][u] exp(+2 pi i ((u - N/2)(x - N/2) +
  (v - N/2)(y - N/2)) / N) / (corr_m[y] corr_l[x]), the grid's DTFT at the image
  pixels divided by a separable correction (for the taper c of the subgrids,
  corr_l[x] = L c(l_x), which makes the division by L^2 c(l) c(m));
* image_to_grid: its adjoint, G[v][u] = sum_{y,x} I[y][x] / (corr_m[y] corr_l[x])
  exp(-2 pi i (...) / N).
"""

import numpy as np


def centred_dft(N, sign):
    """D[a, b] = exp(sign 2 pi i (a - N/2)(b - N/2) / N), exact integer phase mod N."""
    k = np.arange(N, dtype=np.int64) - N // 2
    r = np.mod(np.outer(k, k), N).astype(np.float64)
    return np.exp(sign * 2j * np.pi * r / N)


def grid_to_image(grid, corr_l, corr_m):
    """Image [4, N, N] complex128 from grid [4, N, N]: the grid's DTFT at the image pixels / correction."""
    g = np.asarray(grid, np.complex128)
    N = g.shape[-1]
    d = centred_dft(N, +1)                  # d[x, u]
    corr = np.outer(np.asarray(corr_m, np.float64), np.asarray(corr_l, np.float64))
    return np.stack([d @ g[p] @ d.T for p in range(g.shape[0])]) / corr


def image_to_grid(image, corr_l, corr_m):
    """Grid [4, N, N] complex128 from image [4, N, N]: the adjoint of grid_to_image."""
    im = np.asarray(image, np.complex128)
    N = im.shape[-1]
    d = centred_dft(N, -1)                  # d[u, x]
    corr = np.outer(np.asarray(corr_m, np.float64), np.asarray(corr_l, np.float64))
    x = im / corr
    return np.stack([d @ x[p] @ d.T for p in range(im.shape[0])])


def _centred_row(N, k, sign):
    """exp(sign 2 pi i (j - N/2)(k - N/2) / N) over j = 0 .. N-1, exact integer phase mod N."""
    j = np.arange(N, dtype=np.int64) - N // 2
    r = np.mod(j * (int(k) - N // 2), N).astype(np.float64)
    return np.exp(sign * 2j * np.pi * r / N)


def grid_to_image_at(grid, xs, ys, corr_l, corr_m):
    """image[:, ys[i], xs[i]] of grid_to_image, one pixel at a time (for grids too large for the whole transform)."""
    g = np.asarray(grid)
    N = g.shape[-1]
    out = np.zeros((g.shape[0], len(xs)), np.complex128)
    for p in range(g.shape[0]):
        gp = g[p].astype(np.complex128)
        for i, (x, y) in enumerate(zip(xs, ys)):
            dx, dy = _centred_row(N, x, +1), _centred_row(N, y, +1)
            out[p, i] = dy @ (gp @ dx) / (float(corr_m[y]) * float(corr_l[x]))
    return out


def image_to_grid_at(image, us, vs, corr_l, corr_m):
    """grid[:, vs[i], us[i]] of image_to_grid, one cell at a time."""
    im = np.asarray(image)
    N = im.shape[-1]
    cl = 1.0 / np.asarray(corr_l, np.float64)
    cm = 1.0 / np.asarray(corr_m, np.float64)
    out = np.zeros((im.shape[0], len(us)), np.complex128)
    for p in range(im.shape[0]):
        ip = im[p].astype(np.complex128)
        for i, (u, v) in enumerate(zip(us, vs)):
            du, dv = _centred_row(N, u, -1) * cl, _centred_row(N, v, -1) * cm
            out[p, i] = dv @ (ip @ du)
    return out


def nprime_image(N, S):
    """n'(l_x, m_y) = sqrt(1 - l^2 - m^2) - 1 at the master-grid image pixels [y, x] (0 under the
    square root outside the unit circle, where no sky exists)."""
    l = (np.arange(N) - N // 2) * float(S) / N
    r2 = l[None, :] ** 2 + l[:, None] ** 2
    return np.sqrt(np.maximum(0.0, 1.0 - r2)) - 1.0


def wstack_to_image(grids, w0s, S, corr_l, corr_m):
    """Image [4, N, N] from W-layer grids [layers, 4, N, N] with offsets w0s [layers]:
    sum_j exp(+2 pi i w0_j n'(l, m)) grid_to_image(grids[j]) -- the w-term the layer's subgrids left
    out (w_k - w0_j) put back in the image domain -- divided by the correction."""
    g = np.asarray(grids, np.complex128)
    N = g.shape[-1]
    n1 = nprime_image(N, S)
    ones = np.ones(N)
    img = sum(np.exp(2j * np.pi * float(w0) * n1) * grid_to_image(g[j], ones, ones) for j, w0 in enumerate(w0s))
    return img / np.outer(np.asarray(corr_m, np.float64), np.asarray(corr_l, np.float64))


def image_to_wstack(image, w0s, S, corr_l, corr_m):
    """W-layer grids [layers, 4, N, N]: the adjoint of wstack_to_image."""
    im = np.asarray(image, np.complex128)
    N = im.shape[-1]
    n1 = nprime_image(N, S)
    ones = np.ones(N)
    x = im / np.outer(np.asarray(corr_m, np.float64), np.asarray(corr_l, np.float64))
    return np.stack([image_to_grid(np.exp(-2j * np.pi * float(w0) * n1) * x, ones, ones) for w0 in w0s])


def wstack_to_image_at(grids, w0s, S, xs, ys, corr_l, corr_m):
    """image[:, ys[i], xs[i]] of wstack_to_image, one pixel at a time."""
    g = np.asarray(grids)
    N = g.shape[-1]
    n1 = nprime_image(N, S)[np.asarray(ys), np.asarray(xs)]
    ones = np.ones(N)
    out = sum(np.exp(2j * np.pi * float(w0) * n1)[None, :] * grid_to_image_at(g[j], xs, ys, ones, ones)
              for j, w0 in enumerate(w0s))
    cl, cm = np.asarray(corr_l, np.float64), np.asarray(corr_m, np.float64)
    return out / (cm[np.asarray(ys)] * cl[np.asarray(xs)])[None, :]


def image_to_wstack_at(image, w0s, S, us, vs, corr_l, corr_m):
    """grids[:, :, vs[i], us[i]] of image_to_wstack ([layers, 4, len(us)]), one cell at a time."""
    im = np.asarray(image)
    N = im.shape[-1]
    n1 = nprime_image(N, S)
    ones = np.ones(N)
    x = im / np.outer(np.asarray(corr_m, np.float64), np.asarray(corr_l, np.float64))
    return np.stack([image_to_grid_at(np.exp(-2j * np.pi * float(w0) * n1) * x, us, vs, ones, ones) for w0 in w0s])
