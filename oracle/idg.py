"""Image-domain gridding and degridding, subgrid by subgrid, in float64 (oracle).

Conventions (each is a reading of the paper; the list of readings is kept with
the design notes of the repository):

* Master grid ``grid[pol][y][x]`` (complex), x <-> u, y <-> v; grid pixel x
  has u_x = (x - N/2) / S, the uv cell being du = 1/S.
* Subgrid p has corner (x0, y0) and centre pixel (x0 + L/2, y0 + L/2), so
  u_0p = (x0 + L/2 - N/2) / S (the central pixel of §3.2 lies on the grid
  lattice because the adder shifts by whole pixels).
* Subgrid image pixel (j, i) (row j <-> m, column i <-> l) sits at
  l_i = (i - L/2) S / L, m_j = (j - L/2) S / L -- the pixel positions of §2
  with L_p pixels across S -- and n'_ij = sqrt(1 - l_i^2 - m_j^2) - 1.
* Polarised data (§3.4): a sample is the 2x2 matrix Y = [[XX, XY], [YX, YY]];
  an A-term is a 2x2 Jones matrix per (slot, station, pixel), row-major
  [J00, J01, J10, J11].  With stations s1 < s2 of the baseline, gridding
  applies c * A_s1^H Y A_s2 per pixel and degridding applies c * A_s1 B A_s2^H;
  these reduce to c^* y (Algorithm 1) and c I (Algorithm 2) in the scalar case,
  where the per-block kernel is g_s1^* g_s2 (§2, definition of A_k) and the
  multiplication by the kernel is moved out of the visibility loop (§3.4).
* Subgrid transform (Algorithm 1, "FFT"): the centred forward DFT
  V[b][a] = sum_{j,i} I[j][i] exp(-2 pi i ((a-L/2)(i-L/2) + (b-L/2)(j-L/2)) / L),
  unnormalised.  Degridding (Algorithm 2, "IFFT") uses its conjugate
  transpose, also unnormalised, so that degridding is the exact adjoint of
  gridding on the planned samples.
* W-offset: subgrid p of W-layer j has w_0p = j * w_step (Algorithms 1 and 2
  subtract w_0p; without layers w_step = 0 and the whole w-term is carried by
  w_k n'_ij).  With layers the master grid is one [4, N, N] grid per layer,
  ``grid[j - wlayer_min]``; the image steps apply exp(+-2 pi i w_0 n') per layer.
"""

import numpy as np

from .plan import C0, F


def lmn(L, S):
    """l_i (by column), m_j (by row) and n'_ij of the subgrid image lattice (§2, §3.3)."""
    idx = (np.arange(L, dtype=np.float64) - L // 2) * (S / L)
    l = idx[None, :]
    m = idx[:, None]
    nprime = np.sqrt(1.0 - l * l - m * m) - 1.0
    return np.broadcast_to(l, (L, L)), np.broadcast_to(m, (L, L)), nprime


def centred_dft_matrix(L, sign=-1):
    """D[a, i] = exp(sign * 2 pi i (a - L/2)(i - L/2) / L), exact integer phase mod L."""
    k = np.arange(L, dtype=np.int64) - L // 2
    r = np.mod(np.outer(k, k), L).astype(np.float64)
    return np.exp(sign * 2j * np.pi * r / L)


def subgrid_centre(sub, N, L, S):
    u0 = (sub[F["x0"]] + L // 2 - N // 2) / S
    v0 = (sub[F["y0"]] + L // 2 - N // 2) / S
    return u0, v0


def sample_uvw(uvw, freqs, bl, tc):
    """(u, v, w) in wavelengths of the samples (t, c) of baseline ``bl`` (§2: u_k = u_ijr / lambda_q)."""
    t, c = tc[:, 0], tc[:, 1]
    lam_inv = freqs[c] / C0
    return uvw[bl, t, 0] * lam_inv, uvw[bl, t, 1] * lam_inv, uvw[bl, t, 2] * lam_inv


def _jones(aterms, slot, st, L):
    a = np.asarray(aterms[slot, st], dtype=np.complex128).reshape(L * L, 2, 2)
    return a


def _as_matrices(x4):
    return x4.reshape(-1, 2, 2)


def phasor_matrix(du, dv, w, l, m, nprime, sign):
    """E[k, pix] = exp(sign 2 pi i (du_k l + dv_k m + w_k n'))  -- the phase of eq. ShiftedDirectImaging."""
    ph = (du[:, None] * l.reshape(1, -1) + dv[:, None] * m.reshape(1, -1)
          + w[:, None] * nprime.reshape(1, -1))
    return np.exp(sign * 2j * np.pi * ph)


def grid_subgrid_image(plan, p, uvw, freqs, vis, aterms, taper):
    """Subgrid image I_p [4, L, L] before the transform (Algorithm 1, inner loops; §3.4)."""
    N, L, S = plan.grid_size, plan.subgrid_size, plan.image_size
    sub = plan.subgrids[p]
    tc = plan.subgrid_samples(p)
    bl = sub[F["bl"]]
    u, v, w = sample_uvw(uvw, freqs, bl, tc)
    u0, v0 = subgrid_centre(sub, N, L, S)
    l, m, nprime = lmn(L, S)
    e = phasor_matrix(u - u0, v - v0, w - plan.w_offset(p), l, m, nprime, +1.0)   # [K, L*L]
    y = np.asarray(vis[bl, tc[:, 0], tc[:, 1]], dtype=np.complex128)     # [K, 4]
    s = e.T @ y                                                         # [L*L, 4]
    a1 = _jones(aterms, sub[F["slot"]], sub[F["st1"]], L)
    a2 = _jones(aterms, sub[F["slot"]], sub[F["st2"]], L)
    img = np.conj(np.transpose(a1, (0, 2, 1))) @ _as_matrices(s) @ a2   # A1^H S A2
    img = img.reshape(L * L, 4) * np.asarray(taper, np.float64).reshape(L * L, 1)
    return img.T.reshape(4, L, L)


def forward_subgrid_dft(img):
    L = img.shape[-1]
    d = centred_dft_matrix(L, -1)
    return np.stack([d @ img[pol] @ d.T for pol in range(img.shape[0])])


def inverse_subgrid_dft(sg):
    L = sg.shape[-1]
    d = centred_dft_matrix(L, +1)
    return np.stack([d @ sg[pol] @ d.T for pol in range(sg.shape[0])])


def grid_subgrid(plan, p, uvw, freqs, vis, aterms, taper):
    """Subgrid V_p [4, L, L] in the uv domain: image, then the centred DFT (Algorithm 1)."""
    return forward_subgrid_dft(grid_subgrid_image(plan, p, uvw, freqs, vis, aterms, taper))


def layer_grid(plan, g, p):
    """The [4, N, N] grid of subgrid p's W-layer inside g ([4, N, N], or [layers, 4, N, N] with layers)."""
    return g[plan.subgrids[p, F["wlayer"]] - plan.wlayer_min] if plan.w_step > 0 else g


def grid(plan, uvw, freqs, vis, aterms, taper, subgrid_ids=None, out=None):
    """Master grid complex128, [4, N, N] ([nr_wlayers, 4, N, N] with W-layers): the sum of all
    subgrids added at their corners."""
    N, L = plan.grid_size, plan.subgrid_size
    shape = (plan.nr_wlayers, 4, N, N) if plan.w_step > 0 else (4, N, N)
    g = np.zeros(shape, np.complex128) if out is None else out
    ids = range(plan.nr_subgrids) if subgrid_ids is None else subgrid_ids
    for p in ids:
        sub = plan.subgrids[p]
        x0, y0 = sub[F["x0"]], sub[F["y0"]]
        layer_grid(plan, g, p)[:, y0:y0 + L, x0:x0 + L] += grid_subgrid(plan, p, uvw, freqs, vis, aterms, taper)
    return g


def degrid_subgrid(plan, p, uvw, freqs, grid_in, aterms, taper):
    """Visibilities [K_p, 4] of subgrid p: split, inverse DFT, A-terms and taper, sum (Algorithm 2)."""
    N, L, S = plan.grid_size, plan.subgrid_size, plan.image_size
    sub = plan.subgrids[p]
    x0, y0 = sub[F["x0"]], sub[F["y0"]]
    vp = np.asarray(layer_grid(plan, grid_in, p)[:, y0:y0 + L, x0:x0 + L], dtype=np.complex128)
    img = inverse_subgrid_dft(vp).reshape(4, L * L).T                  # [L*L, 4]
    a1 = _jones(aterms, sub[F["slot"]], sub[F["st1"]], L)
    a2 = _jones(aterms, sub[F["slot"]], sub[F["st2"]], L)
    b = a1 @ _as_matrices(img) @ np.conj(np.transpose(a2, (0, 2, 1)))  # A1 I A2^H
    b = b.reshape(L * L, 4) * np.asarray(taper, np.float64).reshape(L * L, 1)
    tc = plan.subgrid_samples(p)
    u, v, w = sample_uvw(uvw, freqs, sub[F["bl"]], tc)
    u0, v0 = subgrid_centre(sub, N, L, S)
    l, m, nprime = lmn(L, S)
    e = phasor_matrix(u - u0, v - v0, w - plan.w_offset(p), l, m, nprime, -1.0)  # [K, L*L]
    return e @ b


def degrid(plan, uvw, freqs, grid_in, aterms, taper, subgrid_ids=None):
    """Visibilities [nbl, nt, nch, 4] complex128; unplanned (flagged or dropped) samples are 0."""
    out = np.zeros((plan.nr_baselines, plan.nr_timesteps, plan.nr_channels, 4), np.complex128)
    ids = range(plan.nr_subgrids) if subgrid_ids is None else subgrid_ids
    for p in ids:
        tc = plan.subgrid_samples(p)
        out[plan.subgrids[p, F["bl"]], tc[:, 0], tc[:, 1]] = degrid_subgrid(
            plan, p, uvw, freqs, grid_in, aterms, taper)
    return out
