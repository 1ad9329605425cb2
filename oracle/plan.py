"""Partitioning of visibilities into subgrids (oracle).

The paper (§3.2 Partitioning, Fig. 2) partitions the data into P blocks, each
holding one baseline, several timesteps and several channels, such that the
support of every visibility in the block lies inside a box of L x L pixels --
the subgrid -- whose central pixel is (u_0p, v_0p) and whose corner in the
master grid is (q_0p, r_0p).  Subgrids may overlap and need not cover the grid.
§3.4 (Variations) adds that blocks may be cut so that one image-domain kernel
(A-term) applies per block.  The paper gives no algorithm beyond the box
criterion, so this module fixes one deterministic rule; the C++ planner of the
library implements the same rule independently.

Rule (all geometry in float64, no fused multiply-add):

* s_c = f_c / c0; u = uvw_u * s_c (wavelengths, the definition of u_k in §2);
  pixel coordinate x = u * S + N/2, y = v * S + N/2 (grid pixel x has
  u_x = (x - N/2)/S); w-support wpix = ceil((|w| * S) * S) pixels.
* A set of samples fits iff  (max x - min x) + (beta + max wpix) <= L - 1  and
  the same for y.  Flags do not enter the geometry.
* W-layers (w_step > 0; the offset w_0p of Algorithms 1 and 2): a block's
  layer is j = floor(w_mid / w_step + 0.5) with w_mid = (w(t0, c_lo) +
  w(t0, c_hi)) * 0.5 the mid-band w of its first timestep (w is linear in
  frequency), its offset w_0p = j * w_step, and the w-support of a sample
  becomes ceil((|w - w_0p| * S) * S).  In the channel-group step a timestep
  taken alone uses its own layer.  With w_step = 0 every layer is 0 and
  w_0p = 0.
* Per baseline, channels are grouped first: start from one group with all
  channels; a group of more than one channel that does not fit at some
  timestep (taking that timestep's samples alone) is split into a lower half
  of floor(n/2) channels and an upper half, recursively.
* Per channel group, time is scanned greedily from t = 0: a block starting at
  t0 takes timesteps t0, t0+1, ... while t - t0 < T_max, t lies in the A-term
  slot of t0 (slot = t // aterm_timesteps) and the union of the block's
  samples fits.  A timestep whose samples do not fit even alone has its
  unflagged samples dropped.
* A finished block with K_p unflagged samples (K_p > 0) gets its centre pixel
  cx = floor((min x + max x) * 0.5 + 0.5) and corner x0 = cx - L/2 (same for
  y).  If 0 <= x0, x0 + L <= N, 0 <= y0, y0 + L <= N it becomes a subgrid,
  otherwise its samples are dropped (no wrap-around).
* Subgrids are ordered by baseline, channel group, then time; each subgrid's
  samples are its unflagged (t, c) in t-major, c-minor order.

Output: ``Plan.subgrids`` int64 [P, 13] with the columns of ``FIELDS`` and
``Plan.samples`` int64 [K, 2] of absolute (t, c).
"""

from dataclasses import dataclass

import numpy as np

C0 = 299792458.0

FIELDS = ("bl", "t0", "nt", "c0", "nc", "x0", "y0", "slot", "st1", "st2", "nvis", "vis_offset", "wlayer")
F = {name: i for i, name in enumerate(FIELDS)}


@dataclass
class Plan:
    grid_size: int
    image_size: float
    subgrid_size: int
    kernel_size: int
    max_timesteps: int
    aterm_timesteps: int
    nr_baselines: int
    nr_timesteps: int
    nr_channels: int
    subgrids: np.ndarray      # int64 [P, 13]
    samples: np.ndarray       # int64 [K, 2]  (t, c)
    nr_gridded: int
    nr_dropped: int
    nr_flagged: int
    w_step: float = 0.0

    @property
    def nr_subgrids(self):
        return self.subgrids.shape[0]

    @property
    def wlayer_min(self):
        return int(self.subgrids[:, F["wlayer"]].min()) if self.nr_subgrids else 0

    @property
    def nr_wlayers(self):
        return int(self.subgrids[:, F["wlayer"]].max()) - self.wlayer_min + 1 if self.nr_subgrids else 1

    def w_offset(self, p):
        """w_0p of subgrid p in wavelengths."""
        return float(self.subgrids[p, F["wlayer"]]) * self.w_step

    def subgrid_samples(self, p):
        off, n = self.subgrids[p, F["vis_offset"]], self.subgrids[p, F["nvis"]]
        return self.samples[off:off + n]


def _fits(span_x, span_y, wmax, beta, L):
    ext = float(beta) + wmax
    return (span_x + ext <= L - 1.0) & (span_y + ext <= L - 1.0)


def make_plan(grid_size, image_size, subgrid_size, kernel_size, max_timesteps, aterm_timesteps,
              baselines, uvw, freqs, flags=None, w_step=0.0):
    N, S, L, beta = int(grid_size), float(image_size), int(subgrid_size), int(kernel_size)
    tmax, aslot = int(max_timesteps), int(aterm_timesteps)
    uvw = np.asarray(uvw, dtype=np.float64)
    freqs = np.asarray(freqs, dtype=np.float64)
    nbl, nt, _ = uvw.shape
    nch = freqs.size
    half_n = N / 2.0
    s = freqs / C0

    rows, samples = [], []
    n_grid = n_drop = 0
    n_flag = 0 if flags is None else int(np.count_nonzero(flags))

    w_step = float(w_step)
    for b in range(nbl):
        x = uvw[b, :, 0][:, None] * s[None, :] * S + half_n          # [nt, nch]
        y = uvw[b, :, 1][:, None] * s[None, :] * S + half_n
        w = uvw[b, :, 2][:, None] * s[None, :]                       # wavelengths
        unflagged = np.ones((nt, nch), bool) if flags is None else (np.asarray(flags[b]) == 0)

        def layers(lo, hi):
            """W-layer of each timestep taken as a block start, for channels [lo, hi)."""
            if w_step <= 0.0:
                return np.zeros(nt)
            return np.floor((w[:, lo] + w[:, hi - 1]) * 0.5 / w_step + 0.5)

        def wsupport(lo, hi, w0):
            """[nt] max over channels of ceil(|w - w0| S^2), w0 per timestep."""
            return np.ceil(np.abs(w[:, lo:hi] - w0[:, None]) * S * S).max(1)

        def group_stats(lo, hi):
            return (x[:, lo:hi].min(1), x[:, lo:hi].max(1), y[:, lo:hi].min(1), y[:, lo:hi].max(1),
                    wsupport(lo, hi, layers(lo, hi) * w_step))

        groups = []

        def split(lo, hi):
            if hi - lo == 1:
                groups.append((lo, hi))
                return
            mnx, mxx, mny, mxy, wm = group_stats(lo, hi)
            if np.all(_fits(mxx - mnx, mxy - mny, wm, beta, L)):
                groups.append((lo, hi))
                return
            mid = lo + (hi - lo) // 2
            split(lo, mid)
            split(mid, hi)

        if nt > 0 and nch > 0:
            split(0, nch)

        for lo, hi in groups:
            mnx, mxx, mny, mxy, wm = group_stats(lo, hi)
            alone = _fits(mxx - mnx, mxy - mny, wm, beta, L)
            lay = layers(lo, hi)
            t = 0
            while t < nt:
                if not alone[t]:
                    n_drop += int(unflagged[t, lo:hi].sum())
                    t += 1
                    continue
                t_lim = min(nt, t + tmax, (t // aslot + 1) * aslot)
                cmnx = np.minimum.accumulate(mnx[t:t_lim])
                cmxx = np.maximum.accumulate(mxx[t:t_lim])
                cmny = np.minimum.accumulate(mny[t:t_lim])
                cmxy = np.maximum.accumulate(mxy[t:t_lim])
                w0 = np.full(nt, lay[t] * w_step)                   # the block's offset for every timestep
                cwm = np.maximum.accumulate(wsupport(lo, hi, w0)[t:t_lim])
                ok = _fits(cmxx - cmnx, cmxy - cmny, cwm, beta, L)
                bad = np.flatnonzero(~ok)
                n_ok = ok.size if bad.size == 0 else int(bad[0])
                t0, t1 = t, t + n_ok                                  # block [t0, t1)
                t = t1
                sel = unflagged[t0:t1, lo:hi]
                kp = int(sel.sum())
                if kp == 0:
                    continue
                bx0, bx1 = cmnx[n_ok - 1], cmxx[n_ok - 1]
                by0, by1 = cmny[n_ok - 1], cmxy[n_ok - 1]
                x0 = np.floor((bx0 + bx1) * 0.5 + 0.5) - L // 2
                y0 = np.floor((by0 + by1) * 0.5 + 0.5) - L // 2
                if not (x0 >= 0 and x0 + L <= N and y0 >= 0 and y0 + L <= N):
                    n_drop += kp
                    continue
                tt, cc = np.nonzero(sel)
                samples.append(np.stack([tt + t0, cc + lo], axis=1))
                rows.append([b, t0, t1 - t0, lo, hi - lo, int(x0), int(y0), t0 // aslot,
                             int(baselines[b][0]), int(baselines[b][1]), kp, n_grid, int(lay[t0])])
                n_grid += kp

    sub = np.array(rows, dtype=np.int64).reshape(-1, len(FIELDS))
    smp = np.concatenate(samples).astype(np.int64, copy=False) if samples else np.zeros((0, 2), np.int64)
    return Plan(N, S, L, beta, tmax, aslot, nbl, nt, nch, sub, smp, n_grid, n_drop, n_flag, w_step)


def plan_workload(wl, w_step=0.0):
    """Plan a ``synth.Workload`` (convenience wrapper)."""
    return make_plan(wl.grid_size, wl.image_size, wl.subgrid_size, wl.kernel_size, wl.max_timesteps,
                     wl.aterm_timesteps, wl.baselines, wl.uvw, wl.freqs, wl.flags, w_step)
