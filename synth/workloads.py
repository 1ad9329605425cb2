"""Seeded synthetic workloads with the shapes of the paper's gridding problems.

Geometry follows the measurement equation's conventions (§2): visibilities are
indexed by (baseline, timestep, channel), uvw are per (baseline, timestep) in
metres, and a sample's uvw in wavelengths is uvw * f_c / c0 (the definition of
u_k, v_k, w_k after the measurement equation).  Station positions are local
East/North/Up coordinates; baseline vectors are rotated to uvw for a source at
declination ``dec`` observed at hour angle H(t) = H0 + omega_earth * t.

Workloads (sizes are the defaults; ``subset`` cuts them down):

* ``tiny``      8 stations in a 1 km-radius disk, 32 x 10 s, 4 channels at
                150-151 MHz, w = 0, identity A-terms, L = 24, 512^2 grid at 1'.
* ``lofar``     48 stations, radius |N(0, 3 km)|, 2048 x 1 s at dec 52 deg,
                16 channels at 120-180 MHz, |w| up to ~2e3 wavelengths,
                L = 32 with 128-timestep blocks, 4096^2 grid at 2.5",
                near-identity A-terms changing every 256 s.
* ``skalow``    512 stations on 3 log-spiral arms to 35 km, 64 x 1 s,
                16 channels at 50-350 MHz, L = 32, 8192^2 grid at 1",
                A-terms changing every 32 timesteps, 10 % random flags.
* ``precision`` the ``lofar`` geometry and A-terms with a 10 Jy point
                source at (l, m) = (sin 5 deg, 0), visibilities from the
                measurement equation in FP64 with identity gains.

Nothing here performs any part of image-domain gridding.
"""

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

from .taper import pswf_taper_2d

C0 = 299792458.0                      # speed of light, m/s
OMEGA_EARTH = 7.2921159e-5            # rad/s
ARCSEC = np.pi / (180.0 * 3600.0)
ARCMIN = 60.0 * ARCSEC
SEED_BASE = 1909_07226

WORKLOAD_NAMES = ("tiny", "lofar", "skalow", "precision")


@dataclass
class Workload:
    name: str
    grid_size: int            # N
    image_size: float         # S = N * cell (direction-cosine units)
    subgrid_size: int         # L
    kernel_size: int          # beta, taper support in uv pixels
    max_timesteps: int        # T_max per subgrid
    aterm_timesteps: int      # A-term slot length in timesteps
    nr_stations: int
    baselines: np.ndarray     # int32 [nbl, 2] station pairs p < q
    uvw: np.ndarray           # float64 [nbl, nt, 3] metres
    freqs: np.ndarray         # float64 [nch] Hz
    flags: Optional[np.ndarray]  # uint8 [nbl, nt, nch] (nonzero = flagged) or None
    vis: Optional[np.ndarray]    # complex64 [nbl, nt, nch, 4] XX, XY, YX, YY
    aterms: np.ndarray        # complex64 [nslot, nst, L, L, 4] Jones row-major
    taper: np.ndarray         # float32 [L, L]
    meta: dict = field(default_factory=dict)

    @property
    def nr_baselines(self):
        return self.uvw.shape[0]

    @property
    def nr_timesteps(self):
        return self.uvw.shape[1]

    @property
    def nr_channels(self):
        return self.freqs.shape[0]

    @property
    def nr_slots(self):
        return self.aterms.shape[0]

    @property
    def nr_samples(self):
        return self.nr_baselines * self.nr_timesteps * self.nr_channels


# ----------------------------------------------------------------------------
# geometry


def _baseline_pairs(nst):
    p, q = np.triu_indices(nst, k=1)
    return np.stack([p, q], axis=1).astype(np.int32)


def _enu_to_xyz(enu, lat):
    e, n, u = enu[..., 0], enu[..., 1], enu[..., 2]
    x = -np.sin(lat) * n + np.cos(lat) * u
    y = e
    z = np.cos(lat) * n + np.sin(lat) * u
    return np.stack([x, y, z], axis=-1)


def _uvw_tracks(bxyz, hour_angles, dec):
    """Rotate equatorial baseline vectors [nbl, 3] to uvw [nbl, nt, 3] (metres)."""
    x = bxyz[:, 0][:, None]
    y = bxyz[:, 1][:, None]
    z = bxyz[:, 2][:, None]
    sh = np.sin(hour_angles)[None, :]
    ch = np.cos(hour_angles)[None, :]
    sd, cd = np.sin(dec), np.cos(dec)
    u = sh * x + ch * y
    v = -sd * ch * x + sd * sh * y + cd * z
    w = cd * ch * x - cd * sh * y + sd * z
    return np.stack([u, v, w], axis=-1)


def _channel_centres(f_lo, f_hi, nch):
    return f_lo + (np.arange(nch, dtype=np.float64) + 0.5) * (f_hi - f_lo) / nch


def _complex_normal(rng, shape, scale=1.0):
    """Circular complex normal with E|z|^2 = scale^2, complex64."""
    re = rng.standard_normal(size=shape, dtype=np.float32)
    im = rng.standard_normal(size=shape, dtype=np.float32)
    s = np.float32(scale * np.sqrt(0.5))
    out = np.empty(shape, dtype=np.complex64)
    out.real = re * s
    out.imag = im * s
    return out


def _identity_aterms(nslot, nst, L):
    a = np.zeros((nslot, nst, L, L, 4), dtype=np.complex64)
    a[..., 0] = 1.0
    a[..., 3] = 1.0
    return a


def _near_identity_aterms(rng, nslot, nst, L, scale=0.05):
    a = _identity_aterms(nslot, nst, L)
    a += _complex_normal(rng, a.shape, scale)
    return a


def _point_source_vis(uvw, freqs, l, m, flux):
    """Visibilities of an unpolarised point source from the measurement equation.

    y = flux * exp(-2 pi i (u l + v m + w n')), n' = sqrt(1 - l^2 - m^2) - 1,
    with (u, v, w) = uvw * f / c0 (§2, eq. of the measurement equation with the
    n' convention of the same section).  XX = YY = y, XY = YX = 0.  FP64, then
    cast to complex64.
    """
    nprime = np.sqrt(1.0 - l * l - m * m) - 1.0
    s = freqs / C0
    nbl, nt, _ = uvw.shape
    out = np.zeros((nbl, nt, freqs.size, 4), dtype=np.complex64)
    for b in range(nbl):
        ph = (uvw[b, :, 0, None] * l + uvw[b, :, 1, None] * m + uvw[b, :, 2, None] * nprime) * s[None, :]
        y = flux * np.exp(-2j * np.pi * ph)
        out[b, :, :, 0] = y
        out[b, :, :, 3] = y
    return out


def _max_abs_w_wavelengths(bxyz, h0, nt, dt, dec, f_max):
    # w only, on every 4th timestep plus the last one (used only to choose H0)
    t = np.unique(np.append(np.arange(0, nt, 4), nt - 1))
    h = h0 + OMEGA_EARTH * dt * t
    cd, sd = np.cos(dec), np.sin(dec)
    w = (cd * np.cos(h))[None, :] * bxyz[:, 0, None] - (cd * np.sin(h))[None, :] * bxyz[:, 1, None] \
        + sd * bxyz[:, 2, None]
    return np.abs(w).max() * f_max / C0


def _solve_h0_for_wmax(bxyz, nt, dt, dec, f_max, target):
    """Smallest |H0| (H0 <= 0) at which the track's max |w| reaches ``target`` wavelengths."""
    step = np.deg2rad(1.5)            # 6 minutes of hour angle
    lo, hi = 0.0, None
    h = 0.0
    for _ in range(240):
        if _max_abs_w_wavelengths(bxyz, h, nt, dt, dec, f_max) >= target:
            hi = h
            break
        lo = h
        h -= step
    if hi is None:
        return lo
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if _max_abs_w_wavelengths(bxyz, mid, nt, dt, dec, f_max) >= target:
            hi = mid
        else:
            lo = mid
    return lo


# ----------------------------------------------------------------------------
# workloads


def _tiny(seed, with_vis, nt=32, nch=4):
    # the defaults are the tiny workload; longer / wider variants keep 10 s steps and 0.25 MHz channels
    rng = np.random.default_rng(seed)
    nst, dt = 8, 10.0
    L, N, beta = 24, 512, 7
    cell = ARCMIN
    lat, dec = np.deg2rad(52.9), np.deg2rad(52.0)
    r = 1000.0 * np.sqrt(rng.random(nst))
    th = 2 * np.pi * rng.random(nst)
    enu = np.stack([r * np.cos(th), r * np.sin(th), np.zeros(nst)], axis=1)
    bl = _baseline_pairs(nst)
    xyz = _enu_to_xyz(enu, lat)
    bxyz = xyz[bl[:, 1]] - xyz[bl[:, 0]]
    h = OMEGA_EARTH * dt * np.arange(nt)
    uvw = _uvw_tracks(bxyz, h, dec)
    uvw[..., 2] = 0.0
    freqs = _channel_centres(150e6, 150e6 + 0.25e6 * nch, nch)
    aterms = _identity_aterms(1, nst, L)
    vis = None
    if with_vis:
        vis = _complex_normal(rng, (bl.shape[0], nt, nch, 4))
        vis += _point_source_vis(uvw, freqs, 37.3 * cell, -21.7 * cell, 1.0)
    return Workload("tiny", N, N * cell, L, beta, 16, nt, nst, bl, uvw, freqs, None, vis,
                    aterms, pswf_taper_2d(L, beta),
                    dict(cell=cell, dt=dt, h0=0.0, dec=dec, lat=lat, source_px=(37.3, -21.7)))


def _lofar_geometry(rng):
    nst, nt, dt, nch = 48, 2048, 1.0, 16
    lat, dec = np.deg2rad(52.9), np.deg2rad(52.0)
    r = np.abs(rng.normal(0.0, 3000.0, nst))
    th = 2 * np.pi * rng.random(nst)
    enu = np.stack([r * np.cos(th), r * np.sin(th), np.zeros(nst)], axis=1)
    bl = _baseline_pairs(nst)
    xyz = _enu_to_xyz(enu, lat)
    bxyz = xyz[bl[:, 1]] - xyz[bl[:, 0]]
    freqs = _channel_centres(120e6, 180e6, nch)
    h0 = _solve_h0_for_wmax(bxyz, nt, dt, dec, freqs.max(), 1950.0)
    h = h0 + OMEGA_EARTH * dt * np.arange(nt)
    uvw = _uvw_tracks(bxyz, h, dec)
    return nst, nt, dt, bl, uvw, freqs, dict(dt=dt, h0=h0, dec=dec, lat=lat)


def _lofar(seed, with_vis):
    rng = np.random.default_rng(seed)
    nst, nt, dt, bl, uvw, freqs, meta = _lofar_geometry(rng)
    L, N, beta = 32, 4096, 7
    cell = 2.5 * ARCSEC
    aslot = 256
    nslot = -(-nt // aslot)
    aterms = _near_identity_aterms(rng, nslot, nst, L)
    vis = _complex_normal(rng, (bl.shape[0], nt, freqs.size, 4)) if with_vis else None
    meta.update(cell=cell)
    return Workload("lofar", N, N * cell, L, beta, 128, aslot, nst, bl, uvw, freqs, None, vis,
                    aterms, pswf_taper_2d(L, beta), meta)


def _precision(seed, with_vis):
    # the station layout, track and A-terms of ``lofar`` (drawn from that workload's seed, in its
    # order); the data are a point source with identity gains, so ``seed`` draws nothing here
    rng = np.random.default_rng(SEED_BASE + 2)
    nst, nt, dt, bl, uvw, freqs, meta = _lofar_geometry(rng)
    L, N, beta = 32, 4096, 7
    cell = 2.5 * ARCSEC
    aslot = 256
    nslot = -(-nt // aslot)
    aterms = _near_identity_aterms(rng, nslot, nst, L)
    src = (np.sin(np.deg2rad(5.0)), 0.0)
    vis = _point_source_vis(uvw, freqs, src[0], src[1], 10.0) if with_vis else None
    meta.update(cell=cell, source_lm=src, flux=10.0)
    return Workload("precision", N, N * cell, L, beta, 128, aslot, nst, bl, uvw, freqs, None, vis,
                    aterms, pswf_taper_2d(L, beta), meta)


def _skalow(seed, with_vis):
    rng = np.random.default_rng(seed)
    nst, nt, dt, nch = 512, 64, 1.0, 16
    L, N, beta = 32, 8192, 7
    cell = ARCSEC
    lat = dec = np.deg2rad(-26.82)
    arm = np.arange(nst) % 3
    r = 35.0 * np.exp(rng.random(nst) * np.log(1000.0))
    ang = 2 * np.pi * arm / 3 + 2.0 * np.log(r / 35.0) + rng.normal(0.0, 0.05, nst)
    enu = np.stack([r * np.cos(ang), r * np.sin(ang), np.zeros(nst)], axis=1)
    bl = _baseline_pairs(nst)
    xyz = _enu_to_xyz(enu, lat)
    bxyz = xyz[bl[:, 1]] - xyz[bl[:, 0]]
    h0 = -0.5 * nt * dt * OMEGA_EARTH
    h = h0 + OMEGA_EARTH * dt * np.arange(nt)
    uvw = _uvw_tracks(bxyz, h, dec)
    freqs = _channel_centres(50e6, 350e6, nch)
    aslot = 32
    nslot = -(-nt // aslot)
    aterms = _near_identity_aterms(rng, nslot, nst, L)
    flags = (rng.random((bl.shape[0], nt, nch), dtype=np.float32) < np.float32(0.1)).view(np.uint8)
    vis = _complex_normal(rng, (bl.shape[0], nt, nch, 4)) if with_vis else None
    return Workload("skalow", N, N * cell, L, beta, 32, aslot, nst, bl, uvw, freqs, flags, vis,
                    aterms, pswf_taper_2d(L, beta),
                    dict(cell=cell, dt=dt, h0=h0, dec=dec, lat=lat))


_BUILDERS = {"tiny": (_tiny, 1), "lofar": (_lofar, 2), "skalow": (_skalow, 3), "precision": (_precision, 5)}


def make_workload(name, with_vis=True, seed=None, **sizes):
    """Build a named workload.  ``seed`` defaults to 1909_07226 + the workload's index.

    ``tiny`` accepts ``nt`` and ``nch`` to make a longer or wider variant of the same array.
    """
    fn, idx = _BUILDERS[name]
    return fn(SEED_BASE + idx if seed is None else seed, with_vis, **sizes)


def subset(wl, baselines=None, nt=None, channels=None):
    """Cut a workload down: baseline index array, first ``nt`` timesteps, channel slice.

    The time cut keeps timestep 0, so A-term slots stay aligned.
    """
    bsel = np.arange(wl.nr_baselines) if baselines is None else np.asarray(baselines)
    nt = wl.nr_timesteps if nt is None else int(nt)
    csel = slice(None) if channels is None else channels
    uvw = np.ascontiguousarray(wl.uvw[bsel, :nt])
    freqs = np.ascontiguousarray(wl.freqs[csel])
    flags = None if wl.flags is None else np.ascontiguousarray(wl.flags[bsel, :nt][:, :, csel])
    vis = None if wl.vis is None else np.ascontiguousarray(wl.vis[bsel, :nt][:, :, csel])
    nslot = -(-nt // wl.aterm_timesteps)
    aterms = np.ascontiguousarray(wl.aterms[:nslot])
    return replace(wl, baselines=np.ascontiguousarray(wl.baselines[bsel]), uvw=uvw, freqs=freqs,
                   flags=flags, vis=vis, aterms=aterms, meta=dict(wl.meta, subset=True))
