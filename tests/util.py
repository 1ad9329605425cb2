"""Small hand-made workloads for the tests.

uvw are given directly in wavelengths by choosing channel frequencies near c0
(so that u_k = uvw * f / c0 ~= uvw), which keeps the geometry readable.
"""

import numpy as np

from synth import C0, Workload


def make_mini(uvw, freqs=(C0,), N=64, L=16, beta=3, S=None, tmax=64, aslot=64, nst=None, baselines=None,
              vis=None, aterms=None, taper=None, flags=None, seed=0, random_aterms=False, random_taper=False):
    rng = np.random.default_rng(seed)
    uvw = np.asarray(uvw, np.float64)
    nbl, nt, _ = uvw.shape
    freqs = np.asarray(freqs, np.float64)
    nch = freqs.size
    if baselines is None:
        baselines = np.stack([np.zeros(nbl, np.int32), np.arange(1, nbl + 1, dtype=np.int32)], 1)
    baselines = np.asarray(baselines, np.int32)
    nst = int(baselines.max()) + 1 if nst is None else nst
    S = 1.0 if S is None else S
    nslot = -(-nt // aslot)
    if aterms is None:
        aterms = np.zeros((nslot, nst, L, L, 4), np.complex64)
        aterms[..., 0] = 1
        aterms[..., 3] = 1
        if random_aterms:
            aterms += (0.3 * (rng.standard_normal(aterms.shape) + 1j * rng.standard_normal(aterms.shape))).astype(
                np.complex64)
    if taper is None:
        taper = np.ones((L, L), np.float32)
        if random_taper:
            taper = (0.5 + rng.random((L, L))).astype(np.float32)
    if vis is None:
        vis = (rng.standard_normal((nbl, nt, nch, 4)) + 1j * rng.standard_normal((nbl, nt, nch, 4))).astype(
            np.complex64)
    return Workload("mini", N, S, L, beta, tmax, aslot, nst, baselines, uvw, freqs, flags, vis, aterms, taper, {})


def random_track_workload(seed=1, N=64, L=16, beta=3, nbl=3, nt=20, nch=3, wscale=1.5, **kw):
    """A few baselines with smooth random uv tracks (in pixels ~ wavelengths at S = 1) and nonzero w."""
    rng = np.random.default_rng(seed)
    uvw = np.zeros((nbl, nt, 3))
    for b in range(nbl):
        start = rng.uniform(-N / 8, N / 8, 2)
        vel = rng.uniform(-1.2, 1.2, 2)
        t = np.arange(nt)
        uvw[b, :, 0] = start[0] + vel[0] * t
        uvw[b, :, 1] = start[1] + vel[1] * t
        uvw[b, :, 2] = rng.uniform(-wscale, wscale) + 0.05 * t
    freqs = C0 * (1.0 + 0.02 * np.arange(nch))
    return make_mini(uvw, freqs=freqs, N=N, L=L, beta=beta, seed=seed, **kw)


def plan_of(wl):
    from oracle.plan import plan_workload
    return plan_workload(wl)
