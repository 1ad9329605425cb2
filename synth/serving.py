"""Seeded request trace for the serving benchmark: arrivals, job kinds and job windows.

Jobs arrive as a Poisson process (mean ``rate`` jobs/s).  Half are gridding
and half degridding jobs; half are of the small class (the 8-station array,
N = 512, L = 24) and half of the LOFAR-like class (48 stations, N = 4096,
L = 32).  A job covers a window of its class's dataset: nt ~ U{64..2048}
timesteps starting on an A-term slot boundary and nch ~ U{4..16} contiguous
channels.  Requests repeat a limited set of windows (``n_windows`` per class),
as repeated observations of the same fields would.  This module only draws
numbers; building plans and device arrays is the caller's business.
"""

import numpy as np

SEED = 1909_07226 + 4
CLASSES = ("tiny", "lofar")


def job_windows(rng, nt_total, nch_total, aslot, n):
    out = []
    for _ in range(n):
        nt = int(rng.integers(64, min(2048, nt_total) + 1))
        nch = int(rng.integers(4, min(16, nch_total) + 1))
        starts = np.arange(0, nt_total - nt + 1, aslot)
        t0 = int(rng.choice(starts))
        c0 = int(rng.integers(0, nch_total - nch + 1))
        out.append(dict(t0=t0, nt=nt, c0=c0, nch=nch))
    return out


def serving_trace(n_jobs=400, rate=50.0, n_windows=16, seed=SEED, sizes=None):
    """Arrivals (s from trace start), kinds, classes and window indices of ``n_jobs`` requests.

    ``sizes`` maps a class to (nt_total, nch_total, aterm_timesteps) of its dataset.
    """
    sizes = sizes or {"tiny": (2048, 16, 2048), "lofar": (2048, 16, 256)}
    rng = np.random.default_rng(seed)
    windows = {c: job_windows(rng, *sizes[c], n_windows) for c in CLASSES}
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_jobs))
    kinds = np.where(rng.random(n_jobs) < 0.5, "grid", "degrid")
    classes = np.where(rng.random(n_jobs) < 0.5, "tiny", "lofar")
    win = rng.integers(0, n_windows, n_jobs)
    return dict(arrivals=arrivals, kinds=kinds, classes=classes, windows=windows, window_ids=win)
