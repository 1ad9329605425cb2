"""Helpers for the GPU tests: device upload of a workload, error metrics, tolerances."""

import sys

import numpy as np

# Tolerances for float32 phase / accumulation against the float64 oracle (the
# paper states none; float32 rounding of ~1e3-term sums and of the phase gives
# a few 1e-6 relative error, so 1e-5 leaves margin without hiding mistakes,
# which show up at 1e-3 or worse).
GRID_RMS_TOL = 1e-5
GRID_MAX_TOL = 1e-4       # per element, relative to the largest |value|
VIS_RMS_TOL = 1e-5
ADJOINT_TOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def require_gpu():
    import torch
    import paper_1909_07226_amd as idg
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    idg.lib()          # raises if libidg.so is missing


def to_dev(wl):
    import torch
    dev = "cuda"
    out = dict(uvw=torch.from_numpy(np.ascontiguousarray(wl.uvw)).to(dev),
               freqs=torch.from_numpy(np.ascontiguousarray(wl.freqs)).to(dev),
               aterms=torch.from_numpy(np.ascontiguousarray(wl.aterms)).to(dev),
               taper=torch.from_numpy(np.ascontiguousarray(wl.taper)).to(dev))
    if wl.vis is not None:
        out["vis"] = torch.from_numpy(np.ascontiguousarray(wl.vis)).to(dev)
    return out


def rms_rel(got, ref):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    return float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel()))


def max_rel(got, ref):
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    return float(np.abs(got - ref).max() / np.abs(ref).max())
