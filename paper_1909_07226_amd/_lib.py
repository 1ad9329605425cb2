"""ctypes binding of libidg.so (include/idg.h).  Argument marshalling only.

Device arrays are torch tensors on a HIP device; every step of gridding and
degridding runs in the library's kernels.  There is no fallback: if the
library has not been built, loading it raises.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# IDG_LIBRARY: another build of the same library (the host-sanitized one of build.py)
LIB_PATH = os.environ.get("IDG_LIBRARY") or os.path.join(_HERE, "libidg.so")

IDG_OK, IDG_EINVAL, IDG_ENOMEM, IDG_EHIP, IDG_ERANGE, IDG_ESTATE = 0, -1, -2, -3, -4, -5
IDG_STRICT = 1 << 0
IDG_PHASE_FP32 = 1 << 1

SUBGRID_FIELDS = ("bl", "t0", "nt", "c0", "nc", "x0", "y0", "slot", "s1", "s2", "nvis", "vis_offset", "wlayer")

EXPORTED = ("idg_plan", "idg_plan_stats", "idg_plan_export", "idg_plan_destroy", "idg_grid", "idg_degrid",
            "idg_grid_subgrids", "idg_subgrid_fft", "idg_add_subgrids", "idg_split_subgrids", "idg_sync",
            "idg_last_error", "idg_version", "idg_profile", "idg_profile_read", "idg_plan_set_tuning",
            "idg_plan_get_tuning", "idg_grid_to_image", "idg_image_to_grid", "idg_taper_optimal",
            "idg_taper_correction", "idg_plan_wlayers", "idg_wstack_to_image", "idg_image_to_wstack",
            "idg_grid_noalloc", "idg_plan_sum_paths", "idg_device_rates",
            "idg_trim_scratch")
NOALLOC_SCRATCH_BYTES = 128 << 20          # IDG_NOALLOC_SCRATCH_BYTES
FORM_PLAIN, FORM_PERSISTENT = 0, 1
DEGRID_STANDARD, DEGRID_WIDE = 0, 1
SUM_AUTO, SUM_DIRECT = 0, 1
STAGES = ("gridder", "adder", "degridder", "zero")


class Params(ctypes.Structure):
    _fields_ = [("grid_size", ctypes.c_int32), ("subgrid_size", ctypes.c_int32), ("kernel_size", ctypes.c_int32),
                ("max_timesteps", ctypes.c_int32), ("aterm_timesteps", ctypes.c_int32),
                ("nr_stations", ctypes.c_int32), ("nr_baselines", ctypes.c_int32), ("nr_timesteps", ctypes.c_int32),
                ("nr_channels", ctypes.c_int32), ("flags", ctypes.c_uint32), ("image_size", ctypes.c_double),
                ("scratch_bytes", ctypes.c_int64), ("w_step", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("grid_form", ctypes.c_int32), ("degrid_form", ctypes.c_int32),
                ("grid_blocks_per_cu", ctypes.c_int32), ("degrid_blocks_per_cu", ctypes.c_int32),
                ("adder_chunk", ctypes.c_int32), ("degrid_shape", ctypes.c_int32), ("sum_path", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_FORMS = {"plain": FORM_PLAIN, "persistent": FORM_PERSISTENT}
_FORM_NAMES = {v: k for k, v in _FORMS.items()}
_SHAPES = {"standard": DEGRID_STANDARD, "wide": DEGRID_WIDE}
_SHAPE_NAMES = {v: k for k, v in _SHAPES.items()}
_SUMS = {"auto": SUM_AUTO, "direct": SUM_DIRECT}
_SUM_NAMES = {v: k for k, v in _SUMS.items()}


class IDGError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{message} (code {code})")
        self.code = code


_lib = None


def lib():
    """The loaded library (loads it on first use)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1909_07226_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        L.idg_plan.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, ctypes.POINTER(vp)]
        L.idg_plan_stats.argtypes = [vp, vp, vp, vp, vp]
        L.idg_plan_export.argtypes = [vp, vp, vp]
        L.idg_plan_destroy.argtypes = [vp]
        L.idg_plan_destroy.restype = None
        L.idg_grid.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.idg_grid_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.idg_degrid.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.idg_grid_subgrids.argtypes = [vp, vp, vp, vp, vp, vp, i64, i64, i32, vp, vp]
        L.idg_subgrid_fft.argtypes = [vp, i64, i32, i32, vp]
        L.idg_add_subgrids.argtypes = [vp, vp, i64, i64, vp, vp]
        L.idg_split_subgrids.argtypes = [vp, vp, i64, i64, vp, vp]
        L.idg_sync.argtypes = [vp]
        L.idg_last_error.restype = ctypes.c_char_p
        L.idg_last_error.argtypes = []
        L.idg_version.argtypes = []
        L.idg_profile.argtypes = [ctypes.c_int]
        L.idg_profile_read.argtypes = [vp, vp, ctypes.c_int]
        L.idg_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.idg_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.idg_grid_to_image.argtypes = [vp, i32, vp, vp, vp, vp]
        L.idg_image_to_grid.argtypes = [vp, i32, vp, vp, vp, vp]
        L.idg_taper_optimal.argtypes = [i32, ctypes.c_double, vp, vp]
        L.idg_taper_correction.argtypes = [i32, ctypes.c_double, vp, i32, vp]
        L.idg_plan_wlayers.argtypes = [vp, vp, vp]
        L.idg_plan_sum_paths.argtypes = [vp, vp, vp]
        L.idg_device_rates.argtypes = [vp, vp, vp]
        L.idg_trim_scratch.argtypes = [ctypes.c_uint64]
        L.idg_wstack_to_image.argtypes = [vp, i32, vp, i32, ctypes.c_double, vp, vp, vp, vp]
        L.idg_image_to_wstack.argtypes = [vp, i32, ctypes.c_double, vp, vp, i32, vp, vp, vp]
        for name in EXPORTED:
            if name not in ("idg_plan_destroy", "idg_last_error"):
                getattr(L, name).restype = ctypes.c_int
        del u32
        _lib = L
    return _lib


def check(rc):
    if rc != IDG_OK:
        raise IDGError(rc, lib().idg_last_error().decode(errors="replace"))
    return rc


def _host_ptr(a, dtype, shape=None, name="array"):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None and arr.shape != tuple(shape):
        raise ValueError(f"{name}: shape {arr.shape}, expected {tuple(shape)}")
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def _dev_ptr(t, dtype, shape, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor on a HIP device")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: must be on a HIP device, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Plan:
    """A subgrid plan (idg_plan).  Host arrays in, opaque handle kept."""

    def __init__(self, grid_size, image_size, subgrid_size, kernel_size, max_timesteps, aterm_timesteps,
                 nr_stations, baselines, uvw, freqs, flags=None, strict=False, phase_fp32=False, scratch_bytes=0,
                 w_step=0.0):
        uvw = np.asarray(uvw)
        nbl, nt = uvw.shape[0], uvw.shape[1]
        nch = int(np.asarray(freqs).size)
        self.params = Params(int(grid_size), int(subgrid_size), int(kernel_size), int(max_timesteps),
                             int(aterm_timesteps), int(nr_stations), nbl, nt, nch,
                             (IDG_STRICT if strict else 0) | (IDG_PHASE_FP32 if phase_fp32 else 0),
                             float(image_size), int(scratch_bytes), float(w_step))
        self._keep = []
        bl, blp = _host_ptr(baselines, np.int32, (nbl, 2), "baselines")
        uv, uvp = _host_ptr(uvw, np.float64, (nbl, nt, 3), "uvw")
        fr, frp = _host_ptr(freqs, np.float64, (nch,), "freqs")
        fl, flp = _host_ptr(flags, np.uint8, (nbl, nt, nch), "flags")
        h = ctypes.c_void_p()
        self._handle = None
        check(lib().idg_plan(ctypes.byref(self.params), blp, uvp, frp, flp, ctypes.byref(h)))
        self._handle = h

    @classmethod
    def from_workload(cls, wl, **kw):
        return cls(wl.grid_size, wl.image_size, wl.subgrid_size, wl.kernel_size, wl.max_timesteps,
                   wl.aterm_timesteps, wl.nr_stations, wl.baselines, wl.uvw, wl.freqs, wl.flags, **kw)

    def __del__(self):
        if getattr(self, "_handle", None) is not None and _lib is not None:
            _lib.idg_plan_destroy(self._handle)
            self._handle = None

    @property
    def handle(self):
        return self._handle

    @property
    def grid_size(self):
        return self.params.grid_size

    @property
    def subgrid_size(self):
        return self.params.subgrid_size

    def stats(self):
        v = [ctypes.c_int64() for _ in range(4)]
        check(lib().idg_plan_stats(self._handle, *[ctypes.byref(x) for x in v]))
        return dict(zip(("nr_subgrids", "nr_gridded", "nr_dropped", "nr_flagged"), (x.value for x in v)))

    def sum_paths(self):
        """Subgrids and samples per evaluation of the subgrid sums under the current tuning:
        {"separable0": (subgrids, samples), "separable1": ..., "direct": ...}."""
        ns = (ctypes.c_int64 * 3)()
        nv = (ctypes.c_int64 * 3)()
        check(lib().idg_plan_sum_paths(self._handle, ns, nv))
        return {k: (int(ns[i]), int(nv[i])) for i, k in enumerate(("separable0", "separable1", "direct"))}

    @property
    def nr_subgrids(self):
        return self.stats()["nr_subgrids"]

    def wlayers(self):
        """(wlayer_min, nr_wlayers): the grid is [nr_wlayers][4][N][N], layer j at index j - wlayer_min."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        check(lib().idg_plan_wlayers(self._handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def w_offsets(self):
        """w offset (wavelengths) of each layer grid, in grid order."""
        lo, n = self.wlayers()
        return [(lo + j) * self.params.w_step for j in range(n)]

    def set_tuning(self, form=None, blocks_per_cu=None, adder_chunk=None, grid_form=None, degrid_form=None,
                   grid_blocks_per_cu=None, degrid_blocks_per_cu=None, degrid_shape=None, sum_path=None):
        """Scheduling knobs (idg_plan_set_tuning).  ``form`` / ``blocks_per_cu`` set both directions;
        the grid_/degrid_ arguments set one; ``degrid_shape`` is "standard" or "wide"; ``sum_path`` is
        "auto" (separable form on the matrix cores where it applies) or "direct".  Unspecified knobs
        keep their value."""
        cur = self.get_tuning()
        gf = grid_form if grid_form is not None else (form if form is not None else cur["grid_form"])
        df = degrid_form if degrid_form is not None else (form if form is not None else cur["degrid_form"])
        gb = grid_blocks_per_cu if grid_blocks_per_cu is not None else (
            blocks_per_cu if blocks_per_cu is not None else cur["grid_blocks_per_cu"])
        db = degrid_blocks_per_cu if degrid_blocks_per_cu is not None else (
            blocks_per_cu if blocks_per_cu is not None else cur["degrid_blocks_per_cu"])
        ds = cur["degrid_shape"] if degrid_shape is None else degrid_shape
        sp = cur["sum_path"] if sum_path is None else sum_path
        t = Tuning(_FORMS.get(gf, gf), _FORMS.get(df, df), int(gb), int(db),
                   cur["adder_chunk"] if adder_chunk is None else int(adder_chunk), _SHAPES.get(ds, ds),
                   _SUMS.get(sp, sp))
        check(lib().idg_plan_set_tuning(self._handle, ctypes.byref(t)))

    def get_tuning(self):
        t = Tuning()
        check(lib().idg_plan_get_tuning(self._handle, ctypes.byref(t)))
        return dict(grid_form=_FORM_NAMES.get(t.grid_form, t.grid_form),
                    degrid_form=_FORM_NAMES.get(t.degrid_form, t.degrid_form),
                    grid_blocks_per_cu=t.grid_blocks_per_cu, degrid_blocks_per_cu=t.degrid_blocks_per_cu,
                    adder_chunk=t.adder_chunk, degrid_shape=_SHAPE_NAMES.get(t.degrid_shape, t.degrid_shape),
                    sum_path=_SUM_NAMES.get(t.sum_path, t.sum_path))

    def export(self):
        """(subgrids int64 [P, 13] with SUBGRID_FIELDS columns, samples int32 [K, 2] of (t, c))."""
        st = self.stats()
        sub = np.zeros((st["nr_subgrids"], len(SUBGRID_FIELDS)), np.int64)
        smp = np.zeros((st["nr_gridded"], 2), np.int32)
        check(lib().idg_plan_export(self._handle, sub.ctypes.data_as(ctypes.c_void_p),
                                    smp.ctypes.data_as(ctypes.c_void_p)))
        return sub, smp

    # shapes of the device arrays
    def shapes(self, nr_slots=None):
        p = self.params
        L, N = p.subgrid_size, p.grid_size
        ns = -(-p.nr_timesteps // p.aterm_timesteps) if nr_slots is None else nr_slots
        return dict(uvw=(p.nr_baselines, p.nr_timesteps, 3), freqs=(p.nr_channels,),
                    vis=(p.nr_baselines, p.nr_timesteps, p.nr_channels, 4), aterms=(ns, p.nr_stations, L, L, 4),
                    taper=(L, L), grid=(4, N, N) if p.w_step == 0 else (self.wlayers()[1], 4, N, N))


def _common(plan, uvw_d, freqs_d, aterms_d, taper_d):
    import torch
    sh = plan.shapes()
    return (_dev_ptr(uvw_d, torch.float64, sh["uvw"], "uvw"), _dev_ptr(freqs_d, torch.float64, sh["freqs"], "freqs"),
            _dev_ptr(aterms_d, torch.complex64, sh["aterms"], "aterms"),
            _dev_ptr(taper_d, torch.float32, sh["taper"], "taper"))


def grid(plan, uvw_d, freqs_d, vis_d, aterms_d, taper_d, grid_d, stream=None):
    """idg_grid: accumulate the plan's visibilities into grid_d complex64, [4, N, N] (or
    [nr_wlayers, 4, N, N] for a plan with W-layers: plan.shapes()["grid"])."""
    import torch
    sh = plan.shapes()
    u, f, a, t = _common(plan, uvw_d, freqs_d, aterms_d, taper_d)
    check(lib().idg_grid(plan.handle, u, f, _dev_ptr(vis_d, torch.complex64, sh["vis"], "vis"), a, t,
                         _dev_ptr(grid_d, torch.complex64, sh["grid"], "grid"), _stream_ptr(stream)))


def grid_noalloc(plan, uvw_d, freqs_d, vis_d, aterms_d, taper_d, grid_d, stream=None):
    """idg_grid_noalloc: idg_grid with the library's fixed device scratch (no allocation).  The plan must
    already have a device copy on this device and batches that fit NOALLOC_SCRATCH_BYTES."""
    import torch
    sh = plan.shapes()
    u, f, a, t = _common(plan, uvw_d, freqs_d, aterms_d, taper_d)
    check(lib().idg_grid_noalloc(plan.handle, u, f, _dev_ptr(vis_d, torch.complex64, sh["vis"], "vis"), a, t,
                                 _dev_ptr(grid_d, torch.complex64, sh["grid"], "grid"), _stream_ptr(stream)))


def degrid(plan, uvw_d, freqs_d, grid_d, aterms_d, taper_d, vis_d, stream=None):
    """idg_degrid: overwrite vis_d [nbl, nt, nch, 4] complex64 with predictions from grid_d."""
    import torch
    sh = plan.shapes()
    u, f, a, t = _common(plan, uvw_d, freqs_d, aterms_d, taper_d)
    check(lib().idg_degrid(plan.handle, u, f, _dev_ptr(grid_d, torch.complex64, sh["grid"], "grid"), a, t,
                           _dev_ptr(vis_d, torch.complex64, sh["vis"], "vis"), _stream_ptr(stream)))


def grid_subgrids(plan, uvw_d, freqs_d, vis_d, aterms_d, taper_d, first, count, stage, out_d, stream=None):
    """idg_grid_subgrids: subgrids [count, 4, L, L] before (stage 0) or after (stage 1) the transform."""
    import torch
    sh = plan.shapes()
    L = plan.subgrid_size
    u, f, a, t = _common(plan, uvw_d, freqs_d, aterms_d, taper_d)
    check(lib().idg_grid_subgrids(plan.handle, u, f, _dev_ptr(vis_d, torch.complex64, sh["vis"], "vis"), a, t,
                                  int(first), int(count), int(stage),
                                  _dev_ptr(out_d, torch.complex64, (count, 4, L, L), "out"), _stream_ptr(stream)))


def subgrid_fft(data_d, direction, stream=None):
    """idg_subgrid_fft in place on data_d [count, 4, L, L] complex64; direction -1 forward, +1 inverse."""
    import torch
    if data_d.dim() != 4 or data_d.shape[1] != 4 or data_d.shape[2] != data_d.shape[3]:
        raise ValueError("data: expected shape [count, 4, L, L]")
    p = _dev_ptr(data_d, torch.complex64, None, "data")
    check(lib().idg_subgrid_fft(p, int(data_d.shape[0]), int(data_d.shape[2]), int(direction), _stream_ptr(stream)))


def add_subgrids(plan, subgrids_d, first, grid_d, stream=None):
    """idg_add_subgrids: grid_d += subgrids_d [count, 4, L, L] at the corners of plan subgrids first..."""
    import torch
    L = plan.subgrid_size
    count = int(subgrids_d.shape[0])
    check(lib().idg_add_subgrids(plan.handle, _dev_ptr(subgrids_d, torch.complex64, (count, 4, L, L), "subgrids"),
                                 int(first), count,
                                 _dev_ptr(grid_d, torch.complex64, plan.shapes()["grid"], "grid"),
                                 _stream_ptr(stream)))


def split_subgrids(plan, grid_d, first, out_d, stream=None):
    """idg_split_subgrids: out_d [count, 4, L, L] = grid_d windows of plan subgrids first..."""
    import torch
    L = plan.subgrid_size
    count = int(out_d.shape[0])
    check(lib().idg_split_subgrids(plan.handle, _dev_ptr(grid_d, torch.complex64, plan.shapes()["grid"], "grid"),
                                   int(first), count, _dev_ptr(out_d, torch.complex64, (count, 4, L, L), "out"),
                                   _stream_ptr(stream)))


def _image_args(src_d, dst_d, corr_l_d, corr_m_d):
    import torch
    if src_d.dim() != 3 or src_d.shape[0] != 4 or src_d.shape[1] != src_d.shape[2]:
        raise ValueError("expected a [4, N, N] complex64 array")
    N = int(src_d.shape[-1])
    src = _dev_ptr(src_d, torch.complex64, (4, N, N), "input")
    dst = _dev_ptr(dst_d, torch.complex64, (4, N, N), "output")
    if (corr_l_d is None) != (corr_m_d is None):
        raise ValueError("give both corrections or neither")
    cl = None if corr_l_d is None else _dev_ptr(corr_l_d, torch.float32, (N,), "corr_l")
    cm = None if corr_m_d is None else _dev_ptr(corr_m_d, torch.float32, (N,), "corr_m")
    return src, N, cl, cm, dst


def grid_to_image(grid_d, corr_l_d, corr_m_d, image_d, stream=None):
    """idg_grid_to_image: image_d [4, N, N] = the grid's DTFT at the image pixels / (corr_m[y] corr_l[x])."""
    src, N, cl, cm, dst = _image_args(grid_d, image_d, corr_l_d, corr_m_d)
    check(lib().idg_grid_to_image(src, N, cl, cm, dst, _stream_ptr(stream)))


def image_to_grid(image_d, corr_l_d, corr_m_d, grid_d, stream=None):
    """idg_image_to_grid: grid_d [4, N, N] = the adjoint transform of image_d / (corr_m[y] corr_l[x])."""
    src, N, cl, cm, dst = _image_args(image_d, grid_d, corr_l_d, corr_m_d)
    check(lib().idg_image_to_grid(src, N, cl, cm, dst, _stream_ptr(stream)))


def taper_shift_for_plan(L, kernel_size):
    """max_shift to design a taper for the plans of idg_plan: (L - kernel_size)/2 uv pixels, half a
    pixel beyond the largest sample shift those plans produce, (L - 1 - kernel_size)/2."""
    return (int(L) - float(kernel_size)) / 2


def _wstack_args(image_d, grids_d, w0s, corr_l_d, corr_m_d):
    import torch
    if grids_d.dim() != 4 or grids_d.shape[1] != 4 or grids_d.shape[2] != grids_d.shape[3]:
        raise ValueError("grids: expected [nr_wlayers, 4, N, N] complex64")
    nl, N = int(grids_d.shape[0]), int(grids_d.shape[-1])
    w0 = np.ascontiguousarray(w0s, np.float64)
    if w0.shape != (nl,):
        raise ValueError(f"w0s: expected {nl} offsets, got shape {w0.shape}")
    if (corr_l_d is None) != (corr_m_d is None):
        raise ValueError("give both corrections or neither")
    cl = None if corr_l_d is None else _dev_ptr(corr_l_d, torch.float32, (N,), "corr_l")
    cm = None if corr_m_d is None else _dev_ptr(corr_m_d, torch.float32, (N,), "corr_m")
    return (_dev_ptr(image_d, torch.complex64, (4, N, N), "image"),
            _dev_ptr(grids_d, torch.complex64, (nl, 4, N, N), "grids"), nl, N, w0, cl, cm)


def wstack_to_image(grids_d, w0s, image_size, corr_l_d, corr_m_d, image_d, stream=None):
    """idg_wstack_to_image: image_d = sum_j exp(+2 pi i w0s[j] n') T(grids_d[j]) / correction."""
    img, g, nl, N, w0, cl, cm = _wstack_args(image_d, grids_d, w0s, corr_l_d, corr_m_d)
    check(lib().idg_wstack_to_image(g, nl, w0.ctypes.data, N, float(image_size), cl, cm, img, _stream_ptr(stream)))


def image_to_wstack(image_d, image_size, corr_l_d, corr_m_d, w0s, grids_d, stream=None):
    """idg_image_to_wstack: grids_d[j] = T^H(image_d exp(-2 pi i w0s[j] n') / correction)."""
    img, g, nl, N, w0, cl, cm = _wstack_args(image_d, grids_d, w0s, corr_l_d, corr_m_d)
    check(lib().idg_image_to_wstack(img, N, float(image_size), cl, cm, nl, w0.ctypes.data, g, _stream_ptr(stream)))


def optimal_taper(L, max_shift):
    """idg_taper_optimal: (taper [L] float64 with taper[L/2] = 1, eps).  Raises IDGError (IDG_ERANGE)
    when eps^2 is beyond float64 resolution."""
    import numpy as np
    a = np.zeros(int(L), np.float64)
    eps = ctypes.c_double(0.0)
    check(lib().idg_taper_optimal(int(L), float(max_shift), a.ctypes.data, ctypes.addressof(eps)))
    return a, eps.value


def taper_correction(taper, max_shift, N):
    """idg_taper_correction: corr [N] float32 (host) for the 1-D subgrid taper (float64 [L])."""
    import numpy as np
    a = np.ascontiguousarray(taper, np.float64)
    out = np.zeros(int(N), np.float32)
    check(lib().idg_taper_correction(int(a.size), float(max_shift), a.ctypes.data, int(N), out.ctypes.data))
    return out


def sync(stream=None):
    check(lib().idg_sync(_stream_ptr(stream)))


def version():
    return lib().idg_version()


def profile(enable=True):
    """Turn the library's per-stage HIP-event timing on or off (idg_profile)."""
    check(lib().idg_profile(1 if enable else 0))


def trim_scratch(keep_bytes=0):
    """idg_trim_scratch: return the library pool's unused scratch beyond keep_bytes (waits for the device)."""
    check(lib().idg_trim_scratch(int(keep_bytes)))


def device_rates():
    """idg_device_rates: {"fp32_fma_tflops", "sincos_ginstr_per_s", "fp16_mfma_tflops"} on the current device."""
    v = [ctypes.c_double() for _ in range(3)]
    check(lib().idg_device_rates(*[ctypes.byref(x) for x in v]))
    return {"fp32_fma_tflops": v[0].value / 1e12, "sincos_ginstr_per_s": v[1].value / 1e9,
            "fp16_mfma_tflops": v[2].value / 1e12}


def profile_read(reset=True):
    """{stage: (milliseconds, launches)} accumulated since the last reset (idg_profile_read)."""
    ms = np.zeros(len(STAGES), np.float64)
    n = np.zeros(len(STAGES), np.int64)
    check(lib().idg_profile_read(ms.ctypes.data_as(ctypes.c_void_p), n.ctypes.data_as(ctypes.c_void_p),
                                 1 if reset else 0))
    return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}
