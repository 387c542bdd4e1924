"""MI355X-native SMLM localization: Python binding of libdloc (ctypes).

This module only marshals arguments: every step of the localization path runs
in the HIP kernels of ``_build/libdloc.so`` (built by ``_build.build()``).
PyTorch is used for device memory and streams.  If the library has not been
built, importing this package raises ``ImportError`` -- there is no fallback.

Names follow the C ABI in ``include/dloc.h``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_build", "libdloc.so")

DL_OK = 0
DL_ERR_INVALID_ARG = -1
DL_ERR_BAD_WEIGHTS = -2
DL_ERR_UNSUPPORTED = -3
DL_ERR_OOM = -4
DL_ERR_DEVICE = -5
DL_ERR_CAPACITY = -6
STATUS_NAMES = {0: "DL_OK", -1: "DL_ERR_INVALID_ARG", -2: "DL_ERR_BAD_WEIGHTS", -3: "DL_ERR_UNSUPPORTED",
                -4: "DL_ERR_OOM", -5: "DL_ERR_DEVICE", -6: "DL_ERR_CAPACITY"}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp8": 2, "bf16x3": 3}
DL_FLAG_GATE = 1
NOALLOC_SCRATCH_BYTES = 64 << 20      # DL_NOALLOC_SCRATCH_BYTES
NOALLOC_MAX_FRAMES = 64               # DL_NOALLOC_MAX_FRAMES
STAGES = ("stem", "conv", "conv_head", "detect", "scan", "emit", "gate", "conv_1x1", "unet")
NSTAGES = 10

EMITTER_DTYPE = np.dtype([("frame", "<i4"), ("row", "<i4"), ("col", "<i4"), ("x_px", "<f4"),
                          ("y_px", "<f4"), ("z_nm", "<f4"), ("photons", "<f4"), ("prob", "<f4")])
assert EMITTER_DTYPE.itemsize == 32
UNCERTAINTY_DTYPE = np.dtype([("sigma_x_px", "<f4"), ("sigma_y_px", "<f4"), ("sigma_z_nm", "<f4"),
                              ("sigma_photons", "<f4"), ("background", "<f4")])
assert UNCERTAINTY_DTYPE.itemsize == 20


class DLConfig(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("threshold", ctypes.c_float), ("gain", ctypes.c_float),
                ("offset", ctypes.c_float), ("device", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("max_workspace_bytes", ctypes.c_uint64), ("tile_rows", ctypes.c_int32),
                ("max_sigma_px", ctypes.c_float), ("in_scale_override", ctypes.c_float),
                ("tile_w", ctypes.c_int32), ("tile_queue", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class DLRoi(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("h", ctypes.c_int32), ("w", ctypes.c_int32),
                ("row_stride", ctypes.c_int64)]


class DLNetInfo(ctypes.Structure):
    _fields_ = [("C", ctypes.c_int32), ("nblocks", ctypes.c_int32), ("dilation", ctypes.c_int32 * 8),
                ("in_scale", ctypes.c_float), ("z_scale", ctypes.c_float), ("ph_scale", ctypes.c_float),
                ("receptive_radius", ctypes.c_int32), ("nparams", ctypes.c_int64),
                ("head_outputs", ctypes.c_int32), ("dense_layers", ctypes.c_int16),
                ("dense_growth", ctypes.c_int16), ("unet_levels", ctypes.c_int32), ("reserved2_", ctypes.c_int32 * 3)]


class DLTuneResult(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32 * 8), ("strip", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("configs_timed", ctypes.c_int32), ("ms_default", ctypes.c_float), ("ms_best", ctypes.c_float)]


class DlocError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


def _load():
    # The library must run on the same HIP runtime instance as PyTorch, whose
    # device pointers and streams it receives.  PyTorch ships its own
    # libamdhip64.so.7; loading torch first makes the dynamic loader resolve
    # libdloc's dependency to that already-loaded copy.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libdloc.so is not built ({LIB_PATH}); run "
                          "`python -m paper_2410_02314_amd._build` (or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P, I, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    sig = {
        "dl_abi_version": (ctypes.c_uint32, []),
        "dl_default_config": (I, [ctypes.POINTER(DLConfig)]),
        "dl_create_net": (I, [P, Z, ctypes.POINTER(DLConfig), ctypes.POINTER(P)]),
        "dl_inspect_weights": (I, [P, Z, ctypes.POINTER(DLNetInfo)]),
        "dl_destroy_net": (None, [P]),
        "dl_last_error": (ctypes.c_char_p, [P]),
        "dl_set_config": (I, [P, ctypes.POINTER(DLConfig)]),
        "dl_localize_device": (I, [P, P, I, I, I, P, P, Z, P]),
        "dl_localize_device_unc": (I, [P, P, I, I, I, P, P, P, Z, P]),
        "dl_localize_device_noalloc": (I, [P, P, I, I, I, P, P, Z, P]),
        "dl_localize_rois_device_unc": (I, [P, ctypes.POINTER(DLRoi), I, P, P, P, Z, P]),
        "dl_maps_device": (I, [P, P, I, I, I, P, P]),
        "dl_localize": (I, [P, P, I, I, I, P, Z, ctypes.POINTER(Z)]),
        "dl_localize_pipelined": (I, [P, P, I, I, I, I, I, P, Z, ctypes.POINTER(Z)]),
        "dl_localize_pipelined_unc": (I, [P, P, I, I, I, I, I, P, P, Z, ctypes.POINTER(Z)]),
        "dl_localize_unc": (I, [P, P, I, I, I, P, P, Z, ctypes.POINTER(Z)]),
        "dl_localize_rois_device": (I, [P, ctypes.POINTER(DLRoi), I, P, P, Z, P]),
        "dl_localize_rois": (I, [P, ctypes.POINTER(DLRoi), I, P, Z, ctypes.POINTER(Z)]),
        "dl_localize_maps": (I, [P, P, I, I, I, P]),
        "dl_debug_compact": (I, [P, P, P, I, I, I, P, P, Z, P]),
        "dl_maps_rois_device": (I, [P, ctypes.POINTER(DLRoi), I, P, P]),
        "dl_host_alloc": (I, [Z, ctypes.POINTER(P)]),
        "dl_measure_rate": (I, [I, Z, I, ctypes.POINTER(ctypes.c_double)]),
        "dl_set_camera_maps": (I, [P, P, P, I, I]),
        "dl_gate_pool_net": (I, [P, P, I, I, I, P, P]),
        "dl_host_free": (None, [P]),
        "dl_debug_conv_layer": (I, [P, P, P, I, I, I, I, I, P, P]),
        "dl_debug_detect": (I, [P, P, I, I, I, ctypes.c_float, P, P]),
        "dl_profile_enable": (I, [P, I]),
        "dl_set_gate": (I, [P, P, ctypes.c_float]),
        "dl_graph_create": (I, [P, P, I, I, I, P, Z, P, ctypes.POINTER(P)]),
        "dl_graph_create_rois": (I, [P, ctypes.POINTER(DLRoi), I, P, Z, P, ctypes.POINTER(P)]),
        "dl_graph_launch": (I, [P, P]),
        "dl_graph_create_rois_dynamic": (I, [P, I, I, I, ctypes.c_int64, P, Z, P, ctypes.POINTER(P)]),
        "dl_graph_launch_rois": (I, [P, ctypes.POINTER(DLRoi), I, P]),
        "dl_autotune": (I, [P, P, I, I, I, P, I, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float)]),
        "dl_graph_destroy": (None, [P]),
        "dl_autotune_ex": (I, [P, P, I, I, I, P, I, ctypes.c_char_p, ctypes.POINTER(DLTuneResult)]),
        "dl_gate_keep_map": (I, [P, P, P, Z, ctypes.POINTER(Z)]),
        "dl_gate_pool": (I, [P, I, I, I, ctypes.c_float, ctypes.c_float, ctypes.c_float, P, P]),
        "dl_gate_forward": (I, [P, I, P, P, P]),
        "dl_gate_backward": (I, [P, I, P, P, P, P, P, P]),
        "dl_gate_bce": (I, [P, P, I, P, P, P]),
        "dl_gate_adam": (I, [P, P, P, P, I, I, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, P]),
        "dl_profile_read": (I, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
        "dl_train_grad": (I, [P, P, I, I, I, P, P, I, P, P, P]),
        "dl_train_step": (I, [P, P, I, I, I, P, P, I, P, ctypes.c_float, P]),
        "dl_get_params": (I, [P, P, Z]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


_lib = _load()


def lib():
    """The loaded ctypes library."""
    return _lib


def abi_version() -> int:
    return int(_lib.dl_abi_version())


def last_error(handle=None) -> str:
    s = _lib.dl_last_error(handle)
    return s.decode() if s else ""


def _check(rc: int, handle=None):
    if rc != DL_OK:
        raise DlocError(rc, last_error(handle))


def make_config(precision: str = "fp32", threshold: float = 0.3, gain: float = 0.5, offset: float = 100.0,
                device: int = 0, flags: int = 0, max_workspace_bytes: int = 0, tile_rows: int = 0,
                max_sigma_px: float = 0.0, in_scale_override: float = 0.0, tile_w: int = 0,
                tile_queue: int = 0) -> DLConfig:
    c = DLConfig()
    _lib.dl_default_config(ctypes.byref(c))
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.threshold = threshold
    c.gain = gain
    c.offset = offset
    c.device = device
    c.flags = flags
    c.max_workspace_bytes = max_workspace_bytes
    c.tile_rows = tile_rows
    c.max_sigma_px = max_sigma_px
    c.in_scale_override = in_scale_override
    c.tile_w = tile_w
    c.tile_queue = tile_queue
    return c


def _ptr(t) -> int:
    """Device (or host) address of a torch tensor / numpy array / int."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _frames_arg(frames, ndim: int = 3):
    """A device frame batch as the C ABI reads it: dense rows of 16-bit
    pixels.  A sliced, transposed or wrongly typed tensor would be read from
    the wrong addresses, so it is refused here."""
    import torch
    if frames.dim() != ndim:
        raise ValueError(f"frames must have {ndim} dimensions, got shape {tuple(frames.shape)}")
    if frames.dtype not in (torch.uint16, torch.int16):
        raise ValueError(f"frames must hold 16-bit pixels (torch.uint16), got {frames.dtype}")
    if not frames.is_contiguous():
        raise ValueError("frames must be contiguous (call .contiguous() first)")
    return frames


def _host_frames(frames, ndim: int) -> np.ndarray:
    F = np.asarray(frames)
    if F.dtype != np.uint16:
        raise ValueError(f"host frames must be uint16, got {F.dtype}")
    if F.ndim != ndim:
        raise ValueError(f"host frames must have {ndim} dimensions, got shape {F.shape}")
    return np.ascontiguousarray(F)


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def inspect_weights(weights: bytes) -> dict:
    """Validate a DLW1 or DLD1 blob on the host and describe the network (no GPU needed)."""
    info = DLNetInfo()
    buf = ctypes.create_string_buffer(bytes(weights), len(weights))
    _check(_lib.dl_inspect_weights(buf, len(weights), ctypes.byref(info)))
    return {"C": info.C, "nblocks": info.nblocks, "dilations": tuple(info.dilation[:info.nblocks]),
            "in_scale": info.in_scale, "z_scale": info.z_scale, "ph_scale": info.ph_scale,
            "receptive_radius": info.receptive_radius, "nparams": info.nparams, "head_outputs": info.head_outputs,
            "dense_layers": info.dense_layers, "dense_growth": info.dense_growth, "unet_levels": info.unet_levels}


def create_net(weights: bytes, **cfg) -> "Net":
    return Net(weights, **cfg)


class Net:
    """Handle of one network on one device (``dl_create_net``)."""

    def __init__(self, weights: bytes, **cfg):
        self.config = make_config(**cfg)
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(bytes(weights), len(weights))
        _check(_lib.dl_create_net(buf, len(weights), ctypes.byref(self.config), ctypes.byref(h)))
        self.handle = h
        info = DLNetInfo()
        _check(_lib.dl_inspect_weights(buf, len(weights), ctypes.byref(info)))
        self.head_outputs = int(info.head_outputs)     # planes of the maps: 5, or 10 with uncertainties
        self.nblocks = int(info.nblocks)
        self.nparams = int(info.nparams)

    def close(self):
        if getattr(self, "handle", None):
            _lib.dl_destroy_net(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_config(self, **cfg):
        c = make_config(**cfg)
        _check(_lib.dl_set_config(self.handle, ctypes.byref(c)), self.handle)
        self.config = c

    # ---- device-resident ----
    def localize_device(self, frames, out, counts, stream=None) -> int:
        """frames: cuda uint16 [n, h, w]; out: cuda tensor of cap*32 bytes; counts: cuda int32 [n+1]."""
        n, h, w = _frames_arg(frames).shape
        cap = out.numel() * out.element_size() // 32
        return self._rc(_lib.dl_localize_device(self.handle, _ptr(frames), n, h, w, _stream(stream),
                                                _ptr(out), cap, _ptr(counts)))

    def localize_device_noalloc(self, frames, out, counts, stream=None) -> int:
        """localize_device without any allocation: the work runs in the
        device's fixed scratch array (at most NOALLOC_MAX_FRAMES frames and
        NOALLOC_SCRATCH_BYTES of workspace; calls that overlap on one device
        race)."""
        n, h, w = _frames_arg(frames).shape
        cap = out.numel() * out.element_size() // 32
        return self._rc(_lib.dl_localize_device_noalloc(self.handle, _ptr(frames), n, h, w, _stream(stream),
                                                        _ptr(out), cap, _ptr(counts)))

    def localize_device_unc(self, frames, out, unc, counts, stream=None) -> int:
        """localize_device for a 10-output network, also filling unc (cuda
        tensor of cap * 20 bytes, one dl_uncertainty per record)."""
        n, h, w = _frames_arg(frames).shape
        cap = out.numel() * out.element_size() // 32
        if unc.numel() * unc.element_size() < cap * 20:
            raise ValueError("unc holds fewer records than out")
        return self._rc(_lib.dl_localize_device_unc(self.handle, _ptr(frames), n, h, w, _stream(stream),
                                                    _ptr(out), _ptr(unc), cap, _ptr(counts)))

    def maps_device(self, frames, maps, stream=None) -> int:
        n, h, w = _frames_arg(frames).shape
        return self._rc(_lib.dl_maps_device(self.handle, _ptr(frames), n, h, w, _stream(stream), _ptr(maps)))

    def localize_rois_device(self, rois: Sequence, out, counts, stream=None) -> int:
        """rois: sequence of cuda uint16 [h, w] tensors (rows may be strided)."""
        arr = self._roi_array(rois)
        cap = out.numel() * out.element_size() // 32
        return self._rc(_lib.dl_localize_rois_device(self.handle, arr, len(rois), _stream(stream), _ptr(out),
                                                     cap, _ptr(counts)))

    def localize_rois_device_unc(self, rois: Sequence, out, unc, counts, stream=None) -> int:
        """localize_rois_device for a 10-output network, with uncertainties."""
        arr = self._roi_array(rois)
        cap = out.numel() * out.element_size() // 32
        if unc.numel() * unc.element_size() < cap * 20:
            raise ValueError("unc holds fewer records than out")
        return self._rc(_lib.dl_localize_rois_device_unc(self.handle, arr, len(rois), _stream(stream), _ptr(out),
                                                         _ptr(unc), cap, _ptr(counts)))

    def maps_rois_device(self, rois: Sequence, maps, stream=None) -> int:
        arr = self._roi_array(rois)
        return self._rc(_lib.dl_maps_rois_device(self.handle, arr, len(rois), _stream(stream), _ptr(maps)))

    @staticmethod
    def _roi_array(rois):
        import torch
        arr = (DLRoi * len(rois))()
        for k, r in enumerate(rois):
            if r.dim() != 2 or r.stride(1) != 1 or r.stride(0) < r.shape[1]:
                raise ValueError(f"roi {k}: rows must be dense (stride(1) == 1, stride(0) >= w)")
            if r.dtype not in (torch.uint16, torch.int16):
                raise ValueError(f"roi {k}: pixels must be 16-bit (torch.uint16), got {r.dtype}")
            arr[k].data = _ptr(r)
            arr[k].h = r.shape[0]
            arr[k].w = r.shape[1]
            arr[k].row_stride = r.stride(0)
        return arr

    def debug_conv_layer(self, x, res, blk: int, which: int, out, stream=None) -> int:
        n, h, w, _ = x.shape
        return self._rc(_lib.dl_debug_conv_layer(self.handle, _ptr(x), _ptr(res), n, h, w, blk, which,
                                                 _stream(stream), _ptr(out)))

    def debug_compact(self, det, maps, out, counts, stream=None) -> int:
        """Compaction alone: det cuda uint8 [n, h, w], maps cuda float
        [n, nh, h, w] -> records in out (cap * 32 bytes), counts int32 [n + 1]."""
        n, h, w = det.shape
        if tuple(maps.shape) != (n, self.head_outputs, h, w) or not maps.is_contiguous() or not det.is_contiguous():
            raise ValueError("det must be [n, h, w] and maps [n, nh, h, w], both contiguous")
        cap = out.numel() * out.element_size() // 32
        return self._rc(_lib.dl_debug_compact(self.handle, _ptr(det), _ptr(maps), n, h, w, _stream(stream),
                                              _ptr(out), cap, _ptr(counts)))

    def debug_detect(self, logit, tau: float, det, stream=None) -> int:
        n, h, w = logit.shape
        return self._rc(_lib.dl_debug_detect(self.handle, _ptr(logit), n, h, w, float(tau), _stream(stream),
                                             _ptr(det)))

    # ---- host ----
    def localize(self, frames: np.ndarray, cap: Optional[int] = None) -> np.ndarray:
        """Host frames uint16 [n, h, w] -> structured array of emitters (EMITTER_DTYPE)."""
        return self.localize_pipelined(frames[None], overlap=False, cap=cap)

    def localize_pipelined(self, frames: np.ndarray, overlap: bool = True, cap: Optional[int] = None) -> np.ndarray:
        """Host frames uint16 [nbatch, n, h, w]; batches are copied on a side stream
        while the previous batch is processed (overlap=True)."""
        F = _host_frames(frames, 4)
        nb, n, h, w = F.shape
        if cap is None:
            cap = max(1024, F.size // 16)
        out = np.empty(cap, EMITTER_DTYPE)
        cnt = ctypes.c_size_t()
        rc = _lib.dl_localize_pipelined(self.handle, F.ctypes.data, nb, n, h, w, int(bool(overlap)),
                                        out.ctypes.data, cap, ctypes.byref(cnt))
        if rc == DL_ERR_CAPACITY:
            return self.localize_pipelined(frames, overlap, cap=int(cnt.value))
        _check(rc, self.handle)
        return out[:cnt.value]          # a view: only the filled records were touched

    def localize_pipelined_unc(self, frames: np.ndarray, overlap: bool = True, cap: Optional[int] = None):
        """localize_pipelined for a 10-output network: (records, uncertainties),
        structured arrays of EMITTER_DTYPE and UNCERTAINTY_DTYPE."""
        F = _host_frames(frames, 4)
        nb, n, h, w = F.shape
        if cap is None:
            cap = max(1024, F.size // 16)
        out = np.empty(cap, EMITTER_DTYPE)
        unc = np.empty(cap, UNCERTAINTY_DTYPE)
        cnt = ctypes.c_size_t()
        rc = _lib.dl_localize_pipelined_unc(self.handle, F.ctypes.data, nb, n, h, w, int(bool(overlap)),
                                            out.ctypes.data, unc.ctypes.data, cap, ctypes.byref(cnt))
        if rc == DL_ERR_CAPACITY:
            return self.localize_pipelined_unc(frames, overlap, cap=int(cnt.value))
        _check(rc, self.handle)
        return out[:cnt.value], unc[:cnt.value]

    def localize_rois(self, rois: Sequence[np.ndarray], cap: Optional[int] = None) -> np.ndarray:
        """Host ROIs (2-D uint16 arrays, rows may be strided views) -> records
        with `frame` = the ROI's index (dl_localize_rois)."""
        arr = (DLRoi * len(rois))()
        for k, r in enumerate(rois):
            if not isinstance(r, np.ndarray) or r.dtype != np.uint16 or r.ndim != 2:
                raise ValueError(f"roi {k}: a 2-D uint16 numpy array is required")
            if r.strides[1] != 2 or r.strides[0] % 2 or r.strides[0] < 2 * r.shape[1]:
                raise ValueError(f"roi {k}: rows must be dense (element stride 1, row stride >= w)")
            arr[k].data = r.ctypes.data
            arr[k].h, arr[k].w = r.shape
            arr[k].row_stride = r.strides[0] // 2
        if cap is None:
            cap = max(1024, sum(r.size for r in rois) // 16)
        out = np.empty(cap, EMITTER_DTYPE)
        cnt = ctypes.c_size_t()
        rc = _lib.dl_localize_rois(self.handle, arr, len(rois), out.ctypes.data, cap, ctypes.byref(cnt))
        if rc == DL_ERR_CAPACITY:
            return self.localize_rois(rois, cap=int(cnt.value))
        _check(rc, self.handle)
        return out[:cnt.value]

    def localize_maps(self, frames: np.ndarray) -> np.ndarray:
        """Host frames uint16 [n, h, w] -> host maps float32 [n, nh, h, w]."""
        F = _host_frames(frames, 3)
        n, h, w = F.shape
        maps = np.empty((n, self.head_outputs, h, w), np.float32)
        self._rc(_lib.dl_localize_maps(self.handle, F.ctypes.data, n, h, w, maps.ctypes.data))
        return maps

    def localize_unc(self, frames: np.ndarray, cap: Optional[int] = None):
        """Host frames [n, h, w] of a 10-output network -> (records, uncertainties)."""
        return self.localize_pipelined_unc(frames[None], overlap=False, cap=cap)

    def graph(self, frames, out, counts) -> "Graph":
        """Capture localization of this fixed frame buffer into a HIP graph."""
        n, h, w = _frames_arg(frames).shape
        cap = out.numel() * out.element_size() // 32
        g = ctypes.c_void_p()
        self._rc(_lib.dl_graph_create(self.handle, _ptr(frames), n, h, w, _ptr(out), cap, _ptr(counts),
                                      ctypes.byref(g)))
        return Graph(self, g, (frames, out, counts))

    def graph_rois(self, rois, out, counts) -> "Graph":
        arr = self._roi_array(rois)
        cap = out.numel() * out.element_size() // 32
        g = ctypes.c_void_p()
        self._rc(_lib.dl_graph_create_rois(self.handle, arr, len(rois), _ptr(out), cap, _ptr(counts),
                                           ctypes.byref(g)))
        return Graph(self, g, (rois, out, counts))

    def graph_rois_dynamic(self, max_rois: int, max_h: int, max_w: int, max_pixels: int, out, counts) -> "Graph":
        """Capture one graph that localizes any ROI list within the capacity
        (dl_graph_create_rois_dynamic); replay it with Graph.launch_rois."""
        if counts.numel() < max_rois + 1:
            raise ValueError("counts must hold max_rois + 1 entries")
        cap = out.numel() * out.element_size() // 32
        g = ctypes.c_void_p()
        self._rc(_lib.dl_graph_create_rois_dynamic(self.handle, max_rois, max_h, max_w, max_pixels, _ptr(out), cap,
                                                   _ptr(counts), ctypes.byref(g)))
        return Graph(self, g, (out, counts))

    def autotune(self, frames, reps: int = 3, stream=None):
        """Pick the fastest convolution tile shape for this batch shape; returns
        (rows, {rows: ms per pass})."""
        n, h, w = _frames_arg(frames).shape
        best = ctypes.c_int32()
        ms = (ctypes.c_float * 2)()
        self._rc(_lib.dl_autotune(self.handle, _ptr(frames), n, h, w, _stream(stream), reps, ctypes.byref(best), ms))
        return int(best.value), {8: float(ms[0]), 4: float(ms[1])}

    def autotune_ex(self, frames, reps: int = 3, cache_path: Optional[str] = None, stream=None) -> dict:
        """Tune strip width and per-block tile rows on this batch (dl_autotune_ex);
        with cache_path, reuse or record the result."""
        n, h, w = _frames_arg(frames).shape
        r = DLTuneResult()
        path = cache_path.encode() if cache_path else None
        self._rc(_lib.dl_autotune_ex(self.handle, _ptr(frames), n, h, w, _stream(stream), reps, path,
                                     ctypes.byref(r)))
        nb = self.nblocks
        return {"rows": list(r.rows[:nb]), "strip": int(r.strip), "from_cache": bool(r.from_cache),
                "configs_timed": int(r.configs_timed), "ms_default": float(r.ms_default), "ms_best": float(r.ms_best)}

    # ---- training ----
    def train_grad(self, frames, truth, truth_off, grad=None, loss=None, stream=None):
        """Loss and gradient of one batch (dl_train_grad).  truth: cuda float32
        [E, 4] (x, y, z_nm, photons per true emitter, frame by frame);
        truth_off: cuda int32 [n + 1]; grad: cuda float32 [nparams] or None;
        returns the cuda float32 [4] loss (total, cross-entropy, count, loc)."""
        import torch
        n, h, w = _frames_arg(frames).shape
        if loss is None:
            loss = torch.zeros(4, dtype=torch.float32, device=frames.device)
        ntruth = int(truth.shape[0])
        self._rc(_lib.dl_train_grad(self.handle, _ptr(frames), n, h, w, _ptr(truth) if ntruth else None,
                                    _ptr(truth_off), ntruth, _stream(stream), _ptr(grad) if grad is not None else None,
                                    _ptr(loss)))
        return loss

    def train_step(self, frames, truth, truth_off, lr: float, loss=None, stream=None):
        """One Adam step of the handle's weights on this batch (dl_train_step)."""
        import torch
        n, h, w = _frames_arg(frames).shape
        if loss is None:
            loss = torch.zeros(4, dtype=torch.float32, device=frames.device)
        ntruth = int(truth.shape[0])
        self._rc(_lib.dl_train_step(self.handle, _ptr(frames), n, h, w, _ptr(truth) if ntruth else None,
                                    _ptr(truth_off), ntruth, _stream(stream), float(lr), _ptr(loss)))
        return loss

    def get_params(self) -> np.ndarray:
        """The handle's current weights, flat in blob order (dl_get_params)."""
        out = np.empty(self.nparams, np.float32)
        self._rc(_lib.dl_get_params(self.handle, out.ctypes.data, out.size))
        return out

    def set_gate(self, theta, threshold: float = 0.05):
        """Attach gate parameters (host array of 673 floats, or None to detach)."""
        if theta is None:
            self._rc(_lib.dl_set_gate(self.handle, None, threshold))
            return
        th = np.ascontiguousarray(theta, np.float32)
        assert th.size == GATE_NPARAM
        self._rc(_lib.dl_set_gate(self.handle, th.ctypes.data, float(threshold)))

    def set_camera_maps(self, gain, offset):
        """Per-pixel sCMOS gain and offset maps (host arrays [h][w]), or None
        and None to return to the config's scalars."""
        if gain is None and offset is None:
            self._rc(_lib.dl_set_camera_maps(self.handle, None, None, 0, 0))
            return
        g = np.ascontiguousarray(gain, np.float32)
        o = np.ascontiguousarray(offset, np.float32)
        if g.ndim != 2 or g.shape != o.shape:
            raise ValueError("gain and offset must be 2-D maps of one shape")
        self._rc(_lib.dl_set_camera_maps(self.handle, g.ctypes.data, o.ctypes.data, g.shape[0], g.shape[1]))

    def gate_pool(self, frames, pooled, stream=None):
        """Pool frames into gate tiles with this handle's preprocessing (its
        scalars or camera maps): the tiles its gated runs see."""
        n, h, w = frames.shape
        self._rc(_lib.dl_gate_pool_net(self.handle, _ptr(frames), n, h, w, _stream(stream), _ptr(pooled)))

    def gate_keep_map(self, keep, stream=None) -> int:
        n = ctypes.c_size_t()
        self._rc(_lib.dl_gate_keep_map(self.handle, _stream(stream), _ptr(keep), keep.numel(), ctypes.byref(n)))
        return int(n.value)

    def profile(self, on: bool = True):
        self._rc(_lib.dl_profile_enable(self.handle, int(bool(on))))

    def profile_read(self) -> dict:
        """Per-stage {name: (total_ms, launches)} since the last read (waits for the events)."""
        ms = (ctypes.c_double * NSTAGES)()
        n = (ctypes.c_int64 * NSTAGES)()
        self._rc(_lib.dl_profile_read(self.handle, ms, n))
        return {STAGES[i]: (ms[i], n[i]) for i in range(len(STAGES))}

    def _rc(self, rc):
        _check(rc, self.handle)
        return rc


class Graph:
    """A captured localization (``dl_graph_create``); keeps its buffers alive."""

    def __init__(self, net: Net, handle, buffers):
        self.net, self.handle, self._buffers = net, handle, buffers

    def launch(self, stream=None):
        _check(_lib.dl_graph_launch(self.handle, _stream(stream)), self.net.handle)

    def launch_rois(self, rois: Sequence, stream=None):
        """One replay of a capacity graph over this ROI list (cuda uint16
        [h, w] tensors, rows may be strided); the tensors must stay alive
        until the replay has run."""
        arr = Net._roi_array(rois)
        self._live = list(rois)
        _check(_lib.dl_graph_launch_rois(self.handle, arr, len(rois), _stream(stream)), self.net.handle)

    def close(self):
        if getattr(self, "handle", None):
            _lib.dl_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def uncertainties_from_device(unc, counts_total: int) -> np.ndarray:
    """Copy the first ``counts_total`` dl_uncertainty entries to a numpy structured array."""
    raw = unc.reshape(-1).view(__import__("torch").uint8)[: counts_total * 20].cpu().numpy()
    return raw.view(UNCERTAINTY_DTYPE).copy()


def emitters_from_device(out, counts_total: int) -> np.ndarray:
    """Copy the first ``counts_total`` records of a device record buffer to a numpy structured array."""
    raw = out.reshape(-1).view(__import__("torch").uint8)[: counts_total * 32].cpu().numpy()
    return raw.view(EMITTER_DTYPE).copy()


# ---------------------------------------------------------------- tile gate
GATE_TILE = 256
GATE_NPARAM = 673


def gate_pool(frames, pooled, gain=0.5, offset=100.0, in_scale=0.01, stream=None):
    n, h, w = _frames_arg(frames).shape
    _check(_lib.dl_gate_pool(_ptr(frames), n, h, w, gain, offset, in_scale, _stream(stream), _ptr(pooled)))


def gate_forward(pooled, theta, logits, stream=None):
    _check(_lib.dl_gate_forward(_ptr(pooled), pooled.shape[0], _ptr(theta), _stream(stream), _ptr(logits)))


def gate_backward(pooled, theta, dlogits, work, logits, grad, stream=None):
    _check(_lib.dl_gate_backward(_ptr(pooled), pooled.shape[0], _ptr(theta), _ptr(dlogits), _ptr(work),
                                 _stream(stream), _ptr(logits), _ptr(grad)))


def gate_bce(logits, labels, loss, dlogits, stream=None):
    _check(_lib.dl_gate_bce(_ptr(logits), _ptr(labels), logits.shape[0], _stream(stream), _ptr(loss), _ptr(dlogits)))


def gate_adam(theta, m, v, grad, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    _check(_lib.dl_gate_adam(_ptr(theta), _ptr(m), _ptr(v), _ptr(grad), theta.numel(), int(step), lr, b1, b2, eps,
                             _stream(stream)))


def host_alloc(nbytes: int) -> int:
    p = ctypes.c_void_p()
    _check(_lib.dl_host_alloc(nbytes, ctypes.byref(p)))
    return p.value


def host_free(p: int):
    _lib.dl_host_free(p)


RATE_KINDS = {"fp32": 0, "bf16": 1, "fp8": 2, "hbm_copy": 3}


def measure_rate(kind: str, nbytes: int = 1 << 30, reps: int = 3) -> float:
    """Sustained rate of the current device: dense MFMA TFLOP/s of a form
    ("fp32", "bf16", "fp8") or device copy GB/s ("hbm_copy", read + written)."""
    v = ctypes.c_double()
    _check(_lib.dl_measure_rate(RATE_KINDS[kind], nbytes, reps, ctypes.byref(v)))
    return v.value
