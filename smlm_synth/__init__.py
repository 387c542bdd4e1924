"""Seeded synthetic inputs for the localization path: camera frames and network weights.

This module creates *inputs only*.  It holds none of the localization method's
arithmetic (no preprocessing, convolution, detection or compaction), so both
the FP64 oracle and the HIP library can consume what it produces without
sharing any code with each other.

Frame model (the paper simulates its test data but does not publish it, see
its Sec. 4.1 and Sec. 4.2; these frames stand in for those simulations):

* emitters placed uniformly at random in the continuous frame [0,w) x [0,h)
  (pixel (i, j) spans [j, j+1) x [i, i+1)), count ~ Poisson(density * area);
* pixel-integrated Gaussian PSF (2D, sigma 1.3 px) or an astigmatic 3D PSF
  (sigma_x, sigma_y depend on z, the usual astigmatism model of Sec. 3.2's
  discussion of z encoding), truncated to a +-4 sigma window;
* Poisson shot noise on (background + PSF photons), Gaussian read noise in
  ADU, conversion ADU = photons / gain + offset, rounding and clipping to
  uint16.

Weights: He-normal (std = sqrt(2 / fan_in)) random initialisation with a fixed
seed, stored in the little-endian ``DLW1`` blob the C ABI reads.  A small
deterministic calibration of the 1x1 head (a linear probe of the final
features) makes a random network produce sparse, meaningful detections; its
constants are computed once by ``smlm_synth/make_calibration.py`` with the FP64
oracle and stored in ``calibration.json``.
"""
from __future__ import annotations

import json
import math
import os
import struct
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "FrameModel", "Camera", "scmos_camera", "NetSpec", "NET_A", "NET_B", "CONFIG_MODELS",
    "render_frames", "render_rois", "he_normal_weights", "make_net",
    "serialize_weights", "param_count", "net_flops_per_px", "receptive_radius",
    "TAU_LOGIT", "DLW_MAGIC",
]

#: detection threshold on the logit map: sigma(TAU_LOGIT) = 0.3 exactly
TAU_LOGIT = math.log(0.3 / 0.7)
DLW_MAGIC = b"DLW1"
DLW_VERSION = 1
DLW_MAX_BLOCKS = 8
DLD_MAGIC = b"DLD1"          # dense-connection networks
_HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------------------
# frame model
# --------------------------------------------------------------------------------------
@dataclass(frozen=True)
class FrameModel:
    """Parameters of the synthetic SMLM camera frames."""
    psf: str = "gauss2d"                    # "gauss2d" | "astig"
    sigma_px: float = 1.3                   # in-focus PSF sigma (px)
    pixel_nm: float = 100.0
    density: Tuple[float, float] = (1.0, 1.0)        # emitters / um^2, drawn per frame U(lo, hi)
    photons: Tuple[str, float, float] = ("uniform", 1000.0, 5000.0)  # or ("lognormal", median, sigma)
    background: Tuple[float, float] = (100.0, 100.0)  # photons / px, per frame U(lo, hi)
    read_sd_adu: float = 1.5
    gain: float = 0.5                       # photons per ADU
    offset: float = 100.0                   # ADU
    z_range_nm: Tuple[float, float] = (0.0, 0.0)
    astig_focal_nm: float = 250.0           # the two focal planes sit at +-250 nm
    astig_depth_nm: float = 400.0
    empty_tile: int = 0                      # >0: tile side for structured occupancy
    empty_frac: Tuple[float, float] = (0.0, 0.0)     # per-frame fraction of empty tiles
    # where the empty tiles lie: "iid" = each tile empty independently; "cell" =
    # the occupied tiles form one compact elliptical region (a cell in the field
    # of view) and the empty ones surround it
    empty_layout: str = "iid"

    def sigmas(self, z: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
        if self.psf == "gauss2d":
            s = np.full_like(z, self.sigma_px, dtype=np.float64)
            return s, s.copy()
        if self.psf == "astig":
            sx = self.sigma_px * np.sqrt(1.0 + ((z - self.astig_focal_nm) / self.astig_depth_nm) ** 2)
            sy = self.sigma_px * np.sqrt(1.0 + ((z + self.astig_focal_nm) / self.astig_depth_nm) ** 2)
            return sx, sy
        raise ValueError(f"unknown psf {self.psf!r}")


#: frame models of the workloads: tiny (4 x 128^2), full (16 x 2048^2), uneven ROIs and sparse frames
CONFIG_MODELS: Dict[str, FrameModel] = {
    # 4 x 128^2, 2D Gaussian sigma 1.3, density 1/um^2, photons U(1000,5000), bg 100
    "tiny": FrameModel(),
    # 16 x 2048^2 sCMOS-like, astigmatic 3D PSF, z U(-700,700), density U(0.5,2),
    # photons lognormal(median 3000, sigma 0.5), background U(50,200)
    "full": FrameModel(psf="astig", density=(0.5, 2.0), photons=("lognormal", 3000.0, 0.5),
                       background=(50.0, 200.0), z_range_nm=(-700.0, 700.0)),
    # uneven ROIs: tiny-model PSF/noise, density U(0.1, 5) per frame
    "rois": FrameModel(density=(0.1, 5.0)),
    # sparse frames for the tile gate: 30-70 % of 256^2 tiles empty, density U(0.05,0.5) in the rest
    "sparse": FrameModel(density=(0.05, 0.5), empty_tile=256, empty_frac=(0.3, 0.7)),
    # the same with the empty tiles around one compact occupied region
    "sparse_cell": FrameModel(density=(0.05, 0.5), empty_tile=256, empty_frac=(0.3, 0.7), empty_layout="cell"),
}

ROI_SIDES = (128, 256, 384, 512, 768, 1024)


@dataclass(frozen=True)
class Camera:
    """Per-pixel sCMOS calibration of one sensor, float32 [h][w] maps."""
    gain: np.ndarray       # photons per ADU
    offset: np.ndarray     # ADU
    read_sd: np.ndarray    # read noise, ADU


def scmos_camera(h: int, w: int, seed: int, gain: float = 0.5, offset: float = 100.0, gain_cv: float = 0.05,
                 offset_sd: float = 3.0, read_sd: float = 1.5, read_log_sd: float = 0.3) -> Camera:
    """Seeded sCMOS sensor: gain = gain (1 + gain_cv N) clipped to +-4 gain_cv,
    offset = offset + offset_sd N, read noise sd = read_sd exp(read_log_sd N)
    (N independent standard normals per pixel and map)."""
    rng = np.random.default_rng([seed, 0x5C])
    g = gain * (1.0 + gain_cv * np.clip(rng.standard_normal((h, w)), -4.0, 4.0))
    o = offset + offset_sd * rng.standard_normal((h, w))
    r = read_sd * np.exp(read_log_sd * rng.standard_normal((h, w)))
    return Camera(g.astype(np.float32), o.astype(np.float32), r.astype(np.float32))


# the camera of the render in progress (inherited by forked workers)
_CAMERA: Optional[Camera] = None


def _phi(t: np.ndarray) -> np.ndarray:
    """Standard normal CDF (used only to integrate the simulated PSF over a pixel)."""
    from scipy.special import ndtr
    return ndtr(t)


def _occupancy(nty: int, ntx: int, q: float, layout: str, rng: np.random.Generator) -> np.ndarray:
    """Occupied-tile map with an empty fraction of about ``q``.

    "iid": every tile is empty with probability q.  "cell": the round((1 - q) N)
    tiles whose centres are nearest (in an ellipse's metric) to a random centre
    are occupied: axis ratio U(0.5, 1), orientation U(0, pi), centre uniform
    over the middle half of the grid in each direction."""
    if layout == "iid":
        return rng.random((nty, ntx)) >= q
    if layout != "cell":
        raise ValueError(f"unknown empty-tile layout {layout!r}")
    cy = rng.uniform(0.25, 0.75) * nty
    cx = rng.uniform(0.25, 0.75) * ntx
    ratio = rng.uniform(0.5, 1.0)
    th = rng.uniform(0.0, math.pi)
    yy, xx = np.mgrid[0:nty, 0:ntx]
    dy, dx = yy + 0.5 - cy, xx + 0.5 - cx
    u = dx * math.cos(th) + dy * math.sin(th)
    v = -dx * math.sin(th) + dy * math.cos(th)
    dist = (u * ratio) ** 2 + v ** 2           # the long axis runs along u
    k = int(round((1.0 - q) * nty * ntx))
    occ = np.zeros(nty * ntx, bool)
    occ[np.argsort(dist.ravel(), kind="stable")[:k]] = True
    return occ.reshape(nty, ntx)


def _render_one(h: int, w: int, model: FrameModel, rng: np.random.Generator, camera: Optional[Camera] = None):
    """Render one frame; returns (uint16 frame, truth dict).  With a camera,
    its per-pixel gain, offset and read noise replace the model's scalars."""
    area_um2 = h * w * (model.pixel_nm / 1000.0) ** 2
    rho = rng.uniform(*model.density)
    bg = rng.uniform(*model.background)

    if model.empty_tile > 0:
        t = model.empty_tile
        nty, ntx = -(-h // t), -(-w // t)
        q = rng.uniform(*model.empty_frac)
        occupied = _occupancy(nty, ntx, q, model.empty_layout, rng)
        occ_idx = np.flatnonzero(occupied.ravel())
        # occupied area (clipped tiles at the ragged edge count their real size)
        ty, tx = np.divmod(occ_idx, ntx)
        th = np.minimum(t, h - ty * t)
        tw = np.minimum(t, w - tx * t)
        occ_area = float(np.sum(th * tw)) * (model.pixel_nm / 1000.0) ** 2
        k = rng.poisson(rho * occ_area) if occ_idx.size else 0
        if k:
            p = (th * tw).astype(np.float64)
            pick = rng.choice(occ_idx.size, size=k, p=p / p.sum())
            xs = tx[pick] * t + rng.random(k) * tw[pick]
            ys = ty[pick] * t + rng.random(k) * th[pick]
        else:
            xs = ys = np.zeros(0)
        tile_occupied = occupied
    else:
        k = rng.poisson(rho * area_um2)
        xs = rng.random(k) * w
        ys = rng.random(k) * h
        tile_occupied = None

    kind, a, b = model.photons
    if kind == "uniform":
        nph = rng.uniform(a, b, size=k)
    elif kind == "lognormal":
        nph = a * np.exp(b * rng.standard_normal(k))
    else:
        raise ValueError(kind)
    z = rng.uniform(*model.z_range_nm, size=k) if model.z_range_nm != (0.0, 0.0) else np.zeros(k)
    sx, sy = model.sigmas(z)

    mu = np.full(h * w, bg, dtype=np.float64)
    if k:
        # group emitters by window radius so each group is rendered vectorised
        rad = np.ceil(4.0 * np.maximum(sx, sy)).astype(np.int64)
        for r in np.unique(rad):
            sel = np.flatnonzero(rad == r)
            kk = 2 * r + 1
            cx = np.floor(xs[sel]).astype(np.int64)
            cy = np.floor(ys[sel]).astype(np.int64)
            off = np.arange(-r, r + 1)
            px = cx[:, None] + off[None, :]                       # (E, kk) pixel columns
            py = cy[:, None] + off[None, :]
            gx = _phi((px + 1 - xs[sel, None]) / sx[sel, None]) - _phi((px - xs[sel, None]) / sx[sel, None])
            gy = _phi((py + 1 - ys[sel, None]) / sy[sel, None]) - _phi((py - ys[sel, None]) / sy[sel, None])
            vx = (px >= 0) & (px < w)
            vy = (py >= 0) & (py < h)
            gx = np.where(vx, gx, 0.0)
            gy = np.where(vy, gy, 0.0)
            pxc = np.clip(px, 0, w - 1)
            pyc = np.clip(py, 0, h - 1)
            val = (nph[sel, None, None] * gy[:, :, None] * gx[:, None, :]).ravel()
            idx = (pyc[:, :, None] * w + pxc[:, None, :]).ravel()
            mu += np.bincount(idx, weights=val, minlength=h * w)
    counts = rng.poisson(mu).astype(np.float64)
    if camera is not None:
        assert camera.gain.shape == (h, w), "the camera maps must cover the frame"
        adu = (counts / camera.gain.ravel().astype(np.float64) + camera.offset.ravel().astype(np.float64)
               + camera.read_sd.ravel().astype(np.float64) * rng.standard_normal(h * w))
    else:
        adu = counts / model.gain + model.offset + model.read_sd_adu * rng.standard_normal(h * w)
    frame = np.clip(np.rint(adu), 0, 65535).astype(np.uint16).reshape(h, w)
    truth = {"x": xs, "y": ys, "z_nm": z, "photons": nph, "background": bg, "density": rho,
             "tile_occupied": tile_occupied}
    return frame, truth


def render_frames(n: int, h: int, w: int, model: FrameModel | str, seed: int,
                  frame_ids: Optional[Sequence[int]] = None, with_truth: bool = False,
                  workers: Optional[int] = None, camera: Optional[Camera] = None):
    """Render ``n`` frames of ``h x w`` uint16 (frame k seeded by ``(seed, k)``).

    ``frame_ids`` selects which frame indices of the seeded sequence to render
    (default ``range(n)``), so any frame can be regenerated on its own.
    ``workers`` > 1 renders frames in forked processes (default: automatic).
    ``camera`` (an sCMOS sensor of h x w) gives per-pixel gain, offset and
    read noise.
    """
    global _CAMERA
    if isinstance(model, str):
        model = CONFIG_MODELS[model]
    ids = list(range(n)) if frame_ids is None else list(frame_ids)
    out = np.empty((len(ids), h, w), dtype=np.uint16)
    truths = []
    jobs = [(h, w, model, int(seed), int(fid)) for fid in ids]
    if workers is None:
        workers = min(len(ids), _pool_size()) if len(ids) * h * w >= (1 << 22) else 1
    _CAMERA = camera
    try:
        if workers > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(workers) as pool:
                res = pool.map(_render_job, jobs)
        else:
            res = [_render_job(j) for j in jobs]
    finally:
        _CAMERA = None
    for i, (f, t) in enumerate(res):
        out[i] = f
        truths.append(t)
    return (out, truths) if with_truth else out


TRUTH_DTYPE = np.dtype([("x", "<f8"), ("y", "<f8"), ("z_nm", "<f8"), ("photons", "<f8")])


def truth_array(truth: dict, h: int, w: int) -> np.ndarray:
    """The true emitters of one rendered frame that lie inside it (0 <= x < w,
    0 <= y < h, pixel units), as records (x, y, z_nm, photons)."""
    x, y = np.asarray(truth["x"], np.float64), np.asarray(truth["y"], np.float64)
    keep = (x >= 0) & (x < w) & (y >= 0) & (y < h)
    out = np.zeros(int(keep.sum()), TRUTH_DTYPE)
    for k in TRUTH_DTYPE.names:
        out[k] = np.asarray(truth[k], np.float64)[keep]
    return out


def _pool_size() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _render_job(job):
    h, w, model, seed, fid = job
    return _render_one(h, w, model, np.random.default_rng([seed, fid]), _CAMERA)


def roi_shapes(n: int, seed: int, sides: Sequence[int] = ROI_SIDES) -> List[Tuple[int, int]]:
    """Seeded (h, w) of ``n`` uneven ROIs, each side drawn uniformly from ``sides``."""
    rng = np.random.default_rng([int(seed), 0x5151])
    hs = rng.choice(np.asarray(sides), size=n)
    ws = rng.choice(np.asarray(sides), size=n)
    return [(int(a), int(b)) for a, b in zip(hs, ws)]


def render_rois(n: int, model: FrameModel | str, seed: int, sides: Sequence[int] = ROI_SIDES,
                shapes: Optional[Sequence[Tuple[int, int]]] = None) -> List[np.ndarray]:
    """Render ``n`` uneven ROI frames (list of uint16 arrays of differing shapes)."""
    if isinstance(model, str):
        model = CONFIG_MODELS[model]
    shapes = roi_shapes(n, seed, sides) if shapes is None else list(shapes)
    out = []
    for k, (h, w) in enumerate(shapes):
        rng = np.random.default_rng([int(seed), int(k)])
        f, _ = _render_one(h, w, model, rng)
        out.append(f)
    return out


# --------------------------------------------------------------------------------------
# networks and weights
# --------------------------------------------------------------------------------------
@dataclass(frozen=True)
class NetSpec:
    """Residual dilated localization network: stem 3x3 (1->C), blocks of two 3x3
    convolutions at one dilation each, 1x1 head C->5 (logit, dx, dy, dz, photons)
    or C->10 (those, then the raw uncertainties of x, y, z and photons and the
    background)."""
    name: str
    C: int
    dilations: Tuple[int, ...]
    in_scale: float = 0.01      # photons -> network input units (background 100 -> 1.0)
    z_scale: float = 700.0      # nm per unit of the dz map
    ph_scale: float = 1000.0    # photons per unit of the photon map
    head_outputs: int = 5       # 5, or 10 with the uncertainty planes


@dataclass(frozen=True)
class DenseSpec:
    """Dense-connection dilated network: stem 3x3 (1->C), then one dense block
    per dilation.  Block k at dilation d: ``layers`` 3x3 convolutions at
    dilation d, layer i reading the concatenation of the block input (C
    channels) and the i earlier layers' outputs (``growth`` channels each) and
    giving ``growth`` channels (+ bias, ReLU); a 1x1 transition over the whole
    concatenation (C + layers * growth -> C, + bias, ReLU) gives the block's
    output.  With ``unet`` = 2, a two-stage U-Net follows the blocks (2x2 max
    pooling, 3x3 convolutions C -> C on the way down at levels 1 and 2,
    nearest upsampling and 3x3 convolutions over [skip, upsampled] 2C -> C on
    the way up at levels 1 and 0, each + bias, ReLU).  Then the 1x1 head
    C -> head_outputs."""
    name: str
    C: int
    dilations: Tuple[int, ...]
    layers: int = 4
    growth: int = 16
    in_scale: float = 0.01
    z_scale: float = 700.0
    ph_scale: float = 1000.0
    head_outputs: int = 5
    unet: int = 0


NET_A = NetSpec("A", 32, (1, 2, 4))
NET_B = NetSpec("B", 48, (1, 2, 4, 8, 16))
# the same networks with the uncertainty head (planes 5-9)
NET_AU = NetSpec("AU", 32, (1, 2, 4), head_outputs=10)
NET_BU = NetSpec("BU", 48, (1, 2, 4, 8, 16), head_outputs=10)
# the paper's feature extractor as read here: one coarse-grained and three
# context dense blocks at dilations 2, 4, 8, 16
NET_D = DenseSpec("D", 32, (2, 4, 8, 16))
# ... followed by the fine-grained stage, a two-stage U-Net
NET_DU = DenseSpec("DU", 32, (2, 4, 8, 16), unet=2)
# net D with the uncertainty head (the trained form of the dense network)
NET_DT = DenseSpec("DT", 32, (2, 4, 8, 16), head_outputs=10)
# ... and net DU with it
NET_DUT = DenseSpec("DUT", 32, (2, 4, 8, 16), head_outputs=10, unet=2)
NETS = {"A": NET_A, "B": NET_B, "AU": NET_AU, "BU": NET_BU, "D": NET_D, "DU": NET_DU, "DT": NET_DT, "DUT": NET_DUT}
# pixels (per axis) a two-stage U-Net's output reaches into its input: its
# final 3x3 conv, and through pooling and nearest upsampling the level-1 and
# level-2 convolutions
UNET_REACH = 12


def is_dense(spec) -> bool:
    return isinstance(spec, DenseSpec)


def tensor_layout(spec) -> List[Tuple[str, Tuple[int, ...]]]:
    """Names and shapes of the weight tensors, in blob order."""
    C = spec.C
    lay = [("stem.w", (C, 1, 3, 3)), ("stem.b", (C,))]
    if is_dense(spec):
        G, L = spec.growth, spec.layers
        for k in range(len(spec.dilations)):
            for i in range(L):
                lay += [(f"blk{k}.l{i}.w", (G, C + i * G, 3, 3)), (f"blk{k}.l{i}.b", (G,))]
            lay += [(f"blk{k}.t.w", (C, C + L * G)), (f"blk{k}.t.b", (C,))]
        if spec.unet:
            lay += [("unet.d1.w", (C, C, 3, 3)), ("unet.d1.b", (C,)), ("unet.d2.w", (C, C, 3, 3)), ("unet.d2.b", (C,)),
                    ("unet.u1.w", (C, 2 * C, 3, 3)), ("unet.u1.b", (C,)), ("unet.u0.w", (C, 2 * C, 3, 3)),
                    ("unet.u0.b", (C,))]
        nh = spec.head_outputs
        return lay + [("head.w", (nh, C)), ("head.b", (nh,))]
    for k in range(len(spec.dilations)):
        lay += [(f"blk{k}.w1", (C, C, 3, 3)), (f"blk{k}.b1", (C,)),
                (f"blk{k}.w2", (C, C, 3, 3)), (f"blk{k}.b2", (C,))]
    nh = spec.head_outputs
    lay += [("head.w", (nh, C)), ("head.b", (nh,))]
    return lay


def param_count(spec: NetSpec) -> int:
    return int(sum(np.prod(s) for _, s in tensor_layout(spec)))


def net_flops_per_px(spec) -> int:
    """Algorithmic FLOP per output pixel (2 per multiply-add; stem + blocks + head)."""
    C, B = spec.C, len(spec.dilations)
    if is_dense(spec):
        G, L = spec.growth, spec.layers
        blk = sum(9 * (C + i * G) * G for i in range(L)) + (C + L * G) * C
        # the U-Net per level-0 pixel: level l holds 1/4^l of the pixels
        unet = (9 * C * C / 4 + 9 * C * C / 16 + 9 * 2 * C * C / 4 + 9 * 2 * C * C) if spec.unet else 0
        return int(2 * (9 * C + B * blk + unet + spec.head_outputs * C))
    macs = 9 * C + B * 2 * 9 * C * C + spec.head_outputs * C
    return 2 * macs


def block_flops_per_px(spec: NetSpec) -> int:
    """FLOP per pixel of one 3x3 C->C convolution layer."""
    return 2 * 9 * spec.C * spec.C


def receptive_radius(spec) -> int:
    if is_dense(spec):
        return 1 + spec.layers * sum(spec.dilations) + (UNET_REACH if spec.unet else 0)
    return 1 + 2 * sum(spec.dilations)


def he_normal_weights(spec: NetSpec, seed: int, bias_std: float = 0.0) -> Dict[str, np.ndarray]:
    """He-normal weights (std sqrt(2/fan_in), untruncated), drawn tensor by tensor
    in blob order from ``numpy.random.default_rng(seed)``; biases are 0 unless
    ``bias_std`` > 0 (then N(0, bias_std^2), drawn after all weights)."""
    rng = np.random.default_rng(int(seed))
    out: Dict[str, np.ndarray] = {}
    for name, shape in tensor_layout(spec):
        if name.endswith(".w"):
            fan_in = int(np.prod(shape[1:]))   # (1x1 transitions: their input channels)
            out[name] = (rng.standard_normal(shape) * math.sqrt(2.0 / fan_in)).astype(np.float32)
        elif name.endswith(("w1", "w2")):
            fan_in = int(np.prod(shape[1:]))
            out[name] = (rng.standard_normal(shape) * math.sqrt(2.0 / fan_in)).astype(np.float32)
        else:
            out[name] = np.zeros(shape, dtype=np.float32)
    if bias_std > 0:
        for name, shape in tensor_layout(spec):
            if name.endswith((".b", "b1", "b2")):
                out[name] = (rng.standard_normal(shape) * bias_std).astype(np.float32)
    return out


def load_calibration(spec: NetSpec, seed: int) -> Optional[dict]:
    path = os.path.join(_HERE, "calibration.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    return table.get(f"{spec.name[:1]}:{seed}")


def apply_calibration(weights: Dict[str, np.ndarray], calib: dict) -> Dict[str, np.ndarray]:
    """Replace the 1x1 head's first five rows by the stored calibrated head
    (linear probe of the final features; see ``make_calibration.py``).  The
    uncertainty rows of a 10-output head keep their He-normal draws scaled by
    0.05, with bias -1 (raw values near -1: uncertainties near softplus(-1),
    0.31 units)."""
    w = {k: v.copy() for k, v in weights.items()}
    C = w["head.w"].shape[1]
    w["head.w"][:5] = np.asarray(calib["head_w"], np.float32).reshape(5, C)
    w["head.b"][:5] = np.asarray(calib["head_b"], np.float32).reshape(5)
    if w["head.w"].shape[0] > 5:
        w["head.w"][5:] *= np.float32(0.05)
        w["head.b"][5:] = np.float32(-1.0)
    return w


def make_net(spec: NetSpec | str, seed: int, calibrated: bool = True, bias_std: float = 0.0):
    """Seeded network weights; calibrated head if stored constants exist."""
    if isinstance(spec, str):
        spec = NETS[spec]
    w = he_normal_weights(spec, seed, bias_std=bias_std)
    if calibrated and bias_std == 0.0:
        c = load_calibration(spec, seed)
        if c is not None:
            w = apply_calibration(w, c)
    return spec, w


def serialize_weights(spec, weights: Dict[str, np.ndarray]) -> bytes:
    """Little-endian ``DLW1`` blob.

    Header (64 bytes): magic 'DLW1', u32 version, u32 C, u32 nblocks,
    u32 dilation[8], f32 in_scale, f32 z_scale, f32 ph_scale, u32 head outputs
    (0 = 5),
    then the FP32 tensors of ``tensor_layout`` in order, C-contiguous.
    """
    nb = len(spec.dilations)
    if nb > DLW_MAX_BLOCKS:
        raise ValueError("too many blocks")
    dil = list(spec.dilations) + [0] * (DLW_MAX_BLOCKS - nb)
    body = b"".join(np.ascontiguousarray(weights[name], dtype="<f4").tobytes()
                    for name, _ in tensor_layout(spec))
    if is_dense(spec):
        # 'DLD1' (80 bytes): magic, u32 version, u32 C, u32 nblocks, u32 layers,
        # u32 growth, u32 dilation[8], f32 in_scale, f32 z_scale, f32 ph_scale,
        # u32 head outputs, u32 U-Net levels (0 or 2), 4 zero bytes
        head = DLD_MAGIC + struct.pack("<IIIII8IfffII4x", 1, spec.C, nb, spec.layers, spec.growth, *dil,
                                       spec.in_scale, spec.z_scale, spec.ph_scale, spec.head_outputs, spec.unet)
        assert len(head) == 80
        return head + body
    # the last header word: 0 for the 5-output head, else the head's outputs
    head = DLW_MAGIC + struct.pack("<III8IfffI", DLW_VERSION, spec.C, nb, *dil,
                                   spec.in_scale, spec.z_scale, spec.ph_scale,
                                   0 if spec.head_outputs == 5 else spec.head_outputs)
    assert len(head) == 64
    return head + body


def flat_weights(spec: NetSpec, weights: Dict[str, np.ndarray]) -> np.ndarray:
    """All tensors concatenated in blob order (float32)."""
    return np.concatenate([np.asarray(weights[n], np.float32).ravel() for n, _ in tensor_layout(spec)])


def unflat_weights(spec, flat: np.ndarray) -> Dict[str, np.ndarray]:
    """The tensors of a flat blob-order vector (the inverse of flat_weights)."""
    out, k = {}, 0
    for name, shape in tensor_layout(spec):
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[k:k + n]).reshape(shape)
        k += n
    assert k == len(flat)
    return out


# --------------------------------------------------------------------------------------
# tile-gate network (2 conv layers of 8 channels + global max + linear 8 -> 1)
# --------------------------------------------------------------------------------------
GATE_POOL = 4
GATE_CH = 8
GATE_TILE = 256


def gate_layout() -> List[Tuple[str, Tuple[int, ...]]]:
    c = GATE_CH
    return [("g1.w", (c, 1, 3, 3)), ("g1.b", (c,)), ("g2.w", (c, c, 3, 3)), ("g2.b", (c,)),
            ("fc.w", (c,)), ("fc.b", (1,))]


def gate_init(seed: int) -> Dict[str, np.ndarray]:
    """He-normal gate weights from ``default_rng(seed)``; biases 0."""
    rng = np.random.default_rng(int(seed))
    out = {}
    for name, shape in gate_layout():
        if name.endswith(".w"):
            fan_in = int(np.prod(shape[1:])) if len(shape) > 1 else shape[0]
            out[name] = (rng.standard_normal(shape) * math.sqrt(2.0 / fan_in)).astype(np.float32)
        else:
            out[name] = np.zeros(shape, np.float32)
    return out


def gate_flat(w: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(w[n], np.float32).ravel() for n, _ in gate_layout()])


def gate_unflat(v: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for n, s in gate_layout():
        k = int(np.prod(s))
        out[n] = np.asarray(v[o:o + k], np.float32).reshape(s)
        o += k
    return out
