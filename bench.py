#!/usr/bin/env python3
"""Throughput of the localization path on one MI355X: Mpixel/s from uint16
frames (resident in HBM) to the emitter list (in HBM).

Workload (default): 16 frames of 2048 x 2048 uint16, astigmatic 3D PSF,
density U(0.5, 2) / um^2, lognormal photons, background U(50, 200), sCMOS-like
noise; net B (C = 48, residual blocks at dilations 1, 2, 4, 8, 16), FP32.
A step is one pass of the whole path over the batch: preprocessing + stem,
10 dilated convolutions (head fused into the last), detection, scan, emit.

Prints ONE JSON line.  Besides the throughput it reports the roofline of the
dominant kernel (the 3x3 block convolution: MFMA-bound in FP32, HBM-bound in
BF16 and FP8) from HIP events recorded around each launch on its stream
during the timed steps, the BF16 and FP8 forms measured on the same frames
(under "forms", with their speedup over FP32), and the FP64 CPU oracle timed
on a bounded sample of the same workload, which also scores every form's
emitters on that sample (recall, precision, RMS offset errors).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpixel/s frame->emitter list: FP32 vs BF16/FP8/gated at oracle-matched recall"
PEAKS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0, "bf16x3": 2500.0}   # dense MFMA TFLOP/s, MI355X
# BF16 MFMA products per algorithmic product: the split-BF16 form takes three
MFMA_PER_PRODUCT = {"fp32": 1, "bf16": 1, "fp8": 1, "bf16x3": 3}
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS")
    return min(n, int(omp)) if omp and omp.isdigit() else n


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), for the baseline's record."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp8", "bf16x3"],
                    help="the headline form (value, roofline, dtype)")
    ap.add_argument("--forms", default="bf16x3,bf16,fp8",
                    help="further forms measured on the same frames and reported under 'forms' ('' = none)")
    ap.add_argument("--frames", type=int, default=16)
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--cpu-sample", type=int, default=1536,
                    help="side of the oracle's sample: the top-left crop of frame 0 (the frame size = the whole "
                         "frame; 0 = skip)")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--workload", default="full", choices=["full", "tiny", "rois", "sparse", "pipeline", "train"],
                    help="full: the headline (16 x 2048^2, net B); tiny: 4 x 128^2 net A; rois: 256 uneven "
                         "ROIs, net A; sparse: gated BF16 net B on 64 x 2048^2 sparse frames; pipeline: "
                         "host frames with H2D overlapped on a side stream; train: training steps of net AU (DT / DUT with --net D / DU)")
    ap.add_argument("--sparse-layout", default="iid", choices=["iid", "cell"],
                    help="sparse workload: empty 256^2 tiles chosen independently (iid) or around one "
                         "compact occupied region (cell)")
    ap.add_argument("--train-eval-steps", type=int, default=500,
                    help="train workload: Adam steps of the trained-net evaluation that follows the timed steps "
                         "(0 = leave it out, e.g. under a profiler)")
    ap.add_argument("--net", default="B", choices=["B", "BU", "D", "DU"],
                    help="full workload: net B with the 5-output head, BU, the same net with the "
                         "10-output head (per-pixel uncertainties and background), D, the "
                         "dense-connection network, or DU, D followed by the two-stage U-Net (FP32, scalar "
                         "camera model); train workload: D or DU trains net DT or DUT (D or DU with the "
                         "10-output head) instead of net AU")
    ap.add_argument("--camera", default="scmos", choices=["scmos", "scalar"],
                    help="full and pipeline workloads: frames from a seeded sCMOS sensor whose per-pixel gain "
                         "and offset maps the net is given (scmos), or the scalar camera model (scalar)")
    ap.add_argument("--gen-workers", type=int, default=0,
                    help="processes rendering the frames (0 = automatic; 1 under profilers)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this many MiB first (scale reference for HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "frames are independent, the multi-GPU form is a design note only.", file=sys.stderr)
        sys.exit(2)

    import smlm_synth as S

    if args.workload != "full":
        from bench_workloads import run_workload
        run_workload(args)
        return

    if args.net in ("D", "DU"):
        # the dense kernels run FP32 with the scalar camera model only
        if args.precision != "fp32" or args.camera != "scalar":
            print("--net D and DU run with --precision fp32 --camera scalar", file=sys.stderr)
            sys.exit(2)
        args.forms = ""
    # inputs first, before anything touches the GPU (workers are forked)
    spec, w = S.make_net(args.net, 3 if args.net in ("D", "DU") else 2)
    n, side = args.frames, args.size
    t0 = time.time()
    cam = S.scmos_camera(side, side, 1002) if args.camera == "scmos" else None
    frames = S.render_frames(n, side, side, "full", 1002, workers=args.gen_workers or None, camera=cam)
    log(f"generated {n} x {side}^2 frames in {time.time() - t0:.1f}s ({args.camera} camera)")

    import torch
    import paper_2410_02314_amd as dl

    assert torch.cuda.is_available(), "no HIP device"
    dev = torch.device("cuda:0")
    d_frames = torch.from_numpy(frames).to(dev)
    if args.copy_probe_mib > 0:
        # plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale between counter units and bytes moved
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {nb} bytes read + {nb} bytes written per launch")
        del src, dst

    forms = [args.precision] + [f for f in args.forms.split(",") if f and f != args.precision]
    results = {f: measure_form(args, f, spec, w, d_frames, dl, torch, dev, cam) for f in forms}
    head = results[args.precision]
    # each roofline against the rate this device sustains as well as the published peak
    rates = {}
    for r in results.values():
        rf = r["roofline"]
        kind = "hbm_copy" if rf["bound"] == "hbm" else rf["kernel"].split()[1]
        if kind not in rates:
            rates[kind] = dl.measure_rate(kind, 1 << 30, 3)
            log(f"measured {kind} rate: {rates[kind]:.1f} {rf['unit']}")
        rf["measured_peak"] = round(rates[kind], 1)
        rf["frac_of_measured"] = round(rf["achieved"] / rates[kind], 4)

    cpu, ref = None, None
    if args.cpu_sample > 0:
        cpu, ref = cpu_baseline(args, spec, w, frames, head["net"], dev, head["records"], cam)
        for f, r in results.items():
            r["accuracy_vs_oracle"] = accuracy_on_sample(r["records"], ref)
            r["accuracy_vs_oracle"].update(map_errors_on_sample(r["net"], d_frames, ref, torch, dev))

    def public(r):
        return {k: v for k, v in r.items() if k not in ("net", "records")}

    for r in results.values():
        if r.get("accuracy_vs_oracle"):
            r["accuracy_target"] = accuracy_target(r["accuracy_vs_oracle"])
    n, side = args.frames, args.size
    others = {}
    for f in forms[1:]:
        r = public(results[f])
        sp = round(r["value"] / head["value"], 3)
        r["speedup_vs_" + args.precision] = sp
        # a speedup counts as "at oracle-matched recall" only where the form
        # meets the accuracy target on the oracle's sample
        met = bool(r.get("accuracy_target", {}).get("met"))
        r["speedup_at_matched_recall"] = sp if met else None
        others[f] = r
    res = {
        "metric": METRIC, "value": head["value"], "unit": "Mpixel/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "ms_per_step_median": head["ms_per_step_median"], "ms_per_step_min": head["ms_per_step_min"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.precision,
        "data": "synthetic (seeded astigmatic-PSF SMLM frames; random-init calibrated net)",
        "config": {"workload": f"{n} x {side}x{side} uint16 frames, astigmatic 3D PSF, net {args.net} "
                               f"({net_text(spec)}, {spec.head_outputs}-output head), {args.precision}",
                   "frames": n, "height": side, "width": side, "precision": args.precision,
                   "camera": ("sCMOS per-pixel gain/offset maps (sensor seed 1002)" if cam is not None
                              else "scalar gain 0.5, offset 100"),
                   "parallelism": "single GPU"},
        "roofline": head["roofline"], "stage_ms_per_step": head["stage_ms_per_step"],
        "bandwidth_kernels": head["bandwidth_kernels"],
        "emitters_per_step": head["emitters_per_step"],
        "accuracy_vs_oracle": head.get("accuracy_vs_oracle"),
        "accuracy_target": head.get("accuracy_target"),
        "forms": others,
        "gated_form": "measured by --workload sparse (sparse frames; the gate is trained first), not in this line",
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    for r in results.values():
        r["net"].close()


def net_text(spec):
    import smlm_synth as S
    d = ",".join(str(x) for x in spec.dilations)
    if S.is_dense(spec):
        return (f"dense blocks: C={spec.C}, {spec.layers} 3x3 layers of growth {spec.growth} + 1x1 transition "
                f"per block, d={d}" + (", then the two-stage U-Net" if spec.unet else ""))
    return f"C={spec.C}, d={d}"


def dense_roofline(spec, prof, total_px, steps):
    """Roofline of the dense network's dominant kernel, the plain 3x3 dense
    layer (k_dconv without fusion: the first L - 1 layers of each block; layer
    i reads C + i G channels and writes G, so its FLOP and bytes per pixel grow
    with i); achieved = the mean algorithmic FLOP of those nblocks x (L - 1)
    launches / their mean duration.  Each block's last layer runs fused with
    the block's 1x1 transition (and, in the last block, the head); it is
    reported beside it."""
    C, G, L, nb, nh = spec.C, spec.growth, spec.layers, len(spec.dilations), spec.head_outputs
    CT = C + L * G
    cins = [C + i * G for i in range(L - 1)]
    conv_ms, conv_n = prof["conv"]
    assert conv_n == nb * (L - 1) * steps, (conv_n, nb, L, steps)
    avg_s = conv_ms / conv_n * 1e-3
    flop_launch = 2.0 * 9 * G * (sum(cins) / len(cins)) * total_px
    bytes_launch = 4.0 * (sum(cins) / len(cins) + G) * total_px
    tflops = flop_launch / avg_s / 1e12
    roof = {"bound": "mfma", "achieved": round(tflops, 2), "peak": PEAKS["fp32"], "unit": "TFLOP/s",
            "frac": round(tflops / PEAKS["fp32"], 4),
            "traffic": measured_traffic(dense_traffic_key(spec, total_px), DENSE_SOURCES),
            "kernel": f"k_dconv fp32 (3x3 dilated dense layer, growth {G} over {cins[0]}..{cins[-1]} input channels; "
                      f"mean of the {nb * (L - 1)} unfused launches)",
            "avg_launch_ms": round(avg_s * 1e3, 3), "flop_per_launch": flop_launch,
            "algorithmic_bytes_per_launch": round(bytes_launch),
            "hbm_gb_s": round(bytes_launch / avg_s / 1e9, 1)}
    # the fused last layers: 3x3 over C + (L - 1) G channels, then the 1x1
    # transition CT -> C (and the head C -> nh in the last block)
    cin = C + (L - 1) * G
    fused = []
    for stage, head in (("conv_1x1", False), ("conv_head", True)):
        t_ms, t_n = prof[stage]
        if not t_n:
            continue
        ts = t_ms / t_n * 1e-3
        if head and spec.unet:       # the U-Net's last conv (2C -> C at level 0) with the head
            tf = (2.0 * 9 * 2 * C * C + 2.0 * C * nh) * total_px
            tb = (4.0 * 2 * C + 4.0 * nh) * total_px
            name = f"k_dconv fp32 fused (U-Net 3x3 {2 * C} -> {C}, head {C} -> {nh})"
        else:
            tf = (2.0 * 9 * G * cin + 2.0 * CT * C + (2.0 * C * nh if head else 0.0)) * total_px
            tb = (4.0 * (cin + C) + (4.0 * nh - 4.0 * C if head else 0.0)) * total_px
            name = (f"k_dconv fp32 fused (3x3 {cin} -> {G}, 1x1 transition {CT} -> {C}"
                    + (f", head {C} -> {nh})" if head else ")"))
        fused.append({"kernel": name, "launches_per_step": t_n // steps, "avg_launch_ms": round(ts * 1e3, 3),
                      "tflop_s": round(tf / ts / 1e12, 2), "mfma_frac": round(tf / ts / 1e12 / PEAKS["fp32"], 4),
                      "gb_s": round(tb / ts / 1e9, 1)})
    roof["fused_last_layers"] = fused
    if spec.unet and prof["unet"][1]:
        # pooling, upsampling and the level-1 and level-2 convolutions, per step
        roof["unet_stage_ms_per_step"] = round(prof["unet"][0] / steps, 3)
    return roof


def dense_traffic_key(spec, total_px):
    return f"k_dconv fp32 unfused net {spec.name} {total_px}px"


def measure_form(args, precision, spec, w, d_frames, dl, torch, dev, cam=None):
    """Time `steps` passes of the whole path in one form on the resident frames;
    returns throughput, per-stage HIP-event times and the dominant kernel's
    roofline (the 3x3 block convolution; its launches are bracketed by HIP
    events on the stream they run on)."""
    import smlm_synth as S
    n, side = args.frames, args.size
    net = dl.Net(S.serialize_weights(spec, w), precision=precision, tile_rows=args.tile_rows)
    if cam is not None:
        net.set_camera_maps(cam.gain, cam.offset)
    cap = n * side * side // 64
    d_out = torch.empty((cap, 8), dtype=torch.int32, device=dev)
    d_counts = torch.zeros(n + 1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    if net.head_outputs == 10:               # records and their uncertainties
        d_unc = torch.empty((cap * 5,), dtype=torch.float32, device=dev)
        run = lambda: net.localize_device_unc(d_frames, d_out, d_unc, d_counts, stream)  # noqa: E731
    else:
        run = lambda: net.localize_device(d_frames, d_out, d_counts, stream)  # noqa: E731
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    net.profile(True)
    net.profile_read()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    wall0 = time.perf_counter()
    for k in range(args.steps):
        run()
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    prof = net.profile_read()
    net.profile(False)
    ms_step = evs[0].elapsed_time(evs[-1]) / args.steps
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    total_px = n * side * side
    value = total_px / (ms_step * 1e-3) / 1e6
    counts = d_counts.cpu().numpy()
    log(f"[{precision}] {ms_step:.2f} ms/step, {value:.1f} Mpx/s, wall {wall / args.steps * 1e3:.2f} ms/step, "
        f"{int(counts[n])} emitters/step")
    log(f"[{precision}] stages: " + ", ".join(f"{k} {v[0] / max(1, v[1]):.3f} ms x{v[1]}" for k, v in prof.items() if v[1]))

    C = spec.C
    if S.is_dense(spec):
        roofline = dense_roofline(spec, prof, total_px, args.steps)
        pt_bytes = 4 * C                      # the stem writes C channels of each point
    else:
        roofline, pt_bytes = conv_roofline(args, precision, spec, prof, total_px)
    # the bandwidth-bound stages against the HBM peak, from their algorithmic
    # bytes: the stem reads the uint16 frame (+ the 8-byte camera map per pixel
    # with sCMOS maps) and writes one stored point per pixel; detection reads
    # the logit plane and writes one mask bit per pixel
    bw = {}
    for stage, nbytes in (("stem", total_px * (2 + (8 if cam is not None else 0) + pt_bytes)),
                          ("detect", total_px * (4 + 1 / 8))):
        if prof.get(stage, (0, 0))[1]:
            t = prof[stage][0] / prof[stage][1] * 1e-3
            bw[stage] = {"gb_s": round(nbytes / t / 1e9, 1), "frac_of_hbm_peak": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 3),
                         "algorithmic_bytes": round(nbytes), "avg_ms": round(t * 1e3, 3)}
    recs = dl.emitters_from_device(d_out, min(int(counts[n]), cap))
    return {"value": round(value, 2), "ms_per_step": round(ms_step, 3),
            "ms_per_step_median": round(float(np.median(step_ms)), 3), "ms_per_step_min": round(min(step_ms), 3),
            "roofline": roofline,
            "stage_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in prof.items() if v[1]},
            "bandwidth_kernels": bw,
            "emitters_per_step": int(counts[n]), "net": net, "records": recs}


def conv_roofline(args, precision, spec, prof, total_px):
    """Roofline of the residual network's dominant kernel, the 3x3 block
    convolution (mean of its non-head launches)."""
    n, side, C = args.frames, args.size, spec.C
    conv_ms, conv_n = prof["conv"]
    avg_s = conv_ms / conv_n * 1e-3
    flop_launch = 2.0 * 9 * C * C * total_px
    tflops = flop_launch / avg_s / 1e12
    # bytes per activation point: FP32 / BF16 values, FP8 codes + 2 group scale bytes
    pt_bytes = {"fp32": 4 * C, "bf16": 2 * C, "fp8": C + 2, "bf16x3": 4 * C}[precision]
    # algorithmic HBM bytes of the mean non-head conv launch: input + output for
    # all nine, + the residual for the four second convolutions of blocks 1-4
    nb = len(spec.dilations)
    n_conv = 2 * nb - 1
    bytes_launch = total_px * pt_bytes * (2 * n_conv + (nb - 1)) / n_conv
    gbs = bytes_launch / avg_s / 1e9
    key = f"k_conv {precision} C={C} {n}x{side}x{side}"
    if precision == "fp32":
        roofline = {"bound": "mfma", "achieved": round(tflops, 2), "peak": PEAKS[precision], "unit": "TFLOP/s",
                    "frac": round(tflops / PEAKS[precision], 4)}
    else:
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "mfma_frac": round(MFMA_PER_PRODUCT[precision] * tflops / PEAKS[precision], 4)}
    roofline.update({"traffic": measured_traffic(key),
                     "kernel": f"k_conv {precision} (3x3 dilated conv, C={C}; mean of the {n_conv} non-head launches)",
                     "avg_launch_ms": round(avg_s * 1e3, 3), "flop_per_launch": flop_launch,
                     "algorithmic_bytes_per_launch": round(bytes_launch)})
    return roofline, pt_bytes


RECALL_TARGET = 0.995
OFFSET_RMS_TARGET_PX = 0.01


def accuracy_target(acc):
    """The accuracy bar a form's speedup is judged at: recall >= 0.995 against
    the FP64 oracle's detections (one-to-one within 1 px) and RMS offset error
    <= 0.01 px, taken as the larger of the x and y RMS differences of the
    detections both put at the same pixel (the offset heads' own error; a
    maximum that moves to a neighbour pixel is a recall question)."""
    off = max(acc.get("same_pixel_rms_dx_px", math.inf), acc.get("same_pixel_rms_dy_px", math.inf))
    rec = acc.get("recall", 0.0)
    return {"recall": rec, "recall_min": RECALL_TARGET, "offset_rms_px": round(off, 6),
            "offset_rms_max_px": OFFSET_RMS_TARGET_PX,
            "offset_rms_used": "max(same_pixel_rms_dx_px, same_pixel_rms_dy_px)",
            "met": bool(rec >= RECALL_TARGET and off <= OFFSET_RMS_TARGET_PX)}


def accuracy_on_sample(recs, ref):
    """Emitters of frame 0 inside the oracle's exact region against the oracle's
    records there: one-to-one matching within 1 px (recall, precision, RMS
    coordinate errors of matched pairs) and the RMS coordinate errors of
    detections at the same pixel."""
    from tests.parity import match_by_distance
    lim = ref["limit"]
    got = recs[(recs["frame"] == 0) & (recs["row"] < lim) & (recs["col"] < lim)]
    rr = ref["records"]
    m = match_by_distance(got, rr, 1.0)
    # detections at the same pixel in both: the offset heads' error from the
    # form's arithmetic alone (a maximum that moved to a neighbour pixel
    # carries a whole-pixel change of the reconstructed position instead)
    gk = {(int(r), int(c)): i for i, (r, c) in enumerate(zip(got["row"], got["col"]))}
    pairs = [(gk[(int(r), int(c))], j) for j, (r, c) in enumerate(zip(rr["row"], rr["col"])) if (int(r), int(c)) in gk]
    if pairs:
        gi = np.array([p_[0] for p_ in pairs])
        ri = np.array([p_[1] for p_ in pairs])
        d = {k: np.asarray(got[kg], np.float64)[gi] - np.asarray(rr[kr], np.float64)[ri]
             for k, kg, kr in (("x", "x_px", "x"), ("y", "y_px", "y"), ("z", "z_nm", "z"))}
        m.update({"same_pixel_pairs": len(pairs),
                  "same_pixel_rms_dx_px": float(np.sqrt(np.mean(d["x"] ** 2))),
                  "same_pixel_rms_dy_px": float(np.sqrt(np.mean(d["y"] ** 2))),
                  "same_pixel_rms_dz_nm": float(np.sqrt(np.mean(d["z"] ** 2)))})
    return {k: (round(v, 6) if isinstance(v, float) else v) for k, v in m.items()}


def map_errors_on_sample(net, d_frames, ref, torch, dev):
    """The form's maps of frame 0 against the FP64 oracle's on the region where
    the oracle's maps are exact: max and RMS absolute logit error, RMS error of
    the dx, dy (px) and dz (units of the dz map) planes."""
    side = d_frames.shape[1]
    maps = torch.empty((1, net.head_outputs, side, d_frames.shape[2]), dtype=torch.float32, device=dev)
    net.maps_device(d_frames[:1], maps)
    torch.cuda.synchronize()
    e = ref["map_extent"]
    g = maps[0, :, :e, :e].cpu().numpy().astype(np.float64)
    d = g - ref["maps"]
    return {"max_logit_err": round(float(np.max(np.abs(d[0]))), 6),
            "rms_logit_err": round(float(np.sqrt(np.mean(d[0] ** 2))), 6),
            "rms_dx_map_err_px": round(float(np.sqrt(np.mean(d[1] ** 2))), 6),
            "rms_dy_map_err_px": round(float(np.sqrt(np.mean(d[2] ** 2))), 6),
            "rms_dz_map_err": round(float(np.sqrt(np.mean(d[3] ** 2))), 6),
            "map_region": f"{e}x{e}"}


CONV_SOURCES = ("kernels_conv.hip", "dloc_internal.h")
DENSE_SOURCES = ("kernels_dense.hip", "dloc_internal.h")


def conv_source_sha256(sources=CONV_SOURCES):
    """Hash of the sources that decide a conv kernel's memory traffic (the
    kernel and the tile order / layouts it includes)."""
    import hashlib
    h = hashlib.sha256()
    for name in sources:
        h.update(open(os.path.join(ROOT, "paper_2410_02314_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic(key, sources=CONV_SOURCES):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (scaled by a plain copy kernel), or None if
    there is no record for this kernel/workload or the kernel source changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path)).get(key)
        sha = conv_source_sha256(sources)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("kernel_source_sha256") != sha:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(args, spec, w, frames, net, dev, recs, cam=None):
    """FP64 oracle on a bounded sample: the top-left s x s crop of frame 0
    (1536^2 by default, about 20 s on 16 host threads).  Also checks the GPU maps and detections where the
    oracle's result is exact: all of a whole frame; in a smaller crop, the part
    at least R pixels from the crop's inner edges (and one more pixel for the
    detections, whose neighbours must be exact too)."""
    import torch
    import oracle
    import smlm_synth as S
    from tests.parity import exempt_mask, map_rel_err
    s = min(args.cpu_sample, args.size)
    crop = np.ascontiguousarray(frames[0, :s, :s])
    t0 = time.perf_counter()
    camera = {} if cam is None else {"gain": cam.gain[:s, :s], "offset": cam.offset[:s, :s]}
    rec, ref_maps = oracle.localize(crop[None], spec, w, return_maps=True, **camera)
    dt = time.perf_counter() - t0
    whole = s == args.size
    R = S.receptive_radius(spec)
    e = s if whole else s - R                 # exact maps on [0, e)^2
    lim = e if whole else e - 1               # exact detections on [0, lim)^2
    maps = torch.empty((1, net.head_outputs, args.size, args.size), dtype=torch.float32, device=dev)
    net.maps_device(torch.from_numpy(np.ascontiguousarray(frames[:1])).to(dev), maps)
    torch.cuda.synchronize()
    g = maps[0, :, :e, :e].cpu().numpy()
    err = map_rel_err(g, ref_maps[0, :, :e, :e])
    # the GPU's own emitter records against the oracle's detections there
    ref_det = oracle.detect(ref_maps[0, 0, :e, :e])[:lim, :lim]
    sel = (recs["frame"] == 0) & (recs["row"] < lim) & (recs["col"] < lim)
    got_det = np.zeros_like(ref_det)
    got_det[recs["row"][sel], recs["col"][sel]] = True
    ex = exempt_mask(ref_maps[0, 0, :e, :e])[:lim, :lim]
    mism = int(np.sum((ref_det != got_det) & ~ex))
    matched = int(np.sum(ref_det & got_det))
    rsel = (rec["row"] < lim) & (rec["col"] < lim)
    ref = {"records": rec[rsel], "limit": lim, "maps": ref_maps[0, :, :e, :e], "map_extent": e}
    what = "frame 0" if whole else f"frame 0 crop {s}x{s}"
    return {"value": round(s * s / dt / 1e6, 4), "unit": "Mpixel/s", "cores": cpu_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{what} of the same workload, FP64 oracle (net + detection + records), {dt:.1f} s",
            "sample_check": {"max_map_rel_err": float(err.max()), "oracle_detections": int(ref_det.sum()),
                             "gpu_detections": int(got_det.sum()), "matched": matched,
                             "recall_vs_oracle": matched / max(1, int(ref_det.sum())),
                             "non_exempt_detection_mismatch": mism, "exempt_pixels": int(ex.sum()),
                             "region": f"{lim}x{lim}"}}, ref


if __name__ == "__main__":
    main()
