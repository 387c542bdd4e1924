"""Secondary benchmark workloads of bench.py (``--workload``): the small
latency-bound batch, the uneven ROI batch, the gated sparse batch and the
host-to-device pipelined run.  Each prints one JSON line in bench.py's
format.  Timing: HIP events on the launch stream around K steps after W
warm-up steps; inputs resident in HBM unless the workload says otherwise."""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

from bench import METRIC, PEAKS, cpu_threads, log


def _timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _line(args, value, ms, config, extra):
    res = {"metric": METRIC, "value": round(value, 3), "unit": "Mpixel/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.precision, "data": "synthetic (seeded SMLM frames)",
           "config": config, **extra}
    print(json.dumps(res), flush=True)


def run_workload(args):
    import smlm_synth as S
    if args.workload == "tiny":
        return tiny(args, S)
    if args.workload == "rois":
        return rois(args, S)
    if args.workload == "sparse":
        return sparse(args, S)
    if args.workload == "pipeline":
        return pipeline(args, S)
    if args.workload == "train":
        return train(args, S)
    raise SystemExit(f"unknown workload {args.workload}")


def tiny(args, S):
    """4 x 128^2 frames, net A: eager launches and one HIP-graph replay per step."""
    frames = S.render_frames(4, 128, 128, "tiny", 1001)
    import torch
    import paper_2410_02314_amd as dl
    spec, w = S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w), precision=args.precision)
    dev = torch.device("cuda:0")
    d = torch.from_numpy(frames).to(dev)
    out = torch.empty((8192, 8), dtype=torch.int32, device=dev)
    counts = torch.zeros(5, dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream()
    # the autotuner times both conv tile shapes on this batch and keeps the faster
    rows, tune_ms = net.autotune(d, reps=50, stream=st) if not args.tile_rows else (args.tile_rows, {})
    steps = max(args.steps, 1000)               # latency-scale: a 1000-iteration replay
    ms_eager = _timed(lambda: net.localize_device(d, out, counts, st), steps, max(args.warmup, 20), st)
    g = net.graph(d, out, counts)
    ms_graph = _timed(lambda: g.launch(st), steps, max(args.warmup, 20), st)
    px = 4 * 128 * 128
    _line(args, px / (ms_graph * 1e-3) / 1e6, ms_graph,
          {"workload": "4 x 128x128 uint16 frames, 2D Gaussian PSF, net A (C=32, d=1,2,4)",
           "precision": args.precision, "frames": 4, "height": 128, "width": 128},
          {"eager_ms_per_step": round(ms_eager, 4), "graph_ms_per_step": round(ms_graph, 4),
           "conv_tile_rows": rows, "autotune_ms": {k: round(v, 4) for k, v in tune_ms.items()},
           "eager_mpx_s": round(px / (ms_eager * 1e-3) / 1e6, 3), "emitters_per_step": int(counts[4].item())})
    g.close()


def rois(args, S):
    """256 ROIs with sides from {128, ..., 1024}, net A (or, with --net D, the
    dense-connection net), one call per step (and a graph).  With net D the
    three tile schedules of its conv kernels are timed on the same ROIs:
    static ranges per XCD, an atomic queue per XCD, one global atomic queue."""
    rois_np = S.render_rois(256, "rois", 1004)
    import torch
    import paper_2410_02314_amd as dl
    dense = args.net == "D"
    spec, w = S.make_net("D", 3) if dense else S.make_net("A", 1)
    net = dl.Net(S.serialize_weights(spec, w), precision=args.precision, tile_rows=args.tile_rows)
    dev = torch.device("cuda:0")
    d = [torch.from_numpy(r).to(dev) for r in rois_np]
    px = sum(r.size for r in rois_np)
    cap = px // 32
    out = torch.empty((cap, 8), dtype=torch.int32, device=dev)
    counts = torch.zeros(257, dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream()
    # the autotuner (strip width, per-block tile rows) on a uniform batch of the
    # ROIs' typical size; its choice is used for everything below
    import tempfile
    tune = None
    if not args.tile_rows and not dense:
        probe = torch.from_numpy(S.render_frames(8, 512, 512, "rois", 1004)).to(dev)
        tune = net.autotune_ex(probe, reps=3, cache_path=os.path.join(tempfile.gettempdir(), "dloc_tune.jsonl"),
                               stream=st)
        del probe
        log(f"autotuner: {tune}")
    net.profile(True)
    ms = _timed(lambda: net.localize_rois_device(d, out, counts, st), args.steps, args.warmup, st)
    prof = net.profile_read()
    net.profile(False)
    schedules = None
    if dense:
        # the same ROIs under each tile schedule (results are identical; only
        # the order in which workgroups take tiles differs)
        ref = dl.emitters_from_device(out, int(counts[256].item()))
        schedules = {"static_xcd_ranges_ms": round(ms, 3)}
        for q, name in ((1, "atomic_queue_per_xcd_ms"), (2, "atomic_queue_global_ms")):
            nq = dl.Net(S.serialize_weights(spec, w), precision=args.precision, tile_queue=q)
            nq.profile(True)
            msq = _timed(lambda: nq.localize_rois_device(d, out, counts, st), args.steps, args.warmup, st)
            pq = nq.profile_read()
            nq.close()
            got = dl.emitters_from_device(out, int(counts[256].item()))
            schedules[name] = round(msq, 3)
            schedules[name.replace("_ms", "_conv_ms")] = round(pq["conv"][0] / max(1, pq["conv"][1]), 4)
            schedules[name.replace("_ms", "_same_records")] = bool(np.array_equal(got, ref))
            log(f"tile schedule {q}: {msq:.3f} ms/step (static {ms:.3f})")
        schedules["static_xcd_ranges_conv_ms"] = round(prof["conv"][0] / max(1, prof["conv"][1]), 4)
    g = net.graph_rois(d, out, counts)
    ms_graph = _timed(lambda: g.launch(st), args.steps, args.warmup, st)
    g.close()
    # one capacity graph serving any ROI batch that fits: replayed alternately
    # over this ROI set and a second, differently seeded one
    rois2_np = S.render_rois(256, "rois", 1005)
    d2 = [torch.from_numpy(r).to(dev) for r in rois2_np]
    px_cap = max(px, sum(r.size for r in rois2_np))
    gd = net.graph_rois_dynamic(256, 1024, 1024, px_cap, out, counts)
    sets = [d, d2]
    it = [0]

    def dyn_step():
        gd.launch_rois(sets[it[0] & 1], st)
        it[0] += 1

    ms_dyn = _timed(dyn_step, 2 * (args.steps // 2 + 1), args.warmup, st)
    gd.close()
    torch.cuda.synchronize()
    net.localize_rois_device(d, out, counts, st)          # counts of the headline ROI set again
    conv_ms, conv_n = prof["conv"]
    if dense:       # the unfused dense layers: mean over layers 0 .. L-2 of each block
        cins = [spec.C + i * spec.growth for i in range(spec.layers - 1)]
        flop = 2.0 * 9 * spec.growth * (sum(cins) / len(cins)) * px
    else:
        flop = 2.0 * 9 * spec.C * spec.C * px
    ach = flop / (conv_ms / conv_n * 1e-3) / 1e12
    # load balance: the same net on a uniform batch of about the same pixel
    # count (16 x 2048^2 frames of the same emitter model) in one launch per layer
    uni = S.render_frames(16, 2048, 2048, "rois", 1004, workers=args.gen_workers or None)
    d_uni = torch.from_numpy(uni).to(dev)
    u_out = torch.empty((uni.size // 32, 8), dtype=torch.int32, device=dev)
    u_counts = torch.zeros(17, dtype=torch.int32, device=dev)
    ms_uni = _timed(lambda: net.localize_device(d_uni, u_out, u_counts, st), args.steps, args.warmup, st)
    mpx, mpx_uni = px / (ms * 1e-3) / 1e6, uni.size / (ms_uni * 1e-3) / 1e6
    del d_uni, u_out
    _line(args, mpx, ms,
          {"workload": f"256 uneven ROIs (sides 128..1024), {px / 1e6:.1f} Mpx, net {'D' if dense else 'A'}",
           "precision": args.precision, "frames": 256, "pixels": px},
          {"graph_ms_per_step": round(ms_graph, 3),
           "capacity_graph_ms_per_step": round(ms_dyn, 3),
           "capacity_graph": "one capture (256 ROIs up to 1024 x 1024) replayed alternately over two ROI sets",
           "autotune": tune,
           "tile_schedules": schedules,
           "emitters_per_step": int(counts[256].item()),
           "uniform_16x2048sq_mpx_s": round(mpx_uni, 2), "load_balance_efficiency": round(mpx / mpx_uni, 4),
           "roofline": {"bound": "mfma", "achieved": round(ach, 2), "peak": PEAKS[args.precision],
                        "unit": "TFLOP/s", "frac": round(ach / PEAKS[args.precision], 4), "traffic": None}})


def sparse(args, S):
    """Tile gate on sparse frames: train the gate on separately seeded frames
    (labels = the ungated BF16 net's detections), then time gated vs ungated
    BF16 net B on 64 x 2048^2 frames and report skip, speedup and recall."""
    args.precision = "bf16"                          # the gated form runs the BF16 net
    n_eval, side = args.frames if args.frames != 16 else 64, args.size
    model = "sparse" if args.sparse_layout == "iid" else "sparse_cell"
    t0 = time.time()
    ev = S.render_frames(n_eval, side, side, model, 1005, workers=args.gen_workers or None)
    n_train = 313                                    # 313 frames x 64 tiles >= 20,000 tiles
    train_frames = [S.render_frames(16, side, side, model, 2005, frame_ids=range(k, min(k + 16, n_train)),
                                    workers=args.gen_workers or None) for k in range(0, n_train, 16)]
    log(f"generated frames in {time.time() - t0:.1f}s")
    import torch
    import paper_2410_02314_amd as dl
    from paper_2410_02314_amd import gate_train as GT
    dev = torch.device("cuda:0")
    spec, w = S.make_net("B", 2)
    blob = S.serialize_weights(spec, w)
    net = dl.Net(blob, precision="bf16")
    t0 = time.time()
    pooled, labels, counts = GT.labelled_tiles(net, iter(train_frames), dev, with_counts=True)
    pooled, labels, counts = pooled[:20000], labels[:20000], counts[:20000]
    theta0 = S.gate_flat(S.gate_init(3005))
    res = GT.train(pooled, labels, theta0, epochs=60, batch=256, lr=1e-2)
    # threshold: 99.9 % of the held-out tiles' detections kept (a margin over
    # the 99.5 % detection recall the gated form is judged by); the
    # 99.5 %-of-positive-tiles threshold and the fixed 0.05 are reported beside it
    thr = GT.threshold_at_recall(pooled, labels, res.theta, res.val_idx, 0.999, counts)
    thr_tile = GT.threshold_at_recall(pooled, labels, res.theta, res.val_idx, 0.995)
    # non-learned control at the same target: keep a tile when its brightest
    # pooled pixel exceeds a level chosen on the same held-out tiles
    vi = np.asarray(res.val_idx)
    peak = torch.clamp(pooled, min=0).amax(dim=(1, 2)).cpu().numpy()
    level = GT.threshold_for_recall(peak[vi], labels.cpu().numpy()[vi] > 0.5, 0.999, counts[vi])
    bright = np.zeros(S.gate_flat(S.gate_init(0)).size, np.float32)
    bright[4] = 1.0                                  # h1[0] = ReLU(p)
    bright[80 + 4] = 1.0                             # h2[0] = h1[0]
    bright[664] = 50.0                               # g = 50 (max h2[0] - level) + logit(0.05)
    bright[672] = -50.0 * level + math.log(0.05 / 0.95)
    log(f"gate trained in {time.time() - t0:.1f}s: {res.history[-1]}; threshold {thr:.4f}")
    d = torch.from_numpy(ev).to(dev)
    cap = n_eval * side * side // 64
    st = torch.cuda.current_stream()

    stages = {}

    def run(gate_theta, thr=0.05):
        g = dl.Net(blob, precision="bf16", flags=dl.DL_FLAG_GATE if gate_theta is not None else 0)
        if gate_theta is not None:
            g.set_gate(gate_theta, thr)
        out = torch.empty((cap, 8), dtype=torch.int32, device=dev)
        counts = torch.zeros(n_eval + 1, dtype=torch.int32, device=dev)
        ms = _timed(lambda: g.localize_device(d, out, counts, st), args.steps, args.warmup, st)
        g.profile(True)
        g.profile_read()
        g.localize_device(d, out, counts, st)
        torch.cuda.synchronize()
        stages.setdefault(gate_theta is not None, {k: round(v[0], 3) for k, v in g.profile_read().items() if v[1]})
        g.profile(False)
        rec = dl.emitters_from_device(out, min(int(counts[-1].item()), cap))
        keep = None
        if gate_theta is not None:
            k = torch.zeros(n_eval * (side // 256) ** 2, dtype=torch.uint8, device=dev)
            g.gate_keep_map(k)
            torch.cuda.synchronize()
            keep = k.cpu().numpy().astype(bool)
        return ms, rec, keep

    ms0, rec0, _ = run(None)
    ms1, rec1, keep = run(res.theta, thr)
    ms5, rec5, keep5 = run(res.theta, 0.05)
    msT, recT, keepT = run(res.theta, thr_tile)
    msB, recB, keepB = run(bright, 0.05)
    k0 = {(a, b, c) for a, b, c in zip(rec0["frame"], rec0["row"], rec0["col"])}
    k1 = {(a, b, c) for a, b, c in zip(rec1["frame"], rec1["row"], rec1["col"])}
    k5 = {(a, b, c) for a, b, c in zip(rec5["frame"], rec5["row"], rec5["col"])}
    kT = {(a, b, c) for a, b, c in zip(recT["frame"], recT["row"], recT["col"])}
    kB = {(a, b, c) for a, b, c in zip(recB["frame"], recB["row"], recB["col"])}
    px = n_eval * side * side
    _line(args, px / (ms1 * 1e-3) / 1e6, ms1,
          {"workload": f"{n_eval} x {side}x{side} sparse frames (30-70% empty 256^2 tiles, "
                       f"{'independent' if args.sparse_layout == 'iid' else 'around one compact occupied region'})"
                       f", gated BF16 net B",
           "precision": "bf16",
           "gate": f"2 conv x 8 ch + global max pool, threshold {thr:.4f} (99.9% of held-out detections kept)",
           "frames": n_eval},
          {"ungated_ms_per_step": round(ms0, 3), "ungated_mpx_s": round(px / (ms0 * 1e-3) / 1e6, 2),
           "speedup_vs_ungated": round(ms0 / ms1, 3), "skipped_tile_fraction": round(float(1 - keep.mean()), 4),
           "recall_vs_ungated": round(len(k0 & k1) / max(1, len(k0)), 5), "extra_border_detections": len(k1 - k0),
           "at_tile_recall_threshold": {"threshold": round(thr_tile, 4),
                                        "skipped_tile_fraction": round(float(1 - keepT.mean()), 4),
                                        "speedup_vs_ungated": round(ms0 / msT, 3),
                                        "recall_vs_ungated": round(len(k0 & kT) / max(1, len(k0)), 5)},
           "brightness_control": {"rule": f"brightest pooled pixel > {level:.4f} (level for 99.9% of held-out "
                                          "detections)",
                                  "skipped_tile_fraction": round(float(1 - keepB.mean()), 4),
                                  "speedup_vs_ungated": round(ms0 / msB, 3),
                                  "recall_vs_ungated": round(len(k0 & kB) / max(1, len(k0)), 5)},
           "at_threshold_0.05": {"skipped_tile_fraction": round(float(1 - keep5.mean()), 4),
                                 "speedup_vs_ungated": round(ms0 / ms5, 3),
                                 "recall_vs_ungated": round(len(k0 & k5) / max(1, len(k0)), 5)},
           "gate_val": res.history[-1],
           "stage_ms_gated": stages.get(True), "stage_ms_ungated": stages.get(False),
           "note": "stage times of one profiled step (gated: at the chosen threshold)"})


def pipeline(args, S):
    """Host frames: batches copied host->device on a side stream while the
    previous batch is processed, against the serial copy-then-compute order."""
    nb = 4
    cam = S.scmos_camera(args.size, args.size, 1002) if args.camera == "scmos" else None
    frames = S.render_frames(args.frames * nb, args.size, args.size, "full", 1002, workers=args.gen_workers or None,
                             camera=cam).reshape(nb, args.frames, args.size, args.size)
    import torch
    import paper_2410_02314_amd as dl
    spec, w = S.make_net("B", 2)
    net = dl.Net(S.serialize_weights(spec, w), precision=args.precision)
    if cam is not None:
        net.set_camera_maps(cam.gain, cam.offset)
    import ctypes
    pin = dl.host_alloc(frames.nbytes)               # pinned: copied to the GPU without staging
    buf = (ctypes.c_char * frames.nbytes).from_address(pin)
    arr = np.frombuffer(buf, dtype=np.uint16).reshape(frames.shape)
    arr[...] = frames
    out = {}
    for overlap in (1, 0):
        net.localize_pipelined(arr, overlap=bool(overlap))          # warm-up
        t0 = time.perf_counter()
        rec = net.localize_pipelined(arr, overlap=bool(overlap))
        out[overlap] = (time.perf_counter() - t0, len(rec))
    dl.host_free(pin)
    px = frames.size
    _line(args, px / out[1][0] / 1e6, out[1][0] * 1e3 / nb,
          {"workload": f"{nb} batches of {args.frames} x {args.size}^2 host frames (pinned), net B, "
                       f"H2D on a side stream overlapped with compute", "precision": args.precision,
           "camera": args.camera},
          {"serial_mpx_s": round(px / out[0][0] / 1e6, 2), "overlap_speedup": round(out[0][0] / out[1][0], 3),
           "emitters": out[1][1]})


def truth_records(truths):
    """Ground-truth emitters of a list of frames as records (frame, x, y, z)."""
    rows = [(f, t["x"], t["y"], t["z_nm"]) for f, ts in enumerate(truths) for t in ts]
    return np.array(rows, dtype=[("frame", "<i4"), ("x", "<f8"), ("y", "<f8"), ("z", "<f8")])


def train_eval(S, spec, w, steps=500, lr=1e-3, nb=16, npool=64, side=128):
    """What training does to localisation: the net from its initial weights is
    trained for ``steps`` Adam steps on a pool of ``npool`` synthetic frames
    (seed 3001, batches of ``nb`` in turn), and its emitter lists on 8
    held-out frames (seed 3002) are matched to their ground truth within 1 px,
    before and after."""
    import torch
    import paper_2410_02314_amd as dl
    from tests.parity import match_by_distance
    fr, tr = S.render_frames(npool, side, side, "tiny", 3001, with_truth=True)
    tr = [S.truth_array(t, side, side) for t in tr]
    ef, et = S.render_frames(8, side, side, "tiny", 3002, with_truth=True)
    ref = truth_records([S.truth_array(t, side, side) for t in et])
    net = dl.Net(S.serialize_weights(spec, w))
    dev = torch.device("cuda:0")
    batches = []
    for b in range(npool // nb):
        sl = slice(b * nb, (b + 1) * nb)
        off = np.zeros(nb + 1, np.int32)
        rows = []
        for f, t in enumerate(tr[sl]):
            off[f + 1] = off[f] + len(t)
            rows += [[r["x"], r["y"], r["z_nm"], r["photons"]] for r in t]
        batches.append((torch.from_numpy(fr[sl]).to(dev),
                        torch.from_numpy(np.asarray(rows, np.float32).reshape(-1, 4)).to(dev),
                        torch.from_numpy(off).to(dev)))

    def score():
        m = match_by_distance(net.localize(ef), ref, 1.0)
        return {"recall": round(m["recall"], 4), "precision": round(m["precision"], 4),
                "rms_xy_px": round(math.hypot(m["rms_dx_px"], m["rms_dy_px"]) / math.sqrt(2), 4)}
    before = score()
    loss = torch.zeros(4, dtype=torch.float32, device=dev)
    for s in range(steps):
        d, t, o = batches[s % len(batches)]
        net.train_step(d, t, o, lr, loss)
    after = score()
    return {"steps": steps, "lr": lr, "pool_frames": npool, "eval_frames": 8, "match_radius_px": 1.0,
            "true_emitters": len(ref), "loss_after": round(float(loss.cpu()[0]), 3), "before": before, "after": after}


def train(args, S):
    """Training steps on 16 frames of 128 x 128 with their true emitters: the
    10-output residual net (net AU: C = 32, d = 1, 2, 4), or with --net D the
    dense-connection network with the 10-output head (net DT); forward with
    kept activations, the loss, backward and Adam, all on the GPU."""
    import torch
    import paper_2410_02314_amd as dl
    n, side = 16, 128
    frames, truths = S.render_frames(n, side, side, "tiny", 1006, with_truth=True)
    truths = [S.truth_array(t, side, side) for t in truths]
    dense = args.net in ("D", "DU")
    spec, w = S.make_net("DUT" if args.net == "DU" else "DT", 3) if dense else S.make_net("AU", 1)
    net = dl.Net(S.serialize_weights(spec, w))
    dev = torch.device("cuda:0")
    d = torch.from_numpy(frames).to(dev)
    off = np.zeros(n + 1, np.int32)
    rows = []
    for f, t in enumerate(truths):
        off[f + 1] = off[f] + len(t)
        rows += [[r["x"], r["y"], r["z_nm"], r["photons"]] for r in t]
    tr = torch.from_numpy(np.asarray(rows, np.float32).reshape(-1, 4)).to(dev)
    toff = torch.from_numpy(off).to(dev)
    loss = torch.zeros(4, dtype=torch.float32, device=dev)
    st = torch.cuda.current_stream()
    first = float(net.train_step(d, tr, toff, 1e-3, loss, st).cpu()[0])
    ms = _timed(lambda: net.train_step(d, tr, toff, 1e-3, loss, st), args.steps, args.warmup, st)
    last = float(loss.cpu()[0])
    px = n * side * side
    C, nb = spec.C, len(spec.dilations)
    if dense:
        # per block: each layer's 3x3 conv and the 1x1 transition, each run
        # forward, transposed (input gradient) and as a weight gradient
        G, L = spec.growth, spec.layers
        per_px = sum(2 * 9 * G * (C + i * G) for i in range(L)) + 2 * C * (C + L * G)
        flop = 3.0 * per_px * px * nb
        name = "net DT (dense blocks at d=2,4,8,16, C=32, 4 layers of growth 16, 10-output head)"
        if spec.unet:
            # the U-Net's convolutions: u0 (2C -> C) at level 0, d1 (C -> C)
            # and u1 (2C -> C) at level 1, d2 (C -> C) at level 2
            h1, h2 = (side + 1) // 2, (side + 3) // 4
            lv = [n * side * side, n * h1 * h1, n * h2 * h2]
            flop += 3.0 * 2 * 9 * C * (2 * C * lv[0] + 3 * C * lv[1] + C * lv[2])
            name = "net DUT (net DT followed by the two-stage U-Net)"
    else:
        # per block two forward convolutions, two transposed ones and two
        # weight gradients, each 2 9 C^2 per pixel
        flop = 2.0 * 9 * C * C * px * 6 * nb
        name = "net AU (C=32, d=1,2,4, 10-output head)"
    tflops = flop / (ms * 1e-3) / 1e12
    _line(args, px / (ms * 1e-3) / 1e6, ms,
          {"workload": f"training steps, {n} x {side}x{side} frames with their true emitters, {name}, FP32, "
                       f"Adam lr 1e-3",
           "precision": "fp32", "frames": n, "height": side, "width": side},
          {"frames_per_s": round(n / (ms * 1e-3), 1), "emitters_per_batch": int(off[-1]),
           "loss_first_step": round(first, 4), "loss_after": round(last, 4), "steps_timed": args.steps,
           "conv_tflop_per_step": round(flop / 1e12, 4),
           "trained_eval": train_eval(S, spec, w, steps=args.train_eval_steps) if args.train_eval_steps > 0 else None,
           "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": PEAKS["fp32"], "unit": "TFLOP/s",
                        "frac": round(tflops / PEAKS["fp32"], 4), "traffic": None,
                        "kernel": "whole training step (convolution FLOP over the step time)"}})
