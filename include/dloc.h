/*
 * dloc.h -- C ABI of the MI355X localization library (libdloc.so).
 *
 * The library turns raw uint16 SMLM camera frames into an emitter list on the
 * GPU: gain/offset preprocessing (scalar or per-pixel sCMOS maps), a residual
 * network of 3x3 dilated convolutions, a 1x1 head giving per-pixel detection
 * logit, sub-pixel offsets and photons (and, with 10 outputs, their
 * uncertainties and the background), then thresholding, 3x3 local-maximum
 * suppression and an ordered compaction into emitter records.
 *
 * Paper passages the calls follow (An Efficient Inference Frame for Single
 * Molecule Localization Microscopy):
 *   - Sec. 2.2: frames are loaded ahead of time into memory the network reads
 *     from fixed locations (preloading); post-processing is kept in GPU memory
 *     and only the post-processed coordinates leave the device.
 *   - Sec. 3.2: the network's output follows DECODE: per pixel a detection
 *     probability plus the emitter's offset relative to that pixel and the
 *     uncertainty of that position.
 *   - Sec. 3.2.1: feature extraction with dilated 3x3 convolutions whose
 *     dilation sets the receptive field.
 *   - Sec. 3.3: binary cross-entropy (used here to train the tile gate).
 *
 * Conventions
 *   - Every function returns DL_OK (0) or a negative dl_status; nothing throws
 *     or aborts across the ABI.  Arguments are validated on the host before any
 *     HIP call, so argument errors are reported even without a GPU.
 *   - After any error the handle stays usable; dl_last_error() describes it.
 *   - A handle is not thread-safe: use one handle per host thread.
 *   - "device" pointers are HIP device memory (for example torch CUDA tensors)
 *     on the handle's device; "host" pointers are ordinary host memory.
 *   - Work queued by the *_device calls runs on the caller's HIP stream
 *     (hipStream_t passed as void*, NULL = the null stream) and is not
 *     synchronised: results are valid once that stream has completed.
 *   - Frames are uint16 [n][h][w] row-major; maps are float [n][nh][h][w]
 *     (planes: logit, dx, dy, dz, photons; with nh = 10 then the raw
 *     uncertainties of x, y, z, photons and the background); emitter records
 *     are ordered by (frame, row, col).
 */
#ifndef DLOC_H
#define DLOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DL_ABI_VERSION 3u

typedef enum {
    DL_OK = 0,
    DL_ERR_INVALID_ARG = -1,   /* NULL/misaligned pointer, bad size, bad enum */
    DL_ERR_BAD_WEIGHTS = -2,   /* weights blob: bad magic/version/size/NaN    */
    DL_ERR_UNSUPPORTED = -3,   /* shape or precision this build does not run  */
    DL_ERR_OOM = -4,           /* allocation failed or workspace cap exceeded */
    DL_ERR_DEVICE = -5,        /* a HIP call failed; see dl_last_error        */
    DL_ERR_CAPACITY = -6       /* more emitters than the output capacity      */
} dl_status;

/* Arithmetic of the 3x3 block convolutions (preprocessing, stem, head,
 * sigmoid and detection are FP32 in every form):
 *   DL_FP32  FP32 weights, activations and accumulation (the exact form);
 *   DL_BF16  BF16 weights and stored activations (round to nearest even),
 *            FP32 accumulation, bias, residual and ReLU;
 *   DL_FP8   OCP e4m3 weights with one scale per output channel, and stored
 *            activations as e4m3 codes with one power-of-two scale per
 *            32-channel group of each pixel; FP32 accumulation, bias,
 *            residual and ReLU; the last block's output reaches the head
 *            unrounded;
 *   DL_BF16X3 split BF16: FP32 weights and stored activations, each product
 *            formed on the BF16 matrix cores from BF16 halves (v = hi + lo,
 *            hi = bf16(v), lo = bf16(v - hi)) as wh xh + wh xl + wl xh, FP32
 *            accumulation (about 16 significant bits per product).
 * None is part of the paper's method; they are the reduced-precision forms
 * measured against the FP32 path. */
typedef enum { DL_FP32 = 0, DL_BF16 = 1, DL_FP8 = 2, DL_BF16X3 = 3 } dl_precision;

/* flags */
#define DL_FLAG_GATE 1u        /* skip tiles the tile gate predicts empty */

typedef struct {
    int32_t precision;          /* dl_precision of the 3x3 block convolutions      */
    float threshold;            /* detection probability threshold, (0, 1); 0.3    */
    float gain;                 /* photons per ADU; 0.5                            */
    float offset;               /* camera offset in ADU; 100                       */
    int32_t device;             /* HIP device ordinal; 0                           */
    uint32_t flags;             /* DL_FLAG_*                                       */
    uint64_t max_workspace_bytes; /* device workspace cap, 0 = no cap             */
    int32_t tile_rows;          /* conv tile rows 4 or 8; 0 = the form's default   */
    float max_sigma_px;         /* 10-output nets: drop a detection whose sigma_x  */
                                /* or sigma_y exceeds this (px); 0 = keep all      */
    float in_scale_override;    /* > 0: network input units per photon in place of */
                                /* the weights' in_scale; 0 = the weights' value   */
    int32_t tile_w;             /* conv tile lattice columns; 0 = the form's own   */
                                /* (32 FP32/BF16X3, 64 BF16/FP8); other widths are */
                                /* DL_ERR_UNSUPPORTED                              */
    int32_t tile_queue;         /* dense-connection nets: how conv tiles reach the */
                                /* persistent workgroups -- 0 static ranges per    */
                                /* XCD, 1 an atomic queue per XCD, 2 one atomic    */
                                /* queue; residual nets: 0 only                    */
    int32_t reserved[3];        /* must be 0                                       */
} dl_config;

/* One detected emitter, 32 bytes.  x_px = col + 0.5 + dx, y_px = row + 0.5 + dy
 * (the frame spans [0, w) x [0, h) pixels, pixel centres at +0.5), z_nm = dz *
 * z_scale, photons = ph * ph_scale, prob = sigmoid(logit). */
typedef struct {
    int32_t frame, row, col;
    float x_px, y_px, z_nm, photons, prob;
} dl_emitter;

/* The least standard deviation the uncertainty planes express, in the units
 * of the head (px; z_scale; ph_scale): sigma = softplus(u) + DL_SIGMA_FLOOR.
 * The training loss's pixel mixture has no bounded likelihood without it (a
 * target dimension that never varies, such as z in 2D data, lets sigma go to
 * zero). */
#define DL_SIGMA_FLOOR 0.01f

/* Uncertainties of one emitter, 20 bytes, from a network with the 10-output
 * head (Sec. 3.2: each pixel also gives the uncertainty of the position).
 * With u the raw head value, softplus(u) = log(1 + e^u) > 0 and s(u) =
 * softplus(u) + DL_SIGMA_FLOOR:
 * sigma_x_px = s(u5), sigma_y_px = s(u6), sigma_z_nm = s(u7) * z_scale,
 * sigma_photons = s(u8) * ph_scale, background = softplus(u9) / in_scale
 * (photons per pixel). */
typedef struct {
    float sigma_x_px, sigma_y_px, sigma_z_nm, sigma_photons, background;
} dl_uncertainty;

/* One region of interest of an uneven batch (device data). */
typedef struct {
    const uint16_t *data;       /* device pointer to the ROI's first pixel */
    int32_t h, w;               /* 1 <= h, w                               */
    int64_t row_stride;         /* elements between rows, >= w             */
} dl_roi;

typedef struct dl_net dl_net;

/* Network description read from a weights blob (dl_inspect_weights). */
typedef struct {
    int32_t C, nblocks;
    int32_t dilation[8];
    float in_scale, z_scale, ph_scale;
    int32_t receptive_radius;   /* 1 + 2 * sum(dilation) (DLD1: 1 + L * sum(dilation)): halo a tile needs */
    int64_t nparams;            /* FP32 values after the header                  */
    int32_t head_outputs;       /* 5, or 10 with the uncertainty planes          */
    int16_t dense_layers;       /* DLD1: 3x3 layers per block; 0 for DLW1        */
    int16_t dense_growth;       /* DLD1: channels each layer adds; 0 for DLW1    */
    int32_t unet_levels;        /* DLD1: 2 with the two-stage U-Net, else 0      */
    int32_t reserved2_[3];
} dl_net_info;

/* Library ABI version (DL_ABI_VERSION). */
uint32_t dl_abi_version(void);

/* Fill *cfg with the defaults listed in dl_config.  cfg must not be NULL. */
int dl_default_config(dl_config *cfg);

/* Create a network from a little-endian "DLW1" weights blob:
 *   header (64 B): char magic[4] = "DLW1"; u32 version = 1; u32 C; u32 nblocks;
 *   u32 dilation[8]; f32 in_scale; f32 z_scale; f32 ph_scale; u32 nh (the head's
 *   outputs: 0 or 5 = logit, dx, dy, dz, photons; 10 = those, then the raw
 *   uncertainties of x, y, z and photons and the raw background);
 *   then FP32 tensors: stem.w [C][1][3][3], stem.b [C], for each block
 *   w1 [C][C][3][3], b1 [C], w2 [C][C][3][3], b2 [C]; head.w [nh][C], head.b [nh].
 * Network (Sec. 3.2, Sec. 3.2.1): x = (ADU - offset) * gain * in_scale;
 * a = ReLU(conv_1(x)); per block with dilation d: t = ReLU(conv_d(a)),
 * a = ReLU(a + conv_d(t)); maps = head(a).  Supported: C in {16, 32, 48, 64},
 * 1 <= nblocks <= 8, dilations 1..64.
 * Or from a "DLD1" blob, the dense-connection network (Sec. 3.2: within a
 * block every layer takes the outputs of all layers before it; Sec. 3.2.1 /
 * Sec. 4.1.2: one dilation per block):
 *   header (80 B): char magic[4] = "DLD1"; u32 version = 1; u32 C; u32 nblocks;
 *   u32 L (3x3 layers per block); u32 G (growth); u32 dilation[8]; f32 in_scale;
 *   f32 z_scale; f32 ph_scale; u32 nh (5 or 10); u32 U-Net levels (0 or 2);
 *   4 bytes ignored;
 *   then FP32 tensors: stem.w [C][1][3][3], stem.b [C]; for each block, for
 *   i = 0 .. L-1: w [G][C + i G][3][3], b [G]; then the transition w [C][C + L G],
 *   b [C]; with the U-Net: d1.w [C][C][3][3], d1.b [C], d2.w [C][C][3][3],
 *   d2.b [C], u1.w [C][2C][3][3], u1.b [C], u0.w [C][2C][3][3], u0.b [C];
 *   head.w [nh][C], head.b [nh].
 * Network: a = ReLU(conv_1(x)); per block with dilation d, cat = [a] and for
 * each layer cat = [cat, ReLU(conv_d(cat))], then a = ReLU(1x1(cat)).  The
 * two-stage U-Net (Sec. 3.2: fine-grained processing after the extractor):
 * d1 = ReLU(conv_1(pool(a))), d2 = ReLU(conv_1(pool(d1))) at levels 1 and 2,
 * u1 = ReLU(conv_1([d1, up(d2)])), a = ReLU(conv_1([a, up(u1)])), where pool
 * is a 2 x 2 max (level l + 1 is ceil(h/2) x ceil(w/2) of level l; an edge
 * window takes the pixels it has), up is nearest (up(v)[y][x] = v[y/2][x/2])
 * and [u, v] concatenates channels.  maps = head(a).  Supported: C and G in
 * {16, 32}, 1 <= L <= 8, 1 <= nblocks <= 8 (7 with the U-Net), dilations
 * 1..64; FP32 only; with the U-Net, no capacity ROI graph (other precisions, the tile gate, camera
 * maps, the autotuner and dl_debug_conv_layer are DL_ERR_UNSUPPORTED).
 * The blob is copied; the caller keeps ownership.  cfg may be NULL (defaults).
 * *out receives a handle the caller frees with dl_destroy_net.
 * Errors: DL_ERR_INVALID_ARG, DL_ERR_BAD_WEIGHTS, DL_ERR_UNSUPPORTED,
 * DL_ERR_OOM, DL_ERR_DEVICE. */
int dl_create_net(const void *weights, size_t nbytes, const dl_config *cfg, dl_net **out);

/* Validate a weights blob and describe it, on the host only (no HIP call).
 * Same checks and error codes as dl_create_net's blob validation. */
int dl_inspect_weights(const void *weights, size_t nbytes, dl_net_info *info);

/* Free every device and pinned allocation of the handle; NULL is a no-op. */
void dl_destroy_net(dl_net *net);

/* Text of the last error on this handle ("" if none); valid until the next
 * call on the handle.  With net == NULL: the last error of dl_create_net or of
 * a call that had no handle. */
const char *dl_last_error(const dl_net *net);

/* Change precision / threshold / gain / offset of an existing handle. */
int dl_set_config(dl_net *net, const dl_config *cfg);

/* Localize, device-resident (Sec. 2.2: frames already in GPU memory, only the
 * post-processed coordinates are produced).
 *   d_frames  device uint16 [n][h][w]
 *   d_out     device dl_emitter[cap]; records in (frame, row, col) order; only
 *             the first cap records are written
 *   d_counts  device uint32[n + 1]: emitters per frame, then the total
 * n, h and w must be >= 1: an empty batch or a zero-sized frame is
 * DL_ERR_INVALID_ARG, returned before anything is queued (this holds for every
 * entry point that takes n, h, w).  A frame larger than the kernels address is
 * DL_ERR_UNSUPPORTED, also before anything is queued: h * w <= 2^28, n * h <=
 * 2^30, and the frame's stored activations (C values per point, 4 / 2 / 1
 * bytes in FP32 / BF16 / FP8, both sides rounded up to the net's largest
 * phase layout, 16 for dilations up to 16) under 2 GiB.  For C = 48 and
 * dilations up to 16 the largest square frames are 3344 (FP32), 4720 (BF16)
 * and 6688 (FP8) pixels a side; larger images go in as ROIs or tiles.
 * Work is queued on `stream`.  Overflow (total > cap) is visible as
 * d_counts[n] > cap once the stream completes; the call itself returns DL_OK. */
int dl_localize_device(dl_net *net, const uint16_t *d_frames, int n, int h, int w,
                       void *stream, dl_emitter *d_out, size_t cap, uint32_t *d_counts);

/* dl_localize_device for a network with the 10-output head, also writing
 * each record's uncertainties: d_unc device dl_uncertainty[cap], entry i
 * belongs to d_out[i] (4-byte aligned; may be NULL only when cap is 0).
 * DL_ERR_UNSUPPORTED for a 5-output network. */
int dl_localize_device_unc(dl_net *net, const uint16_t *d_frames, int n, int h, int w,
                           void *stream, dl_emitter *d_out, dl_uncertainty *d_unc, size_t cap,
                           uint32_t *d_counts);

/* Allocation-free form of dl_localize_device, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and stream semantics as
 * dl_localize_device, and the same kernels; the activations, maps, masks and
 * row offsets live in one fixed device array of DL_NOALLOC_SCRATCH_BYTES per
 * device (set up by dl_create_net; held until the process ends) instead of
 * the handle's workspace, and the frame descriptors in a ring the handle
 * allocated at creation, so the call performs no allocation.  Limits
 * (DL_ERR_UNSUPPORTED, before anything is queued): n <= DL_NOALLOC_MAX_FRAMES
 * (more if an earlier call on the handle grew its ring), a batch whose
 * workspace exceeds the array (net A in FP32: about 150k pixels, e.g. 4 x
 * 128 x 128 frames fit; net B in FP32: about 100k pixels), and gated runs.
 * Nothing in the array needs to start at zero: every kernel writes what the
 * next one reads.  Every call on a device shares that device's array, from any
 * handle: calls whose work overlaps on one device (other streams, other host
 * threads) race and give wrong results; order them on one stream. */
#define DL_NOALLOC_SCRATCH_BYTES (64u << 20)
#define DL_NOALLOC_MAX_FRAMES 64
int dl_localize_device_noalloc(dl_net *net, const uint16_t *d_frames, int n, int h, int w,
                               void *stream, dl_emitter *d_out, size_t cap, uint32_t *d_counts);

/* Per-pixel maps of the network, device-resident (Sec. 3.2: the DECODE-style
 * output, per pixel a detection logit, the emitter's offset relative to the
 * pixel and, with 10 outputs, the uncertainties): d_maps float [n][nh][h][w]
 * with nh the head's outputs (5: logit, dx, dy, dz, photons before scaling;
 * 10: then the raw uncertainty and background planes), 4-byte aligned,
 * caller-owned.  Queued on `stream`; errors as dl_localize_device.  For parity
 * checks. */
int dl_maps_device(dl_net *net, const uint16_t *d_frames, int n, int h, int w,
                   void *stream, float *d_maps);

/* Per-pixel camera maps of an sCMOS sensor (host float [h][w] each, row-major,
 * copied into the handle): preprocessing becomes
 * x = (ADU - offset[y][x]) * gain[y][x] * in_scale in place of the config's
 * scalar gain and offset, in the stem and in the tile gate's pooling.  Every
 * frame of a uniform batch must then be h x w (else DL_ERR_INVALID_ARG); ROI
 * lists are refused with DL_ERR_UNSUPPORTED.  gain and offset both NULL
 * clears the maps (the scalars apply again).  gain must be finite and > 0,
 * offset finite.  Waits for all work on the device before it changes the
 * maps.  Graphs captured before the maps were set, cleared or given another
 * shape refuse to launch (DL_ERR_INVALID_ARG); new values of the same shape
 * are used by existing graphs. */
int dl_set_camera_maps(dl_net *net, const float *gain, const float *offset, int h, int w);

/* Localize host frames (synchronous).  The frames are copied host->device on
 * the handle's copy stream (from the caller's buffer directly when it is
 * pinned memory from dl_host_alloc, else through a pinned staging buffer),
 * processed on the compute stream, and the records copied back.
 *   frames  host uint16 [n][h][w]; out host dl_emitter[cap]; *count = total.
 * Returns DL_ERR_CAPACITY (after writing the first cap records) if the total
 * exceeds cap. */
int dl_localize(dl_net *net, const uint16_t *frames, int n, int h, int w,
                dl_emitter *out, size_t cap, size_t *count);

/* Pipelined host localization of `nbatch` consecutive batches of n frames
 * (frames host uint16 [nbatch][n][h][w]): batch k+1 is copied host->device on
 * a side stream while batch k is processed, and the records of batch k are
 * copied back while batch k+1 is processed (Sec. 2.2 preloading and
 * pipelining).  Records of all batches are concatenated in order, with
 * `frame` counted across batches.  overlap = 0 copies, processes and collects
 * each batch before the next starts (the serial workflow, for comparison).
 * The handle keeps two device frame slots of n*h*w*2 bytes, two record slots
 * of min(cap, n*h*w) records and, for unpinned frames, two pinned staging
 * slots; they grow to the largest call and are freed by dl_destroy_net.
 * Synchronous; returns DL_ERR_CAPACITY as dl_localize does. */
int dl_localize_pipelined(dl_net *net, const uint16_t *frames, int nbatch, int n, int h, int w,
                          int overlap, dl_emitter *out, size_t cap, size_t *count);

/* dl_localize and dl_localize_pipelined for a network with the 10-output head,
 * also writing each record's uncertainties to the host array unc[cap] (entry
 * i beside out[i]; may be NULL only when cap is 0).  The handle then also
 * keeps two device slots of min(cap, n*h*w) dl_uncertainty.  Errors as the
 * plain calls, plus DL_ERR_UNSUPPORTED for a 5-output network. */
int dl_localize_unc(dl_net *net, const uint16_t *frames, int n, int h, int w,
                    dl_emitter *out, dl_uncertainty *unc, size_t cap, size_t *count);
int dl_localize_pipelined_unc(dl_net *net, const uint16_t *frames, int nbatch, int n, int h, int w,
                              int overlap, dl_emitter *out, dl_uncertainty *unc, size_t cap, size_t *count);

/* dl_localize_rois_device for ROIs in host memory (Sec. 2.2: frames read from
 * fixed memory locations; only the post-processed coordinates come back):
 * each ROI's rows (h rows of w pixels, row_stride apart, host memory read
 * before the call returns) are copied into one device slot of the handle,
 * localized in one launch per layer on the handle's compute stream, and the
 * records copied into out[cap] (host).  *count = total emitters; the first
 * cap are written and DL_ERR_CAPACITY returned when the total exceeds cap.
 * Synchronous.  Errors otherwise as dl_localize_rois_device. */
int dl_localize_rois(dl_net *net, const dl_roi *rois, int nroi, dl_emitter *out, size_t cap, size_t *count);

/* The network's maps of host frames, into host memory: frames host uint16
 * [n][h][w] -> maps host float [n][nh][h][w] (as dl_maps_device).  The handle
 * keeps a device maps buffer, grown to the largest call.  Synchronous; errors
 * as dl_localize.  For parity checks. */
int dl_localize_maps(dl_net *net, const uint16_t *frames, int n, int h, int w, float *maps);

/* Uneven batch of ROIs (Sec. 4.2.1 and 4.2.2 run frames in batches; here the
 * frames of one batch may differ in shape): device data, the dl_roi array
 * itself host memory (read before the call returns).  All ROIs go through one
 * launch per layer.  Same outputs as dl_localize_device with n = nroi and
 * `frame` = the ROI's index; DL_ERR_INVALID_ARG for a NULL or misaligned ROI,
 * h or w < 1 or row_stride < w, DL_ERR_UNSUPPORTED for an ROI past the frame
 * limits of dl_localize_device or with camera maps set. */
int dl_localize_rois_device(dl_net *net, const dl_roi *rois, int nroi, void *stream,
                            dl_emitter *d_out, size_t cap, uint32_t *d_counts);

/* dl_localize_rois_device for a network with the 10-output head, with each
 * record's uncertainties in d_unc (as dl_localize_device_unc: device
 * dl_uncertainty[cap], entry i beside d_out[i], 4-byte aligned).  Errors as
 * dl_localize_rois_device, plus DL_ERR_UNSUPPORTED for a 5-output network. */
int dl_localize_rois_device_unc(dl_net *net, const dl_roi *rois, int nroi, void *stream,
                                dl_emitter *d_out, dl_uncertainty *d_unc, size_t cap, uint32_t *d_counts);

/* Maps of an uneven ROI batch: ROI k's maps [nh][h_k][w_k] start at
 * d_maps + nh * sum_{j<k} h_j * w_j. */
int dl_maps_rois_device(dl_net *net, const dl_roi *rois, int nroi, void *stream, float *d_maps);

/* ---- autotuning ----
 * (Not from the paper, which fixes no tiling: the conv tile shape is this
 * library's choice.)  Time the network (no post-processing) on the given batch for every
 * candidate convolution tile shape (lattice rows per workgroup: 8, then 4),
 * `reps` times each after one warm-up, with HIP events on `stream`; keep the
 * fastest on the handle (as cfg.tile_rows) and return it in *best_rows.
 * ms (may be NULL) receives the mean time per pass of each candidate.
 * Synchronous. */
#define DL_TUNE_CANDIDATES 2
int dl_autotune(dl_net *net, const uint16_t *d_frames, int n, int h, int w, void *stream, int reps,
                int32_t *best_rows, float *ms /*[DL_TUNE_CANDIDATES]*/);

/* ---- HIP graphs ----
 * Capture the whole localization of one fixed batch (frames at d_frames, or
 * the ROI list) into a HIP graph that owns its workspace and descriptors.
 * Refill the frame buffer in place and replay with dl_graph_launch: one
 * launch per batch instead of ~20 kernel launches (Sec. 2.2: the network reads
 * preloaded frames from fixed memory locations).  Outputs as for
 * dl_localize_device.  The graph holds the handle's weights, precision,
 * threshold, gain, offset and max_sigma_px at creation; after a change of
 * precision (the packed weights move) or of the camera maps' presence or
 * shape, dl_graph_launch refuses with DL_ERR_INVALID_ARG and the graph must
 * be created again.  Destroy graphs before their handle.  Not available with
 * the gate. */
typedef struct dl_graph dl_graph;
int dl_graph_create(dl_net *net, const uint16_t *d_frames, int n, int h, int w, dl_emitter *d_out, size_t cap,
                    uint32_t *d_counts, dl_graph **out);
int dl_graph_create_rois(dl_net *net, const dl_roi *rois, int nroi, dl_emitter *d_out, size_t cap,
                         uint32_t *d_counts, dl_graph **out);
int dl_graph_launch(dl_graph *g, void *stream);

/* A graph that localizes ANY uneven ROI batch within a capacity (Sec. 4.2.1
 * and 4.2.2 run fixed-size batches; here one capture serves every batch that
 * fits): at most max_rois ROIs, each at most max_h x max_w, at most max_pixels
 * pixels in all.  The graph owns a workspace sized for the capacity, a pinned
 * host slot for the ROI list, and device descriptor buffers; its first nodes
 * copy the slot to the device and build the frame descriptors there (prefix
 * sums over the ROIs), and every kernel reads the batch's frame count, rows
 * and tiles from device memory, so nothing is re-captured.  d_out / cap /
 * d_counts as dl_graph_create_rois, except that d_counts must hold
 * max_rois + 1 entries: a replay over n ROIs writes counts[0..n-1] and the
 * total at counts[n].  Gated handles and camera maps are refused
 * (DL_ERR_UNSUPPORTED); max_rois is at most DL_GRAPH_MAX_ROIS.
 * dl_graph_launch_rois: queue one replay on `stream` for the ROI list `rois`
 * (device data; the array is host memory, copied into the graph's slot
 * before the call returns).  It first waits (on the host) until the previous
 * replay has copied the slot.  ROIs past the capacity return DL_ERR_CAPACITY
 * before anything is queued; other errors as dl_localize_rois_device.
 * dl_graph_launch refuses such a graph, and dl_graph_launch_rois a fixed one. */
#define DL_GRAPH_MAX_ROIS 65536
int dl_graph_create_rois_dynamic(dl_net *net, int max_rois, int max_h, int max_w, int64_t max_pixels,
                                 dl_emitter *d_out, size_t cap, uint32_t *d_counts, dl_graph **out);
int dl_graph_launch_rois(dl_graph *g, const dl_roi *rois, int nroi, void *stream);
void dl_graph_destroy(dl_graph *g);

/* Pinned host memory for frames (Sec. 2.2 "specified memory locations"). */
int dl_host_alloc(size_t bytes, void **p);
void dl_host_free(void *p);

/* ---- tile-occupancy gate ----
 * A small learned classifier decides per 256 x 256 tile whether the network
 * needs to run there.  Per tile of preprocessed input x (DL_GATE_TILE pixels
 * square): p = 4x4 mean pooling (64 x 64); h1 = ReLU(conv3x3(p; 1 -> 8, pad 1));
 * h2 = ReLU(conv3x3(h1; 8 -> 8, pad 1)); m = max of h2 over pixels (its
 * gradient goes to the first maximising pixel in raster order);
 * g = fw . m + fb (logit).  theta[DL_GATE_NPARAM] holds W1[8][1][3][3], b1[8],
 * W2[8][8][3][3], b2[8], fw[8], fb in that order (FP32).  Training uses binary
 * cross-entropy on g (paper Sec. 3.3) and Adam.  All pointers are device
 * memory; work is queued on `stream`; these calls need no network handle. */
#define DL_GATE_TILE 256
#define DL_GATE_NPARAM 673

/* d_frames uint16 [n][h][w] (h, w multiples of 256) -> d_pooled float
 * [n * (h/256) * (w/256)][64][64], tiles frame-major then row-major. */
int dl_gate_pool(const uint16_t *d_frames, int n, int h, int w, float gain, float offset, float in_scale,
                 void *stream, float *d_pooled);
/* dl_gate_pool with the handle's own preprocessing: its config's gain and
 * offset and its weights' in_scale, or its camera maps when set (then the
 * frames must be sensor-sized) -- the tiles a gated run of this handle
 * pools, for training its gate.  Same layouts as dl_gate_pool; work is
 * queued on `stream`.  Errors: DL_ERR_INVALID_ARG (NULL pointers, frames not
 * the camera maps' shape), DL_ERR_UNSUPPORTED (h or w not a multiple of 256). */
int dl_gate_pool_net(dl_net *net, const uint16_t *d_frames, int n, int h, int w, void *stream, float *d_pooled);
/* d_logits[ntiles] = g of every pooled tile. */
int dl_gate_forward(const float *d_pooled, int ntiles, const float *d_theta, void *stream, float *d_logits);
/* Forward plus the gradient of sum_b d_dlogits[b] * g_b with respect to theta:
 * d_logits[ntiles], d_grad[DL_GATE_NPARAM].  d_work: float[ntiles * DL_GATE_NPARAM]
 * scratch (per-tile partial gradients, summed in tile order: deterministic). */
int dl_gate_backward(const float *d_pooled, int ntiles, const float *d_theta, const float *d_dlogits,
                     float *d_work, void *stream, float *d_logits, float *d_grad);
/* Mean binary cross-entropy of logits against labels in {0, 1}:
 * d_loss[1] (may be NULL) and d_dlogits[n] = (sigmoid(g) - y) / n (may be NULL). */
int dl_gate_bce(const float *d_logits, const float *d_labels, int n, void *stream, float *d_loss, float *d_dlogits);
/* One Adam step (step counts from 1) on n parameters, in place. */
int dl_gate_adam(float *d_theta, float *d_m, float *d_v, const float *d_grad, int n, int step, float lr, float b1,
                 float b2, float eps, void *stream);

/* Attach a trained gate to a network (theta host float[DL_GATE_NPARAM],
 * copied; NULL detaches).  With DL_FLAG_GATE set in the config, uniform
 * batches whose h and w are multiples of 256 run the gate first; a 256^2 tile
 * is kept iff sigmoid(g) > threshold.  Each convolution layer then computes
 * only the tiles within its remaining receptive radius of a kept tile, so
 * kept tiles get exactly the ungated maps.  Skipped tiles produce no
 * emitters, and their pixels do not count as neighbours in the local-maximum
 * test.  Other shapes return DL_ERR_UNSUPPORTED while the flag is set. */
int dl_set_gate(dl_net *net, const float *theta, float threshold);

/* Copy the keep flags (uint8, 1 = kept) of the handle's most recent run,
 * which must have been gated (a later run reuses the workspace they live in;
 * else DL_ERR_INVALID_ARG), frame-major then row-major over 256^2 tiles, to
 * device memory d_keep (cap bytes), queued on `stream`; *ntiles = number of
 * flags.  DL_ERR_CAPACITY if cap is too small. */
int dl_gate_keep_map(dl_net *net, void *stream, uint8_t *d_keep, size_t cap, size_t *ntiles);

/* Autotuner over the conv tiling, with a cache (the tiling is this library's
 * choice; the paper fixes none).  Starting from the form's default (8-row
 * tiles, tile order in column strips 8 regions wide) it times the network on
 * the caller's batch (`reps` passes after one warm-up, HIP events on
 * `stream`) for strip widths 4, 16 and 32, keeping one only when 1% faster,
 * then toggles each block's tile rows between 8 and 4 in turn under the same
 * rule, and applies the result to the handle (per-block rows; cfg.tile_rows
 * is reset to 0).  cache_path (may be NULL): a text file of JSON lines
 * {"key": ..., "rows": [...], "strip": s, "ms": t}; the key names the device
 * architecture, its CU count, the net (C, dilations, head outputs), the
 * precision and the batch shape.  A line with this key is applied without
 * timing (res->from_cache = 1); otherwise the result is appended.  res
 * receives the chosen rows and strip, the number of tilings timed and the
 * mean ms per pass of the default and of the chosen tiling.  Synchronous.
 * DL_ERR_INVALID_ARG if the cache cannot be appended to (the tuned tiling is
 * still applied). */
typedef struct {
    int32_t rows[8];         /* tile rows of each block's convolutions (4 or 8) */
    int32_t strip;           /* strip width of the tile order, in regions        */
    int32_t from_cache;      /* 1: taken from the cache, nothing timed           */
    int32_t configs_timed;
    float ms_default, ms_best;
} dl_tune_result;
int dl_autotune_ex(dl_net *net, const uint16_t *d_frames, int n, int h, int w, void *stream, int reps,
                   const char *cache_path, dl_tune_result *res);

/* ---- training (Sec. 3.3) ----
 * One true emitter of a training frame: position in pixels (the frame spans
 * [0, w) x [0, h), pixel (row, col) covers [col, col + 1) x [row, row + 1)),
 * axial position in nm and photon count. */
typedef struct {
    float x, y, z_nm, photons;
} dl_truth;

/* Loss and gradient of one batch at the handle's current weights, on the
 * device, queued on `stream`.  The network must have the 10-output head and
 * C = 16 or 32: a residual (DLW1) net, or a dense-connection (DLD1) net of
 * growth 16 with or without the two-stage U-Net (the max pooling's gradient
 * goes to each window's first maximum in raster order); FP32; scalar gain and
 * offset.
 *   d_frames     device uint16 [n][h][w]
 *   d_truth      device dl_truth[], the frames' true emitters, frame by frame,
 *                each inside its frame
 *   d_truth_off  device int32[n + 1]: frame f's emitters are
 *                d_truth[d_truth_off[f] .. d_truth_off[f + 1] - 1]; [0] = 0
 *   ntruth       d_truth_off[n] (the host's copy; sizes the launches)
 *   d_grad       device float[nparams]: the gradient in blob order (may be NULL)
 *   d_loss       device float[4]: batch means of the loss and of its three
 *                terms {total, cross-entropy, count, localisation}
 * Per frame of P pixels, with p = sigmoid(logit), y = 1 on pixels holding a
 * true emitter, mu = sum p, v = sum p (1 - p) + 1e-4, E emitters:
 *   cross-entropy  (1/P) sum [softplus(logit) - y logit]
 *   count          log(2 pi v) / 2 + (E - mu)^2 / (2 v)
 *   localisation   -sum_e log sum_k (p_k / mu) prod_d N(t_ed; m_kd, s_kd^2),
 *                  m_k = (col + 0.5 + dx, row + 0.5 + dy, dz, ph), s = softplus
 *                  of the raw uncertainty planes + DL_SIGMA_FLOOR, t_e = (x, y,
 *                  z_nm / z_scale, photons / ph_scale)
 * and the batch loss is the mean over frames.  A batch holds at most 2^26
 * pixels and a frame row at most 2^20 (DL_ERR_UNSUPPORTED beyond).  Training
 * buffers are the handle's (grown on demand).  Errors: DL_ERR_INVALID_ARG,
 * DL_ERR_UNSUPPORTED, DL_ERR_OOM, DL_ERR_DEVICE. */
int dl_train_grad(dl_net *net, const uint16_t *d_frames, int n, int h, int w, const dl_truth *d_truth,
                  const int32_t *d_truth_off, int ntruth, void *stream, float *d_grad, float *d_loss);

/* dl_train_grad, then one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, the
 * handle's own moments and step count) of learning rate lr on the handle's
 * weights; later localize calls use the updated weights. */
int dl_train_step(dl_net *net, const uint16_t *d_frames, int n, int h, int w, const dl_truth *d_truth,
                  const int32_t *d_truth_off, int ntruth, void *stream, float lr, float *d_loss);

/* The handle's current weights, flat in blob order (nparams floats), to the
 * host; waits for the device. */
int dl_get_params(dl_net *net, float *params, size_t count);

/* ---- stage timing ----
 * With profiling on, every kernel launch of the path is bracketed by two HIP
 * events recorded on the stream it runs on.  dl_profile_read waits for the
 * recorded events and returns, per stage, the summed elapsed milliseconds and
 * the number of launches since the previous read. */
enum {
    DL_STAGE_STEM = 0,       /* preprocessing + stem convolution              */
    DL_STAGE_CONV = 1,       /* 3x3 block convolutions without the head       */
                             /* (DLD1 networks: the dense layers)             */
    DL_STAGE_CONV_HEAD = 2,  /* last block convolution with the fused head    */
                             /* (DLD1: last layer + transition + head fused)  */
    DL_STAGE_DETECT = 3,     /* threshold + 3x3 local maximum, masks + counts */
    DL_STAGE_SCAN = 4,       /* row offsets and per-frame counts              */
    DL_STAGE_EMIT = 5,       /* ordered emitter records                       */
    DL_STAGE_GATE = 6,       /* tile gate inference and tile selection        */
    DL_STAGE_CONV_1X1 = 7,   /* DLD1: a block's last layer fused with its 1x1 */
                             /* transition (all blocks but the last)          */
    DL_STAGE_UNET = 8,       /* DLD1 U-Net: pooling, upsampling and its       */
                             /* convolutions but the last (which is CONV_HEAD)*/
    DL_NSTAGES = 10
};
int dl_profile_enable(dl_net *net, int on);
int dl_profile_read(dl_net *net, double *ms /*[DL_NSTAGES]*/, int64_t *launches /*[DL_NSTAGES]*/);

/* ---- debug / parity entry points (device pointers, queued on stream) ---- */

/* One 3x3 dilated convolution layer (Sec. 3.2.1) of an FP32 or BF16X3 handle on NHWC
 * FP32 tensors: d_in float [n][h][w][C] -> d_out float [n][h][w][C] (16-byte
 * aligned, caller-owned; d_res optional, same layout),
 * out = ReLU(conv_d(in; block `blk` conv `which` (0 or 1)) + (d_res ? res : 0)),
 * zero padding at the frame border.  DL_ERR_UNSUPPORTED unless the handle's
 * precision is DL_FP32 or DL_BF16X3 (the forms that store FP32 activations);
 * DL_ERR_INVALID_ARG for a bad blk / which. */
int dl_debug_conv_layer(dl_net *net, const float *d_in, const float *d_res, int n, int h, int w,
                        int blk, int which, void *stream, float *d_out);

/* Threshold + 3x3 local-maximum test (the post-processing Sec. 2.2 keeps on
 * the GPU) on a logit plane stack: d_logit float [n][h][w] (4-byte aligned)
 * -> d_det uint8 [n][h][w] (1 = detected; caller-owned).  tau is the logit
 * threshold (ln(p / (1 - p))), finite; ties between neighbours go to the
 * earlier pixel in raster order. */
int dl_debug_detect(dl_net *net, const float *d_logit, int n, int h, int w, float tau,
                    void *stream, uint8_t *d_det);

/* Compaction alone (Sec. 2.2 post-processing; Sec. 4.2.1: converting the
 * offsets to coordinates is part of the cost): detection flags d_det uint8
 * [n][h][w] (non-zero = detected) and maps d_maps float [n][nh][h][w] (nh =
 * the handle's head outputs) -> records d_out (16-byte aligned, cap entries)
 * in (frame, row, col) order and d_counts uint32 [n + 1] (per frame, then the
 * total), exactly as the last stages of dl_localize_device produce them
 * (uncertainties are not written).  Records past cap are dropped; the counts
 * still hold the totals. */
int dl_debug_compact(dl_net *net, const uint8_t *d_det, const float *d_maps, int n, int h, int w,
                     void *stream, dl_emitter *d_out, size_t cap, uint32_t *d_counts);

/* ---- measured ceilings ----
 * Sustained rates of the current device, quoted beside the published peaks
 * in rooflines.  what:
 *   DL_RATE_MFMA_FP32 / _BF16 / _FP8  dense MFMA rate in TFLOP/s: every SIMD
 *       runs register-resident chains of the MFMA each form's convolution
 *       uses (16x16x4 f32, 16x16x32 bf16, 16x16x128 scaled e4m3); `bytes`
 *       is ignored;
 *   DL_RATE_HBM_COPY  GB/s read plus written by the best of three
 *       device-to-device copies of `bytes` (a multiple of 16) each way: the
 *       runtime's copy, a grid-stride kernel and a chunked kernel.
 * *value = the best of `reps` timed launches (after one untimed launch).
 * Synchronous; allocates and frees its own buffers and stream.  Returns
 * DL_ERR_INVALID_ARG or DL_ERR_DEVICE; no handle records the text. */
enum { DL_RATE_MFMA_FP32 = 0, DL_RATE_MFMA_BF16 = 1, DL_RATE_MFMA_FP8 = 2, DL_RATE_HBM_COPY = 3 };
int dl_measure_rate(int what, size_t bytes, int reps, double *value);

#ifdef __cplusplus
}
#endif
#endif /* DLOC_H */
