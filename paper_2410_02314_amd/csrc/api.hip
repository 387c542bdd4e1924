// C ABI of libdloc: argument validation, weights parsing, device workspace,
// streams, and the launch sequence of the localization path.
//
// Launch sequence for a batch (paper Sec. 2.2: everything after the copy of
// the preloaded frames stays on the GPU):
//   stem (preprocess + 3x3 conv 1->C) -> per block: conv_d, conv_d + residual
//   (last one with the 1x1 head fused, writing the 5 planar maps) ->
//   detect (threshold + 3x3 local max, 64-bit masks + per-row counts) ->
//   scan (row offsets, per-frame counts) -> emit (ordered records).
#include "dloc_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace dloc;

// Workspace of dl_localize_device_noalloc: a fixed array in device memory,
// one copy per device the library runs on, held until the process ends.  In
// host code `scratch` names a host-side stand-in, not the device address:
// host code only ever uses the address hipGetSymbolAddress returns for it on
// each device (scratch_ptr below).
static __device__ __align__(256) char scratch[DL_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int DESC_SLOTS = 8;
constexpr size_t ALIGN = 256;
constexpr int MAX_DEVICES = 64;

// device address of `scratch` on each device, looked up once per device
std::mutex g_scratch_mu;
char *g_scratch_ptr[MAX_DEVICES] = {};

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

thread_local std::string g_err;   // errors with no handle

size_t param_count(int C, int nb, int nh)
{
    return (size_t)C * 9 + C + (size_t)nb * 2 * ((size_t)C * C * 9 + C) + (size_t)nh * C + nh;
}

// dense-connection network: stem, per block L layers (G x (C + i G) x 3 x 3 + G)
// and a transition (C x (C + L G) + C), head
size_t dense_param_count(int C, int nb, int L, int G, int nh, int unet)
{
    size_t blk = 0;
    for (int i = 0; i < L; ++i) blk += (size_t)G * (C + i * G) * 9 + G;
    blk += (size_t)C * (C + L * G) + C;
    // the U-Net: two C -> C and two 2C -> C 3x3 convolutions
    const size_t un = unet ? 2 * ((size_t)C * C * 9 + C) + 2 * ((size_t)C * 2 * C * 9 + C) : 0;
    return (size_t)C * 9 + C + (size_t)nb * blk + un + (size_t)nh * C + nh;
}

}  // namespace

struct dl_net {
    dl_config cfg{};
    int dev = 0, ncu = 256;
    int C = 0, nb = 0;
    int nh = 5;                     // head outputs: 5, or 10 with the uncertainty planes
    int dil[8] = {0};
    float in_scale = 0.f, z_scale = 0.f, ph_scale = 0.f;
    std::vector<float> params;

    float *d_stem = nullptr;        // w [C][9] then b [C]
    float *d_head = nullptr;        // w [5][C] then b [5]
    float *d_bias = nullptr;        // [nb][2][C]
    void *d_wpk = nullptr;          // packed conv weights [nb][2][...]
    float *d_wscale = nullptr;      // FP8 per-output-channel weight scales [nb][2][C]
    int *d_dil = nullptr;           // dilations [nb]
    size_t wpk_stride = 0;
    int packed_precision = -1;
    uint64_t packed_gen = 0;        // counts repacks (graphs check it: they hold d_wpk)

    char *ws = nullptr;
    size_t ws_bytes = 0;
    char *scratch = nullptr;        // this device's `scratch` (dl_localize_device_noalloc)
    // Ordering of runs that share the workspace: ws_ev is recorded on the
    // stream of the last run that used it (ws_stream); a run on another
    // stream first waits for it on the device.
    hipEvent_t ws_ev = nullptr;
    hipStream_t ws_stream = nullptr;
    bool ws_used = false;

    FrameDesc *h_desc = nullptr;    // pinned, DESC_SLOTS * desc_cap
    FrameDesc *d_desc = nullptr;    // device, DESC_SLOTS * desc_cap
    int desc_cap = 0;
    hipEvent_t desc_ev[DESC_SLOTS] = {};
    int desc_next = 0;

    hipStream_t copy_stream = nullptr, compute_stream = nullptr;
    std::string err;

    // tile gate
    float *d_gate_theta = nullptr;  // [673]
    float gate_tau = 0.f;           // keep a tile iff its logit > gate_tau
    bool gate_set = false;
    int *d_radius = nullptr;        // [1 + 2 nb]: stem radius, then per conv layer
    int64_t last_gate_tiles = 0;
    size_t last_keep_off = 0;

    // per-stage timing with HIP events recorded on the launch stream
    bool profiling = false;
    struct Ev { int stage; hipEvent_t a, b; };
    std::vector<Ev> prof_pending;
    std::vector<hipEvent_t> ev_pool;

    // host-frame pipeline (dl_localize, dl_localize_pipelined): two slots of
    // frames, pinned staging, records and counts; grow-only, freed with the net
    uint16_t *pl_frames[2] = {};
    uint16_t *pl_stage[2] = {};
    dl_emitter *pl_out[2] = {};
    dl_uncertainty *pl_unc[2] = {};   // record uncertainties (10-output nets, on demand)
    uint32_t *pl_dcounts = nullptr;   // device [2][n + 1]
    uint32_t *pl_hcounts = nullptr;   // pinned [2][n + 1]
    float *pl_maps = nullptr;         // device maps of dl_localize_maps (grow-only)
    size_t pl_maps_bytes = 0;
    size_t pl_frame_bytes = 0, pl_stage_bytes = 0, pl_out_cap = 0, pl_unc_cap = 0;
    int pl_counts_n = 0;
    hipEvent_t pl_copied[2] = {}, pl_used[2] = {}, pl_counted[2] = {};

    // per-pixel camera maps (sCMOS): {offset, gain * in_scale} per pixel of
    // a cam_h x cam_w sensor; null = the scalar gain and offset of the config.
    // cam_gen counts every change of shape or presence (graphs check it).
    float2 *d_cam = nullptr;
    int cam_h = 0, cam_w = 0;
    uint64_t cam_gen = 0;

    // conv tiling chosen by the autotuner: tile rows per block (0 = the form's
    // default) and the strip width of the tile order (0 = 8); cfg.tile_rows,
    // when set, overrides the rows of every block
    int tune_rows[MAXBLK] = {0};
    uint32_t tune_strip = 0;

    // dense-connection networks (DLD1 blobs): layers per block and growth
    // (0 for the residual network), the packed weights and biases of every
    // conv in run order ([block][layer 0 .. L-1, transition]) at float
    // offsets dense_w / dense_b of d_dense, then the head's (rows padded to 16)
    int dL = 0, dG = 0;
    int unet = 0;                   // U-Net levels after the dense blocks: 0 or 2

    // training (dl_train_*): the weights being trained (blob order), their
    // gradient and Adam moments, the packed forward and transposed conv
    // weights, and the batch buffers (grow-only); t_dirty: the trained
    // weights have not been handed to the inference path yet
    float *t_params = nullptr, *t_grad = nullptr, *t_m = nullptr, *t_v = nullptr, *t_pack = nullptr;
    PackJob *t_jobs = nullptr;      // dense networks: the weight packs' job table (device)
    int t_njobs = 0;
    int64_t t_jobs_total = 0;
    char *t_ws = nullptr;
    size_t t_ws_bytes = 0;
    int t_step = 0;
    bool t_dirty = false;
    float *d_dense = nullptr;
    std::vector<size_t> dense_w, dense_b;
    size_t dense_head_w = 0;
};

namespace {

// the input scaling in use: the config's override when set, else the blob's
float in_scale_of(const dl_net *net)
{
    return net->cfg.in_scale_override > 0.f ? net->cfg.in_scale_override : net->in_scale;
}

int fail(dl_net *net, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (net) net->err = buf; else g_err = buf;
    return code;
}

#define HIPCHK(net, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((net), DL_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool finite_all(const float *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int check_config(dl_net *net, const dl_config *c)
{
    if (c->precision < DL_FP32 || c->precision > DL_BF16X3)
        return fail(net, DL_ERR_INVALID_ARG, "precision %d is not one of DL_FP32/DL_BF16/DL_FP8/DL_BF16X3",
                    c->precision);
    if (!(c->threshold > 0.f && c->threshold < 1.f))
        return fail(net, DL_ERR_INVALID_ARG, "threshold must lie in (0, 1)");
    if (!std::isfinite(c->gain) || !(c->gain > 0.f))
        return fail(net, DL_ERR_INVALID_ARG, "gain must be finite and > 0");
    if (!std::isfinite(c->offset)) return fail(net, DL_ERR_INVALID_ARG, "offset must be finite");
    if (!std::isfinite(c->max_sigma_px) || c->max_sigma_px < 0.f)
        return fail(net, DL_ERR_INVALID_ARG, "max_sigma_px must be finite and >= 0");
    if (c->device < 0) return fail(net, DL_ERR_INVALID_ARG, "device must be >= 0");
    if (!(c->tile_rows == 0 || c->tile_rows == 4 || c->tile_rows == 8))
        return fail(net, DL_ERR_INVALID_ARG, "tile_rows must be 0, 4 or 8");
    if (c->flags & ~DL_FLAG_GATE) return fail(net, DL_ERR_INVALID_ARG, "unknown flag bits");
    if (!std::isfinite(c->in_scale_override) || c->in_scale_override < 0.f)
        return fail(net, DL_ERR_INVALID_ARG, "in_scale_override must be finite and >= 0 (0 = the weights' in_scale)");
    if (c->tile_w < 0) return fail(net, DL_ERR_INVALID_ARG, "tile_w must be >= 0");
    if (c->tile_w) {
        int tr = 0, tc = 0;
        conv_tile_shape(48, c->precision, 0, &tr, &tc);
        if (c->tile_w != tc)
            return fail(net, DL_ERR_UNSUPPORTED, "tile_w %d: this form's conv kernel is built for %d lattice columns",
                        c->tile_w, tc);
    }
    if (c->tile_queue < 0 || c->tile_queue > 2) return fail(net, DL_ERR_INVALID_ARG, "tile_queue must be 0, 1 or 2");
    for (int k = 0; k < 3; ++k)
        if (c->reserved[k]) return fail(net, DL_ERR_INVALID_ARG, "reserved config fields must be 0");
    return DL_OK;
}

// What the dense-connection kernels support of a config: FP32, their fixed
// tile, no tile gate.
int check_dense_config(dl_net *net, const dl_config *c)
{
    if (c->precision != DL_FP32)
        return fail(net, DL_ERR_UNSUPPORTED, "the dense-connection network runs in FP32 only");
    if (c->tile_rows || c->tile_w)
        return fail(net, DL_ERR_UNSUPPORTED, "the dense-connection kernels have a fixed tile: tile_rows and tile_w must be 0");
    if (c->flags & DL_FLAG_GATE)
        return fail(net, DL_ERR_UNSUPPORTED, "the tile gate does not run with the dense-connection network");
    return DL_OK;
}

int tile_rows_of(const dl_net *net) { return net->cfg.tile_rows ? net->cfg.tile_rows : 0; }

// The conv tiling of a batch: the form's tile (its default rows in g.tr), each
// block's rows (config override, else the autotuner's choice, else the
// default) and the strip width of the tile order.
void set_tiling(const dl_net *net, Geometry &g)
{
    if (net->dL) {                      // the dense kernels' fixed tile
        g.tr = dense_tile_rows();
        g.tc = dense_tile_cols();
        for (int b = 0; b < MAXBLK; ++b) g.trb[b] = g.tr;
        g.strip = 8;
        return;
    }
    conv_tile_shape(net->C, net->cfg.precision, tile_rows_of(net), &g.tr, &g.tc);
    for (int b = 0; b < MAXBLK; ++b) {
        const int rows = net->cfg.tile_rows ? net->cfg.tile_rows : b < net->nb ? net->tune_rows[b] : 0;
        int tc = 0;
        conv_tile_shape(net->C, net->cfg.precision, rows, &g.trb[b], &tc);
    }
    g.strip = net->tune_strip ? net->tune_strip : 8;
}

// Activation layout of block b's layers (input, intermediate and residual):
// the phase layout of its dilation when that is a power of two, plain NHWC
// for the first block (the stem writes plain rows) and other dilations.
int block_layout(const dl_net *net, int b)
{
    if (net->dL) return 1;              // dense networks: plain NHWC throughout
    const int d = net->dil[b];
    return b > 0 && d > 1 && (d & (d - 1)) == 0 ? d : 1;
}

// activation points one frame needs: the largest layout the net uses
int64_t frame_act_points(const dl_net *net, int h, int w)
{
    int64_t m = act_points(h, w, 1);
    for (int b = 0; b < net->nb; ++b) m = std::max(m, act_points(h, w, block_layout(net, b)));
    return m;
}

// the conv kernels address a frame's activations with 32-bit byte offsets
bool frame_act_fits(const dl_net *net, int h, int w)
{
    if (net->dL) return true;           // the dense kernels address with 64-bit offsets
    // FP32 4, BF16 2, FP8 1 byte per value (FP8 scales: 2 bytes per point, also within range)
    const int pr = net->cfg.precision;
    const int64_t esz = pr == DL_FP32 || pr == DL_BF16X3 ? 4 : pr == DL_BF16 ? 2 : 1;
    return frame_act_points(net, h, w) * net->C * esz < ((int64_t)1 << 31);
}

// Build the frame descriptors of a uniform batch or a ROI list.
void build_geometry(const dl_net *net, int n, const int *hs, const int *ws_, const uint16_t *const *data,
                    const int64_t *strides, std::vector<FrameDesc> &fd, Geometry &g)
{
    fd.resize(n);
    g = Geometry{};
    g.nf = n;
    set_tiling(net, g);
    g.minor_blk = net->nb - 1;        // its head writes plain planar maps
    for (int f = 0; f < n; ++f) {
        FrameDesc &d = fd[f];
        std::memset(&d, 0, sizeof d);
        d.data = data[f];
        d.stride = strides[f];
        d.h = hs[f];
        d.w = ws_[f];
        d.px_off = g.total_px;
        d.act_off = g.total_act;
        d.row_start = g.total_rows;
        d.mask_start = g.total_words;
        d.words = (d.w + 63) / 64;
        d.gtx = d.w / GATE_TILE;
        d.gty = d.h / GATE_TILE;
        d.keep_start = g.gate_tiles;
        for (int b = 0; b < net->nb; ++b) {
            d.tile_start[b] = g.tiles[b];
            const int64_t nt = conv_tiles(d.h, d.w, net->dil[b], g.trb[b], g.tc);
            g.tiles[b] += nt;
            g.max_frame_tiles = std::max(g.max_frame_tiles, nt);
        }
        g.gate_tiles += (int64_t)d.gtx * d.gty;
        g.total_px += (int64_t)d.h * d.w;
        g.total_act += frame_act_points(net, d.h, d.w);
        g.total_rows += d.h;
        g.total_words += (int64_t)d.h * d.words;
        if (d.w > g.maxw) g.maxw = d.w;
        if (d.h > g.maxh) g.maxh = d.h;
    }
    for (int b = 0; b < net->nb; ++b) g.max_tiles = std::max(g.max_tiles, g.tiles[b]);
    if (net->unet) {
        // the U-Net's last convolution (level 0, d = 1) in tile slot nblocks;
        // levels 1 and 2 get descriptors of their own after the n frames'
        const int nb = net->nb;
        for (int f = 0; f < n; ++f) {
            fd[f].tile_start[nb] = g.tiles[nb];
            g.tiles[nb] += conv_tiles(fd[f].h, fd[f].w, 1, g.trb[nb], g.tc);
        }
        g.lv_pts[0] = g.total_act;
        g.lv_tiles[0] = g.tiles[nb];
        fd.resize((size_t)3 * n);
        for (int l = 1; l <= 2; ++l)
            for (int f = 0; f < n; ++f) {
                const FrameDesc &up = fd[(size_t)(l - 1) * n + f];
                FrameDesc &d = fd[(size_t)l * n + f];
                std::memset(&d, 0, sizeof d);
                d.h = (up.h + 1) / 2;
                d.w = (up.w + 1) / 2;
                d.act_off = g.lv_pts[l];
                d.tile_start[0] = g.lv_tiles[l];
                g.lv_pts[l] += (int64_t)d.h * d.w;
                g.lv_tiles[l] += conv_tiles(d.h, d.w, 1, g.tr, g.tc);
            }
        for (int l = 0; l <= 2; ++l) g.max_tiles = std::max(g.max_tiles, g.lv_tiles[l]);
    }
}

// frame descriptors per frame: the U-Net's levels 1 and 2 have their own
int desc_per_frame(const dl_net *net) { return net->unet ? 3 : 1; }

struct Plan {
    char *ws = nullptr;             // workspace base the offsets refer to
    // activations: act0 / act2 alternate as block input and output, act1
    // holds the intermediate of a block (a block writes its output in the next
    // block's layout, so it cannot overwrite its own input in place)
    size_t act0 = 0, act1 = 0, act2 = 0, maps = 0, mask = 0, rc = 0, roff = 0, total = 0;
    size_t queue = 0;               // dense tile queues: 8 counters per conv launch (tile_queue != 0)
    size_t unet = 0;                // U-Net levels 1 and 2: 96 floats per level-1 point, 64 per level-2 point
    bool gated = false;
    size_t pooled = 0, glog = 0, keep = 0, lists = 0, lcount = 0;
};

bool gated_run(const dl_net *net) { return (net->cfg.flags & DL_FLAG_GATE) && net->gate_set; }

Plan make_plan(const dl_net *net, const Geometry &g, bool ext_maps)
{
    // bytes per activation point: FP32 / BF16 values, or FP8 codes plus two
    // group scale bytes (the scales follow all codes of the buffer)
    // (dense networks: FP32 concatenations of C + L G channels, two buffers)
    const int prec = net->cfg.precision;
    const size_t pt_bytes = net->dL                               ? 4 * (size_t)(net->C + net->dL * net->dG)
                            : prec == DL_FP32 || prec == DL_BF16X3 ? 4 * (size_t)net->C
                            : prec == DL_BF16                     ? 2 * (size_t)net->C
                                                                  : net->C + 2;
    Plan p;
    size_t o = 0;
    p.act0 = o; o = align_up(o + (size_t)g.total_act * pt_bytes);
    p.act1 = o; if (!net->dL) o = align_up(o + (size_t)g.total_act * pt_bytes);
    p.act2 = o; o = align_up(o + (size_t)g.total_act * pt_bytes);
    p.maps = o; if (!ext_maps) o = align_up(o + (size_t)g.total_px * net->nh * 4);
    p.mask = o; o = align_up(o + (size_t)g.total_words * 8);
    p.rc = o; o = align_up(o + (size_t)g.total_rows * 4);
    p.roff = o; o = align_up(o + (size_t)(g.total_rows + 1) * 4);
    if (net->dL && net->cfg.tile_queue) {
        p.queue = o; o = align_up(o + (size_t)net->nb * net->dL * 8 * 4);
    }
    if (net->unet) {
        p.unet = o; o = align_up(o + ((size_t)96 * g.lv_pts[1] + (size_t)64 * g.lv_pts[2]) * 4);
    }
    if (gated_run(net)) {
        const int L = 2 * net->nb;
        p.gated = true;
        p.pooled = o; o = align_up(o + (size_t)g.gate_tiles * 4096 * 4);
        p.glog = o; o = align_up(o + (size_t)g.gate_tiles * 4);
        p.keep = o; o = align_up(o + (size_t)g.gate_tiles);
        p.lists = o; o = align_up(o + (size_t)L * g.max_tiles * 4);
        p.lcount = o; o = align_up(o + (size_t)L * 4);
    }
    p.total = o;
    return p;
}

// Release a library buffer and clear its pointer whatever the release
// returns: an error here (a call may report an earlier asynchronous failure)
// must never leave a pointer that a later release would free again.
template <class T>
hipError_t free_dev(T *&p)
{
    const hipError_t e = p ? hipFree(p) : hipSuccess;
    p = nullptr;
    return e;
}
template <class T>
hipError_t free_host(T *&p)
{
    const hipError_t e = p ? hipHostFree(p) : hipSuccess;
    p = nullptr;
    return e;
}

// A run on stream s that uses the handle's workspace is ordered after the
// previous such run: when that one was queued on another stream, s waits
// for it on the device (no host synchronisation).  Skipped while s is being
// captured into a graph, where an event recorded outside the capture cannot
// be waited on.
int ws_acquire(dl_net *net, hipStream_t s)
{
    if (!net->ws_used || net->ws_stream == s) return DL_OK;
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    HIPCHK(net, hipStreamIsCapturing(s, &cst));
    if (cst != hipStreamCaptureStatusNone) return DL_OK;
    HIPCHK(net, hipStreamWaitEvent(s, net->ws_ev, 0));
    return DL_OK;
}

int ws_release(dl_net *net, hipStream_t s)
{
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    HIPCHK(net, hipStreamIsCapturing(s, &cst));
    if (cst != hipStreamCaptureStatusNone) return DL_OK;
    HIPCHK(net, hipEventRecord(net->ws_ev, s));
    net->ws_stream = s;
    net->ws_used = true;
    return DL_OK;
}

int ensure_workspace(dl_net *net, size_t bytes, hipStream_t s)
{
    if (bytes <= net->ws_bytes) return DL_OK;
    if (net->cfg.max_workspace_bytes && bytes > net->cfg.max_workspace_bytes)
        return fail(net, DL_ERR_OOM, "workspace of %zu bytes exceeds max_workspace_bytes %llu", bytes,
                    (unsigned long long)net->cfg.max_workspace_bytes);
    if (net->ws) {
        HIPCHK(net, hipStreamSynchronize(s));
        HIPCHK(net, hipDeviceSynchronize());
        const hipError_t e = free_dev(net->ws);
        net->ws_bytes = 0;
        net->last_gate_tiles = 0;           // the keep map lived in the old workspace
        HIPCHK(net, e);
    }
    hipError_t e = hipMalloc(&net->ws, bytes);
    if (e != hipSuccess) {
        net->ws = nullptr;
        (void)hipGetLastError();
        return fail(net, DL_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    net->ws_bytes = bytes;
    return DL_OK;
}

// Grow the descriptor ring (pinned host + device, DESC_SLOTS slots) to hold
// batches of n frames; waits for the slots' last uploads first.
int grow_desc(dl_net *net, int n)
{
    if (n <= net->desc_cap) return DL_OK;
    for (int i = 0; i < DESC_SLOTS; ++i)
        if (net->desc_ev[i]) HIPCHK(net, hipEventSynchronize(net->desc_ev[i]));
    const hipError_t eh = free_host(net->h_desc), ed = free_dev(net->d_desc);
    net->desc_cap = 0;
    HIPCHK(net, eh);
    HIPCHK(net, ed);
    int cap = DL_NOALLOC_MAX_FRAMES;
    while (cap < n) cap *= 2;
    HIPCHK(net, hipHostMalloc((void **)&net->h_desc, sizeof(FrameDesc) * cap * DESC_SLOTS, hipHostMallocDefault));
    HIPCHK(net, hipMalloc((void **)&net->d_desc, sizeof(FrameDesc) * cap * DESC_SLOTS));
    net->desc_cap = cap;
    return DL_OK;
}

// Upload descriptors into the next ring slot; returns the device pointer.
int upload_desc(dl_net *net, const std::vector<FrameDesc> &fd, hipStream_t s, FrameDesc **out)
{
    const int n = (int)fd.size();
    int rc;
    if ((rc = grow_desc(net, n))) return rc;
    const int slot = net->desc_next;
    net->desc_next = (slot + 1) % DESC_SLOTS;
    HIPCHK(net, hipEventSynchronize(net->desc_ev[slot]));
    FrameDesc *h = net->h_desc + (size_t)slot * net->desc_cap;
    FrameDesc *d = net->d_desc + (size_t)slot * net->desc_cap;
    std::memcpy(h, fd.data(), sizeof(FrameDesc) * n);
    HIPCHK(net, hipMemcpyAsync(d, h, sizeof(FrameDesc) * n, hipMemcpyHostToDevice, s));
    *out = d;
    return slot;
}

// stem, head and (residual nets) conv biases from net->params to the device
int upload_small_weights(dl_net *net)
{
    const int C = net->C, nb = net->nb;
    const float *p = net->params.data();
    const size_t nstem = (size_t)C * 9 + C, nhead = (size_t)net->nh * C + net->nh;
    HIPCHK(net, hipMemcpy(net->d_stem, p, nstem * 4, hipMemcpyHostToDevice));
    HIPCHK(net, hipMemcpy(net->d_head, p + net->params.size() - nhead, nhead * 4, hipMemcpyHostToDevice));
    if (!net->dL) {
        std::vector<float> bias((size_t)nb * 2 * C);
        const float *q = p + nstem;
        for (int k = 0; k < nb; ++k)
            for (int j = 0; j < 2; ++j) {
                q += (size_t)C * C * 9;
                std::memcpy(bias.data() + (size_t)(k * 2 + j) * C, q, C * 4);
                q += C;
            }
        HIPCHK(net, hipMemcpy(net->d_bias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice));
    }
    return DL_OK;
}

// Trained weights reach the inference path: copied back into net->params,
// the small tensors re-uploaded, the conv weights repacked on next use.
int sync_trained(dl_net *net)
{
    if (!net->t_dirty) return DL_OK;
    HIPCHK(net, hipDeviceSynchronize());
    HIPCHK(net, hipMemcpy(net->params.data(), net->t_params, net->params.size() * 4, hipMemcpyDeviceToHost));
    int rc = upload_small_weights(net);
    if (rc) return rc;
    net->t_dirty = false;
    net->packed_precision = -1;
    return DL_OK;
}

// Dense networks: every conv's weights in the k_dconv layout and its bias,
// in run order, in one device buffer (FP32; packed once).
int pack_dense(dl_net *net)
{
    const int C = net->C, L = net->dL, G = net->dG, CT = C + L * G;
    std::vector<float> host;
    net->dense_w.clear();
    net->dense_b.clear();
    const float *p = net->params.data() + (size_t)C * 9 + C;
    auto put = [&](int cout, int cin, int taps) {
        const size_t nw = (size_t)cout * cin * taps;
        const size_t ow = (host.size() + 63) / 64 * 64;
        host.resize(ow + nw);
        pack_dense_weights(cout, cin, taps, p, host.data() + ow);
        p += nw;
        const size_t ob = (host.size() + 63) / 64 * 64;
        host.resize(ob + cout);
        std::memcpy(host.data() + ob, p, sizeof(float) * cout);
        p += cout;
        net->dense_w.push_back(ow);
        net->dense_b.push_back(ob);
    };
    for (int b = 0; b < net->nb; ++b) {
        for (int i = 0; i < L; ++i) put(G, C + i * G, 9);
        put(C, CT, 1);
    }
    if (net->unet) {                    // d1, d2 (C -> C), u1, u0 (2C -> C)
        put(C, C, 9);
        put(C, C, 9);
        put(C, 2 * C, 9);
        put(C, 2 * C, 9);
    }
    // the head (fused into the last block's last layer) as a 16-row 1x1 conv
    std::vector<float> head16((size_t)16 * C, 0.f);
    std::memcpy(head16.data(), p, sizeof(float) * net->nh * C);
    net->dense_head_w = (host.size() + 63) / 64 * 64;
    host.resize(net->dense_head_w + head16.size());
    pack_dense_weights(16, C, 1, head16.data(), host.data() + net->dense_head_w);
    net->packed_precision = -1;     // not packed until the new buffer holds the weights
    if (net->d_dense) {             // a repack (trained weights): kernels still queued may read the old buffer
        HIPCHK(net, hipDeviceSynchronize());
        HIPCHK(net, free_dev(net->d_dense));
    }
    HIPCHK(net, hipMalloc(&net->d_dense, host.size() * sizeof(float)));
    HIPCHK(net, hipMemcpy(net->d_dense, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice));
    net->packed_precision = DL_FP32;
    ++net->packed_gen;
    return DL_OK;
}

int ensure_packed(dl_net *net)
{
    if (int rc = sync_trained(net)) return rc;
    if (net->packed_precision == net->cfg.precision) return DL_OK;
    if (net->dL) return pack_dense(net);
    const int C = net->C;
    const size_t per = conv_packed_bytes(C, net->cfg.precision);
    const size_t stride = align_up(per);
    std::vector<char> host(stride * net->nb * 2);
    std::vector<float> wscale((size_t)net->nb * 2 * C, 0.f);
    const float *p = net->params.data() + (size_t)C * 9 + C;
    for (int b = 0; b < net->nb; ++b)
        for (int k = 0; k < 2; ++k) {
            pack_conv_weights(C, net->cfg.precision, p, host.data() + (size_t)(b * 2 + k) * stride,
                              wscale.data() + (size_t)(b * 2 + k) * C);
            p += (size_t)C * C * 9 + C;
        }
    // kernels still queued on any stream may read the old weights and scales
    HIPCHK(net, hipDeviceSynchronize());
    if (!net->d_wscale) HIPCHK(net, hipMalloc(&net->d_wscale, wscale.size() * sizeof(float)));
    HIPCHK(net, hipMemcpy(net->d_wscale, wscale.data(), wscale.size() * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(net, free_dev(net->d_wpk));
    HIPCHK(net, hipMalloc(&net->d_wpk, host.size()));
    HIPCHK(net, hipMemcpy(net->d_wpk, host.data(), host.size(), hipMemcpyHostToDevice));
    net->wpk_stride = stride;
    net->packed_precision = net->cfg.precision;
    ++net->packed_gen;
    return DL_OK;
}

// Profiling: when enabled, every launch of the path is bracketed by two HIP
// events on its stream; dl_profile_read sums the elapsed times per stage.
hipEvent_t pool_event(dl_net *net)
{
    if (!net->ev_pool.empty()) {
        hipEvent_t e = net->ev_pool.back();
        net->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct StageTimer {
    dl_net *net;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(dl_net *n, int st, hipStream_t str) : net(n), stage(st), s(str)
    {
        if (!net->profiling) return;
        a = pool_event(net);
        b = pool_event(net);
        if (a && b) (void)hipEventRecord(a, s);
    }
    ~StageTimer()
    {
        if (!net->profiling || !a || !b) return;
        (void)hipEventRecord(b, s);
        net->prof_pending.push_back({stage, a, b});
    }
};

// Gated runs: pool the input per 256^2 tile, run the gate, keep tiles whose
// logit exceeds the threshold, and build each conv layer's list of tiles that
// lie within that layer's remaining receptive radius of a kept tile.
int run_gate(dl_net *net, const FrameDesc *d_fd, const Geometry &g, const Plan &p, const uint16_t *d_frames,
             int n, int h, int w, hipStream_t s)
{
    StageTimer t(net, DL_STAGE_GATE, s);
    float *pooled = reinterpret_cast<float *>(p.ws + p.pooled);
    float *glog = reinterpret_cast<float *>(p.ws + p.glog);
    uint8_t *keep = reinterpret_cast<uint8_t *>(p.ws + p.keep);
    HIPCHK(net, launch_gate_pool(d_frames, n, h, w, net->cfg.offset, net->cfg.gain * in_scale_of(net), net->d_cam, pooled, s));
    HIPCHK(net, launch_gate(pooled, (int)g.gate_tiles, net->d_gate_theta, glog, nullptr, nullptr, s));
    HIPCHK(net, launch_gate_keep(glog, g.gate_tiles, net->gate_tau, keep, s));
    HIPCHK(net, launch_active_lists(d_fd, g, keep, net->d_radius + 1, net->d_dil, 2 * net->nb,
                                    reinterpret_cast<int32_t *>(p.ws + p.lists),
                                    reinterpret_cast<uint32_t *>(p.ws + p.lcount), s));
    net->last_gate_tiles = g.gate_tiles;
    net->last_keep_off = (size_t)(p.ws - net->ws) + p.keep;
    return DL_OK;
}

// The two-stage U-Net on the extractor's output a0 (channels 0 .. C-1 of B0,
// points of 2C floats at level 0).  Level buffers: B1 [d1 | x] (2C floats per
// level-1 point; x is pool(a0), later up(d2)), B2 [d2 | pool(d1)] (2C per
// level-2 point), U1 (C per level-1 point); B0's channels C .. 2C-1 take
// up(u1), and the last convolution reads [a0, up(u1)] with the head fused.
int run_unet(dl_net *net, const FrameDesc *d_fd, const Geometry &g, const Plan &p, float *B0, float *maps,
             hipStream_t s)
{
    const int C = net->C, n = g.nf, C2 = 2 * C;
    const FrameDesc *fd0 = d_fd, *fd1 = d_fd + n, *fd2 = d_fd + 2 * (size_t)n;
    float *B1 = reinterpret_cast<float *>(p.ws + p.unet);
    float *B2 = B1 + (size_t)C2 * g.lv_pts[1];
    float *U1 = B2 + (size_t)C2 * g.lv_pts[2];
    Geometry g1 = g, g2 = g;
    g1.tiles[0] = g.lv_tiles[1];
    g2.tiles[0] = g.lv_tiles[2];
    const size_t k0 = (size_t)net->nb * (net->dL + 1);   // the U-Net's convs in run order
    auto conv = [&](const FrameDesc *fd, const Geometry &gg, int blk, const float *in, int cin, float *out, int cso,
                    size_t k, int fuse) {
        DenseConvArgs a{};
        a.in = in;
        a.csi = C2;
        a.cin = cin;
        a.out = out;
        a.cso = cso;
        a.co = 0;
        a.w = net->d_dense + net->dense_w[k];
        a.bias = net->d_dense + net->dense_b[k];
        a.fd = fd;
        a.d = 1;
        a.blk = blk;
        if (fuse) {
            a.wh = net->d_dense + net->dense_head_w;
            a.bh = net->d_head + (size_t)net->nh * C;
            a.nh = net->nh;
            a.maps = maps;
        }
        return launch_dconv(C / 16, fuse, 1, a, gg, net->ncu, s);
    };
    {
        StageTimer t(net, DL_STAGE_UNET, s);
        HIPCHK(net, launch_pool2(fd0, fd1, n, g.lv_pts[1], B0, C2, B1 + C, C2, C, s));
        HIPCHK(net, conv(fd1, g1, 0, B1 + C, C, B1, C2, k0, 0));                  // d1
        HIPCHK(net, launch_pool2(fd1, fd2, n, g.lv_pts[2], B1, C2, B2 + C, C2, C, s));
        HIPCHK(net, conv(fd2, g2, 0, B2 + C, C, B2, C2, k0 + 1, 0));              // d2
        HIPCHK(net, launch_up2(fd2, fd1, n, g.lv_pts[1], B2, C2, B1 + C, C2, C, s));
        HIPCHK(net, conv(fd1, g1, 0, B1, C2, U1, C, k0 + 2, 0));                  // u1
        HIPCHK(net, launch_up2(fd1, fd0, n, g.lv_pts[0], U1, C, B0 + C, C2, C, s));
    }
    StageTimer t(net, DL_STAGE_CONV_HEAD, s);
    HIPCHK(net, conv(fd0, g, net->nb, B0, C2, nullptr, 0, k0 + 3, 3));             // u0 + head
    return DL_OK;
}

// Dense networks: stem into channels 0 .. C-1 of buffer A; per block, each
// layer appends its G channels to A, and the last one, fused with the block's
// transition, writes the next block's input into B (channels 0 .. C-1), after
// which A and B swap; in the last block the head is fused after the
// transition and writes the maps.
int run_dense(dl_net *net, const FrameDesc *d_fd, const Geometry &g, const Plan &p, float *maps, hipStream_t s)
{
    const int C = net->C, L = net->dL, G = net->dG, CT = C + L * G;
    float *A = reinterpret_cast<float *>(p.ws + p.act0), *B = reinterpret_cast<float *>(p.ws + p.act2);
    uint32_t *queue = net->cfg.tile_queue ? reinterpret_cast<uint32_t *>(p.ws + p.queue) : nullptr;
    if (queue) HIPCHK(net, launch_zero_u32(queue, (int64_t)net->nb * L * 8, s));
    {
        StageTimer t(net, DL_STAGE_STEM, s);
        HIPCHK(net, launch_dstem(C, d_fd, g, net->d_stem, net->d_stem + C * 9, net->cfg.offset,
                                 net->cfg.gain * in_scale_of(net), A, CT, s));
    }
    for (int b = 0; b < net->nb; ++b) {
        const size_t k0 = (size_t)b * (L + 1);          // this block's first conv in run order
        for (int i = 0; i < L; ++i) {
            const bool last = i == L - 1;
            const int fuse = !last ? 0 : b == net->nb - 1 && !net->unet ? 2 : 1;
            DenseConvArgs a{};
            a.in = A;
            a.csi = CT;
            a.cin = C + i * G;
            a.out = A;
            a.cso = CT;
            a.co = C + i * G;
            a.w = net->d_dense + net->dense_w[k0 + i];
            a.bias = net->d_dense + net->dense_b[k0 + i];
            a.fd = d_fd;
            a.d = net->dil[b];
            a.blk = b;
            if (queue) {
                a.queue = queue + ((size_t)b * L + i) * 8;
                a.queue_mode = net->cfg.tile_queue;
            }
            if (fuse) {
                a.wt = net->d_dense + net->dense_w[k0 + L];
                a.bt = net->d_dense + net->dense_b[k0 + L];
                a.tout = B;
                a.cst = b == net->nb - 1 ? 2 * C : CT;   // the U-Net's [a0, up(u1)] at level 0
            }
            if (fuse == 2) {
                a.wh = net->d_dense + net->dense_head_w;
                a.bh = net->d_head + (size_t)net->nh * C;
                a.nh = net->nh;
                a.maps = maps;
            }
            StageTimer t(net, fuse == 0 ? DL_STAGE_CONV : fuse == 1 ? DL_STAGE_CONV_1X1 : DL_STAGE_CONV_HEAD, s);
            HIPCHK(net, launch_dconv(G / 16, fuse, C / 16, a, g, net->ncu, s));
        }
        std::swap(A, B);
    }
    if (net->unet) return run_unet(net, d_fd, g, p, A, maps, s);
    return DL_OK;
}

// Run stem + blocks (+ fused head into maps).
int run_net(dl_net *net, const FrameDesc *d_fd, const Geometry &g, const Plan &p, float *maps, hipStream_t s)
{
    if (net->dL) return run_dense(net, d_fd, g, p, maps, s);
    const int C = net->C;
    void *a0 = p.ws + p.act0;
    void *a1 = p.ws + p.act1;
    const float scale = net->cfg.gain * in_scale_of(net);
    const uint8_t *keep = p.gated ? reinterpret_cast<const uint8_t *>(p.ws + p.keep) : nullptr;
    const int32_t *lists = p.gated ? reinterpret_cast<const int32_t *>(p.ws + p.lists) : nullptr;
    const uint32_t *lcount = p.gated ? reinterpret_cast<const uint32_t *>(p.ws + p.lcount) : nullptr;
    int stem_r = 0;
    for (int b = 0; b < net->nb; ++b) stem_r += 2 * net->dil[b];
    {
        StageTimer t(net, DL_STAGE_STEM, s);
        HIPCHK(net, launch_stem(C, d_fd, g, net->d_stem, net->d_stem + C * 9, net->cfg.offset, scale, net->d_cam,
                                a0, net->cfg.precision, keep, stem_r, s));
    }
    void *x = a0, *xn = p.ws + p.act2;      // block input, block output (alternating)
    for (int b = 0; b < net->nb; ++b) {
        const int maxg = conv_max_grid(C, net->cfg.precision, g.trb[b], net->ncu);
        int grid = (int)std::min<int64_t>(g.tiles[b], maxg);
        grid = std::max(8, grid / 8 * 8);
        const int lay = block_layout(net, b);
        const int lay_next = b + 1 < net->nb ? block_layout(net, b + 1) : 1;
        ConvArgs a{};
        a.fd = d_fd;
        a.d = net->dil[b];
        a.blk = b;
        a.tr = g.trb[b];
        a.in_phase = lay == net->dil[b] && lay > 1;
        a.out_shift = __builtin_ctz((unsigned)lay);
        if (net->cfg.precision == DL_FP8) a.wscale = net->d_wscale + (size_t)(b * 2) * C;
        a.in = x;
        a.out = a1;
        a.res = nullptr;
        a.wpk = static_cast<char *>(net->d_wpk) + (size_t)(b * 2) * net->wpk_stride;
        a.bias = net->d_bias + (size_t)(b * 2) * C;
        if (lists) {
            a.list = lists + (size_t)(2 * b) * g.max_tiles;
            a.list_count = lcount + 2 * b;
        }
        {
            StageTimer t(net, DL_STAGE_CONV, s);
            HIPCHK(net, launch_conv(C, net->cfg.precision, a, g, grid, s));
        }
        a.in = a1;
        a.res = x;
        a.out = xn;
        a.out_shift = __builtin_ctz((unsigned)lay_next);
        a.wpk = static_cast<char *>(net->d_wpk) + (size_t)(b * 2 + 1) * net->wpk_stride;
        a.bias = net->d_bias + (size_t)(b * 2 + 1) * C;
        if (net->cfg.precision == DL_FP8) a.wscale = net->d_wscale + (size_t)(b * 2 + 1) * C;
        if (lists) {
            a.list = lists + (size_t)(2 * b + 1) * g.max_tiles;
            a.list_count = lcount + 2 * b + 1;
        }
        if (b == net->nb - 1) {
            a.head = net->d_head;
            a.maps = maps;
            a.nh = net->nh;
            a.out = nullptr;
        }
        StageTimer t(net, b == net->nb - 1 ? DL_STAGE_CONV_HEAD : DL_STAGE_CONV, s);
        HIPCHK(net, launch_conv(C, net->cfg.precision, a, g, grid, s));
        std::swap(x, xn);
    }
    return DL_OK;
}

// The uncertainty filter as a bound on the raw sigma planes: sigma =
// softplus(u) + DL_SIGMA_FLOOR <= s iff u <= log(e^(s - floor) - 1)
// (softplus is increasing); -inf when s is at or below the floor (no sigma
// passes), +inf when the filter is off or the net has no uncertainty planes.
float sigma_limit_raw(const dl_net *net)
{
    const double s = net->cfg.max_sigma_px;
    if (net->nh != 10 || !(s > 0.0)) return INFINITY;
    const double r = s - (double)DL_SIGMA_FLOOR;
    if (!(r > 0.0)) return -INFINITY;
    return (float)(r > 30.0 ? r : std::log(std::expm1(r)));
}

int run_post(dl_net *net, const FrameDesc *d_fd, const Geometry &g, const Plan &p, const float *maps,
             dl_emitter *d_out, size_t cap, uint32_t *d_counts, hipStream_t s, dl_uncertainty *d_unc = nullptr)
{
    const float thr = net->cfg.threshold;
    const float tau = (float)std::log((double)thr / (1.0 - (double)thr));
    uint64_t *mask = reinterpret_cast<uint64_t *>(p.ws + p.mask);
    uint32_t *rc = reinterpret_cast<uint32_t *>(p.ws + p.rc);
    uint32_t *roff = reinterpret_cast<uint32_t *>(p.ws + p.roff);
    {
        StageTimer t(net, DL_STAGE_DETECT, s);
        const uint8_t *keep = p.gated ? reinterpret_cast<const uint8_t *>(p.ws + p.keep) : nullptr;
        HIPCHK(net, launch_detect_mask(maps, net->nh, d_fd, g, tau, sigma_limit_raw(net), keep, mask, rc, s));
    }
    {
        StageTimer t(net, DL_STAGE_SCAN, s);
        HIPCHK(net, launch_scan(rc, d_fd, g, roff, d_counts, s));
    }
    {
        StageTimer t(net, DL_STAGE_EMIT, s);
        HIPCHK(net, launch_emit(maps, net->nh, mask, roff, d_fd, g, net->z_scale, net->ph_scale, 1.f / in_scale_of(net),
                                d_out, d_unc, cap, s));
    }
    return DL_OK;
}

int check_uniform(dl_net *net, const void *frames, int n, int h, int w)
{
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    if (!frames) return fail(net, DL_ERR_INVALID_ARG, "frames is NULL");
    if (reinterpret_cast<uintptr_t>(frames) % 2) return fail(net, DL_ERR_INVALID_ARG, "frames must be 2-byte aligned");
    if (n <= 0 || h <= 0 || w <= 0) return fail(net, DL_ERR_INVALID_ARG, "n, h, w must be > 0 (got %d, %d, %d)", n, h, w);
    if ((int64_t)h * w > (int64_t)1 << 28 || !frame_act_fits(net, h, w))
        return fail(net, DL_ERR_UNSUPPORTED, "frame of %d x %d pixels is too large", h, w);
    if ((int64_t)n * h > (int64_t)1 << 30) return fail(net, DL_ERR_UNSUPPORTED, "too many rows in the batch");
    return DL_OK;
}

int set_device(dl_net *net) { HIPCHK(net, hipSetDevice(net->dev)); return DL_OK; }

int uniform_geometry(dl_net *net, const uint16_t *d_frames, int n, int h, int w, std::vector<FrameDesc> &fd, Geometry &g)
{
    std::vector<int> hs(n, h), ws(n, w);
    std::vector<const uint16_t *> ptr(n);
    std::vector<int64_t> st(n, w);
    for (int f = 0; f < n; ++f) ptr[f] = d_frames ? d_frames + (size_t)f * h * w : nullptr;
    build_geometry(net, n, hs.data(), ws.data(), ptr.data(), st.data(), fd, g);
    return DL_OK;
}

// Camera maps cover one sensor: they apply to uniform batches of frames of
// exactly that shape and not to ROI lists.
int check_camera(dl_net *net, bool uniform, int h, int w)
{
    if (!net->d_cam) return DL_OK;
    if (!uniform) return fail(net, DL_ERR_UNSUPPORTED, "camera maps apply to uniform batches of sensor frames, not ROI lists");
    if (h != net->cam_h || w != net->cam_w)
        return fail(net, DL_ERR_INVALID_ARG, "frames are %d x %d but the camera maps are %d x %d", h, w, net->cam_h,
                    net->cam_w);
    return DL_OK;
}

// fixed_ws (fixed_cap bytes): run in this memory instead of the handle's
// workspace, which is then neither grown nor touched (the allocation-free
// entry point; ungated runs only)
int localize_geom(dl_net *net, const std::vector<FrameDesc> &fd, const Geometry &g, hipStream_t s,
                  dl_emitter *d_out, size_t cap, uint32_t *d_counts, float *ext_maps,
                  const uint16_t *d_frames = nullptr, int n = 0, int h = 0, int w = 0,
                  dl_uncertainty *d_unc = nullptr, char *fixed_ws = nullptr, size_t fixed_cap = 0)
{
    int rc;
    if ((rc = check_camera(net, d_frames != nullptr, h, w))) return rc;
    if ((rc = set_device(net))) return rc;
    if ((rc = ensure_packed(net))) return rc;
    if (gated_run(net)) {
        if (!d_frames) return fail(net, DL_ERR_UNSUPPORTED, "the tile gate runs on uniform batches only (not ROI lists)");
        if (h % GATE_TILE || w % GATE_TILE)
            return fail(net, DL_ERR_UNSUPPORTED, "the tile gate needs h and w multiples of %d (got %d x %d)", GATE_TILE, h, w);
    }
    Plan p = make_plan(net, g, ext_maps != nullptr);
    if (fixed_ws) {
        if (p.gated) return fail(net, DL_ERR_UNSUPPORTED, "gated runs need the handle's workspace");
        if (p.total > fixed_cap)
            return fail(net, DL_ERR_UNSUPPORTED, "the batch needs %zu bytes of workspace; the allocation-free entry "
                        "point has %zu", p.total, fixed_cap);
        p.ws = fixed_ws;
    } else {
        if ((rc = ensure_workspace(net, p.total, s))) return rc;
        if ((rc = ws_acquire(net, s))) return rc;
        p.ws = net->ws;
    }
    FrameDesc *d_fd = nullptr;
    const int slot = upload_desc(net, fd, s, &d_fd);
    if (slot < 0) return slot;
    float *maps = ext_maps ? ext_maps : reinterpret_cast<float *>(p.ws + p.maps);
    net->last_gate_tiles = 0;               // this run reuses the workspace
    if (p.gated && (rc = run_gate(net, d_fd, g, p, d_frames, n, h, w, s))) return rc;
    if ((rc = run_net(net, d_fd, g, p, maps, s))) return rc;
    if (d_out || d_counts)
        if ((rc = run_post(net, d_fd, g, p, maps, d_out, cap, d_counts, s, d_unc))) return rc;
    HIPCHK(net, hipEventRecord(net->desc_ev[slot], s));
    return fixed_ws ? DL_OK : ws_release(net, s);
}

// This device's `scratch`: its address is looked up once per device (with
// that device current) and kept; every handle on the device shares it.
int scratch_init(dl_net *net)
{
    if (net->dev >= MAX_DEVICES) return fail(net, DL_ERR_UNSUPPORTED, "device ordinal %d >= %d", net->dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[net->dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(net, DL_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        g_scratch_ptr[net->dev] = static_cast<char *>(p);
    }
    net->scratch = g_scratch_ptr[net->dev];
    return DL_OK;
}

}  // namespace

// A captured localization of one fixed batch geometry: its own workspace and
// descriptor buffer (so later calls on the handle can never move memory the
// graph points at), the kernel sequence as a hipGraphExec.
struct dl_graph {
    dl_net *net = nullptr;
    int dev = 0;                    // the net's device (destroying the graph does not touch the net)
    char *ws = nullptr;
    FrameDesc *d_fd = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t cam_gen = 0;           // the handle's camera-map generation at capture
    uint64_t packed_gen = 0;        // and its weight-packing generation
    // ROI graphs of any batch within a capacity: the ROI list goes into a
    // pinned slot the graph's first node copies to the device, where a kernel
    // builds the descriptors and the frame counts (dyn)
    bool dynamic = false;
    int cap_rois = 0, cap_h = 0, cap_w = 0;
    int64_t cap_px = 0, cap_act = 0, cap_rows = 0, cap_words = 0;
    char *h_slot = nullptr, *d_slot = nullptr;   // [int64 n][dl_roi x cap_rois]
    int64_t *d_dyn = nullptr;
    hipEvent_t copied = nullptr;    // recorded in the graph after the slot's copy
};

static int check_rois(dl_net *net, const dl_roi *rois, int nroi);
static void roi_geometry(dl_net *net, const dl_roi *rois, int nroi, std::vector<FrameDesc> &fd, Geometry &g);

namespace {

int graph_build(dl_net *net, const std::vector<FrameDesc> &fd, const Geometry &g, dl_emitter *d_out, size_t cap,
                uint32_t *d_counts, dl_graph **out, dl_graph *dyn_proto = nullptr)
{
    int rc;
    if ((rc = set_device(net))) return rc;
    if ((rc = ensure_packed(net))) return rc;
    if (gated_run(net)) return fail(net, DL_ERR_UNSUPPORTED, "graph capture of gated runs is not supported");
    dl_graph *gr = new (std::nothrow) dl_graph();
    if (!gr) return fail(net, DL_ERR_OOM, "out of host memory");
    if (dyn_proto) *gr = *dyn_proto;        // capacity fields of a dynamic ROI graph
    gr->net = net;
    gr->dev = net->dev;
    gr->cam_gen = net->cam_gen;
    gr->packed_gen = net->packed_gen;       // ensure_packed ran above
    auto bail = [&](int code) {
        if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
        if (gr->graph) (void)hipGraphDestroy(gr->graph);
        if (gr->ws) (void)hipFree(gr->ws);
        if (gr->d_fd) (void)hipFree(gr->d_fd);
        if (gr->d_slot) (void)hipFree(gr->d_slot);
        if (gr->d_dyn) (void)hipFree(gr->d_dyn);
        if (gr->h_slot) (void)hipHostFree(gr->h_slot);
        if (gr->copied) (void)hipEventDestroy(gr->copied);
        delete gr;
        return code;
    };
    Plan p = make_plan(net, g, false);
    if (net->cfg.max_workspace_bytes && p.total > net->cfg.max_workspace_bytes)
        return bail(fail(net, DL_ERR_OOM, "graph workspace of %zu bytes exceeds max_workspace_bytes", p.total));
    if (hipMalloc(&gr->ws, p.total) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(net, DL_ERR_OOM, "hipMalloc(%zu) for the graph workspace failed", p.total));
    }
    Geometry gg = g;
    const size_t slot_bytes = 8 + sizeof(dl_roi) * (size_t)gr->cap_rois;
    if (gr->dynamic) {
        if (hipMalloc(&gr->d_fd, sizeof(FrameDesc) * gr->cap_rois) != hipSuccess ||
            hipMalloc(&gr->d_slot, slot_bytes) != hipSuccess ||
            hipMalloc(&gr->d_dyn, sizeof(int64_t) * DYN_WORDS) != hipSuccess ||
            hipHostMalloc((void **)&gr->h_slot, slot_bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(net, DL_ERR_OOM, "allocation of the graph's ROI slots failed"));
        }
        std::memset(gr->h_slot, 0, slot_bytes);
        if (hipEventCreateWithFlags(&gr->copied, hipEventDisableTiming) != hipSuccess)
            return bail(fail(net, DL_ERR_DEVICE, "hipEventCreate failed"));
        gg.dyn = gr->d_dyn;
    } else if (hipMalloc(&gr->d_fd, sizeof(FrameDesc) * fd.size()) != hipSuccess ||
               hipMemcpy(gr->d_fd, fd.data(), sizeof(FrameDesc) * fd.size(), hipMemcpyHostToDevice) != hipSuccess) {
        return bail(fail(net, DL_ERR_DEVICE, "descriptor upload failed"));
    }
    p.ws = gr->ws;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(net, DL_ERR_DEVICE, "hipStreamCreate failed"));
    const bool prof = net->profiling;
    net->profiling = false;           // no timing events inside the graph
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        float *maps = reinterpret_cast<float *>(p.ws + p.maps);
        rc = DL_OK;
        if (gr->dynamic) {
            // the ROI list of this replay: pinned slot -> device, then the
            // descriptors and frame counts built on the device
            EnumArgs ea{};
            ea.nb = net->nb;
            for (int b = 0; b < MAXBLK; ++b) ea.tr[b] = g.trb[b];
            ea.tc = g.tc;
            ea.layouts[ea.nl++] = 1;
            for (int b = 0; b < net->nb; ++b) {
                ea.dil[b] = net->dil[b];
                const int l = block_layout(net, b);
                bool seen = false;
                for (int i = 0; i < ea.nl; ++i) seen |= ea.layouts[i] == l;
                if (!seen) ea.layouts[ea.nl++] = l;
            }
            if (hipMemcpyAsync(gr->d_slot, gr->h_slot, slot_bytes, hipMemcpyHostToDevice, cs) != hipSuccess ||
                hipEventRecord(gr->copied, cs) != hipSuccess || launch_enumerate(gr->d_slot, ea, gr->d_fd, gr->d_dyn, cs) != hipSuccess)
                rc = fail(net, DL_ERR_DEVICE, "capturing the ROI list's copy and enumeration failed");
        }
        if (!rc) rc = run_net(net, gr->d_fd, gg, p, maps, cs);
        if (!rc) rc = run_post(net, gr->d_fd, gg, p, maps, d_out, cap, d_counts, cs);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        gr->graph = graph;
        if (!rc && e2 != hipSuccess) rc = fail(net, DL_ERR_DEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e2));
        if (!rc && hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0) != hipSuccess)
            rc = fail(net, DL_ERR_DEVICE, "hipGraphInstantiate failed");
    } else {
        rc = fail(net, DL_ERR_DEVICE, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
    }
    net->profiling = prof;
    (void)hipStreamDestroy(cs);
    if (rc) return bail(rc);
    *out = gr;
    return DL_OK;
}

}  // namespace

// ---- training ----
namespace {

// float offsets of a residual net's tensors in blob order
struct ParamOffsets {
    size_t stem_w, stem_b, w1[MAXBLK], b1[MAXBLK], w2[MAXBLK], b2[MAXBLK], head_w, head_b, total;
};
ParamOffsets param_offsets(const dl_net *net)
{
    const size_t C = net->C;
    ParamOffsets o{};
    size_t k = 0;
    o.stem_w = k; k += C * 9;
    o.stem_b = k; k += C;
    for (int b = 0; b < net->nb; ++b) {
        o.w1[b] = k; k += C * C * 9;
        o.b1[b] = k; k += C;
        o.w2[b] = k; k += C * C * 9;
        o.b2[b] = k; k += C;
    }
    o.head_w = k; k += (size_t)net->nh * C;
    o.head_b = k; k += net->nh;
    o.total = k;
    return o;
}

// float offsets of a dense network's tensors in blob order: stem, per block
// the L layers' weights and biases then the transition's, the U-Net's
// convolutions (d1, d2, u1, u0), the head
struct DenseOffsets {
    size_t stem_w = 0, stem_b = 0, head_w = 0, head_b = 0;
    std::vector<size_t> lw, lb, tw, tb;          // lw/lb [block L + layer]
    size_t uw[4] = {0, 0, 0, 0}, ub[4] = {0, 0, 0, 0};
};
DenseOffsets dense_offsets(const dl_net *net)
{
    const size_t C = net->C, L = net->dL, G = net->dG, CT = C + L * G;
    DenseOffsets o;
    size_t k = 0;
    o.stem_w = k; k += C * 9;
    o.stem_b = k; k += C;
    for (int b = 0; b < net->nb; ++b) {
        for (size_t i = 0; i < L; ++i) {
            o.lw.push_back(k); k += G * (C + i * G) * 9;
            o.lb.push_back(k); k += G;
        }
        o.tw.push_back(k); k += C * CT;
        o.tb.push_back(k); k += C;
    }
    if (net->unet)
        for (int u = 0; u < 4; ++u) {                // d1, d2: C -> C; u1, u0: 2C -> C
            o.uw[u] = k; k += C * (u < 2 ? C : 2 * C) * 9;
            o.ub[u] = k; k += C;
        }
    o.head_w = k; k += (size_t)net->nh * C;
    o.head_b = k;
    return o;
}

// The dense network's weight packs for training, as pack jobs in a fixed
// order: per block, each layer's forward pack (16 rows over its C + i G
// inputs, 9 taps), the transition's (C rows over CT inputs, 1 tap) for the
// fused last layer, and each layer's transposed convolution (G inputs ->
// C + i G outputs) in slices of at most 80 output rows, one conv launch each.
struct DensePackPlan {
    std::vector<PackJob> jobs;
    std::vector<int> fw, tw;                      // job index: fw [block L + layer], tw [block]
    std::vector<std::vector<int>> tr;             // [block L + layer]: the slices' job indices
    int ufw[4] = {0, 0, 0, 0}, utr[4] = {0, 0, 0, 0};   // the U-Net's convs, forward and transposed
    int64_t total = 0;
};
DensePackPlan dense_pack_plan(const dl_net *net)
{
    const int C = net->C, L = net->dL, G = net->dG, CT = C + L * G;
    const DenseOffsets o = dense_offsets(net);
    DensePackPlan pl;
    auto add = [&](size_t src, int cout, int cin, int taps, int flip, int row0, int nrows) {
        PackJob j{};
        j.src = (int64_t)src;
        j.cout = cout;
        j.cin = cin;
        j.taps = taps;
        j.flip = flip;
        j.row0 = row0;
        j.nrows = nrows;
        j.start = pl.total;
        j.dst = (pl.total + 63) / 64 * 64;       // 256-byte aligned packs
        const int64_t n = (int64_t)nrows * (flip ? cout : cin) * taps;
        j.start = j.dst;
        pl.total = j.dst + n;
        pl.jobs.push_back(j);
        return (int)pl.jobs.size() - 1;
    };
    for (int b = 0; b < net->nb; ++b) {
        for (int i = 0; i < L; ++i) pl.fw.push_back(add(o.lw[(size_t)b * L + i], G, C + i * G, 9, 0, 0, G));
        pl.tw.push_back(add(o.tw[b], C, CT, 1, 0, 0, C));
        for (int i = 0; i < L; ++i) {
            std::vector<int> sl;
            for (int r = 0; r < C + i * G; r += 80)
                sl.push_back(add(o.lw[(size_t)b * L + i], G, C + i * G, 9, 1, r, std::min(80, C + i * G - r)));
            pl.tr.push_back(sl);
        }
    }
    if (net->unet)
        for (int u = 0; u < 4; ++u) {
            const int cin = u < 2 ? C : 2 * C;
            pl.ufw[u] = add(o.uw[u], C, cin, 9, 0, 0, C);
            pl.utr[u] = add(o.uw[u], C, cin, 9, 1, 0, cin);
        }
    return pl;
}

int train_check(dl_net *net, const uint16_t *d_frames, int n, int h, int w, const dl_truth *d_truth,
                const int32_t *d_off, int ntruth, float *d_loss)
{
    int rc = check_uniform(net, d_frames, n, h, w);
    if (rc) return rc;
    if (net->nh != 10 || !(net->C == 16 || net->C == 32) || (net->dL && net->dG != 16))
        return fail(net, DL_ERR_UNSUPPORTED,
                    "training runs the residual or the dense network (growth 16) with the 10-output head and C = 16 "
                    "or 32");
    if (net->d_cam) return fail(net, DL_ERR_UNSUPPORTED, "training uses the scalar gain and offset (clear the camera maps)");
    if (!d_off || !d_loss || (ntruth > 0 && !d_truth) || ntruth < 0)
        return fail(net, DL_ERR_INVALID_ARG, "d_truth_off and d_loss must be given, d_truth when ntruth > 0");
    if ((int64_t)n * h * w > ((int64_t)1 << 26))
        return fail(net, DL_ERR_UNSUPPORTED, "a training batch holds at most 2^26 pixels");
    // the weight-gradient kernels address within a row with 32-bit byte
    // offsets (up to 96 floats per point)
    if (w > (1 << 20)) return fail(net, DL_ERR_UNSUPPORTED, "training frame rows hold at most 2^20 pixels (got %d)", w);
    return DL_OK;
}

// device copies of the weights and the Adam state, made on first use
int train_init(dl_net *net)
{
    if (net->t_params) return DL_OK;
    const size_t np = net->params.size(), C = net->C;
    HIPCHK(net, hipMalloc(&net->t_params, np * 4));
    HIPCHK(net, hipMalloc(&net->t_grad, np * 4));
    HIPCHK(net, hipMalloc(&net->t_m, np * 4));
    HIPCHK(net, hipMalloc(&net->t_v, np * 4));
    if (net->dL) {
        const DensePackPlan pl = dense_pack_plan(net);
        HIPCHK(net, hipMalloc(&net->t_pack, (size_t)pl.total * 4));
        HIPCHK(net, hipMalloc(&net->t_jobs, pl.jobs.size() * sizeof(PackJob)));
        HIPCHK(net, hipMemcpy(net->t_jobs, pl.jobs.data(), pl.jobs.size() * sizeof(PackJob), hipMemcpyHostToDevice));
        net->t_njobs = (int)pl.jobs.size();
        net->t_jobs_total = pl.total;
    } else {
        HIPCHK(net, hipMalloc(&net->t_pack, (size_t)net->nb * 4 * C * C * 9 * 4));
    }
    HIPCHK(net, hipMemcpy(net->t_params, net->params.data(), np * 4, hipMemcpyHostToDevice));
    HIPCHK(net, hipMemset(net->t_m, 0, np * 4));
    HIPCHK(net, hipMemset(net->t_v, 0, np * 4));
    net->t_step = 0;
    return DL_OK;
}

// frame descriptors and conv geometry of a uniform training batch (frame f's
// points from f h w, its tiles per block from f times a frame's); with the
// U-Net, the level-0 convolution in tile slot nb and levels 1 and 2 with
// descriptors of their own after the n frames' (g1, g2: their geometry)
int train_geometry(dl_net *net, const uint16_t *d_frames, int n, int h, int w, hipStream_t s, Geometry &g,
                   FrameDesc **d_fd, Geometry *g1 = nullptr, Geometry *g2 = nullptr)
{
    std::vector<FrameDesc> fd((size_t)n * desc_per_frame(net));
    g = Geometry{};
    g.nf = n;
    g.tr = dense_tile_rows();
    g.tc = dense_tile_cols();
    for (int f = 0; f < n; ++f) {
        FrameDesc &d = fd[f];
        std::memset(&d, 0, sizeof d);
        d.data = d_frames + (size_t)f * h * w;
        d.stride = w;
        d.h = h;
        d.w = w;
        d.px_off = d.act_off = (int64_t)f * h * w;
        d.row_start = (int64_t)f * h;
        for (int b = 0; b < net->nb; ++b) d.tile_start[b] = (int64_t)f * conv_tiles(h, w, net->dil[b], g.tr, g.tc);
    }
    for (int b = 0; b < net->nb; ++b) g.tiles[b] = (int64_t)n * conv_tiles(h, w, net->dil[b], g.tr, g.tc);
    g.total_rows = (int64_t)n * h;
    g.total_px = g.total_act = (int64_t)n * h * w;
    if (net->unet) {
        const int nb = net->nb;
        for (int f = 0; f < n; ++f) fd[f].tile_start[nb] = (int64_t)f * conv_tiles(h, w, 1, g.tr, g.tc);
        g.tiles[nb] = (int64_t)n * conv_tiles(h, w, 1, g.tr, g.tc);
        int hl = h, wl = w;
        for (int l = 1; l <= 2; ++l) {
            hl = (hl + 1) / 2;
            wl = (wl + 1) / 2;
            Geometry &gl = l == 1 ? *g1 : *g2;
            gl = g;
            gl.tiles[0] = (int64_t)n * conv_tiles(hl, wl, 1, g.tr, g.tc);
            for (int f = 0; f < n; ++f) {
                FrameDesc &d = fd[(size_t)l * n + f];
                std::memset(&d, 0, sizeof d);
                d.h = hl;
                d.w = wl;
                d.act_off = (int64_t)f * hl * wl;
                d.tile_start[0] = (int64_t)f * conv_tiles(hl, wl, 1, g.tr, g.tc);
            }
        }
    }
    return upload_desc(net, fd, s, d_fd);
}

// The dense network: forward with every concatenation kept (block b's in A[b],
// CT = C + L G channels per point; the last transition's output in tl), the
// loss, backward.  Backward through block b: the transition's
// pre-activation gradient gtp (the head's, or the next block's input gradient
// masked where the transition's ReLU was off) gives the transition's weight
// gradient and, through the transposed 1x1 map, the concatenation's gradient
// ga; then from the last layer to the first, the layer's output channels of
// ga masked where its ReLU was off (gl) give its weight gradient, and the
// transposed 3x3 convolution of gl is added to ga's channels 0 .. C + i G - 1.
int train_run_dense(dl_net *net, const uint16_t *d_frames, int n, int h, int w, const dl_truth *d_truth,
                    const int32_t *d_off, int ntruth, hipStream_t s, float *d_grad, float *d_loss)
{
    const int C = net->C, L = net->dL, G = net->dG, CT = C + L * G, nb = net->nb, C2 = 2 * C;
    const int64_t P = (int64_t)n * h * w;
    const int h1 = (h + 1) / 2, w1 = (w + 1) / 2, h2 = (h1 + 1) / 2, w2 = (w1 + 1) / 2;
    const int64_t P1 = net->unet ? (int64_t)n * h1 * w1 : 0, P2 = net->unet ? (int64_t)n * h2 * w2 : 0;
    const DenseOffsets o = dense_offsets(net);
    const DensePackPlan pl = dense_pack_plan(net);
    const int nblk = (n * h + wgrad_rows_per_block(n, h) - 1) / wgrad_rows_per_block(n, h);
    // the largest weight gradient (floats per partial): a layer's, the
    // transition's, or the U-Net's 2C -> C convolutions'
    const size_t wmax = std::max({(size_t)G * (C + (L - 1) * G) * 9, (size_t)C * CT,
                                  net->unet ? (size_t)C * C2 * 9 : (size_t)0});
    size_t off = 0;
    auto take = [&](size_t floats) { size_t at = off; off = align_up(off + floats * 4); return at; };
    std::vector<size_t> A(nb);
    for (int b = 0; b < nb; ++b) A[b] = take((size_t)P * CT);
    const size_t tl = take((size_t)P * C), ga = take((size_t)P * CT), gl = take((size_t)P * G), gtp = take((size_t)P * C);
    const size_t maps = take((size_t)P * 10), gm = take((size_t)P * 10);
    const size_t stats = take((size_t)3 * n), lse = take((size_t)train_lse_floats(h, w, ntruth));
    const size_t term = take((size_t)9 * P + 48 * (size_t)n), occ = take((size_t)(P + 3) / 4);
    const size_t part = take((size_t)nblk * wmax), pb = take((size_t)nblk * 32);
    const size_t tmp = take((size_t)32 * (wmax + 32) + (size_t)32 * (10 * C + 10));
    const size_t gpart = take((size_t)grad_chunks(P) * (10 * C + 10));
    // the U-Net (level 0 points P, level 1 P1, level 2 P2): c0 = [a0, up(u1)],
    // p1 = pool(a0), c1 = [d1, up(d2)], p2 = pool(d1), d2, u1, u0, and their
    // gradients
    const size_t c0 = take((size_t)P * C2 * !!net->unet), u0 = take((size_t)P * C * !!net->unet);
    const size_t p1 = take((size_t)P1 * C), c1 = take((size_t)P1 * C2), p2 = take((size_t)P2 * C);
    const size_t d2 = take((size_t)P2 * C), u1 = take((size_t)P1 * C);
    const size_t gc0 = take((size_t)P * C2 * !!net->unet), gu1 = take((size_t)P1 * C), gc1 = take((size_t)P1 * C2);
    const size_t gd2 = take((size_t)P2 * C), gp2 = take((size_t)P2 * C), gd1 = take((size_t)P1 * C);
    const size_t gp1 = take((size_t)P1 * C);
    if (off > net->t_ws_bytes) {
        HIPCHK(net, hipDeviceSynchronize());
        const hipError_t e = free_dev(net->t_ws);
        net->t_ws_bytes = 0;
        HIPCHK(net, e);
        if (hipMalloc(&net->t_ws, off) != hipSuccess) return fail(net, DL_ERR_OOM, "training buffers of %zu bytes", off);
        net->t_ws_bytes = off;
    }
    auto F = [&](size_t at) { return reinterpret_cast<float *>(net->t_ws + at); };
    float *prm = net->t_params, *grd = d_grad ? d_grad : net->t_grad;
    Geometry g, g1, g2;
    FrameDesc *d_fd = nullptr;
    const int slot = train_geometry(net, d_frames, n, h, w, s, g, &d_fd, &g1, &g2);
    if (slot < 0) return slot;
    const FrameDesc *fd1 = d_fd + n, *fd2 = d_fd + 2 * (size_t)n;
    HIPCHK(net, launch_pack_jobs(net->t_jobs, net->t_njobs, net->t_jobs_total, prm, net->t_pack, s));
    auto pk = [&](int job) { return net->t_pack + pl.jobs[job].dst; };
    auto conv = [&](int b, float *in, int csi, int cin, float *out, int cso, int co, const float *wpk,
                    const float *bias, const float *res, int relu) {
        DenseConvArgs a{};
        a.in = in;
        a.csi = csi;
        a.cin = cin;
        a.out = out;
        a.cso = cso;
        a.co = co;
        a.w = wpk;
        a.bias = bias;
        a.fd = d_fd;
        a.d = net->dil[b];
        a.blk = b;
        a.res = res;
        a.rcs = cso;
        a.relu = relu;
        return a;
    };
    const float scale = net->cfg.gain * in_scale_of(net);
    // forward
    HIPCHK(net, launch_dstem(C, d_fd, g, prm + o.stem_w, prm + o.stem_b, net->cfg.offset, scale, F(A[0]), CT, s));
    for (int b = 0; b < nb; ++b) {
        for (int i = 0; i < L; ++i) {
            const size_t li = (size_t)b * L + i;
            DenseConvArgs a = conv(b, F(A[b]), CT, C + i * G, F(A[b]), CT, C + i * G, pk(pl.fw[li]), prm + o.lb[li],
                                   nullptr, 1);
            if (i < L - 1) {
                HIPCHK(net, launch_dconv_train(G / 16, a, g, net->ncu, s));
            } else {
                a.wt = pk(pl.tw[b]);
                a.bt = prm + o.tb[b];
                a.tout = b + 1 < nb ? F(A[b + 1]) : net->unet ? F(c0) : F(tl);
                a.cst = b + 1 < nb ? CT : net->unet ? C2 : C;
                HIPCHK(net, launch_dconv_train_fused(C / 16, a, g, net->ncu, s));
            }
        }
    }
    // a U-Net convolution (3x3, d = 1) at a level: fd, geometry, tile slot
    auto uconv = [&](const FrameDesc *fd, const Geometry &gg, int blk, float *in, int csi, int cin, float *out,
                     int cso, int nbo, const float *wpk, const float *bias, int relu) {
        DenseConvArgs a{};
        a.in = in;
        a.csi = csi;
        a.cin = cin;
        a.out = out;
        a.cso = cso;
        a.w = wpk;
        a.bias = bias;
        a.fd = fd;
        a.d = 1;
        a.blk = blk;
        a.relu = relu;
        return launch_dconv_train(nbo, a, gg, net->ncu, s);
    };
    if (net->unet) {
        const int nbc = C / 16, nbc2 = C2 / 16;
        HIPCHK(net, launch_pool2(d_fd, fd1, n, P1, F(c0), C2, F(p1), C, C, s));
        HIPCHK(net, uconv(fd1, g1, 0, F(p1), C, C, F(c1), C2, nbc, pk(pl.ufw[0]), prm + o.ub[0], 1));     // d1
        HIPCHK(net, launch_pool2(fd1, fd2, n, P2, F(c1), C2, F(p2), C, C, s));
        HIPCHK(net, uconv(fd2, g2, 0, F(p2), C, C, F(d2), C, nbc, pk(pl.ufw[1]), prm + o.ub[1], 1));       // d2
        HIPCHK(net, launch_up2(fd2, fd1, n, P1, F(d2), C, F(c1) + C, C2, C, s));
        HIPCHK(net, uconv(fd1, g1, 0, F(c1), C2, C2, F(u1), C, nbc, pk(pl.ufw[2]), prm + o.ub[2], 1));     // u1
        HIPCHK(net, launch_up2(fd1, d_fd, n, P, F(u1), C, F(c0) + C, C2, C, s));
        HIPCHK(net, uconv(d_fd, g, nb, F(c0), C2, C2, F(u0), C, nbc, pk(pl.ufw[3]), prm + o.ub[3], 1));    // u0
        (void)nbc2;
    }
    float *last = net->unet ? F(u0) : F(tl);
    HIPCHK(net, launch_train_loss(C, last, prm + o.head_w, prm + o.head_b, n, h, w, d_truth, d_off, ntruth,
                                  net->z_scale, net->ph_scale, F(maps), F(stats), F(lse), F(gm), d_loss, F(term),
                                  reinterpret_cast<uint8_t *>(net->t_ws + occ), s));
    // backward
    float *mid = F(tmp);
    HIPCHK(net, launch_head_backward(C, F(gm), last, prm + o.head_w, n, h, w, grd + o.head_w, F(gpart), mid, F(gtp),
                                     s));
    if (net->unet) {
        // gtp: u0's pre-activation gradient
        const int nbc = C / 16, nbc2 = C2 / 16;
        HIPCHK(net, launch_wgrad_ex(C, 9, F(gtp), C, F(c0), C2, C2, n, h, w, 1, F(part), F(pb), mid, grd + o.uw[3],
                                    grd + o.ub[3], s));
        HIPCHK(net, uconv(d_fd, g, nb, F(gtp), C, C, F(gc0), C2, nbc2, pk(pl.utr[3]), nullptr, 0));
        HIPCHK(net, launch_up2_back(F(gc0) + C, C2, F(gu1), C, n, h, w, C, s));
        HIPCHK(net, launch_mask_slice(F(gu1), C, 0, F(u1), C, 0, C, P1, F(gu1), C, s));
        HIPCHK(net, launch_wgrad_ex(C, 9, F(gu1), C, F(c1), C2, C2, n, h1, w1, 1, F(part), F(pb), mid, grd + o.uw[2],
                                    grd + o.ub[2], s));
        HIPCHK(net, uconv(fd1, g1, 0, F(gu1), C, C, F(gc1), C2, nbc2, pk(pl.utr[2]), nullptr, 0));
        HIPCHK(net, launch_up2_back(F(gc1) + C, C2, F(gd2), C, n, h1, w1, C, s));
        HIPCHK(net, launch_mask_slice(F(gd2), C, 0, F(d2), C, 0, C, P2, F(gd2), C, s));
        HIPCHK(net, launch_wgrad_ex(C, 9, F(gd2), C, F(p2), C, C, n, h2, w2, 1, F(part), F(pb), mid, grd + o.uw[1],
                                    grd + o.ub[1], s));
        HIPCHK(net, uconv(fd2, g2, 0, F(gd2), C, C, F(gp2), C, nbc, pk(pl.utr[1]), nullptr, 0));
        // d1's output gradient: from u1 (gc1's first C channels) and through the pooling from d2
        HIPCHK(net, launch_pool2_back(F(c1), C2, F(gp2), C, F(gc1), C2, n, h1, w1, C, s));
        HIPCHK(net, launch_mask_slice(F(gc1), C2, 0, F(c1), C2, 0, C, P1, F(gd1), C, s));
        HIPCHK(net, launch_wgrad_ex(C, 9, F(gd1), C, F(p1), C, C, n, h1, w1, 1, F(part), F(pb), mid, grd + o.uw[0],
                                    grd + o.ub[0], s));
        HIPCHK(net, uconv(fd1, g1, 0, F(gd1), C, C, F(gp1), C, nbc, pk(pl.utr[0]), nullptr, 0));
        // a0's gradient: from u0 (gc0's first C channels) and through the pooling from d1
        HIPCHK(net, launch_pool2_back(F(c0), C2, F(gp1), C, F(gc0), C2, n, h, w, C, s));
    }
    for (int b = nb - 1; b >= 0; --b) {
        if (b + 1 < nb)   // the next block's input gradient, where this block's transition was on
            HIPCHK(net, launch_mask_slice(F(ga), CT, 0, F(A[b + 1]), CT, 0, C, P, F(gtp), C, s));
        else if (net->unet)   // the U-Net's input gradient, where the last transition was on
            HIPCHK(net, launch_mask_slice(F(gc0), C2, 0, F(c0), C2, 0, C, P, F(gtp), C, s));
        // the transition: weight gradient (16-row pieces when CT is not a multiple of C), input gradient
        if (CT % C == 0) {
            HIPCHK(net, launch_wgrad_ex(C, 1, F(gtp), C, F(A[b]), CT, CT, n, h, w, 1, F(part), F(pb), mid,
                                        grd + o.tw[b], grd + o.tb[b], s));
        } else {
            for (int r = 0; r < C; r += 16)
                HIPCHK(net, launch_wgrad_ex(16, 1, F(gtp) + r, C, F(A[b]), CT, CT, n, h, w, 1, F(part), F(pb), mid,
                                            grd + o.tw[b] + (size_t)r * CT, grd + o.tb[b] + r, s));
        }
        HIPCHK(net, launch_1x1_back(C, F(gtp), prm + o.tw[b], CT, P, F(ga), s));
        for (int i = L - 1; i >= 0; --i) {
            const size_t li = (size_t)b * L + i;
            const int lo = C + i * G;
            HIPCHK(net, launch_mask_slice(F(ga), CT, lo, F(A[b]), CT, lo, G, P, F(gl), G, s));
            HIPCHK(net, launch_wgrad_ex(G, 9, F(gl), G, F(A[b]), CT, lo, n, h, w, net->dil[b], F(part), F(pb), mid,
                                        grd + o.lw[li], grd + o.lb[li], s));
            for (int job : pl.tr[li]) {
                const PackJob &J = pl.jobs[job];
                DenseConvArgs a = conv(b, F(gl), G, G, F(ga), CT, J.row0, pk(job), nullptr, F(ga) + J.row0, 0);
                HIPCHK(net, launch_dconv_train(J.nrows / 16, a, g, net->ncu, s));
            }
        }
    }
    // the stem: its output's gradient where its ReLU was on
    HIPCHK(net, launch_mask_slice(F(ga), CT, 0, F(A[0]), CT, 0, C, P, F(gtp), C, s));
    HIPCHK(net, launch_stem_grad(F(gtp), d_frames, n, h, w, net->cfg.offset, scale, C, grd + o.stem_w, F(gpart), mid,
                                 s));
    HIPCHK(net, hipEventRecord(net->desc_ev[slot], s));
    return DL_OK;
}

// Forward with every activation kept, the loss and its gradient, backward.
// Buffers (P = n h w points of C floats): act[0 .. nb], T[0 .. nb-1], two
// gradient buffers and ds; maps and gm (10 P); stats, lse; the weight-gradient
// partials.
int train_run(dl_net *net, const uint16_t *d_frames, int n, int h, int w, const dl_truth *d_truth,
              const int32_t *d_off, int ntruth, hipStream_t s, float *d_grad, float *d_loss)
{
    int rc;
    if ((rc = set_device(net)) || (rc = train_init(net))) return rc;
    if (net->dL) return train_run_dense(net, d_frames, n, h, w, d_truth, d_off, ntruth, s, d_grad, d_loss);
    const int C = net->C, nb = net->nb;
    const int64_t P = (int64_t)n * h * w;
    const ParamOffsets o = param_offsets(net);
    const int nblk = (n * h + wgrad_rows_per_block(n, h) - 1) / wgrad_rows_per_block(n, h);
    size_t off = 0;
    auto take = [&](size_t floats) { size_t at = off; off = align_up(off + floats * 4); return at; };
    size_t act[MAXBLK + 1], T[MAXBLK];
    for (int b = 0; b <= nb; ++b) act[b] = take((size_t)P * C);
    for (int b = 0; b < nb; ++b) T[b] = take((size_t)P * C);
    const size_t g0 = take((size_t)P * C), g1 = take((size_t)P * C), dsb = take((size_t)P * C);
    const size_t maps = take((size_t)P * 10), gm = take((size_t)P * 10);
    const size_t stats = take((size_t)3 * n), lse = take((size_t)train_lse_floats(h, w, ntruth));
    const size_t term = take((size_t)9 * P + 48 * (size_t)n), occ = take((size_t)(P + 3) / 4);
    const size_t part = take((size_t)nblk * 9 * C * C), pb = take((size_t)nblk * C);
    const size_t tmp = take((size_t)32 * (9 * C * C + C));
    const size_t gpart = take((size_t)grad_chunks(P) * (10 * C + 10));
    if (off > net->t_ws_bytes) {
        HIPCHK(net, hipDeviceSynchronize());
        const hipError_t e = free_dev(net->t_ws);
        net->t_ws_bytes = 0;
        HIPCHK(net, e);
        if (hipMalloc(&net->t_ws, off) != hipSuccess) return fail(net, DL_ERR_OOM, "training buffers of %zu bytes", off);
        net->t_ws_bytes = off;
    }
    auto F = [&](size_t at) { return reinterpret_cast<float *>(net->t_ws + at); };
    float *prm = net->t_params, *grd = d_grad ? d_grad : net->t_grad;
    Geometry g;
    FrameDesc *d_fd = nullptr;
    const int slot = train_geometry(net, d_frames, n, h, w, s, g, &d_fd);
    if (slot < 0) return slot;
    // packed conv weights: [block][conv 1, 2][forward, transposed]
    auto pk = [&](int b, int k, int tr) { return net->t_pack + ((size_t)(b * 2 + k) * 2 + tr) * C * C * 9; };
    // (the blob holds w1, b1, w2, b2 of each block in turn: the 3x3 weights
    // follow one another 9 C^2 + C floats apart)
    HIPCHK(net, launch_pack_convs(prm + o.w1[0], (int64_t)9 * C * C + C, 2 * nb, C, net->t_pack, s));
    auto conv = [&](int b, int k, int tr, float *in, float *out, const float *bias, const float *res,
                    const float *mask, int relu) {
        DenseConvArgs a{};
        a.in = in;
        a.csi = C;
        a.cin = C;
        a.out = out;
        a.cso = C;
        a.co = 0;
        a.w = pk(b, k, tr);
        a.bias = bias;
        a.fd = d_fd;
        a.d = net->dil[b];
        a.blk = b;
        a.res = res;
        a.rcs = C;
        a.mask = mask;
        a.mcs = C;
        a.relu = relu;
        return launch_dconv_train(C / 16, a, g, net->ncu, s);
    };
    const float scale = net->cfg.gain * in_scale_of(net);
    // forward
    HIPCHK(net, launch_dstem(C, d_fd, g, prm + o.stem_w, prm + o.stem_b, net->cfg.offset, scale, F(act[0]), C, s));
    for (int b = 0; b < nb; ++b) {
        HIPCHK(net, conv(b, 0, 0, F(act[b]), F(T[b]), prm + o.b1[b], nullptr, nullptr, 1));
        HIPCHK(net, conv(b, 1, 0, F(T[b]), F(act[b + 1]), prm + o.b2[b], F(act[b]), nullptr, 1));
    }
    HIPCHK(net, launch_train_loss(C, F(act[nb]), prm + o.head_w, prm + o.head_b, n, h, w, d_truth, d_off, ntruth,
                                  net->z_scale, net->ph_scale, F(maps), F(stats), F(lse), F(gm), d_loss, F(term),
                                  reinterpret_cast<uint8_t *>(net->t_ws + occ), s));
    // backward: du is the gradient at the pre-activation of block b's output
    float *du = F(g0), *dn = F(g1);
    HIPCHK(net, launch_head_backward(C, F(gm), F(act[nb]), prm + o.head_w, n, h, w, grd + o.head_w, F(gpart),
                                     F(tmp) + 9 * C * C, du, s));
    for (int b = nb - 1; b >= 0; --b) {
        HIPCHK(net, launch_wgrad(C, du, F(T[b]), n, h, w, net->dil[b], F(part), F(pb), F(tmp), grd + o.w2[b],
                                 grd + o.b2[b], s));
        HIPCHK(net, conv(b, 1, 1, du, F(dsb), nullptr, nullptr, F(T[b]), 0));            // ds
        HIPCHK(net, launch_wgrad(C, F(dsb), F(act[b]), n, h, w, net->dil[b], F(part), F(pb), F(tmp), grd + o.w1[b],
                                 grd + o.b1[b], s));
        HIPCHK(net, conv(b, 0, 1, F(dsb), dn, nullptr, du, F(act[b]), 0));              // (du + W1^T ds) at a_b > 0
        std::swap(du, dn);
    }
    HIPCHK(net, launch_stem_grad(du, d_frames, n, h, w, net->cfg.offset, scale, C, grd + o.stem_w, F(gpart),
                                 F(tmp) + 9 * C * C, s));
    HIPCHK(net, hipEventRecord(net->desc_ev[slot], s));
    return DL_OK;
}

}  // namespace

// ---- autotuner with a cache ----
namespace {

std::string tune_key(dl_net *net, int n, int h, int w)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, net->dev) == hipSuccess) arch = prop.gcnArchName;
    std::string k = "arch=" + arch + ";cu=" + std::to_string(net->ncu) + ";C=" + std::to_string(net->C) + ";dil=";
    for (int b = 0; b < net->nb; ++b) k += (b ? "," : "") + std::to_string(net->dil[b]);
    k += ";nh=" + std::to_string(net->nh) + ";prec=" + std::to_string(net->cfg.precision) + ";batch=" +
         std::to_string(n) + "x" + std::to_string(h) + "x" + std::to_string(w);
    return k;
}

// one cache line: {"key": "<key>", "rows": [r0, r1, ...], "strip": s, "ms": t}
bool tune_cache_find(const char *path, const std::string &key, int nb, int *rows, int *strip)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    const std::string want = "{\"key\": \"" + key + "\", \"rows\": [";
    while (!found && std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, want.c_str(), want.size()) != 0) continue;
        const char *q = line + want.size();
        int r[MAXBLK], k = 0;
        bool ok = true;
        for (; k < nb && ok; ++k) {
            char *end = nullptr;
            const long v = std::strtol(q, &end, 10);
            ok = end != q && (v == 4 || v == 8);
            r[k] = (int)v;
            q = end;
            while (*q == ',' || *q == ' ') ++q;
        }
        const char *sp = std::strstr(q, "\"strip\": ");
        if (!ok || *q != ']' || !sp) continue;
        const long sv = std::strtol(sp + 9, nullptr, 10);
        if (sv < 1 || sv > 64) continue;
        for (int b = 0; b < nb; ++b) rows[b] = r[b];
        *strip = (int)sv;
        found = true;
    }
    std::fclose(f);
    return found;
}

}  // namespace

// ============================================================== public ABI
extern "C" {

uint32_t dl_abi_version(void) { return DL_ABI_VERSION; }

int dl_default_config(dl_config *cfg)
{
    if (!cfg) return fail(nullptr, DL_ERR_INVALID_ARG, "cfg is NULL");
    std::memset(cfg, 0, sizeof *cfg);
    cfg->precision = DL_FP32;
    cfg->threshold = 0.3f;
    cfg->gain = 0.5f;
    cfg->offset = 100.f;
    return DL_OK;
}

const char *dl_last_error(const dl_net *net) { return net ? net->err.c_str() : g_err.c_str(); }

// "DLD1": the dense-connection network (header of 80 bytes, see dl_create_net)
static int parse_dense(const unsigned char *b, size_t nbytes, dl_net_info *info, std::vector<float> *params)
{
    if (nbytes < 80) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "weights blob of %zu bytes is shorter than its header", nbytes);
    uint32_t hdr[13];
    std::memcpy(hdr, b + 4, sizeof hdr);
    const uint32_t version = hdr[0], C = hdr[1], nb = hdr[2], L = hdr[3], G = hdr[4];
    float sc[3];
    std::memcpy(sc, b + 56, sizeof sc);
    uint32_t nh, unet;
    std::memcpy(&nh, b + 68, 4);
    std::memcpy(&unet, b + 72, 4);
    if (version != 1) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "unsupported weights version %u", version);
    if (nh != 5 && nh != 10) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "head outputs %u: 5 or 10 supported", nh);
    if (nb < 1 || nb > MAXBLK) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "nblocks %u outside 1..%d", nb, MAXBLK);
    if (unet != 0 && unet != 2) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "U-Net levels %u: 0 or 2 supported", unet);
    if (unet && nb > MAXBLK - 1)    // the U-Net's last convolution takes tile slot nblocks
        return fail(nullptr, DL_ERR_UNSUPPORTED, "a U-Net after %u blocks (at most %d)", nb, MAXBLK - 1);
    if (L < 1 || L > 8) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "layers per block %u outside 1..8", L);
    if (!(C == 16 || C == 32)) return fail(nullptr, DL_ERR_UNSUPPORTED, "dense network with C = %u (16 or 32)", C);
    if (!(G == 16 || G == 32)) return fail(nullptr, DL_ERR_UNSUPPORTED, "dense network with growth %u (16 or 32)", G);
    for (uint32_t k = 0; k < nb; ++k)
        if (hdr[5 + k] < 1 || hdr[5 + k] > 64) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "dilation %u of block %u outside 1..64", hdr[5 + k], k);
    if (!finite_all(sc, 3) || !(sc[0] > 0.f)) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "bad in_scale/z_scale/ph_scale");
    const size_t np = dense_param_count((int)C, (int)nb, (int)L, (int)G, (int)nh, (int)unet);
    if (nbytes != 80 + np * 4)
        return fail(nullptr, DL_ERR_BAD_WEIGHTS, "blob is %zu bytes, expected %zu for a dense network with C=%u, %u "
                    "blocks of %u layers, growth %u", nbytes, 80 + np * 4, C, nb, L, G);
    std::vector<float> tmp(np);
    std::memcpy(tmp.data(), b + 80, np * 4);
    if (!finite_all(tmp.data(), np)) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "weights contain NaN or Inf");
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->C = (int32_t)C;
        info->nblocks = (int32_t)nb;
        int R = 1;
        for (uint32_t k = 0; k < nb; ++k) {
            info->dilation[k] = (int32_t)hdr[5 + k];
            R += (int)L * (int)hdr[5 + k];
        }
        info->in_scale = sc[0];
        info->z_scale = sc[1];
        info->ph_scale = sc[2];
        info->nparams = (int64_t)np;
        info->head_outputs = (int32_t)nh;
        // the U-Net's output reaches 12 pixels into its input (its last 3x3
        // conv, and through pooling and upsampling the level-1 and level-2 ones)
        info->receptive_radius = R + (unet ? 12 : 0);
        info->dense_layers = (int16_t)L;
        info->dense_growth = (int16_t)G;
        info->unet_levels = (int32_t)unet;
    }
    if (params) *params = std::move(tmp);
    return DL_OK;
}

static int parse_weights(const void *weights, size_t nbytes, dl_net_info *info, std::vector<float> *params)
{
    if (!weights) return fail(nullptr, DL_ERR_INVALID_ARG, "weights is NULL");
    const unsigned char *b = static_cast<const unsigned char *>(weights);
    if (nbytes >= 4 && std::memcmp(b, "DLD1", 4) == 0) return parse_dense(b, nbytes, info, params);
    if (nbytes < 64) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "weights blob of %zu bytes is shorter than its header", nbytes);
    if (std::memcmp(b, "DLW1", 4) != 0) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "bad magic (expected DLW1 or DLD1)");
    // header: magic, u32 version, u32 C, u32 nblocks, u32 dilation[8], f32 in_scale,
    // f32 z_scale, f32 ph_scale, u32 head outputs (0 = 5)
    uint32_t hdr[11];
    std::memcpy(hdr, b + 4, sizeof hdr);
    const uint32_t version = hdr[0], C = hdr[1], nb = hdr[2];
    float sc[3];
    std::memcpy(sc, b + 4 + 11 * 4, sizeof sc);
    if (version != 1) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "unsupported weights version %u", version);
    uint32_t nh_word;                                  // the header's last word (byte 60)
    std::memcpy(&nh_word, b + 60, 4);
    const uint32_t nh = nh_word == 0 ? 5u : nh_word;
    if (nh != 5 && nh != 10) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "head outputs %u: 5 or 10 supported", nh);
    if (nb < 1 || nb > 8) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "nblocks %u outside 1..8", nb);
    if (!(C == 16 || C == 32 || C == 48 || C == 64))
        return fail(nullptr, DL_ERR_UNSUPPORTED, "C = %u not supported (16, 32, 48 or 64)", C);
    for (uint32_t k = 0; k < nb; ++k)
        if (hdr[3 + k] < 1 || hdr[3 + k] > 64) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "dilation %u of block %u outside 1..64", hdr[3 + k], k);
    if (!finite_all(sc, 3) || !(sc[0] > 0.f)) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "bad in_scale/z_scale/ph_scale");
    const size_t np = param_count((int)C, (int)nb, (int)nh);
    if (nbytes != 64 + np * 4)
        return fail(nullptr, DL_ERR_BAD_WEIGHTS, "blob is %zu bytes, expected %zu for C=%u, %u blocks", nbytes, 64 + np * 4, C, nb);
    std::vector<float> tmp(np);
    std::memcpy(tmp.data(), b + 64, np * 4);
    if (!finite_all(tmp.data(), np)) return fail(nullptr, DL_ERR_BAD_WEIGHTS, "weights contain NaN or Inf");
    if (info) {
        std::memset(info, 0, sizeof *info);
        info->C = (int32_t)C;
        info->nblocks = (int32_t)nb;
        for (uint32_t k = 0; k < nb; ++k) info->dilation[k] = (int32_t)hdr[3 + k];
        info->in_scale = sc[0];
        info->z_scale = sc[1];
        info->ph_scale = sc[2];
        info->nparams = (int64_t)np;
        info->head_outputs = (int32_t)nh;
        int R = 1;
        for (uint32_t k = 0; k < nb; ++k) R += 2 * (int)hdr[3 + k];
        info->receptive_radius = R;
    }
    if (params) *params = std::move(tmp);
    return DL_OK;
}

int dl_inspect_weights(const void *weights, size_t nbytes, dl_net_info *info)
{
    if (!info) return fail(nullptr, DL_ERR_INVALID_ARG, "info is NULL");
    return parse_weights(weights, nbytes, info, nullptr);
}

int dl_create_net(const void *weights, size_t nbytes, const dl_config *cfg, dl_net **out)
{
    if (!out) return fail(nullptr, DL_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!weights) return fail(nullptr, DL_ERR_INVALID_ARG, "weights is NULL");
    dl_config c;
    dl_default_config(&c);
    if (cfg) c = *cfg;
    int rc = check_config(nullptr, &c);
    if (rc) return rc;
    dl_net_info info;
    std::vector<float> params;
    if ((rc = parse_weights(weights, nbytes, &info, &params))) return rc;
    if (c.max_sigma_px > 0.f && info.head_outputs != 10)
        return fail(nullptr, DL_ERR_UNSUPPORTED, "max_sigma_px needs a network with the uncertainty head");
    const bool dense = info.dense_layers > 0;
    if (dense && (rc = check_dense_config(nullptr, &c))) return rc;
    if (!dense && c.tile_queue)
        return fail(nullptr, DL_ERR_UNSUPPORTED, "tile_queue applies to the dense-connection kernels only");
    if (!dense && !conv_supported(info.C, c.precision, info.head_outputs))
        return fail(nullptr, DL_ERR_UNSUPPORTED, "C = %d does not fit the %s conv kernel's LDS", info.C,
                    c.precision == DL_FP32 ? "FP32" : c.precision == DL_BF16 ? "BF16" : c.precision == DL_FP8 ? "FP8"
                                                                                                           : "BF16X3");
    const uint32_t C = (uint32_t)info.C, nb = (uint32_t)info.nblocks;

    // ---- arguments are valid; device work starts here ----
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(nullptr, DL_ERR_DEVICE, "no HIP device: %s", hipGetErrorString(e));
    if (c.device >= ndev) return fail(nullptr, DL_ERR_INVALID_ARG, "device %d >= device count %d", c.device, ndev);

    dl_net *net = new (std::nothrow) dl_net();
    if (!net) return fail(nullptr, DL_ERR_OOM, "out of host memory");
    net->cfg = c;
    net->dev = c.device;
    net->C = (int)C;
    net->nb = (int)nb;
    for (uint32_t k = 0; k < nb; ++k) net->dil[k] = info.dilation[k];
    net->in_scale = info.in_scale;
    net->z_scale = info.z_scale;
    net->ph_scale = info.ph_scale;
    net->nh = info.head_outputs;
    net->dL = info.dense_layers;
    net->dG = info.dense_growth;
    net->unet = info.unet_levels;
    net->params = std::move(params);

    auto bail = [&](int code) {
        g_err = net->err;
        dl_destroy_net(net);
        return code;
    };
    if ((rc = set_device(net))) return bail(rc);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, net->dev) == hipSuccess) net->ncu = prop.multiProcessorCount;
    const float *p = net->params.data();
    const size_t nstem = (size_t)C * 9 + C, nhead = (size_t)net->nh * C + net->nh;
    if (hipMalloc(&net->d_stem, nstem * 4) != hipSuccess || hipMalloc(&net->d_head, nhead * 4) != hipSuccess ||
        (!dense && hipMalloc(&net->d_bias, (size_t)nb * 2 * C * 4) != hipSuccess))
        return bail(fail(net, DL_ERR_OOM, "hipMalloc of weights failed"));
    if (hipMemcpy(net->d_stem, p, nstem * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->d_head, p + net->params.size() - nhead, nhead * 4, hipMemcpyHostToDevice) != hipSuccess)
        return bail(fail(net, DL_ERR_DEVICE, "weight upload failed"));
    if (!dense) {
        std::vector<float> bias((size_t)nb * 2 * C);
        const float *q = p + nstem;
        for (uint32_t k = 0; k < nb; ++k)
            for (int j = 0; j < 2; ++j) {
                q += (size_t)C * C * 9;
                std::memcpy(bias.data() + (size_t)(k * 2 + j) * C, q, C * 4);
                q += C;
            }
        if (hipMemcpy(net->d_bias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(net, DL_ERR_DEVICE, "bias upload failed"));
    }
    for (int i = 0; i < DESC_SLOTS; ++i)
        if (hipEventCreateWithFlags(&net->desc_ev[i], hipEventDisableTiming) != hipSuccess)
            return bail(fail(net, DL_ERR_DEVICE, "hipEventCreate failed"));
    if (hipEventCreateWithFlags(&net->ws_ev, hipEventDisableTiming) != hipSuccess)
        return bail(fail(net, DL_ERR_DEVICE, "hipEventCreate failed"));
    // the allocation-free entry point's memory: the device's scratch array
    // and a descriptor ring for DL_NOALLOC_MAX_FRAMES frames
    if ((rc = scratch_init(net))) return bail(rc);
    if ((rc = grow_desc(net, DL_NOALLOC_MAX_FRAMES * desc_per_frame(net)))) return bail(rc);
    if (hipStreamCreateWithFlags(&net->copy_stream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&net->compute_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(net, DL_ERR_DEVICE, "hipStreamCreate failed"));
    {
        // remaining receptive radius after each layer: stem, then every conv
        std::vector<int> rad(1 + 2 * nb);
        int r = 0;
        for (int b = (int)nb - 1; b >= 0; --b) {
            rad[1 + 2 * b + 1] = r;
            r += net->dil[b];
            rad[1 + 2 * b] = r;
            r += net->dil[b];
        }
        rad[0] = r;
        if (hipMalloc(&net->d_radius, rad.size() * sizeof(int)) != hipSuccess ||
            hipMemcpy(net->d_radius, rad.data(), rad.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
            hipMalloc(&net->d_dil, nb * sizeof(int)) != hipSuccess ||
            hipMemcpy(net->d_dil, net->dil, nb * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(net, DL_ERR_DEVICE, "radius upload failed"));
    }
    if ((rc = ensure_packed(net))) return bail(rc);
    *out = net;
    return DL_OK;
}

void dl_destroy_net(dl_net *net)
{
    if (!net) return;
    (void)hipSetDevice(net->dev);
    (void)hipDeviceSynchronize();
    for (auto &e : net->prof_pending) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto e : net->ev_pool) (void)hipEventDestroy(e);
    if (net->ws) (void)hipFree(net->ws);
    if (net->d_stem) (void)hipFree(net->d_stem);
    if (net->d_head) (void)hipFree(net->d_head);
    if (net->d_bias) (void)hipFree(net->d_bias);
    if (net->d_wpk) (void)hipFree(net->d_wpk);
    if (net->d_dense) (void)hipFree(net->d_dense);
    for (float *q : {net->t_params, net->t_grad, net->t_m, net->t_v, net->t_pack})
        if (q) (void)hipFree(q);
    if (net->t_jobs) (void)hipFree(net->t_jobs);
    if (net->t_ws) (void)hipFree(net->t_ws);
    if (net->d_gate_theta) (void)hipFree(net->d_gate_theta);
    if (net->d_radius) (void)hipFree(net->d_radius);
    if (net->d_dil) (void)hipFree(net->d_dil);
    if (net->d_wscale) (void)hipFree(net->d_wscale);
    if (net->h_desc) (void)hipHostFree(net->h_desc);
    if (net->d_desc) (void)hipFree(net->d_desc);
    for (int i = 0; i < DESC_SLOTS; ++i)
        if (net->desc_ev[i]) (void)hipEventDestroy(net->desc_ev[i]);
    if (net->ws_ev) (void)hipEventDestroy(net->ws_ev);
    for (int i = 0; i < 2; ++i) {
        if (net->pl_frames[i]) (void)hipFree(net->pl_frames[i]);
        if (net->pl_stage[i]) (void)hipHostFree(net->pl_stage[i]);
        if (net->pl_out[i]) (void)hipFree(net->pl_out[i]);
        if (net->pl_unc[i]) (void)hipFree(net->pl_unc[i]);
        for (hipEvent_t e : {net->pl_copied[i], net->pl_used[i], net->pl_counted[i]})
            if (e) (void)hipEventDestroy(e);
    }
    if (net->pl_dcounts) (void)hipFree(net->pl_dcounts);
    if (net->pl_maps) (void)hipFree(net->pl_maps);
    if (net->pl_hcounts) (void)hipHostFree(net->pl_hcounts);
    if (net->d_cam) (void)hipFree(net->d_cam);
    if (net->copy_stream) (void)hipStreamDestroy(net->copy_stream);
    if (net->compute_stream) (void)hipStreamDestroy(net->compute_stream);
    delete net;
}

int dl_set_config(dl_net *net, const dl_config *cfg)
{
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    if (!cfg) return fail(net, DL_ERR_INVALID_ARG, "cfg is NULL");
    int rc = check_config(net, cfg);
    if (rc) return rc;
    if (cfg->device != net->cfg.device) return fail(net, DL_ERR_INVALID_ARG, "device cannot change");
    if (cfg->max_sigma_px > 0.f && net->nh != 10)
        return fail(net, DL_ERR_UNSUPPORTED, "max_sigma_px needs a network with the uncertainty head");
    if (net->dL && (rc = check_dense_config(net, cfg))) return rc;
    if (!net->dL && cfg->tile_queue)
        return fail(net, DL_ERR_UNSUPPORTED, "tile_queue applies to the dense-connection kernels only");
    if (!net->dL && !conv_supported(net->C, cfg->precision, net->nh))
        return fail(net, DL_ERR_UNSUPPORTED, "C = %d does not fit this form's conv kernel", net->C);
    const float new_scale = cfg->in_scale_override > 0.f ? cfg->in_scale_override : net->in_scale;
    if (net->d_cam && new_scale != in_scale_of(net))
        return fail(net, DL_ERR_INVALID_ARG, "the input scaling cannot change while camera maps are set (clear them first)");
    const int old = net->cfg.precision;
    net->cfg = *cfg;
    if (cfg->precision != old) {
        if ((rc = set_device(net))) return rc;
        if ((rc = ensure_packed(net))) {
            net->cfg.precision = old;
            return rc;
        }
    }
    return DL_OK;
}

int dl_set_camera_maps(dl_net *net, const float *gain, const float *offset, int h, int w)
{
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    if (!gain != !offset) return fail(net, DL_ERR_INVALID_ARG, "give both camera maps or neither");
    if (gain && (h <= 0 || w <= 0 || (int64_t)h * w > ((int64_t)1 << 28)))
        return fail(net, DL_ERR_INVALID_ARG, "camera maps must be h x w with 0 < h * w <= 2^28 (got %d x %d)", h, w);
    if (gain && net->dL)
        return fail(net, DL_ERR_UNSUPPORTED, "camera maps do not apply to the dense-connection network");
    int rc;
    if ((rc = set_device(net))) return rc;
    auto clear = [&]() {
        if (net->d_cam) (void)hipFree(net->d_cam);
        net->d_cam = nullptr;
        net->cam_h = net->cam_w = 0;
        ++net->cam_gen;
    };
    if (!gain) {
        if (net->d_cam) {
            HIPCHK(net, hipDeviceSynchronize());
            clear();
        }
        return DL_OK;
    }
    const size_t npx = (size_t)h * w;
    std::vector<float2> host(npx);
    for (size_t p = 0; p < npx; ++p) {
        if (!std::isfinite(gain[p]) || !(gain[p] > 0.f) || !std::isfinite(offset[p]))
            return fail(net, DL_ERR_INVALID_ARG, "camera map pixel %zu: gain must be finite and > 0, offset finite", p);
        host[p] = make_float2(offset[p], gain[p] * in_scale_of(net));   // the scalar path's FP32 product
    }
    HIPCHK(net, hipDeviceSynchronize());        // nothing in flight still reads the old maps
    if (!net->d_cam || h != net->cam_h || w != net->cam_w) {
        clear();
        if (hipMalloc(&net->d_cam, npx * sizeof(float2)) != hipSuccess) {
            (void)hipGetLastError();
            net->d_cam = nullptr;
            return fail(net, DL_ERR_OOM, "hipMalloc for %d x %d camera maps failed", h, w);
        }
        net->cam_h = h;
        net->cam_w = w;
    }
    hipError_t e = hipMemcpy(net->d_cam, host.data(), npx * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        clear();
        return fail(net, DL_ERR_DEVICE, "camera map upload failed: %s", hipGetErrorString(e));
    }
    return DL_OK;
}

int dl_localize_device(dl_net *net, const uint16_t *d_frames, int n, int h, int w, void *stream,
                       dl_emitter *d_out, size_t cap, uint32_t *d_counts)
{
    int rc = check_uniform(net, d_frames, n, h, w);
    if (rc) return rc;
    if (!d_counts) return fail(net, DL_ERR_INVALID_ARG, "d_counts is NULL");
    if (cap > 0 && !d_out) return fail(net, DL_ERR_INVALID_ARG, "d_out is NULL with cap > 0");
    if (reinterpret_cast<uintptr_t>(d_out) % 16 || reinterpret_cast<uintptr_t>(d_counts) % 4)
        return fail(net, DL_ERR_INVALID_ARG, "d_out must be 16-byte and d_counts 4-byte aligned");
    std::vector<FrameDesc> fd;
    Geometry g;
    uniform_geometry(net, d_frames, n, h, w, fd, g);
    return localize_geom(net, fd, g, static_cast<hipStream_t>(stream), d_out, cap, d_counts, nullptr, d_frames, n, h, w);
}

int dl_localize_device_unc(dl_net *net, const uint16_t *d_frames, int n, int h, int w, void *stream,
                           dl_emitter *d_out, dl_uncertainty *d_unc, size_t cap, uint32_t *d_counts)
{
    int rc = check_uniform(net, d_frames, n, h, w);
    if (rc) return rc;
    if (net->nh != 10) return fail(net, DL_ERR_UNSUPPORTED, "the network has no uncertainty head (%d outputs)", net->nh);
    if (!d_counts) return fail(net, DL_ERR_INVALID_ARG, "d_counts is NULL");
    if (cap > 0 && (!d_out || !d_unc)) return fail(net, DL_ERR_INVALID_ARG, "d_out or d_unc is NULL with cap > 0");
    if (reinterpret_cast<uintptr_t>(d_out) % 16 || reinterpret_cast<uintptr_t>(d_counts) % 4 ||
        reinterpret_cast<uintptr_t>(d_unc) % 4)
        return fail(net, DL_ERR_INVALID_ARG, "d_out must be 16-byte, d_unc and d_counts 4-byte aligned");
    std::vector<FrameDesc> fd;
    Geometry g;
    uniform_geometry(net, d_frames, n, h, w, fd, g);
    return localize_geom(net, fd, g, static_cast<hipStream_t>(stream), d_out, cap, d_counts, nullptr, d_frames, n, h, w,
                         cap ? d_unc : nullptr);
}

int dl_localize_device_noalloc(dl_net *net, const uint16_t *d_frames, int n, int h, int w, void *stream,
                               dl_emitter *d_out, size_t cap, uint32_t *d_counts)
{
    int rc = check_uniform(net, d_frames, n, h, w);
    if (rc) return rc;
    if (!d_counts) return fail(net, DL_ERR_INVALID_ARG, "d_counts is NULL");
    if (cap > 0 && !d_out) return fail(net, DL_ERR_INVALID_ARG, "d_out is NULL with cap > 0");
    if (reinterpret_cast<uintptr_t>(d_out) % 16 || reinterpret_cast<uintptr_t>(d_counts) % 4)
        return fail(net, DL_ERR_INVALID_ARG, "d_out must be 16-byte and d_counts 4-byte aligned");
    if ((int64_t)n * desc_per_frame(net) > net->desc_cap)
        return fail(net, DL_ERR_UNSUPPORTED, "at most %d frames per allocation-free call (got %d)",
                    net->desc_cap / desc_per_frame(net), n);
    if (gated_run(net)) return fail(net, DL_ERR_UNSUPPORTED, "gated runs need the handle's workspace");
    if (net->packed_precision != net->cfg.precision || !net->scratch)
        return fail(net, DL_ERR_DEVICE, "the handle's weights or scratch memory are not set up");
    std::vector<FrameDesc> fd;
    Geometry g;
    uniform_geometry(net, d_frames, n, h, w, fd, g);
    const bool prof = net->profiling;
    net->profiling = false;            // timing events may need creating
    rc = localize_geom(net, fd, g, static_cast<hipStream_t>(stream), d_out, cap, d_counts, nullptr, d_frames, n, h, w,
                       nullptr, net->scratch, DL_NOALLOC_SCRATCH_BYTES);
    net->profiling = prof;
    return rc;
}

int dl_maps_device(dl_net *net, const uint16_t *d_frames, int n, int h, int w, void *stream, float *d_maps)
{
    int rc = check_uniform(net, d_frames, n, h, w);
    if (rc) return rc;
    if (!d_maps) return fail(net, DL_ERR_INVALID_ARG, "d_maps is NULL");
    if (reinterpret_cast<uintptr_t>(d_maps) % 4) return fail(net, DL_ERR_INVALID_ARG, "d_maps must be 4-byte aligned");
    std::vector<FrameDesc> fd;
    Geometry g;
    uniform_geometry(net, d_frames, n, h, w, fd, g);
    return localize_geom(net, fd, g, static_cast<hipStream_t>(stream), nullptr, 0, nullptr, d_maps, d_frames, n, h, w);
}

static int check_rois(dl_net *net, const dl_roi *rois, int nroi)
{
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    if (!rois || nroi <= 0) return fail(net, DL_ERR_INVALID_ARG, "rois is NULL or nroi <= 0");
    int64_t rows = 0;
    for (int k = 0; k < nroi; ++k) {
        const dl_roi &r = rois[k];
        if (!r.data || reinterpret_cast<uintptr_t>(r.data) % 2) return fail(net, DL_ERR_INVALID_ARG, "roi %d: NULL or misaligned data", k);
        if (r.h <= 0 || r.w <= 0) return fail(net, DL_ERR_INVALID_ARG, "roi %d: h and w must be > 0", k);
        if (r.row_stride < r.w) return fail(net, DL_ERR_INVALID_ARG, "roi %d: row_stride < w", k);
        if ((int64_t)r.h * r.w > (int64_t)1 << 28 || !frame_act_fits(net, r.h, r.w))
            return fail(net, DL_ERR_UNSUPPORTED, "roi %d too large", k);
        rows += r.h;
    }
    if (rows > (int64_t)1 << 30) return fail(net, DL_ERR_UNSUPPORTED, "too many rows in the batch");
    return DL_OK;
}

static void roi_geometry(dl_net *net, const dl_roi *rois, int nroi, std::vector<FrameDesc> &fd, Geometry &g)
{
    std::vector<int> hs(nroi), ws(nroi);
    std::vector<const uint16_t *> ptr(nroi);
    std::vector<int64_t> st(nroi);
    for (int k = 0; k < nroi; ++k) {
        hs[k] = rois[k].h;
        ws[k] = rois[k].w;
        ptr[k] = rois[k].data;
        st[k] = rois[k].row_stride;
    }
    build_geometry(net, nroi, hs.data(), ws.data(), ptr.data(), st.data(), fd, g);
}

int dl_localize_rois_device(dl_net *net, const dl_roi *rois, int nroi, void *stream, dl_emitter *d_out,
                            size_t cap, uint32_t *d_counts)
{
    int rc = check_rois(net, rois, nroi);
    if (rc) return rc;
    if (!d_counts) return fail(net, DL_ERR_INVALID_ARG, "d_counts is NULL");
    if (cap > 0 && !d_out) return fail(net, DL_ERR_INVALID_ARG, "d_out is NULL with cap > 0");
    std::vector<FrameDesc> fd;
    Geometry g;
    roi_geometry(net, rois, nroi, fd, g);
    return localize_geom(net, fd, g, static_cast<hipStream_t>(stream), d_out, cap, d_counts, nullptr);
}

int dl_localize_rois_device_unc(dl_net *net, const dl_roi *rois, int nroi, void *stream, dl_emitter *d_out,
                                dl_uncertainty *d_unc, size_t cap, uint32_t *d_counts)
{
    int rc = check_rois(net, rois, nroi);
    if (rc) return rc;
    if (net->nh != 10) return fail(net, DL_ERR_UNSUPPORTED, "the network has no uncertainty head (%d outputs)", net->nh);
    if (!d_counts) return fail(net, DL_ERR_INVALID_ARG, "d_counts is NULL");
    if (cap > 0 && (!d_out || !d_unc)) return fail(net, DL_ERR_INVALID_ARG, "d_out or d_unc is NULL with cap > 0");
    if (reinterpret_cast<uintptr_t>(d_unc) % 4) return fail(net, DL_ERR_INVALID_ARG, "d_unc must be 4-byte aligned");
    std::vector<FrameDesc> fd;
    Geometry g;
    roi_geometry(net, rois, nroi, fd, g);
    return localize_geom(net, fd, g, static_cast<hipStream_t>(stream), d_out, cap, d_counts, nullptr, nullptr, 0, 0, 0,
                         cap ? d_unc : nullptr);
}

int dl_maps_rois_device(dl_net *net, const dl_roi *rois, int nroi, void *stream, float *d_maps)
{
    int rc = check_rois(net, rois, nroi);
    if (rc) return rc;
    if (!d_maps) return fail(net, DL_ERR_INVALID_ARG, "d_maps is NULL");
    std::vector<FrameDesc> fd;
    Geometry g;
    roi_geometry(net, rois, nroi, fd, g);
    return localize_geom(net, fd, g, static_cast<hipStream_t>(stream), nullptr, 0, nullptr, d_maps);
}

int dl_host_alloc(size_t bytes, void **p)
{
    if (!p) return fail(nullptr, DL_ERR_INVALID_ARG, "p is NULL");
    *p = nullptr;
    if (bytes == 0) return fail(nullptr, DL_ERR_INVALID_ARG, "bytes is 0");
    hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(nullptr, DL_ERR_OOM, "hipHostMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    return DL_OK;
}

void dl_host_free(void *p)
{
    if (p) (void)hipHostFree(p);
}

static bool is_pinned(const void *p)
{
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeHost;
}

// Grow the pipeline's slot buffers to hold batches of `fbytes` frame bytes,
// `out_cap` records and n + 1 counts.  Waits for all work on the device before
// it frees anything.
static int ensure_pipeline(dl_net *net, size_t fbytes, bool staged, size_t out_cap, int n, bool unc)
{
    const bool grow = fbytes > net->pl_frame_bytes || (staged && fbytes > net->pl_stage_bytes) ||
                      out_cap > net->pl_out_cap || n + 1 > net->pl_counts_n || (unc && out_cap > net->pl_unc_cap);
    if (!grow && net->pl_copied[0]) return DL_OK;
    HIPCHK(net, hipDeviceSynchronize());
    for (int i = 0; i < 2; ++i) {
        if (!net->pl_copied[i]) {
            HIPCHK(net, hipEventCreateWithFlags(&net->pl_copied[i], hipEventDisableTiming));
            HIPCHK(net, hipEventCreateWithFlags(&net->pl_used[i], hipEventDisableTiming));
            HIPCHK(net, hipEventCreateWithFlags(&net->pl_counted[i], hipEventDisableTiming));
        }
    }
    if (fbytes > net->pl_frame_bytes) {
        net->pl_frame_bytes = 0;
        for (auto &p : net->pl_frames) HIPCHK(net, free_dev(p));
        for (auto &p : net->pl_frames)
            if (hipMalloc(&p, fbytes) != hipSuccess) {
                (void)hipGetLastError();
                return fail(net, DL_ERR_OOM, "hipMalloc(%zu) for a frame slot failed", fbytes);
            }
        net->pl_frame_bytes = fbytes;
    }
    if (staged && fbytes > net->pl_stage_bytes) {
        net->pl_stage_bytes = 0;
        for (auto &p : net->pl_stage) HIPCHK(net, free_host(p));
        for (auto &p : net->pl_stage)
            if (hipHostMalloc((void **)&p, fbytes, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return fail(net, DL_ERR_OOM, "hipHostMalloc(%zu) for a staging slot failed", fbytes);
            }
        net->pl_stage_bytes = fbytes;
    }
    if (out_cap > net->pl_out_cap) {
        net->pl_out_cap = 0;
        for (auto &p : net->pl_out) HIPCHK(net, free_dev(p));
        for (auto &p : net->pl_out)
            if (hipMalloc(&p, out_cap * sizeof(dl_emitter)) != hipSuccess) {
                (void)hipGetLastError();
                return fail(net, DL_ERR_OOM, "hipMalloc for %zu records failed", out_cap);
            }
        net->pl_out_cap = out_cap;
    }
    if (unc && out_cap > net->pl_unc_cap) {
        net->pl_unc_cap = 0;
        for (auto &p : net->pl_unc) HIPCHK(net, free_dev(p));
        for (auto &p : net->pl_unc)
            if (hipMalloc(&p, out_cap * sizeof(dl_uncertainty)) != hipSuccess) {
                (void)hipGetLastError();
                return fail(net, DL_ERR_OOM, "hipMalloc for %zu record uncertainties failed", out_cap);
            }
        net->pl_unc_cap = out_cap;
    }
    if (n + 1 > net->pl_counts_n) {
        const hipError_t ed = free_dev(net->pl_dcounts), eh = free_host(net->pl_hcounts);
        net->pl_counts_n = 0;
        HIPCHK(net, ed);
        HIPCHK(net, eh);
        HIPCHK(net, hipMalloc(&net->pl_dcounts, (size_t)2 * (n + 1) * 4));
        HIPCHK(net, hipHostMalloc((void **)&net->pl_hcounts, (size_t)2 * (n + 1) * 4, hipHostMallocDefault));
        net->pl_counts_n = n + 1;
    }
    return DL_OK;
}

// Host-frame localization of nbatch batches (unc: the records'
// uncertainties too, for 10-output nets; else null).
static int localize_pipelined(dl_net *net, const uint16_t *frames, int nbatch, int n, int h, int w, int overlap,
                              dl_emitter *out, dl_uncertainty *unc, size_t cap, size_t *count)
{
    int rc = check_uniform(net, frames, n, h, w);
    if (rc) return rc;
    if (nbatch <= 0) return fail(net, DL_ERR_INVALID_ARG, "nbatch must be > 0");
    if (!count) return fail(net, DL_ERR_INVALID_ARG, "count is NULL");
    if (cap > 0 && !out) return fail(net, DL_ERR_INVALID_ARG, "out is NULL with cap > 0");
    if ((rc = set_device(net))) return rc;
    *count = 0;
    const size_t fbytes = (size_t)n * h * w * 2;
    const bool pinned = is_pinned(frames);
    // a batch yields at most one record per pixel
    const size_t slot_cap = std::max<size_t>(1, std::min<size_t>(cap, (size_t)n * h * w));
    if ((rc = ensure_pipeline(net, fbytes, !pinned, slot_cap, n, unc != nullptr))) return rc;

    // Slot k & 1 holds batch k's frames, records and counts.  With overlap the
    // copy of batch k (copy stream) waits on the device for the compute that
    // last read its slot, the compute of batch k waits for that copy, and the
    // host collects batch k - 1 only after batch k is queued, so the compute
    // stream never waits for the host.  Without overlap every batch is copied,
    // processed and collected before the next one starts.
    hipStream_t cs = net->compute_stream, xs = overlap ? net->copy_stream : net->compute_stream;
    const size_t cn = (size_t)n + 1;
    size_t written = 0;        // records copied to `out` so far
    size_t total = 0;
    int result = DL_OK;
    auto drain = [&]() {
        (void)hipStreamSynchronize(cs);
        (void)hipStreamSynchronize(xs);
    };
#define PCHK(expr)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) {                                                                     \
            result = fail(net, DL_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
            drain();                                                                                \
            return result;                                                                          \
        }                                                                                           \
    } while (0)
    // Copy batch j's records to the host: the counts are in pinned memory once
    // its compute has finished; the first min(total, room) records are the
    // same whatever room the kernels were given (they are placed by prefix).
    auto collect = [&](int j) -> int {
        const int sl = j & 1;
        PCHK(hipEventSynchronize(net->pl_counted[sl]));
        const uint32_t tot = net->pl_hcounts[sl * cn + n];
        const size_t take = std::min<size_t>(tot, cap - written);
        if (take) {
            PCHK(hipMemcpyAsync(out + written, net->pl_out[sl], take * sizeof(dl_emitter), hipMemcpyDeviceToHost, xs));
            if (unc)
                PCHK(hipMemcpyAsync(unc + written, net->pl_unc[sl], take * sizeof(dl_uncertainty),
                                    hipMemcpyDeviceToHost, xs));
            PCHK(hipStreamSynchronize(xs));
            for (size_t r = 0; r < take; ++r) out[written + r].frame += j * n;
        }
        written += take;
        total += tot;
        return DL_OK;
    };
    for (int k = 0; k < nbatch; ++k) {
        const int sl = k & 1;
        const uint16_t *src = frames + (size_t)k * n * h * w;
        if (!pinned) {
            PCHK(hipEventSynchronize(net->pl_copied[sl]));   // batch k - 2's copy out of this stage is done
            std::memcpy(net->pl_stage[sl], src, fbytes);
            src = net->pl_stage[sl];
        }
        if (xs != cs) PCHK(hipStreamWaitEvent(xs, net->pl_used[sl], 0));
        PCHK(hipMemcpyAsync(net->pl_frames[sl], src, fbytes, hipMemcpyHostToDevice, xs));
        PCHK(hipEventRecord(net->pl_copied[sl], xs));
        if (xs != cs) PCHK(hipStreamWaitEvent(cs, net->pl_copied[sl], 0));
        std::vector<FrameDesc> fd;
        Geometry g;
        uniform_geometry(net, net->pl_frames[sl], n, h, w, fd, g);
        // an upper bound on the room left: batches not yet collected take none
        const size_t room = std::min(slot_cap, cap - std::min(cap, written));
        rc = localize_geom(net, fd, g, cs, room ? net->pl_out[sl] : nullptr, room, net->pl_dcounts + sl * cn,
                           nullptr, net->pl_frames[sl], n, h, w, unc && room ? net->pl_unc[sl] : nullptr);
        if (rc) { drain(); return rc; }
        PCHK(hipEventRecord(net->pl_used[sl], cs));
        PCHK(hipMemcpyAsync(net->pl_hcounts + sl * cn, net->pl_dcounts + sl * cn, cn * 4, hipMemcpyDeviceToHost, cs));
        PCHK(hipEventRecord(net->pl_counted[sl], cs));
        if (!overlap) {
            if ((rc = collect(k))) return rc;
        } else if (k > 0) {
            if ((rc = collect(k - 1))) return rc;
        }
    }
    if (overlap && (rc = collect(nbatch - 1))) return rc;
#undef PCHK
    *count = total;
    if (total > cap) return fail(net, DL_ERR_CAPACITY, "%zu emitters exceed capacity %zu", total, cap);
    return DL_OK;
}

int dl_localize_pipelined(dl_net *net, const uint16_t *frames, int nbatch, int n, int h, int w, int overlap,
                          dl_emitter *out, size_t cap, size_t *count)
{
    return localize_pipelined(net, frames, nbatch, n, h, w, overlap, out, nullptr, cap, count);
}

int dl_localize_pipelined_unc(dl_net *net, const uint16_t *frames, int nbatch, int n, int h, int w, int overlap,
                              dl_emitter *out, dl_uncertainty *unc, size_t cap, size_t *count)
{
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    if (net->nh != 10) return fail(net, DL_ERR_UNSUPPORTED, "the network has no uncertainty head (%d outputs)", net->nh);
    if (cap > 0 && !unc) return fail(net, DL_ERR_INVALID_ARG, "unc is NULL with cap > 0");
    return localize_pipelined(net, frames, nbatch, n, h, w, overlap, out, cap ? unc : nullptr, cap, count);
}

int dl_localize(dl_net *net, const uint16_t *frames, int n, int h, int w, dl_emitter *out, size_t cap, size_t *count)
{
    return localize_pipelined(net, frames, 1, n, h, w, 0, out, nullptr, cap, count);
}

int dl_localize_unc(dl_net *net, const uint16_t *frames, int n, int h, int w, dl_emitter *out, dl_uncertainty *unc,
                    size_t cap, size_t *count)
{
    return dl_localize_pipelined_unc(net, frames, 1, n, h, w, 0, out, unc, cap, count);
}

int dl_localize_rois(dl_net *net, const dl_roi *rois, int nroi, dl_emitter *out, size_t cap, size_t *count)
{
    int rc = check_rois(net, rois, nroi);
    if (rc) return rc;
    if (!count) return fail(net, DL_ERR_INVALID_ARG, "count is NULL");
    if (cap > 0 && !out) return fail(net, DL_ERR_INVALID_ARG, "out is NULL with cap > 0");
    if ((rc = check_camera(net, false, 0, 0))) return rc;
    if ((rc = set_device(net))) return rc;
    *count = 0;
    size_t px = 0;
    for (int k = 0; k < nroi; ++k) px += (size_t)rois[k].h * rois[k].w;
    const size_t slot_cap = std::max<size_t>(1, std::min(cap, px));
    if ((rc = ensure_pipeline(net, px * 2, false, slot_cap, nroi, false))) return rc;
    hipStream_t cs = net->compute_stream;
    // the ROIs, packed densely one after another into the frame slot
    std::vector<dl_roi> dev(nroi);
    size_t off = 0;
    for (int k = 0; k < nroi; ++k) {
        const dl_roi &r = rois[k];
        uint16_t *dst = net->pl_frames[0] + off;
        HIPCHK(net, hipMemcpy2DAsync(dst, (size_t)r.w * 2, r.data, (size_t)r.row_stride * 2, (size_t)r.w * 2, r.h,
                                     hipMemcpyHostToDevice, cs));
        dev[k] = dl_roi{dst, r.h, r.w, r.w};
        off += (size_t)r.h * r.w;
    }
    std::vector<FrameDesc> fd;
    Geometry g;
    roi_geometry(net, dev.data(), nroi, fd, g);
    uint32_t *dc = net->pl_dcounts;
    if ((rc = localize_geom(net, fd, g, cs, cap ? net->pl_out[0] : nullptr, cap ? slot_cap : 0, dc, nullptr))) return rc;
    HIPCHK(net, hipMemcpyAsync(net->pl_hcounts, dc, (size_t)(nroi + 1) * 4, hipMemcpyDeviceToHost, cs));
    HIPCHK(net, hipStreamSynchronize(cs));
    const size_t total = net->pl_hcounts[nroi];
    const size_t take = std::min(total, cap);
    if (take) {
        HIPCHK(net, hipMemcpyAsync(out, net->pl_out[0], take * sizeof(dl_emitter), hipMemcpyDeviceToHost, cs));
        HIPCHK(net, hipStreamSynchronize(cs));
    }
    *count = total;
    if (total > cap) return fail(net, DL_ERR_CAPACITY, "%zu emitters exceed capacity %zu", total, cap);
    return DL_OK;
}

int dl_localize_maps(dl_net *net, const uint16_t *frames, int n, int h, int w, float *maps)
{
    int rc = check_uniform(net, frames, n, h, w);
    if (rc) return rc;
    if (!maps) return fail(net, DL_ERR_INVALID_ARG, "maps is NULL");
    if ((rc = set_device(net))) return rc;
    const size_t fbytes = (size_t)n * h * w * 2, mbytes = (size_t)n * net->nh * h * w * 4;
    if ((rc = ensure_pipeline(net, fbytes, false, 1, n, false))) return rc;
    hipStream_t cs = net->compute_stream;
    if (mbytes > net->pl_maps_bytes) {
        HIPCHK(net, hipStreamSynchronize(cs));
        net->pl_maps_bytes = 0;
        HIPCHK(net, free_dev(net->pl_maps));
        if (hipMalloc(&net->pl_maps, mbytes) != hipSuccess) {
            (void)hipGetLastError();
            net->pl_maps = nullptr;
            return fail(net, DL_ERR_OOM, "hipMalloc(%zu) for the maps failed", mbytes);
        }
        net->pl_maps_bytes = mbytes;
    }
    HIPCHK(net, hipMemcpyAsync(net->pl_frames[0], frames, fbytes, hipMemcpyHostToDevice, cs));
    std::vector<FrameDesc> fd;
    Geometry g;
    uniform_geometry(net, net->pl_frames[0], n, h, w, fd, g);
    if ((rc = localize_geom(net, fd, g, cs, nullptr, 0, nullptr, net->pl_maps, net->pl_frames[0], n, h, w))) return rc;
    HIPCHK(net, hipMemcpyAsync(maps, net->pl_maps, mbytes, hipMemcpyDeviceToHost, cs));
    HIPCHK(net, hipStreamSynchronize(cs));
    return DL_OK;
}

int dl_debug_compact(dl_net *net, const uint8_t *d_det, const float *d_maps, int n, int h, int w, void *stream,
                     dl_emitter *d_out, size_t cap, uint32_t *d_counts)
{
    int rc = check_uniform(net, d_det, n, h, w);
    if (rc) return rc;
    if (!d_maps || !d_counts) return fail(net, DL_ERR_INVALID_ARG, "d_maps or d_counts is NULL");
    if (cap > 0 && !d_out) return fail(net, DL_ERR_INVALID_ARG, "d_out is NULL with cap > 0");
    if (reinterpret_cast<uintptr_t>(d_maps) % 4 || reinterpret_cast<uintptr_t>(d_out) % 16 ||
        reinterpret_cast<uintptr_t>(d_counts) % 4)
        return fail(net, DL_ERR_INVALID_ARG, "d_maps and d_counts must be 4-byte, d_out 16-byte aligned");
    if ((rc = set_device(net))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<FrameDesc> fd;
    Geometry g;
    uniform_geometry(net, nullptr, n, h, w, fd, g);
    Plan p = make_plan(net, g, true);
    if ((rc = ensure_workspace(net, p.total, s))) return rc;
    if ((rc = ws_acquire(net, s))) return rc;
    p.ws = net->ws;
    FrameDesc *d_fd = nullptr;
    const int slot = upload_desc(net, fd, s, &d_fd);
    if (slot < 0) return slot;
    uint64_t *mask = reinterpret_cast<uint64_t *>(p.ws + p.mask);
    uint32_t *rcnt = reinterpret_cast<uint32_t *>(p.ws + p.rc);
    uint32_t *roff = reinterpret_cast<uint32_t *>(p.ws + p.roff);
    HIPCHK(net, launch_mask_from_u8(d_det, d_fd, g, mask, rcnt, s));
    HIPCHK(net, launch_scan(rcnt, d_fd, g, roff, d_counts, s));
    HIPCHK(net, launch_emit(d_maps, net->nh, mask, roff, d_fd, g, net->z_scale, net->ph_scale, 1.f / in_scale_of(net),
                            d_out, nullptr, cap, s));
    HIPCHK(net, hipEventRecord(net->desc_ev[slot], s));
    return ws_release(net, s);
}

int dl_debug_conv_layer(dl_net *net, const float *d_in, const float *d_res, int n, int h, int w, int blk,
                        int which, void *stream, float *d_out)
{
    int rc = check_uniform(net, d_in, n, h, w);
    if (rc) return rc;
    if (!d_out) return fail(net, DL_ERR_INVALID_ARG, "d_out is NULL");
    if (net->dL) return fail(net, DL_ERR_UNSUPPORTED, "dl_debug_conv_layer runs the residual network's layers");
    if (blk < 0 || blk >= net->nb || which < 0 || which > 1) return fail(net, DL_ERR_INVALID_ARG, "bad blk/which");
    if (net->cfg.precision != DL_FP32 && net->cfg.precision != DL_BF16X3)
        return fail(net, DL_ERR_UNSUPPORTED, "debug conv layer takes FP32 tensors; set precision FP32 or BF16X3");
    if (reinterpret_cast<uintptr_t>(d_in) % 16 || reinterpret_cast<uintptr_t>(d_out) % 16 ||
        reinterpret_cast<uintptr_t>(d_res) % 16)
        return fail(net, DL_ERR_INVALID_ARG, "tensors must be 16-byte aligned");
    if ((rc = set_device(net))) return rc;
    if ((rc = ensure_packed(net))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<FrameDesc> fd;
    Geometry g;
    uniform_geometry(net, reinterpret_cast<const uint16_t *>(d_in), n, h, w, fd, g);
    for (FrameDesc &d : fd) d.act_off = d.px_off;    // caller tensors: plain NHWC, frame after frame
    FrameDesc *d_fd = nullptr;
    const int slot = upload_desc(net, fd, s, &d_fd);
    if (slot < 0) return slot;
    ConvArgs a{};
    a.fd = d_fd;
    a.in_phase = 0;
    a.out_shift = 0;
    a.d = net->dil[blk];
    a.blk = blk;
    a.in = d_in;
    a.res = d_res;
    a.out = d_out;
    a.wpk = static_cast<char *>(net->d_wpk) + (size_t)(blk * 2 + which) * net->wpk_stride;
    a.bias = net->d_bias + (size_t)(blk * 2 + which) * net->C;
    a.tr = g.trb[blk];
    const int maxg = conv_max_grid(net->C, net->cfg.precision, g.trb[blk], net->ncu);
    int grid = (int)std::min<int64_t>(g.tiles[blk], maxg);
    grid = std::max(8, grid / 8 * 8);
    HIPCHK(net, launch_conv(net->C, net->cfg.precision, a, g, grid, s));
    HIPCHK(net, hipEventRecord(net->desc_ev[slot], s));
    return DL_OK;
}

int dl_debug_detect(dl_net *net, const float *d_logit, int n, int h, int w, float tau, void *stream, uint8_t *d_det)
{
    int rc = check_uniform(net, d_logit, n, h, w);
    if (rc) return rc;
    if (!d_det) return fail(net, DL_ERR_INVALID_ARG, "d_det is NULL");
    if (!std::isfinite(tau)) return fail(net, DL_ERR_INVALID_ARG, "tau must be finite");
    if (reinterpret_cast<uintptr_t>(d_logit) % 4) return fail(net, DL_ERR_INVALID_ARG, "d_logit must be 4-byte aligned");
    if ((rc = set_device(net))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<FrameDesc> fd;
    Geometry g;
    uniform_geometry(net, nullptr, n, h, w, fd, g);
    Plan p = make_plan(net, g, true);
    if ((rc = ensure_workspace(net, p.total, s))) return rc;
    if ((rc = ws_acquire(net, s))) return rc;
    p.ws = net->ws;
    FrameDesc *d_fd = nullptr;
    const int slot = upload_desc(net, fd, s, &d_fd);
    if (slot < 0) return slot;
    uint64_t *mask = reinterpret_cast<uint64_t *>(p.ws + p.mask);
    uint32_t *rcnt = reinterpret_cast<uint32_t *>(p.ws + p.rc);
    HIPCHK(net, launch_detect_mask(d_logit, 1, d_fd, g, tau, INFINITY, nullptr, mask, rcnt, s));
    HIPCHK(net, launch_mask_to_u8(mask, d_fd, g, d_det, s));
    HIPCHK(net, hipEventRecord(net->desc_ev[slot], s));
    return ws_release(net, s);
}

int dl_graph_create(dl_net *net, const uint16_t *d_frames, int n, int h, int w, dl_emitter *d_out, size_t cap,
                    uint32_t *d_counts, dl_graph **out)
{
    if (!out) return fail(net, DL_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_uniform(net, d_frames, n, h, w);
    if (rc) return rc;
    if (!d_counts) return fail(net, DL_ERR_INVALID_ARG, "d_counts is NULL");
    if (cap > 0 && !d_out) return fail(net, DL_ERR_INVALID_ARG, "d_out is NULL with cap > 0");
    if ((rc = check_camera(net, true, h, w))) return rc;
    std::vector<FrameDesc> fd;
    Geometry g;
    uniform_geometry(net, d_frames, n, h, w, fd, g);
    return graph_build(net, fd, g, d_out, cap, d_counts, out);
}

int dl_graph_create_rois(dl_net *net, const dl_roi *rois, int nroi, dl_emitter *d_out, size_t cap, uint32_t *d_counts,
                         dl_graph **out)
{
    if (!out) return fail(net, DL_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = check_rois(net, rois, nroi);
    if (rc) return rc;
    if (!d_counts) return fail(net, DL_ERR_INVALID_ARG, "d_counts is NULL");
    if (cap > 0 && !d_out) return fail(net, DL_ERR_INVALID_ARG, "d_out is NULL with cap > 0");
    if ((rc = check_camera(net, false, 0, 0))) return rc;
    std::vector<FrameDesc> fd;
    Geometry g;
    roi_geometry(net, rois, nroi, fd, g);
    return graph_build(net, fd, g, d_out, cap, d_counts, out);
}

int dl_graph_create_rois_dynamic(dl_net *net, int max_rois, int max_h, int max_w, int64_t max_pixels,
                                 dl_emitter *d_out, size_t cap, uint32_t *d_counts, dl_graph **out)
{
    if (!out) return fail(net, DL_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    if (max_rois < 1 || max_rois > DL_GRAPH_MAX_ROIS || max_h < 1 || max_w < 1 || max_pixels < 1)
        return fail(net, DL_ERR_INVALID_ARG, "capacity: 1 <= max_rois <= %d, max_h, max_w, max_pixels >= 1",
                    DL_GRAPH_MAX_ROIS);
    if ((int64_t)max_h * max_w > (int64_t)1 << 28 || !frame_act_fits(net, max_h, max_w))
        return fail(net, DL_ERR_UNSUPPORTED, "an ROI of %d x %d pixels is too large", max_h, max_w);
    if (!d_counts) return fail(net, DL_ERR_INVALID_ARG, "d_counts is NULL");
    if (cap > 0 && !d_out) return fail(net, DL_ERR_INVALID_ARG, "d_out is NULL with cap > 0");
    int rc;
    if ((rc = check_camera(net, false, 0, 0))) return rc;
    if (net->unet)
        return fail(net, DL_ERR_UNSUPPORTED, "the U-Net's level descriptors are built on the host: no capacity graph");
    dl_graph proto;
    proto.dynamic = true;
    proto.cap_rois = max_rois;
    proto.cap_h = max_h;
    proto.cap_w = max_w;
    proto.cap_px = std::min<int64_t>(max_pixels, (int64_t)max_rois * max_h * max_w);
    proto.cap_rows = std::min<int64_t>((int64_t)max_rois * max_h, proto.cap_px);
    const int64_t cols = std::min<int64_t>((int64_t)max_rois * max_w, proto.cap_px);
    int L = 1;
    for (int b = 0; b < net->nb; ++b) L = std::max(L, block_layout(net, b));
    // a frame's largest layout holds at most (h + L - 1)(w + L - 1) points
    proto.cap_act = proto.cap_px + (int64_t)(L - 1) * (proto.cap_rows + cols) + (int64_t)max_rois * (L - 1) * (L - 1);
    proto.cap_words = (proto.cap_px + 63) / 64 + proto.cap_rows;
    if (proto.cap_rows > (int64_t)1 << 30) return fail(net, DL_ERR_UNSUPPORTED, "capacity has too many rows");
    Geometry g;
    g.nf = max_rois;
    set_tiling(net, g);
    g.minor_blk = net->nb - 1;
    g.total_px = proto.cap_px;
    g.total_act = proto.cap_act;
    g.total_rows = proto.cap_rows;
    g.total_words = proto.cap_words;
    for (int b = 0; b < net->nb; ++b) g.tiles[b] = (int64_t)1 << 40;   // persistent grids: the full chip
    g.max_tiles = 0;
    g.maxh = max_h;
    g.maxw = max_w;
    std::vector<FrameDesc> none;
    return graph_build(net, none, g, d_out, cap, d_counts, out, &proto);
}

int dl_graph_launch_rois(dl_graph *g, const dl_roi *rois, int nroi, void *stream)
{
    if (!g) return fail(nullptr, DL_ERR_INVALID_ARG, "graph is NULL");
    dl_net *net = g->net;
    if (!g->dynamic) return fail(net, DL_ERR_INVALID_ARG, "this graph was captured for one fixed batch (dl_graph_launch)");
    int rc = check_rois(net, rois, nroi);
    if (rc) return rc;
    if (nroi > g->cap_rois) return fail(net, DL_ERR_CAPACITY, "%d ROIs exceed the graph's capacity of %d", nroi, g->cap_rois);
    int64_t px = 0, act = 0, rows = 0, words = 0;
    for (int k = 0; k < nroi; ++k) {
        const dl_roi &r = rois[k];
        if (r.h > g->cap_h || r.w > g->cap_w)
            return fail(net, DL_ERR_CAPACITY, "roi %d is %d x %d; the graph holds ROIs up to %d x %d", k, r.h, r.w,
                        g->cap_h, g->cap_w);
        px += (int64_t)r.h * r.w;
        act += frame_act_points(net, r.h, r.w);
        rows += r.h;
        words += (int64_t)r.h * ((r.w + 63) / 64);
    }
    if (px > g->cap_px || act > g->cap_act || rows > g->cap_rows || words > g->cap_words)
        return fail(net, DL_ERR_CAPACITY, "the ROIs' %lld pixels exceed the graph's capacity of %lld", (long long)px,
                    (long long)g->cap_px);
    if (g->cam_gen != net->cam_gen)
        return fail(net, DL_ERR_INVALID_ARG, "the camera maps were set, cleared or reshaped after this graph was captured");
    if (g->packed_gen != net->packed_gen)
        return fail(net, DL_ERR_INVALID_ARG, "the handle's precision changed after this graph was captured (its weights moved)");
    if ((rc = set_device(net))) return rc;
    // the previous replay has copied the slot once this event has passed
    HIPCHK(net, hipEventSynchronize(g->copied));
    const int64_t n64 = nroi;
    std::memcpy(g->h_slot, &n64, 8);
    std::memcpy(g->h_slot + 8, rois, sizeof(dl_roi) * (size_t)nroi);
    HIPCHK(net, hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return DL_OK;
}

int dl_graph_launch(dl_graph *g, void *stream)
{
    if (!g) return fail(nullptr, DL_ERR_INVALID_ARG, "graph is NULL");
    dl_net *net = g->net;
    if (g->dynamic) return fail(net, DL_ERR_INVALID_ARG, "this graph takes a ROI list at each launch (dl_graph_launch_rois)");
    int rc;
    if (g->cam_gen != net->cam_gen)
        return fail(net, DL_ERR_INVALID_ARG, "the camera maps were set, cleared or reshaped after this graph was captured");
    if (g->packed_gen != net->packed_gen)
        return fail(net, DL_ERR_INVALID_ARG, "the handle's precision changed after this graph was captured (its weights moved)");
    if ((rc = set_device(net))) return rc;
    HIPCHK(net, hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return DL_OK;
}

void dl_graph_destroy(dl_graph *g)
{
    if (!g) return;
    (void)hipSetDevice(g->dev);
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ws) (void)hipFree(g->ws);
    if (g->d_fd) (void)hipFree(g->d_fd);
    if (g->d_slot) (void)hipFree(g->d_slot);
    if (g->d_dyn) (void)hipFree(g->d_dyn);
    if (g->h_slot) (void)hipHostFree(g->h_slot);
    if (g->copied) (void)hipEventDestroy(g->copied);
    delete g;
}

int dl_autotune(dl_net *net, const uint16_t *d_frames, int n, int h, int w, void *stream, int reps,
                int32_t *best_rows, float *ms)
{
    int rc = check_uniform(net, d_frames, n, h, w);
    if (rc) return rc;
    if (reps <= 0 || reps > 1000) return fail(net, DL_ERR_INVALID_ARG, "reps must lie in 1..1000");
    if (net->dL) return fail(net, DL_ERR_UNSUPPORTED, "the dense-connection kernels have a fixed tile (nothing to tune)");
    if ((rc = set_device(net))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    static const int cand[DL_TUNE_CANDIDATES] = {8, 4};
    const int saved = net->cfg.tile_rows;
    const bool prof = net->profiling;
    net->profiling = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(net, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(net, DL_ERR_DEVICE, "hipEventCreate failed");
    }
    float best = 0.f;
    int pick = cand[0];
    for (int c = 0; c < DL_TUNE_CANDIDATES && rc == DL_OK; ++c) {
        net->cfg.tile_rows = cand[c];
        std::vector<FrameDesc> fd;
        Geometry g;
        uniform_geometry(net, d_frames, n, h, w, fd, g);
        rc = localize_geom(net, fd, g, s, nullptr, 0, nullptr, nullptr, d_frames, n, h, w);   // warm-up
        if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = fail(net, DL_ERR_DEVICE, "hipEventRecord failed");
        for (int r = 0; r < reps && !rc; ++r)
            rc = localize_geom(net, fd, g, s, nullptr, 0, nullptr, nullptr, d_frames, n, h, w);
        float t = 0.f;
        if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess))
            rc = fail(net, DL_ERR_DEVICE, "event timing failed");
        t /= (float)reps;
        if (ms) ms[c] = t;
        if (!rc && (c == 0 || t < best)) {
            best = t;
            pick = cand[c];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    net->profiling = prof;
    net->cfg.tile_rows = rc ? saved : pick;
    if (!rc && best_rows) *best_rows = pick;
    return rc;
}


int dl_autotune_ex(dl_net *net, const uint16_t *d_frames, int n, int h, int w, void *stream, int reps,
                   const char *cache_path, dl_tune_result *res)
{
    int rc = check_uniform(net, d_frames, n, h, w);
    if (rc) return rc;
    if (!res) return fail(net, DL_ERR_INVALID_ARG, "res is NULL");
    if (reps <= 0 || reps > 1000) return fail(net, DL_ERR_INVALID_ARG, "reps must lie in 1..1000");
    if (net->dL) return fail(net, DL_ERR_UNSUPPORTED, "the dense-connection kernels have a fixed tile (nothing to tune)");
    if ((rc = set_device(net))) return rc;
    std::memset(res, 0, sizeof *res);
    const std::string key = tune_key(net, n, h, w);
    int rows[MAXBLK], strip = 8;
    if (cache_path && tune_cache_find(cache_path, key, net->nb, rows, &strip)) {
        net->cfg.tile_rows = 0;
        for (int b = 0; b < net->nb; ++b) net->tune_rows[b] = res->rows[b] = rows[b];
        net->tune_strip = (uint32_t)(res->strip = strip);
        res->from_cache = 1;
        return DL_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int saved_rows = net->cfg.tile_rows;
    int saved_tune[MAXBLK];
    std::memcpy(saved_tune, net->tune_rows, sizeof saved_tune);
    const uint32_t saved_strip = net->tune_strip;
    const bool prof = net->profiling;
    net->profiling = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(net, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(net, DL_ERR_DEVICE, "hipEventCreate failed");
    }
    // mean time of one pass of the network (no post-processing) with this tiling
    auto time_cfg = [&](const int *r, int st, float *ms) -> int {
        net->cfg.tile_rows = 0;
        for (int b = 0; b < net->nb; ++b) net->tune_rows[b] = r[b];
        net->tune_strip = (uint32_t)st;
        std::vector<FrameDesc> fd;
        Geometry g;
        uniform_geometry(net, d_frames, n, h, w, fd, g);
        int e = localize_geom(net, fd, g, s, nullptr, 0, nullptr, nullptr, d_frames, n, h, w);   // warm-up
        if (!e && hipEventRecord(e0, s) != hipSuccess) e = fail(net, DL_ERR_DEVICE, "hipEventRecord failed");
        for (int k = 0; k < reps && !e; ++k) e = localize_geom(net, fd, g, s, nullptr, 0, nullptr, nullptr, d_frames, n, h, w);
        float t = 0.f;
        if (!e && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                   hipEventElapsedTime(&t, e0, e1) != hipSuccess))
            e = fail(net, DL_ERR_DEVICE, "event timing failed");
        *ms = t / (float)reps;
        ++res->configs_timed;
        return e;
    };
    // start from the form's default rows and strip 8; pick the strip width,
    // then each block's rows in turn (kept only when 1% faster)
    for (int b = 0; b < net->nb; ++b) {
        int tr = 0, tc = 0;
        conv_tile_shape(net->C, net->cfg.precision, 0, &tr, &tc);
        rows[b] = tr;
    }
    float best = 0.f, t = 0.f;
    rc = time_cfg(rows, strip, &best);
    res->ms_default = best;
    static const int strips[] = {4, 16, 32};
    for (int k = 0; k < 3 && !rc; ++k) {
        rc = time_cfg(rows, strips[k], &t);
        if (!rc && t < 0.99f * best) {
            best = t;
            strip = strips[k];
        }
    }
    for (int b = 0; b < net->nb && !rc; ++b) {
        const int old = rows[b];
        rows[b] = old == 8 ? 4 : 8;
        rc = time_cfg(rows, strip, &t);
        if (!rc && t < 0.99f * best) best = t;
        else rows[b] = old;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    net->profiling = prof;
    if (rc) {
        net->cfg.tile_rows = saved_rows;
        std::memcpy(net->tune_rows, saved_tune, sizeof saved_tune);
        net->tune_strip = saved_strip;
        return rc;
    }
    net->cfg.tile_rows = 0;
    for (int b = 0; b < net->nb; ++b) net->tune_rows[b] = res->rows[b] = rows[b];
    net->tune_strip = (uint32_t)(res->strip = strip);
    res->ms_best = best;
    if (cache_path) {
        FILE *f = std::fopen(cache_path, "a");
        if (!f) return fail(net, DL_ERR_INVALID_ARG, "cannot append to the tuning cache %s", cache_path);
        std::fprintf(f, "{\"key\": \"%s\", \"rows\": [", key.c_str());
        for (int b = 0; b < net->nb; ++b) std::fprintf(f, "%s%d", b ? ", " : "", rows[b]);
        std::fprintf(f, "], \"strip\": %d, \"ms\": %.4f}\n", strip, best);
        std::fclose(f);
    }
    return DL_OK;
}

int dl_train_grad(dl_net *net, const uint16_t *d_frames, int n, int h, int w, const dl_truth *d_truth,
                  const int32_t *d_truth_off, int ntruth, void *stream, float *d_grad, float *d_loss)
{
    int rc = train_check(net, d_frames, n, h, w, d_truth, d_truth_off, ntruth, d_loss);
    if (rc) return rc;
    return train_run(net, d_frames, n, h, w, d_truth, d_truth_off, ntruth, static_cast<hipStream_t>(stream), d_grad,
                     d_loss);
}

int dl_train_step(dl_net *net, const uint16_t *d_frames, int n, int h, int w, const dl_truth *d_truth,
                  const int32_t *d_truth_off, int ntruth, void *stream, float lr, float *d_loss)
{
    int rc = train_check(net, d_frames, n, h, w, d_truth, d_truth_off, ntruth, d_loss);
    if (rc) return rc;
    if (!(lr > 0.f) || !std::isfinite(lr)) return fail(net, DL_ERR_INVALID_ARG, "lr must be finite and > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = train_run(net, d_frames, n, h, w, d_truth, d_truth_off, ntruth, s, nullptr, d_loss))) return rc;
    HIPCHK(net, launch_adam(net->t_params, net->t_m, net->t_v, net->t_grad, (int)net->params.size(), lr, 0.9f, 0.999f,
                            1e-8f, ++net->t_step, s));
    net->t_dirty = true;
    return DL_OK;
}

int dl_get_params(dl_net *net, float *params, size_t count)
{
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    if (!params || count != net->params.size())
        return fail(net, DL_ERR_INVALID_ARG, "params must hold exactly %zu floats", net->params.size());
    int rc;
    if ((rc = set_device(net)) || (rc = sync_trained(net))) return rc;
    std::memcpy(params, net->params.data(), count * 4);
    return DL_OK;
}

int dl_set_gate(dl_net *net, const float *theta, float threshold)
{
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    if (!theta) {
        net->gate_set = false;
        return DL_OK;
    }
    if (!(threshold > 0.f && threshold < 1.f)) return fail(net, DL_ERR_INVALID_ARG, "gate threshold must lie in (0, 1)");
    if (!finite_all(theta, DL_GATE_NPARAM)) return fail(net, DL_ERR_INVALID_ARG, "gate parameters contain NaN or Inf");
    int rc;
    if ((rc = set_device(net))) return rc;
    if (!net->d_gate_theta) HIPCHK(net, hipMalloc(&net->d_gate_theta, DL_GATE_NPARAM * sizeof(float)));
    HIPCHK(net, hipDeviceSynchronize());
    HIPCHK(net, hipMemcpy(net->d_gate_theta, theta, DL_GATE_NPARAM * sizeof(float), hipMemcpyHostToDevice));
    net->gate_tau = (float)std::log((double)threshold / (1.0 - (double)threshold));
    net->gate_set = true;
    return DL_OK;
}

int dl_gate_keep_map(dl_net *net, void *stream, uint8_t *d_keep, size_t cap, size_t *ntiles)
{
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    if (!ntiles) return fail(net, DL_ERR_INVALID_ARG, "ntiles is NULL");
    *ntiles = (size_t)net->last_gate_tiles;
    if (net->last_gate_tiles == 0) return fail(net, DL_ERR_INVALID_ARG, "the handle's most recent run was not gated");
    if (!d_keep || cap < *ntiles) return fail(net, DL_ERR_CAPACITY, "keep map needs %zu bytes", *ntiles);
    int rc;
    if ((rc = set_device(net))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((rc = ws_acquire(net, s))) return rc;
    HIPCHK(net, hipMemcpyAsync(d_keep, net->ws + net->last_keep_off, *ntiles, hipMemcpyDeviceToDevice, s));
    return ws_release(net, s);
}

int dl_profile_enable(dl_net *net, int on)
{
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    net->profiling = on != 0;
    return DL_OK;
}

int dl_profile_read(dl_net *net, double *ms, int64_t *launches)
{
    if (!net) return fail(nullptr, DL_ERR_INVALID_ARG, "net is NULL");
    if (!ms || !launches) return fail(net, DL_ERR_INVALID_ARG, "ms/launches is NULL");
    for (int i = 0; i < DL_NSTAGES; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    int rc = DL_OK;
    for (auto &e : net->prof_pending) {
        float t = 0.f;
        if (rc == DL_OK) {
            hipError_t err = hipEventSynchronize(e.b);
            if (err == hipSuccess) err = hipEventElapsedTime(&t, e.a, e.b);
            if (err != hipSuccess) rc = fail(net, DL_ERR_DEVICE, "event timing failed: %s", hipGetErrorString(err));
        }
        if (e.stage >= 0 && e.stage < DL_NSTAGES) {
            ms[e.stage] += t;
            launches[e.stage] += 1;
        }
        net->ev_pool.push_back(e.a);
        net->ev_pool.push_back(e.b);
    }
    net->prof_pending.clear();
    return rc;
}

// ------------------------------------------------------------------ gate
#define GCHK(expr)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(nullptr, DL_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int dl_gate_pool_net(dl_net *net, const uint16_t *d_frames, int n, int h, int w, void *stream, float *d_pooled)
{
    int rc = check_uniform(net, d_frames, n, h, w);
    if (rc) return rc;
    if (!d_pooled) return fail(net, DL_ERR_INVALID_ARG, "d_pooled is NULL");
    if (h % GATE_TILE || w % GATE_TILE)
        return fail(net, DL_ERR_UNSUPPORTED, "the tile gate needs h and w multiples of %d (got %d x %d)", GATE_TILE, h, w);
    if ((rc = check_camera(net, true, h, w))) return rc;
    if ((rc = set_device(net))) return rc;
    HIPCHK(net, launch_gate_pool(d_frames, n, h, w, net->cfg.offset, net->cfg.gain * in_scale_of(net), net->d_cam, d_pooled,
                                 static_cast<hipStream_t>(stream)));
    return DL_OK;
}

int dl_gate_pool(const uint16_t *d_frames, int n, int h, int w, float gain, float offset, float in_scale,
                 void *stream, float *d_pooled)
{
    if (!d_frames || !d_pooled) return fail(nullptr, DL_ERR_INVALID_ARG, "NULL pointer");
    if (n <= 0 || h <= 0 || w <= 0) return fail(nullptr, DL_ERR_INVALID_ARG, "n, h, w must be > 0");
    if (h % DL_GATE_TILE || w % DL_GATE_TILE)
        return fail(nullptr, DL_ERR_UNSUPPORTED, "gate tiles need h and w multiples of %d", DL_GATE_TILE);
    if (!std::isfinite(gain) || !std::isfinite(offset) || !std::isfinite(in_scale) || !(gain > 0.f) || !(in_scale > 0.f))
        return fail(nullptr, DL_ERR_INVALID_ARG, "bad gain/offset/in_scale");
    GCHK(launch_gate_pool(d_frames, n, h, w, offset, gain * in_scale, nullptr, d_pooled, static_cast<hipStream_t>(stream)));
    return DL_OK;
}

int dl_gate_forward(const float *d_pooled, int ntiles, const float *d_theta, void *stream, float *d_logits)
{
    if (!d_pooled || !d_theta || !d_logits) return fail(nullptr, DL_ERR_INVALID_ARG, "NULL pointer");
    if (ntiles <= 0) return fail(nullptr, DL_ERR_INVALID_ARG, "ntiles must be > 0");
    GCHK(launch_gate(d_pooled, ntiles, d_theta, d_logits, nullptr, nullptr, static_cast<hipStream_t>(stream)));
    return DL_OK;
}

int dl_gate_backward(const float *d_pooled, int ntiles, const float *d_theta, const float *d_dlogits,
                     float *d_work, void *stream, float *d_logits, float *d_grad)
{
    if (!d_pooled || !d_theta || !d_dlogits || !d_work || !d_logits || !d_grad)
        return fail(nullptr, DL_ERR_INVALID_ARG, "NULL pointer");
    if (ntiles <= 0) return fail(nullptr, DL_ERR_INVALID_ARG, "ntiles must be > 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    GCHK(launch_gate(d_pooled, ntiles, d_theta, d_logits, d_dlogits, d_work, s));
    GCHK(launch_gate_reduce(d_work, ntiles, d_grad, s));
    return DL_OK;
}

int dl_gate_bce(const float *d_logits, const float *d_labels, int n, void *stream, float *d_loss, float *d_dlogits)
{
    if (!d_logits || !d_labels || (!d_loss && !d_dlogits)) return fail(nullptr, DL_ERR_INVALID_ARG, "NULL pointer");
    if (n <= 0) return fail(nullptr, DL_ERR_INVALID_ARG, "n must be > 0");
    GCHK(launch_gate_bce(d_logits, d_labels, n, d_loss, d_dlogits, static_cast<hipStream_t>(stream)));
    return DL_OK;
}

int dl_gate_adam(float *d_theta, float *d_m, float *d_v, const float *d_grad, int n, int step, float lr, float b1,
                 float b2, float eps, void *stream)
{
    if (!d_theta || !d_m || !d_v || !d_grad) return fail(nullptr, DL_ERR_INVALID_ARG, "NULL pointer");
    if (n <= 0 || step <= 0) return fail(nullptr, DL_ERR_INVALID_ARG, "n and step must be > 0");
    if (!(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
        return fail(nullptr, DL_ERR_INVALID_ARG, "bad Adam hyper-parameters");
    GCHK(launch_adam(d_theta, d_m, d_v, d_grad, n, lr, b1, b2, eps, step, static_cast<hipStream_t>(stream)));
    return DL_OK;
}

}  // extern "C"
