// Internal declarations shared by the HIP translation units of libdloc.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#include "dloc.h"

namespace dloc {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int MAXBLK = 8;         // residual blocks a network may have
constexpr int GATE_TILE = 256;    // gate tile side (pixels)

// Convolution tiles.  For a layer of dilation d a frame is cut into regions
// of (tr d) x (tc d) pixels; a region holds d*d phase tiles, and phase (py, px)
// covers the pixels (Y0 + d i, X0 + d j), i < tr, j < tc, with
// Y0 = region_y * tr d + py, X0 = region_x * tc d + px.  On that d-strided
// sub-lattice the dilated 3x3 convolution is an ordinary 3x3 convolution, so a
// tile's input is always (tr + 2) x (tc + 2) lattice points.  Tiles are
// numbered region-major, phase-minor: consecutive tiles cover the same pixels'
// neighbourhood and share cache lines.
__host__ __device__ inline int64_t conv_tiles(int h, int w, int d, int tr, int tc)
{
    const int ry = (h + tr * d - 1) / (tr * d), rx = (w + tc * d - 1) / (tc * d);
    return (int64_t)ry * rx * d * d;
}

// One frame (or ROI) of a batch, as every kernel sees it.  Per-pixel maps
// are packed frame after frame from px_off; activations from act_off, with
// room for the largest phase layout the net uses (see act_points).  Rows,
// detection words, gate tiles and conv tiles (per block, since the tiling
// depends on the dilation) are numbered globally over the batch; the *_start
// fields are the frame's first ones.
struct FrameDesc {
    const uint16_t *data;   // device frame (uint16), rows `stride` elements apart
    int64_t stride;
    int64_t px_off;
    int64_t act_off;        // first activation point of the frame
    int64_t row_start;
    int64_t mask_start;     // first 64-bit detection word of the frame
    int64_t keep_start;     // first gate-tile flag of the frame (gated runs)
    int64_t tile_start[MAXBLK];
    int32_t h, w;
    int32_t words;          // 64-pixel detection words per row = ceil(w / 64)
    int32_t gtx, gty;       // gate tiles per row / column (gated runs)
    int32_t pad_;
};

// Activation layouts.  Layout 1 is plain NHWC.  Phase layout l (a power of
// two) stores the l*l phase sub-images of a frame one after the other, each a
// dense NHWC image of ceil(h/l) x ceil(w/l) points: pixel (y, x) sits in
// sub-image (y mod l, x mod l) at (y div l, x div l).  A dilation-l layer
// reads its phase tiles from contiguous rows of one sub-image.
__host__ __device__ inline int64_t act_points(int h, int w, int l)
{
    const int64_t hd = (h + l - 1) / l, wd = (w + l - 1) / l;
    return (int64_t)l * l * hd * wd;
}

struct Geometry {
    int nf = 0;
    int64_t total_px = 0, total_act = 0, total_rows = 0, total_words = 0, gate_tiles = 0;
    int64_t tiles[MAXBLK] = {0};   // conv tiles of each block's layers
    int64_t max_tiles = 0;
    int64_t max_frame_tiles = 0;   // most conv tiles of one frame in one block
    int tr = 8, tc = 64;           // conv tile shape on the sub-lattice (tr: the form's default rows)
    int trb[MAXBLK] = {8, 8, 8, 8, 8, 8, 8, 8};   // tile rows of each block's layers
    uint32_t strip = 8;            // tile order: column strips of this many regions (see decode_tile)
    int maxw = 0, maxh = 0;
    int minor_blk = -1;            // block whose tiles run phase-minor (see decode_tile)
    // Batches whose frame list is only known on the device (a graph replayed
    // over any ROI set within its capacity): dyn points to DYN_WORDS int64 in
    // device memory -- the frame count, the total rows, then the conv tiles of
    // each block -- which the kernels read in place of nf, total_rows and
    // tiles[].  The other fields then hold capacity bounds (grid sizes,
    // workspace offsets such as the FP8 scale region at total_act * C).
    const int64_t *dyn = nullptr;
    // dense networks with the two-stage U-Net: points and conv tiles of
    // levels 1 and 2 (index 1, 2); their frame descriptors follow the n frame
    // descriptors of the batch, level by level
    int64_t lv_pts[3] = {0, 0, 0}, lv_tiles[3] = {0, 0, 0};
};
constexpr int DYN_NF = 0, DYN_ROWS = 1, DYN_TILES = 2, DYN_WORDS = 2 + MAXBLK;

// Order of one frame's conv tiles for one block.  Phase-major: the d*d phase
// sub-lattices one after another, and within a phase its ry x rx regions in
// column strips `strip` regions wide, row by row inside a strip, so the tile
// below a tile comes at most `strip` tiles later and finds the halo rows they
// share still in L2 (tiles are handed out in order to the resident
// workgroups of an XCD; the strip width is a tuning choice, 8 by default).
// Phase-minor (the last block, whose head writes plain planar maps): the d*d
// phases of one region in a row, regions row by row, so the map pixels a
// region's phases write are written together.
__device__ __forceinline__ void decode_tile(int h, int w, int64_t local, int d, int tr, int tc, bool phase_minor,
                                            uint32_t strip, int &Y0, int &X0)
{
    // a frame has fewer than 2^32 tiles: 32-bit arithmetic suffices
    const uint32_t l = (uint32_t)local, ud = (uint32_t)d;
    const uint32_t ryn = (uint32_t)((h + tr * d - 1) / (tr * d)), rxn = (uint32_t)((w + tc * d - 1) / (tc * d));
    uint32_t ph, ry, rx;
    if (phase_minor) {
        const uint32_t r = l / (ud * ud);
        ph = l - r * ud * ud;
        ry = r / rxn;
        rx = r - ry * rxn;
    } else {
        const uint32_t nreg = ryn * rxn;
        ph = l / nreg;
        const uint32_t r = l - ph * nreg;
        const uint32_t sfull = ryn * strip;                   // tiles of a full strip
        const uint32_t st = r / sfull, in = r - st * sfull;
        const uint32_t sw = min(strip, rxn - st * strip);     // width of this strip
        ry = in / sw;
        rx = st * strip + (in - ry * sw);
    }
    const uint32_t py = ph / ud, px = ph - py * ud;
    Y0 = (int)(ry * (uint32_t)(tr * d) + py);
    X0 = (int)(rx * (uint32_t)(tc * d) + px);
}

// Is any kept gate tile within distance r of the pixel box [y0, y1] x [x0, x1]
// (inclusive)?  keep == nullptr means every tile is kept.
__device__ __forceinline__ bool near_kept(const uint8_t *keep, const FrameDesc &d, int y0, int y1, int x0,
                                          int x1, int r)
{
    if (!keep) return true;
    const int ty0 = max(0, y0 - r) / GATE_TILE, ty1 = min(d.h - 1, y1 + r) / GATE_TILE;
    const int tx0 = max(0, x0 - r) / GATE_TILE, tx1 = min(d.w - 1, x1 + r) / GATE_TILE;
    const uint8_t *k = keep + d.keep_start;
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx)
            if (k[ty * d.gtx + tx]) return true;
    return false;
}

// Read of memory that no kernel writes while the reader runs (descriptors,
// lists and scales made by earlier launches): through the constant address
// space, so uniform addresses become scalar loads, which are not counted with
// the vector memory loads a kernel may have in flight.
template <class T>
__device__ __forceinline__ T ld_const(const T *p)
{
    return *(const __attribute__((address_space(4))) T *)p;
}

// binary search: largest f with key(f) <= idx, for a key increasing in f
template <typename F>
__device__ __forceinline__ int find_frame(const FrameDesc *fd, int nf, int64_t idx, F key)
{
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (key(fd[mid]) <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// two floats -> two BF16 (round to nearest even, v_cvt_pk_bf16_f32), packed
// low value first
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pack2(float lo, float hi)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t{lo, hi}), bf16x2_t));
}

// ---- FP8 activation storage ----
// The FP8 form stores an activation tensor as e4m3 codes, C bytes per point,
// then (from byte offset total_act * C of the same buffer) two E8M0 scale
// bytes per point, one per group of 32 channels: value = code * 2^(byte - 127).
// A group's scale is the smallest power of two s with amax / s <= 448, where
// amax is the largest magnitude in the group; s stays a normal float
// (byte 1..254; an all-zero group gets byte 1).
__device__ __forceinline__ uint32_t fp8_scale_byte(float amax)
{
    const uint32_t u = __float_as_uint(amax);
    const int b = (int)(u >> 23) - ((u & 0x7FFFFFu) <= 0x600000u ? 8 : 7);
    return (uint32_t)(b < 1 ? 1 : b > 254 ? 254 : b);
}
__device__ __forceinline__ float fp8_scale_value(uint32_t byte) { return __uint_as_float(byte << 23); }
typedef short i16x2_t __attribute__((ext_vector_type(2)));
// e4m3 codes (round to nearest even) of v / s for four values with |v| / s <= 448
__device__ __forceinline__ uint32_t fp8_pack4(float v0, float v1, float v2, float v3, float s)
{
    i16x2_t r = {0, 0};
    r = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(r, v0, v1, s, false);
    r = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(r, v2, v3, s, true);
    return __builtin_bit_cast(uint32_t, r);
}
// the four e4m3 codes of a word, each times s
__device__ __forceinline__ v4f fp8_unpack4(uint32_t codes, float s)
{
    const f32x2_t lo = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(codes, s, false);
    const f32x2_t hi = __builtin_amdgcn_cvt_scalef32_pk_f32_fp8(codes, s, true);
    return v4f{lo[0], lo[1], hi[0], hi[1]};
}

// The frame descriptors of a ROI list on the device (one workgroup): from
// in = [int64 n][dl_roi x n] (device copy of a pinned slot), fd[k] of ROI k
// with every offset a prefix sum over the ROIs before it, and dyn (see
// Geometry::dyn).  layouts: the activation layouts the net uses (a frame
// reserves the largest); dil: the blocks' dilations; tr x tc: the conv tile.
struct EnumArgs {
    int nl, nb, tc;
    int layouts[MAXBLK + 1];
    int dil[MAXBLK];
    int tr[MAXBLK];          // tile rows of each block
};
hipError_t launch_enumerate(const void *in, const EnumArgs &e, FrameDesc *fd, int64_t *dyn, hipStream_t s);

// ---- launchers (kernels_*.hip) ----
// all return hipError_t of the launch
// precision: storage of the output activations (FP32, BF16, or FP8 codes
// and group scales)
// cam: per-pixel {offset, gain * in_scale} of the sensor (every frame of
// the batch is sensor-sized), or null for the scalar offset and scale
hipError_t launch_stem(int C, const FrameDesc *fd, const Geometry &g, const float *w, const float *b,
                       float offset, float scale, const float2 *cam, void *act, int precision,
                       const uint8_t *keep, int radius, hipStream_t s);
hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s);
// gated runs: keep[t] = logit[t] > tau_gate; then one compacted list of conv
// tiles per layer (tiles within radius[l] of a kept gate tile)
hipError_t launch_gate_keep(const float *logits, int64_t n, float tau, uint8_t *keep, hipStream_t s);
hipError_t launch_active_lists(const FrameDesc *fd, const Geometry &g, const uint8_t *keep, const int *radius,
                               const int *dil, int nlayers, int32_t *lists, uint32_t *counts, hipStream_t s);

struct ConvArgs {
    const void *in;          // activations (FP32, BF16, or FP8 codes + group scales), frame at act_off
    const void *res;         // residual (same layout as out) or null
    void *out;               // NHWC output (or null when the head is fused)
    const void *wpk;         // packed weights
    const float *bias;       // [C]
    const float *wscale;     // FP8: per-output-channel weight scale [C]
    const float *head;       // fused head: w [nh][C] then b [nh]; null = no head
    float *maps;             // fused head output, planar [nh][h][w] per frame
    int nh;                  // head outputs: 5, or 10 with the uncertainty planes
    const FrameDesc *fd;
    int d;
    int blk;                 // block index: selects the frame's tile numbering
    const int32_t *list;     // active tiles of this layer (gated runs) or null = all tiles
    const uint32_t *list_count;
    int in_phase;            // input and residual in phase layout d (1) or plain NHWC (0)
    int out_shift;           // output in phase layout 1 << out_shift (0: plain NHWC)
    int tr;                  // tile rows of this layer (4 or 8)
};
hipError_t launch_conv(int C, int precision, const ConvArgs &a, const Geometry &g, int grid, hipStream_t s);
// tile shape of the conv kernel: rows = 4 or 8; 0 picks the form's default
// (8, except FP32 with C > 48: 4)
void conv_tile_shape(int C, int precision, int rows, int *tr, int *tc);
int conv_max_grid(int C, int precision, int tr, int ncu);
// does the conv kernel of this channel count and form fit in LDS (both tile heights)?
bool conv_supported(int C, int precision, int nh);
size_t conv_packed_bytes(int C, int precision);
// pack one 3x3 C->C layer W [C][C][3][3]; FP8 also writes scale[C]
void pack_conv_weights(int C, int precision, const float *W, void *dst, float *scale);

// ---- dense-connection networks (kernels_dense.hip) ----
// A block's concatenation lives in one plain NHWC buffer of cs floats per
// point (block input in channels 0 .. C-1, then each layer's growth channels);
// a layer reads channels 0 .. cin-1 of `in` and writes its 16 NB outputs (+
// bias, ReLU) from channel co of `out`.  A block's last layer runs fused with
// its 1x1 transition (CT = cin + 16 NB -> 16 NT, + bias, ReLU), which writes
// channels 0 .. 16 NT - 1 of `tout` (its own outputs are not stored), and in
// the last block with the 1x1 head after it (16 NT -> nh planar maps).
// Tiles: dense_tile_rows() x dense_tile_cols() points of the layer's d-strided
// lattice (conv_tiles / decode_tile numbering, phase-major, strip 8) in the
// tile numbering of slot `blk`.
struct DenseConvArgs {
    const float *in;
    int csi, cin;            // floats per input point, input channels read (multiple of 16)
    float *out;
    int cso, co;             // floats per output point, first output channel
    const float *w;          // packed layer weights (pack_dense_weights, taps 9)
    const float *bias;       // [16 NB]
    const FrameDesc *fd;
    int d, blk;
    // fused transition: packed weights (pack_dense_weights, taps 1, cin + 16 NB
    // -> 16 NT), bias [16 NT], output points of cst floats
    const float *wt, *bt;
    float *tout;
    int cst;
    // fused head: packed weights (16 rows, rows >= nh zero; K = 16 NT), bias [nh]
    const float *wh, *bh;
    int nh;
    float *maps;             // planar [nh][h][w] per frame from px_off
    // tile schedule: null = static ranges per XCD; else 8 zeroed counters, and
    // queue_mode 1 (one atomic queue per XCD over its range) or 2 (counter 0:
    // one queue over all tiles)
    uint32_t *queue;
    int queue_mode;
    // training passes (launch_dconv_train): bias may be null; res (points of
    // rcs floats) is added before the optional ReLU; where mask (points of mcs
    // floats) is <= 0 the output is 0
    const float *res, *mask;
    int rcs, mcs, relu;
};
int dense_tile_rows();
int dense_tile_cols();
// nb_out 1 or 2 (16 or 32 layer outputs); fuse 0 (layer), 1 (+ transition),
// 2 (+ transition + head), 3 (+ head on the layer's outputs); nt = transition
// outputs / 16 (1 or 2)
hipError_t launch_dconv(int nb_out, int fuse, int nt, const DenseConvArgs &a, const Geometry &g, int ncu,
                        hipStream_t s);
// ---- training (kernels_train.hip) ----
// count square 3x3 convs' flat weights [C][C][9], the i-th at W0 + i src_stride,
// into the conv kernel's layout, each as itself (dst + 2 i 9 C^2) and as the
// transposed convolution (dst + (2 i + 1) 9 C^2: cout and cin swapped, taps reversed)
hipError_t launch_pack_convs(const float *W0, int64_t src_stride, int count, int C, float *dst, hipStream_t s);
// head (10 outputs) on the last activations, loss terms, their gradient with
// respect to the maps (gm, planar like maps), batch means into loss[4];
// term: 9 n h w + 48 n floats, occ: n h w bytes, lse: train_lse_floats(h, w,
// ntruth) floats (the log-sum-exps first, then the emitters' constants and the
// per-chunk partials)
int64_t train_lse_floats(int h, int w, int ntruth);
hipError_t launch_train_loss(int C, const float *act, const float *hw, const float *hb, int n, int h, int w,
                             const dl_truth *tr, const int32_t *toff, int ntruth, float zs, float ps, float *maps,
                             float *stats, float *lse, float *gm, float *loss, float *term, uint8_t *occ,
                             hipStream_t s);
// head weight/bias gradients (gwb: head.w then head.b) and the gradient at the
// last block's pre-activation; part: grad_chunks(n h w) x (10 C + 10) floats,
// mid: 32 x (10 C + 10)
int grad_chunks(int64_t npx);
hipError_t launch_head_backward(int C, const float *gm, const float *act, const float *hw, int n, int h, int w,
                                float *gwb, float *part, float *mid, float *du, hipStream_t s);
// 3x3 weight and bias gradients; part holds nblk x 9 C^2 floats and pb nblk C,
// nblk = ceil(n h / wgrad_rows_per_block(n, h)); tmp 32 x (9 C^2 + C)
int wgrad_rows_per_block(int n, int h);
hipError_t launch_wgrad(int C, const float *dy, const float *x, int n, int h, int w, int d, float *part, float *pb,
                        float *tmp, float *gW, float *gb, hipStream_t s);
// the same for CO (16 or 32) outputs over CI inputs (a multiple of CO) of a
// 3x3 (taps 9) or 1x1 (taps 1) conv; dy points of dcs floats, x points of xcs
// floats (channels 0 .. CI-1); gW [CO][CI][taps]; part nblk x CO CI taps, pb
// nblk CO, tmp 32 x (CO CI taps + CO)
hipError_t launch_wgrad_ex(int CO, int taps, const float *dy, int dcs, const float *x, int xcs, int CI, int n, int h,
                           int w, int d, float *part, float *pb, float *tmp, float *gW, float *gb, hipStream_t s);
// one weight pack: the conv at params + src ([cout][cin][taps]), or (flip) its
// transposed convolution, rows row0 .. row0 + nrows - 1 (a multiple of 16),
// into dst .. in the conv kernel's layout; start: the job's first element in
// the launch (jobs in increasing order; elements between one job's last and
// the next job's start are skipped)
struct PackJob {
    int64_t src, dst, start;
    int cout, cin, taps, flip, row0, nrows;
};
hipError_t launch_pack_jobs(const PackJob *jobs, int njobs, int64_t total, const float *params, float *dst,
                            hipStream_t s);
// dst[p][c] = src[p][so + c] where m[p][mo + c] > 0, else 0 (c < nc)
hipError_t launch_mask_slice(const float *src, int scs, int so, const float *m, int mcs, int mo, int nc, int64_t npx,
                             float *dst, int dcs, hipStream_t s);
// U-Net gradients over n uniform frames of h x w at the fine level (coarse:
// ceil(h/2) x ceil(w/2)): pooling -- each window's gradient g (coarse) added
// into out (fine) at the window's first maximum of a (the pooling's input,
// channels 0 .. C-1); upsampling -- out (coarse) = the sum of g (fine) over
// the pixels each coarse pixel fills; points of *cs floats each
hipError_t launch_pool2_back(const float *a, int acs, const float *g, int gcs, float *out, int ocs, int n, int h, int w,
                             int C, hipStream_t s);
hipError_t launch_up2_back(const float *g, int gcs, float *out, int ocs, int n, int h, int w, int C, hipStream_t s);
// out[p][c] = sum_o Wt[o][c] g[p][o]: the 1x1 transition's input gradient (C 16
// or 32; ct a multiple of 16)
hipError_t launch_1x1_back(int C, const float *g, const float *Wt, int ct, int64_t npx, float *out, hipStream_t s);
// stem weight/bias gradients (gwb: stem.w then stem.b); part: grad_chunks(n h w) x 10 C
hipError_t launch_stem_grad(const float *ds, const uint16_t *frames, int n, int h, int w, float offset, float scale,
                            int C, float *gwb, float *part, float *mid, hipStream_t s);

// one plain dense-kernel layer with the training epilogue (see DenseConvArgs),
// nb_out 1 .. 5 blocks of 16 outputs
hipError_t launch_dconv_train(int nb_out, const DenseConvArgs &a, const Geometry &g, int ncu, hipStream_t s);
// a dense block's last layer (16 outputs, written to out at co) fused with the
// block's 1x1 transition (nt = its outputs / 16) as in inference, for the
// training forward pass
hipError_t launch_dconv_train_fused(int nt, const DenseConvArgs &a, const Geometry &g, int ncu, hipStream_t s);
// preprocessing + stem 1 -> C (C 16 or 32) + ReLU into channels 0 .. C-1 of points of cs floats
hipError_t launch_dstem(int C, const FrameDesc *fd, const Geometry &g, const float *w, const float *b, float offset,
                        float scale, float *act, int cs, hipStream_t s);
// U-Net levels (src and dst descriptors of the same frames, npts = the dst
// level's points): 2 x 2 max pooling to the next level, nearest upsampling
// to the level above; C channels read from points of scs floats, written to
// points of dcs floats
hipError_t launch_pool2(const FrameDesc *sfd, const FrameDesc *dfd, int nf, int64_t npts, const float *src, int scs,
                        float *dst, int dcs, int C, hipStream_t s);
hipError_t launch_up2(const FrameDesc *sfd, const FrameDesc *dfd, int nf, int64_t npts, const float *src, int scs,
                      float *dst, int dcs, int C, hipStream_t s);
// W [cout][cin][taps] -> the MFMA layout of k_dconv (cout, cin multiples of 16)
void pack_dense_weights(int cout, int cin, int taps, const float *W, float *dst);

// maps: `planes` planes per frame, the logit plane first (5 for the head
// output, 1 for a plain logit stack)
// u_max: with 10 planes, a candidate is kept only if its raw sigma_x and
// sigma_y values (planes 5, 6) are <= u_max (+inf keeps all)
hipError_t launch_detect_mask(const float *maps, int planes, const FrameDesc *fd, const Geometry &g, float tau,
                              float u_max, const uint8_t *keep, uint64_t *mask, uint32_t *row_counts,
                              hipStream_t s);
hipError_t launch_scan(const uint32_t *row_counts, const FrameDesc *fd, const Geometry &g,
                       uint32_t *row_off, uint32_t *counts, hipStream_t s);
// maps has `planes` planes per frame; with unc (10 planes) each record's
// uncertainties go to unc[i] beside out[i]
hipError_t launch_emit(const float *maps, int planes, const uint64_t *mask, const uint32_t *row_off,
                       const FrameDesc *fd, const Geometry &g, float z_scale, float ph_scale,
                       float bg_scale, dl_emitter *out, dl_uncertainty *unc, uint64_t cap, hipStream_t s);
hipError_t launch_mask_to_u8(const uint64_t *mask, const FrameDesc *fd, const Geometry &g,
                             uint8_t *det, hipStream_t s);
// detection flags (u8 per pixel, planar per frame from px_off) -> mask words + row counts
hipError_t launch_mask_from_u8(const uint8_t *det, const FrameDesc *fd, const Geometry &g, uint64_t *mask,
                               uint32_t *row_counts, hipStream_t s);

// tile gate (kernels_gate.hip)
size_t gate_smem_bytes();
hipError_t launch_gate_pool(const uint16_t *frames, int n, int h, int w, float offset, float scale,
                            const float2 *cam, float *pooled, hipStream_t s);
hipError_t launch_gate(const float *pooled, int ntiles, const float *theta, float *logits,
                       const float *dlogits, float *gpart, hipStream_t s);
hipError_t launch_gate_reduce(const float *gpart, int ntiles, float *grad, hipStream_t s);
hipError_t launch_gate_bce(const float *g, const float *y, int n, float *loss, float *dg, hipStream_t s);
hipError_t launch_adam(float *theta, float *m, float *v, const float *grad, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);

}  // namespace dloc
