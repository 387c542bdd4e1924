// Internal declarations shared by the HIP translation units of libdloc.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#include "dloc.h"

namespace dloc {

typedef float v4f __attribute__((ext_vector_type(4)));

// Tile of the convolution kernels: TILE_ROWS rows (one wave per row) x
// TILE_COLS = 16 * PB columns.
constexpr int PB = 4;             // 16-pixel MFMA column blocks per wave
constexpr int TILE_COLS = 16 * PB;

// One frame (or ROI) of a batch, as every kernel sees it.  Per-pixel buffers
// (activations, maps) are packed frame after frame; px_off is the frame's
// first pixel in that packing.  Rows and conv tiles are numbered globally over
// the batch; row_start / tile_start are the frame's first global row / tile.
struct FrameDesc {
    const uint16_t *data;   // device frame (uint16), rows row_stride apart
    int64_t stride;
    int64_t px_off;
    int64_t row_start;
    int64_t tile_start;
    int64_t mask_start;     // first 64-bit detection word of the frame
    int64_t keep_start;     // first gate-tile flag of the frame (gated runs)
    int32_t h, w;
    int32_t tiles_x;        // conv tiles per tile row
    int32_t words;          // 64-pixel detection words per row = ceil(w / 64)
    int32_t gtx, gty;       // gate tiles per row / column (gated runs)
    int32_t pad_;
};

constexpr int GATE_TILE = 256;

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

struct Geometry {
    int nf = 0;
    int64_t total_px = 0, total_rows = 0, total_tiles = 0, total_words = 0;
    int tile_rows = 0;
    int maxw = 0;
    int64_t gate_tiles = 0;
};

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

// ---- launchers (kernels_*.hip) ----
// all return hipError_t of the launch
hipError_t launch_stem(int C, const FrameDesc *fd, const Geometry &g, const float *w, const float *b,
                       float offset, float scale, void *act, int act_bf16, const uint8_t *keep, int radius,
                       hipStream_t s);
// gated runs: keep[t] = logit[t] > tau_gate; then one compacted list of conv
// tiles per layer (tiles within radius[l] of a kept gate tile)
hipError_t launch_gate_keep(const float *logits, int64_t n, float tau, uint8_t *keep, hipStream_t s);
hipError_t launch_active_lists(const FrameDesc *fd, const Geometry &g, const uint8_t *keep, const int *radius,
                               int nlayers, int32_t *lists, uint32_t *counts, hipStream_t s);

struct ConvArgs {
    const void *in;          // NHWC activations (fp32 or bf16)
    const void *res;         // residual (same layout as out) or null
    void *out;               // NHWC output (or null when the head is fused)
    const void *wpk;         // packed weights
    const float *bias;       // [C]
    const float *head;       // fused head: w [5][C] then b [5]; null = no head
    float *maps;             // fused head output, planar [5][h][w] per frame
    const FrameDesc *fd;
    int d;
    const int32_t *list;       // active tiles of this layer (gated runs) or null = all tiles
    const uint32_t *list_count;
};
hipError_t launch_conv(int C, int precision, const ConvArgs &a, const Geometry &g, int grid,
                       hipStream_t s);
int conv_max_grid(int C, int precision, int tile_rows, int ncu);
size_t conv_packed_bytes(int C, int precision);
void pack_conv_weights(int C, int precision, const float *W /*[C][C][3][3]*/, void *dst);

// maps: `planes` planes per frame, the logit plane first (5 for the head
// output, 1 for a plain logit stack)
hipError_t launch_detect_mask(const float *maps, int planes, const FrameDesc *fd, const Geometry &g, float tau,
                              const uint8_t *keep, uint64_t *mask, uint32_t *row_counts, hipStream_t s);
hipError_t launch_scan(const uint32_t *row_counts, const FrameDesc *fd, const Geometry &g,
                       uint32_t *row_off, uint32_t *counts, hipStream_t s);
hipError_t launch_emit(const float *maps, const uint64_t *mask, const uint32_t *row_off,
                       const FrameDesc *fd, const Geometry &g, float z_scale, float ph_scale,
                       dl_emitter *out, uint64_t cap, hipStream_t s);
hipError_t launch_mask_to_u8(const uint64_t *mask, const FrameDesc *fd, const Geometry &g,
                             uint8_t *det, hipStream_t s);

// tile gate (kernels_gate.hip)
size_t gate_smem_bytes();
hipError_t launch_gate_pool(const uint16_t *frames, int n, int h, int w, float offset, float scale,
                            float *pooled, hipStream_t s);
hipError_t launch_gate(const float *pooled, int ntiles, const float *theta, float *logits,
                       const float *dlogits, float *gpart, hipStream_t s);
hipError_t launch_gate_reduce(const float *gpart, int ntiles, float *grad, hipStream_t s);
hipError_t launch_gate_bce(const float *g, const float *y, int n, float *loss, float *dg, hipStream_t s);
hipError_t launch_adam(float *theta, float *m, float *v, const float *grad, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);

}  // namespace dloc
