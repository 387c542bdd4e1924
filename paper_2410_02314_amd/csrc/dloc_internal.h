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
    int32_t h, w;
    int32_t tiles_x;        // conv tiles per tile row
    int32_t words;          // 64-pixel detection words per row = ceil(w / 64)
};

struct Geometry {
    int nf = 0;
    int64_t total_px = 0, total_rows = 0, total_tiles = 0, total_words = 0;
    int tile_rows = 0;
    int maxw = 0;
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
                       float offset, float scale, void *act, int act_bf16, hipStream_t s);

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
};
hipError_t launch_conv(int C, int precision, const ConvArgs &a, const Geometry &g, int grid,
                       hipStream_t s);
int conv_max_grid(int C, int precision, int tile_rows, int ncu);
size_t conv_packed_bytes(int C, int precision);
void pack_conv_weights(int C, int precision, const float *W /*[C][C][3][3]*/, void *dst);

// maps: `planes` planes per frame, the logit plane first (5 for the head
// output, 1 for a plain logit stack)
hipError_t launch_detect_mask(const float *maps, int planes, const FrameDesc *fd, const Geometry &g, float tau,
                              uint64_t *mask, uint32_t *row_counts, hipStream_t s);
hipError_t launch_scan(const uint32_t *row_counts, const FrameDesc *fd, const Geometry &g,
                       uint32_t *row_off, uint32_t *counts, hipStream_t s);
hipError_t launch_emit(const float *maps, const uint64_t *mask, const uint32_t *row_off,
                       const FrameDesc *fd, const Geometry &g, float z_scale, float ph_scale,
                       dl_emitter *out, uint64_t cap, hipStream_t s);
hipError_t launch_mask_to_u8(const uint64_t *mask, const FrameDesc *fd, const Geometry &g,
                             uint8_t *det, hipStream_t s);

}  // namespace dloc
