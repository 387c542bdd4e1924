// Bandwidth-bound stages: preprocessing + stem convolution, detection
// (threshold + 3x3 local maximum), ordered compaction into emitter records.
//
// Paper Sec. 2.2: pre- and post-processing stay in GPU memory; only the
// post-processed coordinates leave the device.  Sec. 3.2: per pixel the
// network gives a detection probability and the emitter's offset from that
// pixel; the record converts the offset into absolute frame coordinates.
#include "dloc_internal.h"

namespace dloc {

namespace {

// ---------------------------------------------------------------- stem
// x = (ADU - offset) * scale (scale = gain * in_scale), then
// a = ReLU(b + sum_tap w * x) for C channels, 3x3, d = 1, zero padding,
// stored as plain NHWC rows.  Each workgroup takes a contiguous range of the
// batch's rows; a row is done in segments of SSEG pixels whose three input rows (preprocessed,
// with a one-pixel zero border) are staged in LDS.  A thread item is one
// 16-byte piece of a pixel's output (8 BF16 or 4 FP32 channels), so
// consecutive threads store consecutive 16 bytes of the row.  In FP8 storage
// a pixel has four 16-channel items in adjacent lanes (items past C idle):
// each 32-channel group's max comes from its two items by one lane shuffle,
// then each item stores its 16 e4m3 codes and the group's first item its
// scale byte (region at scale_off).
constexpr int SSEG = 1024;

template <int C, int P>
__global__ void __launch_bounds__(256)
k_stem(const FrameDesc *__restrict__ fdp, int nf, int64_t nrows, const int64_t *__restrict__ dyn,
       const float *__restrict__ w, const float *__restrict__ b, float offset, float scale,
       const float2 *__restrict__ cam, void *__restrict__ act, int64_t scale_off, const uint8_t *__restrict__ keep,
       int radius)
{
    if (dyn) {                       // frame count and rows known on the device only
        nf = (int)dyn[DYN_NF];
        nrows = dyn[DYN_ROWS];
    }
    constexpr int CQ = P == DL_FP8 ? 16 : P == DL_BF16 ? 8 : 4;   // channels per item
    constexpr int IPX = P == DL_FP8 ? 4 : C / CQ;                  // items per pixel
    static_assert(P != DL_FP8 || C <= 64, "FP8 stem: at most four 16-channel items");
    constexpr int CP = IPX * CQ;             // channels the items cover (FP8: zero weights past C)
    __shared__ __align__(16) float sw[9 * CP];      // tap-major: an item's channels are contiguous
    __shared__ __align__(16) float sb[CP];
    __shared__ float sx[3][SSEG + 2];
    __shared__ bool sneed[SSEG / 64];
    for (int i = threadIdx.x; i < CP * 9; i += 256) {
        const int t = i / CP, c = i - (i / CP) * CP;
        sw[i] = c < C ? w[c * 9 + t] : 0.f;
    }
    for (int i = threadIdx.x; i < CP; i += 256) sb[i] = i < C ? b[i] : 0.f;

    // a contiguous range of rows per workgroup (mostly one frame)
    const int64_t per = (nrows + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * per, r1 = min(nrows, r0 + per);
    for (int64_t row = r0; row < r1; ++row) {
        const int f = find_frame(fdp, nf, row, [](const FrameDesc &d) { return d.row_start; });
        const FrameDesc &fd = fdp[f];
        const int y = (int)(row - fd.row_start);
        const int H = fd.h, W = fd.w;
        // gated runs: only rows / 64-pixel segments within `radius` of a kept tile
        if (!near_kept(keep, fd, y, y, 0, W - 1, radius)) continue;
        for (int x0 = 0; x0 < W; x0 += SSEG) {
            const int n = min(SSEG, W - x0);
            __syncthreads();                  // previous segment's reads (and the weights) are done
            for (int i = threadIdx.x; i < 3 * (SSEG + 2); i += 256) {
                const int r = i / (SSEG + 2), c = i - r * (SSEG + 2);
                const int yy = y + r - 1, xx = x0 + c - 1;
                const bool ok = c < n + 2 && (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W;
                float v = 0.f;
                if (ok) {
                    const float adu = (float)fd.data[(int64_t)yy * fd.stride + xx];
                    if (cam) {               // sCMOS: this pixel's offset and gain (frames are sensor-sized)
                        const float2 cm = cam[(int64_t)yy * W + xx];
                        v = (adu - cm.x) * cm.y;
                    } else {
                        v = (adu - offset) * scale;
                    }
                }
                sx[r][c] = v;
            }
            // gated runs: which 64-pixel pieces of the segment are needed
            if (threadIdx.x < SSEG / 64) {
                const int xs = x0 + 64 * threadIdx.x;
                sneed[threadIdx.x] = xs < W && near_kept(keep, fd, y, y, xs, min(W - 1, xs + 63), radius);
            }
            __syncthreads();
            for (int i = threadIdx.x; i < n * IPX; i += 256) {
                const int px = i / IPX, q = i - (i / IPX) * IPX;
                const int x = x0 + px;
                if (!sneed[px >> 6]) continue;
                float xin[9];
#pragma unroll
                for (int u = 0; u < 3; ++u)
#pragma unroll
                    for (int v = 0; v < 3; ++v) xin[u * 3 + v] = sx[u][px + v];
                const int64_t base = (fd.act_off + (int64_t)y * W + x) * C + q * CQ;   // plain NHWC
                float o[CQ];
#pragma unroll
                for (int k = 0; k < CQ; ++k) o[k] = sb[q * CQ + k];
#pragma unroll
                for (int t = 0; t < 9; ++t)
#pragma unroll
                    for (int k = 0; k < CQ; ++k) o[k] = fmaf(sw[t * CP + q * CQ + k], xin[t], o[k]);
#pragma unroll
                for (int k = 0; k < CQ; ++k) o[k] = fmaxf(o[k], 0.f);
                if constexpr (P == DL_FP8) {
                    // e4m3 codes under the group's power-of-two scale; the two
                    // items of a group are lanes 2 g and 2 g + 1 of the pixel's four
                    float m = 0.f;
#pragma unroll
                    for (int k = 0; k < CQ; ++k) m = fmaxf(m, o[k]);
                    m = fmaxf(m, __shfl_xor(m, 1));
                    const uint32_t sbyte = fp8_scale_byte(m);
                    const float sv = fp8_scale_value(sbyte);
                    if (q * CQ < C) {
                        *reinterpret_cast<uint4 *>(static_cast<uint8_t *>(act) + base) =
                            uint4{fp8_pack4(o[0], o[1], o[2], o[3], sv), fp8_pack4(o[4], o[5], o[6], o[7], sv),
                                  fp8_pack4(o[8], o[9], o[10], o[11], sv), fp8_pack4(o[12], o[13], o[14], o[15], sv)};
                        if ((q & 1) == 0) {
                            const int64_t pt = fd.act_off + (int64_t)y * W + x;
                            static_cast<uint8_t *>(act)[scale_off + 2 * pt + (q >> 1)] = (uint8_t)sbyte;
                        }
                    }
                } else if constexpr (P == DL_BF16) {
                    const uint4 pk{bf16_pack2(o[0], o[1]), bf16_pack2(o[2], o[3]), bf16_pack2(o[4], o[5]),
                                   bf16_pack2(o[6], o[7])};
                    *reinterpret_cast<uint4 *>(static_cast<uint16_t *>(act) + base) = pk;
                } else {
                    *reinterpret_cast<v4f *>(static_cast<float *>(act) + base) = v4f{o[0], o[1], o[2], o[3]};
                }
            }
        }
    }
}

template <int C>
hipError_t stem_c(const FrameDesc *fd, const Geometry &g, const float *w, const float *b, float offset,
                  float scale, const float2 *cam, void *act, int precision, const uint8_t *keep, int radius,
                  hipStream_t s)
{
    const unsigned grid = (unsigned)std::min<int64_t>(g.total_rows, 8192);
    const int64_t soff = g.total_act * C;        // FP8: byte offset of the group scales
    if (precision == DL_FP8)
        hipLaunchKernelGGL((k_stem<C, DL_FP8>), dim3(grid), dim3(256), 0, s, fd, g.nf, g.total_rows, g.dyn, w, b, offset,
                           scale, cam, act, soff, keep, radius);
    else if (precision == DL_BF16)
        hipLaunchKernelGGL((k_stem<C, DL_BF16>), dim3(grid), dim3(256), 0, s, fd, g.nf, g.total_rows, g.dyn, w, b, offset,
                           scale, cam, act, soff, keep, radius);
    else
        hipLaunchKernelGGL((k_stem<C, DL_FP32>), dim3(grid), dim3(256), 0, s, fd, g.nf, g.total_rows, g.dyn, w, b, offset,
                           scale, cam, act, soff, keep, radius);
    return hipGetLastError();
}

// ------------------------------------------------------------ detection
// Pixel (y, x) is detected iff its logit exceeds tau and beats every in-frame
// 8-neighbour in the order (value, then smaller raster index) -- a strict
// local maximum with a deterministic tie-break, so a plateau yields exactly
// one detection.  With the uncertainty planes and a finite u_max, a local
// maximum whose raw sigma_x or sigma_y exceeds u_max is dropped (its
// neighbours are not promoted): softplus is increasing, so this is
// sigma <= softplus(u_max) + DL_SIGMA_FLOOR without evaluating softplus.
//
// A workgroup (4 waves) takes a band of DBAND rows of one frame.  A wave
// works on chunks of 256 columns (chunk k of the band goes to wave k mod 4),
// as four groups of 64: lane l holds columns x0 + l + 64 e, e = 0..3, so each
// group's decisions form one 64-bit mask word by a ballot.  The wave loads
// the chunk's DBAND + 2 rows (the band and one row above and below) at once,
// 4 (DBAND + 2) logits per lane in flight, plus one halo column per row (the
// pixel left of the chunk in lane 0, right of it in lane 63).  Left and right
// neighbours come from the adjacent lanes (lane shuffles; across a group
// boundary from the neighbouring group's end lane), the rows above and below
// from the registers: each logit is read from HBM once per band (the band's
// two halo rows aside), with no LDS staging and no barrier until the per-row
// counts are summed.  Neighbours off the frame or in a gate tile that was
// skipped are -inf (absent).  The row's count goes to row_counts for the scan.
constexpr int DBAND = 8, DROWS = DBAND + 2;

// GATED: keep is a gate keep map; SIGMA: the uncertainty filter is on
template <bool GATED, bool SIGMA>
__global__ void __launch_bounds__(256)
k_detect_mask(const float *__restrict__ maps, int planes, const FrameDesc *__restrict__ fdp, int bands,
              const int64_t *__restrict__ dyn, float tau, float u_max, const uint8_t *__restrict__ keep,
              uint64_t *__restrict__ mask, uint32_t *__restrict__ row_counts)
{
    __shared__ uint32_t wcnt[DBAND][4];
    // workgroup = (frame, band): bands per frame from the batch's tallest frame
    const int f = blockIdx.x / bands, band = blockIdx.x - f * bands;
    if (dyn && f >= dyn[DYN_NF]) return;                  // past the frames of this batch
    const FrameDesc fd = fdp[f];
    const int H = fd.h, W = fd.w;
    const int y0 = band * DBAND;
    if (y0 >= H) return;                                  // uniform over the workgroup
    const int y1 = min(H, y0 + DBAND);
    const float *L = maps + planes * fd.px_off;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint8_t *kp = GATED ? keep + fd.keep_start : nullptr;
    const int64_t plane = (int64_t)H * W;
    if (lane == 0)
        for (int r = 0; r < DBAND; ++r) wcnt[r][wave] = 0;
    // is (yy, xx) a present pixel: in the frame and in a kept gate tile
    // (branch-free: the keep byte is read at clamped coordinates)
    auto present = [&](int yy, int xx) -> bool {
        const bool in = ((unsigned)yy < (unsigned)H) & ((unsigned)xx < (unsigned)W);
        if constexpr (!GATED) return in;
        const int yc = min(max(yy, 0), H - 1), xc = min(max(xx, 0), W - 1);
        return in & (kp[(yc / GATE_TILE) * fd.gtx + xc / GATE_TILE] != 0);
    };
    // the logit plane as a buffer resource: each load is a per-lane column
    // offset plus the row's offset (uniform) plus the group's immediate, so the
    // many loads in flight cost few address registers; a load past the plane
    // reads zero, and every position off the frame is replaced by -inf below
    const __amdgpu_buffer_rsrc_t rl = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(L), (short)0, (int)min<int64_t>(plane * 4, 0x7FFFFFFF), (int)0x00020000);
    for (int x0 = wave * 256; x0 < W; x0 += 1024) {
        const int hx = lane == 0 ? x0 - 1 : x0 + 256;     // halo column (lanes 0 and 63)
        const int vo = (x0 + lane) * 4, ho = min(max(hx, 0), W - 1) * 4;
        v4f v[DROWS];
        float h[DROWS];
#pragma unroll
        for (int r = 0; r < DROWS; ++r) {
            const int ro = __builtin_amdgcn_readfirstlane(min(max(y0 - 1 + r, 0), H - 1) * W * 4);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[r][e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rl, vo + 256 * e, ro, 0));
            h[r] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rl, ho, ro, 0));
        }
#pragma unroll
        for (int r = 0; r < DROWS; ++r) {
            const int yy = y0 - 1 + r;
#pragma unroll
            for (int e = 0; e < 4; ++e) v[r][e] = present(yy, x0 + lane + 64 * e) ? v[r][e] : -INFINITY;
            h[r] = present(yy, hx) ? h[r] : -INFINITY;
        }
        // left / right neighbours of row r's values (a sliding window of three rows)
        // (DPP whole-wave shifts by one lane: wave_shr1 gives lane i the value
        // of lane i - 1, wave_shl1 that of lane i + 1)
        auto shr1 = [](float x) {
            return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x138, 0xF, 0xF, false));
        };
        auto shl1 = [](float x) {
            return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), 0x130, 0xF, 0xF, false));
        };
        auto lane_val = [](float x, int l) {
            return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), l));
        };
        auto sides = [&](int r, v4f &lf, v4f &rt) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float up = shr1(v[r][e]), dn = shl1(v[r][e]);
                // across a group boundary: the neighbouring group's end lane
                const float pl = e > 0 ? lane_val(v[r][e > 0 ? e - 1 : 0], 63) : h[r];
                const float nx = e < 3 ? lane_val(v[r][e < 3 ? e + 1 : 3], 0) : lane_val(h[r], 63);
                lf[e] = lane == 0 ? pl : up;
                rt[e] = lane == 63 ? nx : dn;
            }
        };
        v4f lf0, rt0, lf1, rt1, lf2, rt2;
        sides(0, lf0, rt0);
        sides(1, lf1, rt1);
#pragma unroll
        for (int r = 0; r < DBAND; ++r) {
            const int yy = y0 + r;
            if (yy >= y1) break;                          // uniform
            sides(r + 2, lf2, rt2);
            uint32_t cnt = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float c = v[r + 1][e];
                // neighbours earlier in raster order must be strictly smaller;
                // later ones may tie
                bool det = c > tau && c > lf0[e] && c > v[r][e] && c > rt0[e] && c > lf1[e] && c >= rt1[e] &&
                           c >= lf2[e] && c >= v[r + 2][e] && c >= rt2[e];
                if (SIGMA && det) {
                    const int64_t idx = (int64_t)yy * W + x0 + lane + 64 * e;
                    det = L[5 * plane + idx] <= u_max && L[6 * plane + idx] <= u_max;
                }
                const uint64_t m = __ballot(det);
                const int xb = x0 + 64 * e;
                if (lane == 0 && xb < W) mask[fd.mask_start + (int64_t)yy * fd.words + (xb >> 6)] = m;
                cnt += (uint32_t)__popcll(m);
            }
            if (lane == 0) wcnt[r][wave] += cnt;
            lf0 = lf1; rt0 = rt1; lf1 = lf2; rt1 = rt2;
        }
    }
    __syncthreads();
    for (int i = tid; i < y1 - y0; i += 256)
        row_counts[fd.row_start + y0 + i] = wcnt[i][0] + wcnt[i][1] + wcnt[i][2] + wcnt[i][3];
}

// ----------------------------------------------------------------- scan
// Exclusive scan of the per-row counts over the whole batch (one workgroup:
// each thread sums a contiguous chunk, the chunk sums are scanned in LDS, and
// each thread writes its chunk's offsets), then per-frame counts and total.
__global__ void __launch_bounds__(1024)
k_scan(const uint32_t *__restrict__ rc, int64_t R, const FrameDesc *__restrict__ fdp, int nf,
       const int64_t *__restrict__ dyn, uint32_t *__restrict__ row_off, uint32_t *__restrict__ counts)
{
    if (dyn) {
        nf = (int)dyn[DYN_NF];
        R = dyn[DYN_ROWS];
    }
    __shared__ uint32_t sh[1024];
    const int tid = threadIdx.x;
    const int64_t per = (R + 1023) / 1024;
    const int64_t lo = (int64_t)tid * per;
    const int64_t hi = lo + per < R ? lo + per : R;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += rc[i];
    sh[tid] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t v = tid >= o ? sh[tid - o] : 0u;
        __syncthreads();
        sh[tid] += v;
        __syncthreads();
    }
    uint32_t run = sh[tid] - s;
    for (int64_t i = lo; i < hi; ++i) {
        row_off[i] = run;
        run += rc[i];
    }
    if (tid == 1023) row_off[R] = sh[1023];
    __syncthreads();
    for (int f = tid; f < nf; f += 1024) {
        const FrameDesc fd = fdp[f];
        counts[f] = row_off[fd.row_start + fd.h] - row_off[fd.row_start];
    }
    if (tid == 0) counts[nf] = sh[1023];
}

// ----------------------------------------------------------------- emit
// One workgroup per global row: each wave takes its mask word, the block
// scans the 4 word counts, and every detected lane writes its record at
// row_off[row] + (detections before it in raster order).  Records beyond
// `cap` are dropped (the total is still reported by the scan).
__global__ void __launch_bounds__(256)
k_emit(const float *__restrict__ maps, int planes, const uint64_t *__restrict__ mask,
       const uint32_t *__restrict__ row_off, const FrameDesc *__restrict__ fdp, int nf,
       const int64_t *__restrict__ dyn, float z_scale, float ph_scale, float bg_scale, dl_emitter *__restrict__ out,
       dl_uncertainty *__restrict__ unc, uint64_t cap)
{
    const int64_t row = blockIdx.x;
    if (dyn) {
        if (row >= dyn[DYN_ROWS]) return;                 // past the rows of this batch
        nf = (int)dyn[DYN_NF];
    }
    const int f = find_frame(fdp, nf, row, [](const FrameDesc &d) { return d.row_start; });
    const FrameDesc fd = fdp[f];
    const int y = (int)(row - fd.row_start);
    const int W = fd.w;
    const int64_t plane = (int64_t)fd.h * W;
    const float *M = maps + planes * fd.px_off + (int64_t)y * W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ uint32_t sc[4];
    uint32_t base = row_off[row];
    for (int xb0 = 0; xb0 < W; xb0 += 256) {
        const int xb = xb0 + wave * 64;
        const uint64_t m = xb < W ? mask[fd.mask_start + (int64_t)y * fd.words + (xb >> 6)] : 0ull;
        __syncthreads();
        if (lane == 0) sc[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t wb = base;
        for (int k = 0; k < wave; ++k) wb += sc[k];
        const uint32_t tot = sc[0] + sc[1] + sc[2] + sc[3];
        if ((m >> lane) & 1ull) {
            const uint64_t below = lane ? (m & ((1ull << lane) - 1ull)) : 0ull;
            const uint64_t idx = (uint64_t)wb + (uint64_t)__popcll(below);
            if (idx < cap) {
                const int x = xb + lane;
                const float lg = M[x];
                dl_emitter e;
                e.frame = f;
                e.row = y;
                e.col = x;
                e.x_px = (float)x + 0.5f + M[plane + x];
                e.y_px = (float)y + 0.5f + M[2 * plane + x];
                e.z_nm = M[3 * plane + x] * z_scale;
                e.photons = M[4 * plane + x] * ph_scale;
                e.prob = 1.f / (1.f + expf(-lg));
                out[idx] = e;
                if (unc) {
                    // softplus(u) = max(u, 0) + log1p(exp(-|u|)): positive, no overflow
                    auto sp = [](float u) { return fmaxf(u, 0.f) + log1pf(expf(-fabsf(u))); };
                    dl_uncertainty q;
                    q.sigma_x_px = sp(M[5 * plane + x]) + DL_SIGMA_FLOOR;
                    q.sigma_y_px = sp(M[6 * plane + x]) + DL_SIGMA_FLOOR;
                    q.sigma_z_nm = (sp(M[7 * plane + x]) + DL_SIGMA_FLOOR) * z_scale;
                    q.sigma_photons = (sp(M[8 * plane + x]) + DL_SIGMA_FLOOR) * ph_scale;
                    q.background = sp(M[9 * plane + x]) * bg_scale;
                    unc[idx] = q;
                }
            }
        }
        base += tot;
    }
}

__global__ void __launch_bounds__(256)
k_mask_to_u8(const uint64_t *__restrict__ mask, const FrameDesc *__restrict__ fdp, int nf,
             uint8_t *__restrict__ det)
{
    const int64_t row = blockIdx.x;
    const int f = find_frame(fdp, nf, row, [](const FrameDesc &d) { return d.row_start; });
    const FrameDesc fd = fdp[f];
    const int y = (int)(row - fd.row_start);
    for (int x = threadIdx.x; x < fd.w; x += 256) {
        const uint64_t m = mask[fd.mask_start + (int64_t)y * fd.words + (x >> 6)];
        det[fd.px_off + (int64_t)y * fd.w + x] = (uint8_t)((m >> (x & 63)) & 1ull);
    }
}

// detection flags (one byte per pixel, non-zero = detected) -> the mask
// words and per-row counts the scan and emit kernels read: one workgroup per
// global row, one 64-bit ballot per wave and 64 pixels
__global__ void __launch_bounds__(256)
k_mask_from_u8(const uint8_t *__restrict__ det, const FrameDesc *__restrict__ fdp, int nf,
               uint64_t *__restrict__ mask, uint32_t *__restrict__ row_counts)
{
    const int64_t row = blockIdx.x;
    const int f = find_frame(fdp, nf, row, [](const FrameDesc &d) { return d.row_start; });
    const FrameDesc fd = fdp[f];
    const int y = (int)(row - fd.row_start);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t cnt = 0;
    for (int xb = wave * 64; xb < fd.w; xb += 256) {
        const int x = xb + lane;
        const bool d = x < fd.w && det[fd.px_off + (int64_t)y * fd.w + x] != 0;
        const uint64_t m = __ballot(d);
        if (lane == 0) mask[fd.mask_start + (int64_t)y * fd.words + (xb >> 6)] = m;
        cnt += (uint32_t)__popcll(m);
    }
    __shared__ uint32_t sc[4];
    if (lane == 0) sc[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) row_counts[row] = sc[0] + sc[1] + sc[2] + sc[3];
}

// ------------------------------------------------ descriptors on the device
// One workgroup turns a ROI list ([int64 n][dl_roi x n], copied from a pinned
// slot by a graph's first node) into the batch's frame descriptors: per ROI
// its pixels, activation points (the largest layout the net uses), rows,
// detection words and conv tiles of every block; each descriptor offset is
// the exclusive prefix sum of that quantity over the ROIs before it (each
// thread sums a contiguous chunk of ROIs, the chunk sums are scanned in
// LDS).  dyn receives the frame count, the total rows and each block's tiles.
constexpr int ENQ = 4 + MAXBLK;      // pixels, activation points, rows, words, tiles per block

__device__ int64_t enum_quantity(int q, int h, int w, const EnumArgs &e)
{
    if (q == 0) return (int64_t)h * w;
    if (q == 1) {
        int64_t m = 0;
        for (int i = 0; i < e.nl; ++i) m = max(m, act_points(h, w, e.layouts[i]));
        return m;
    }
    if (q == 2) return h;
    if (q == 3) return (int64_t)h * ((w + 63) / 64);
    return conv_tiles(h, w, e.dil[q - 4], e.tr[q - 4], e.tc);
}

__global__ void __launch_bounds__(1024)
k_enumerate(const char *__restrict__ in, EnumArgs e, FrameDesc *__restrict__ fd, int64_t *__restrict__ dyn)
{
    __shared__ int64_t sh[1024];
    const int64_t n = *reinterpret_cast<const int64_t *>(in);
    const dl_roi *r = reinterpret_cast<const dl_roi *>(in + 8);
    const int tid = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t k0 = min(n, (int64_t)tid * per), k1 = min(n, k0 + per);
    int64_t base[ENQ];
#pragma unroll
    for (int q = 0; q < ENQ; ++q) {
        base[q] = 0;
        if (q >= 4 + e.nb) continue;                       // uniform
        int64_t sum = 0;
        for (int64_t k = k0; k < k1; ++k) sum += enum_quantity(q, r[k].h, r[k].w, e);
        sh[tid] = sum;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t v = tid >= o ? sh[tid - o] : 0;
            __syncthreads();
            sh[tid] += v;
            __syncthreads();
        }
        base[q] = sh[tid] - sum;
        if (tid == 1023) {
            if (q == 2) dyn[DYN_ROWS] = sh[1023];
            if (q >= 4) dyn[DYN_TILES + q - 4] = sh[1023];
        }
        __syncthreads();
    }
    for (int64_t k = k0; k < k1; ++k) {
        const int h = r[k].h, w = r[k].w;
        FrameDesc d;
        d.data = r[k].data;
        d.stride = r[k].row_stride;
        d.px_off = base[0];
        d.act_off = base[1];
        d.row_start = base[2];
        d.mask_start = base[3];
        d.keep_start = 0;
#pragma unroll
        for (int b = 0; b < MAXBLK; ++b) d.tile_start[b] = b < e.nb ? base[4 + b] : 0;
        d.h = h;
        d.w = w;
        d.words = (w + 63) / 64;
        d.gtx = w / GATE_TILE;
        d.gty = h / GATE_TILE;
        d.pad_ = 0;
        fd[k] = d;
#pragma unroll
        for (int q = 0; q < ENQ; ++q)
            if (q < 4 + e.nb) base[q] += enum_quantity(q, h, w, e);
    }
    if (tid == 0) {
        dyn[DYN_NF] = n;
        for (int b = e.nb; b < MAXBLK; ++b) dyn[DYN_TILES + b] = 0;
    }
}

// ----------------------------------------------------------- gated runs
__global__ void __launch_bounds__(256)
k_gate_keep(const float *__restrict__ logits, int64_t n, float tau, uint8_t *__restrict__ keep)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) keep[t] = logits[t] > tau ? 1 : 0;
}

__global__ void __launch_bounds__(256)
k_zero_u32(uint32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// One thread per conv tile of frame blockIdx.z and block blockIdx.y: append the tile to the
// lists of the block's two layers when their radius brings it within reach
// of a kept gate tile.  A wave appends its (consecutive) tiles as one run with
// one atomic, so a list keeps the tile order within runs of up to 64 tiles
// and the conv kernels keep their L2 locality; the order of the runs depends
// on atomic arrival, which changes only which workgroup computes a tile.
__global__ void __launch_bounds__(256)
k_active_lists(const FrameDesc *__restrict__ fdp, Geometry geo, const uint8_t *__restrict__ keep,
               const int *__restrict__ radius, const int *__restrict__ dil, int32_t *__restrict__ lists,
               uint32_t *__restrict__ counts)
{
    const int b = blockIdx.y, f = blockIdx.z;
    const FrameDesc &fd = fdp[f];           // read in place: tile_start is indexed by the block
    const int64_t first = ld_const(&fd.tile_start[b]);
    const int64_t end = f + 1 < geo.nf ? ld_const(&fdp[f + 1].tile_start[b]) : geo.tiles[b];
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x, t = first + l;
    const int lane = threadIdx.x & 63;
    bool act[2] = {false, false};
    if (t < end) {
        const int d = dil[b];
        int Y0, X0;
        decode_tile(fd.h, fd.w, l, d, geo.trb[b], geo.tc, b == geo.minor_blk, geo.strip, Y0, X0);
        if (Y0 < fd.h && X0 < fd.w) {
            const int y1 = min(fd.h - 1, Y0 + d * (geo.trb[b] - 1)), x1 = min(fd.w - 1, X0 + d * (geo.tc - 1));
            for (int k = 0; k < 2; ++k) act[k] = near_kept(keep, fd, Y0, y1, X0, x1, radius[2 * b + k]);
        }
    }
    for (int k = 0; k < 2; ++k) {
        const int l = 2 * b + k;
        const uint64_t m = __ballot(act[k]);
        if (m == 0) continue;
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&counts[l], (uint32_t)__popcll(m));
        base = __shfl(base, 0);
        if (act[k]) {
            const uint32_t rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            lists[(int64_t)l * geo.max_tiles + base + rank] = (int32_t)t;
        }
    }
}

}  // namespace

hipError_t launch_gate_keep(const float *logits, int64_t n, float tau, uint8_t *keep, hipStream_t s)
{
    hipLaunchKernelGGL(k_gate_keep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, logits, n, tau, keep);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_active_lists(const FrameDesc *fd, const Geometry &g, const uint8_t *keep, const int *radius,
                               const int *dil, int nlayers, int32_t *lists, uint32_t *counts, hipStream_t s)
{
    hipError_t e = launch_zero_u32(counts, nlayers, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_active_lists, dim3((unsigned)((g.max_frame_tiles + 255) / 256), nlayers / 2, g.nf), dim3(256), 0, s,
                       fd, g, keep, radius, dil, lists, counts);
    return hipGetLastError();
}

hipError_t launch_stem(int C, const FrameDesc *fd, const Geometry &g, const float *w, const float *b,
                       float offset, float scale, const float2 *cam, void *act, int precision,
                       const uint8_t *keep, int radius, hipStream_t s)
{
    switch (C) {
    case 16: return stem_c<16>(fd, g, w, b, offset, scale, cam, act, precision, keep, radius, s);
    case 32: return stem_c<32>(fd, g, w, b, offset, scale, cam, act, precision, keep, radius, s);
    case 48: return stem_c<48>(fd, g, w, b, offset, scale, cam, act, precision, keep, radius, s);
    case 64: return stem_c<64>(fd, g, w, b, offset, scale, cam, act, precision, keep, radius, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_detect_mask(const float *maps, int planes, const FrameDesc *fd, const Geometry &g, float tau,
                              float u_max, const uint8_t *keep, uint64_t *mask, uint32_t *row_counts,
                              hipStream_t s)
{
    const int bands = (g.maxh + DBAND - 1) / DBAND;
    const int64_t blocks = (int64_t)bands * g.nf;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    const bool sigma = planes == 10 && u_max < INFINITY;
    auto kern = keep ? (sigma ? k_detect_mask<true, true> : k_detect_mask<true, false>)
                     : (sigma ? k_detect_mask<false, true> : k_detect_mask<false, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, s, maps, planes, fd, bands, g.dyn, tau, u_max, keep,
                       mask, row_counts);
    return hipGetLastError();
}

hipError_t launch_scan(const uint32_t *row_counts, const FrameDesc *fd, const Geometry &g,
                       uint32_t *row_off, uint32_t *counts, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, row_counts, g.total_rows, fd, g.nf, g.dyn, row_off, counts);
    return hipGetLastError();
}

hipError_t launch_emit(const float *maps, int planes, const uint64_t *mask, const uint32_t *row_off,
                       const FrameDesc *fd, const Geometry &g, float z_scale, float ph_scale,
                       float bg_scale, dl_emitter *out, dl_uncertainty *unc, uint64_t cap, hipStream_t s)
{
    hipLaunchKernelGGL(k_emit, dim3((unsigned)g.total_rows), dim3(256), 0, s, maps, planes, mask, row_off, fd, g.nf, g.dyn,
                       z_scale, ph_scale, bg_scale, out, unc, cap);
    return hipGetLastError();
}

hipError_t launch_enumerate(const void *in, const EnumArgs &e, FrameDesc *fd, int64_t *dyn, hipStream_t s)
{
    hipLaunchKernelGGL(k_enumerate, dim3(1), dim3(1024), 0, s, static_cast<const char *>(in), e, fd, dyn);
    return hipGetLastError();
}

hipError_t launch_mask_from_u8(const uint8_t *det, const FrameDesc *fd, const Geometry &g, uint64_t *mask,
                               uint32_t *row_counts, hipStream_t s)
{
    hipLaunchKernelGGL(k_mask_from_u8, dim3((unsigned)g.total_rows), dim3(256), 0, s, det, fd, g.nf, mask, row_counts);
    return hipGetLastError();
}

hipError_t launch_mask_to_u8(const uint64_t *mask, const FrameDesc *fd, const Geometry &g,
                             uint8_t *det, hipStream_t s)
{
    hipLaunchKernelGGL(k_mask_to_u8, dim3((unsigned)g.total_rows), dim3(256), 0, s, mask, fd, g.nf, det);
    return hipGetLastError();
}

}  // namespace dloc
