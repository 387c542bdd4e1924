// 3x3 dilated convolution layers as MFMA implicit GEMM (gfx950).
//
// Operation (paper Sec. 3.2.1, dilated convolution; Sec. 3.2, DECODE-style
// per-pixel head): for every output pixel p and output channel o
//     y[p][o] = b[o] + sum_{tap, c} W[o][c][tap] * x[p + d * off(tap)][c]
// with zero padding at the frame border, then optional residual add, ReLU and
// an optional fused 1x1 head (C -> 5 planar maps).
//
// GEMM view: M = output channels (blocks of 16), N = pixels (blocks of 16),
// K = 9 taps x C input channels.  One wave computes one tile row of
// TILE_COLS = 16 * PB pixels for all C output channels; a workgroup of ROWS
// waves computes ROWS consecutive rows.  Workgroups are persistent: the packed
// weights are staged into LDS once and the workgroup then walks its share of
// the tile list.  Tiles are handed out XCD by XCD in contiguous chunks so that
// tiles that share halo rows run on the same XCD and hit the same L2.
//
// Activations are NHWC, so a K-step's channels of one pixel are one
// contiguous 16-byte load.  FP32 (v_mfma_f32_16x16x4_f32): the K order inside
// a tap is permuted so lane group kq handles channels 16 g + 4 kq + s (s = MFMA
// step), i.e. one float4 feeds 4 consecutive MFMA steps.  BF16
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): K is cut into chunks of 8
// channels of one tap; lane group kq of MFMA step m takes chunk 4 m + kq, so
// one 16-byte load of 8 bf16 is one lane's operand (a K that is not a multiple
// of 32 is padded with zero chunks).  The weights are packed in the same K
// order on the host.
#include "dloc_internal.h"

#include <cstring>

namespace dloc {

namespace {

constexpr int NXCD = 8;
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ v4f relu4(v4f v)
{
    v4f r;
    r[0] = fmaxf(v[0], 0.f); r[1] = fmaxf(v[1], 0.f);
    r[2] = fmaxf(v[2], 0.f); r[3] = fmaxf(v[3], 0.f);
    return r;
}

__device__ __forceinline__ uint32_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

// 4 consecutive channels of one pixel, FP32 or BF16 storage
template <int P> struct Act;
template <> struct Act<DL_FP32> {
    typedef float T;
    static constexpr int ESZ = 4;
    __device__ static v4f load4(const void *base, int64_t idx)
    {
        return *reinterpret_cast<const v4f *>(static_cast<const float *>(base) + idx);
    }
    __device__ static void store4(void *base, int64_t idx, v4f v)
    {
        *reinterpret_cast<v4f *>(static_cast<float *>(base) + idx) = v;
    }
};
template <> struct Act<DL_BF16> {
    static constexpr int ESZ = 2;
    __device__ static v4f load4(const void *base, int64_t idx)
    {
        const uint2 u = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(base) + idx);
        return v4f{__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xFFFF0000u),
                   __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xFFFF0000u)};
    }
    __device__ static void store4(void *base, int64_t idx, v4f v)
    {
        uint2 u;
        u.x = bf16_rne(v[0]) | (bf16_rne(v[1]) << 16);
        u.y = bf16_rne(v[2]) | (bf16_rne(v[3]) << 16);
        *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(base) + idx) = u;
    }
};

// K iterations and packed-weight size per precision
template <int C, int P> struct KPlan;
template <int C> struct KPlan<C, DL_FP32> {
    static constexpr int NIT = 9 * (C / 16);               // float4 = 4 MFMA steps each
    static constexpr int BYTES = 9 * C * C * 4;
};
template <int C> struct KPlan<C, DL_BF16> {
    static constexpr int CH8 = C / 8;                      // 8-channel chunks per tap
    static constexpr int NCH = 9 * CH8;
    static constexpr int NIT = (NCH + 3) / 4;              // one MFMA step each
    static constexpr int BYTES = NIT * (C / 16) * 64 * 16;
};

template <int C, int P>
constexpr size_t conv_smem()
{
    return (size_t)KPlan<C, P>::BYTES + (size_t)C * 4 + (size_t)(5 * C + 5) * 4;
}

// --------------------------------------------------------------- kernel
template <int C, int ROWS, bool RES, bool HEAD, int P>
__global__ void __launch_bounds__(ROWS * 64)
k_conv(ConvArgs a, Geometry geo)
{
    constexpr int NB = C / 16;            // output-channel blocks
    constexpr int NIT = KPlan<C, P>::NIT;
    constexpr int WBYTES = KPlan<C, P>::BYTES;
    extern __shared__ v4f smem[];
    v4f *sW = smem;                                                    // packed weights
    float *sB = reinterpret_cast<float *>(reinterpret_cast<char *>(smem) + WBYTES);   // bias [C]
    float *sH = sB + C;                                                // head [5C + 5]

    {
        const v4f *gw = reinterpret_cast<const v4f *>(a.wpk);
        for (int i = threadIdx.x; i < WBYTES / 16; i += ROWS * 64) sW[i] = gw[i];
        for (int i = threadIdx.x; i < C; i += ROWS * 64) sB[i] = a.bias[i];
        if (HEAD)
            for (int i = threadIdx.x; i < 5 * C + 5; i += ROWS * 64) sH[i] = a.head[i];
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int j = lane & 15;       // pixel within a 16-pixel block
    const int kq = lane >> 4;      // K lane group
    const int dd = a.d;

    const int64_t T = a.list ? (int64_t)*a.list_count : geo.total_tiles;
    const int xcd = blockIdx.x % NXCD;
    const int slot = blockIdx.x / NXCD;
    const int nslot = gridDim.x / NXCD;
    const int64_t chunk = (T + NXCD - 1) / NXCD;
    const int64_t t0 = (int64_t)xcd * chunk;
    const int64_t t1 = t0 + chunk < T ? t0 + chunk : T;

    for (int64_t ti = t0 + slot; ti < t1; ti += nslot) {
        const int64_t t = a.list ? (int64_t)a.list[ti] : ti;
        const int f = find_frame(a.fd, geo.nf, t, [](const FrameDesc &d) { return d.tile_start; });
        const FrameDesc fd = a.fd[f];
        const int64_t local = t - fd.tile_start;
        const int ty = (int)(local / fd.tiles_x);
        const int tx = (int)(local - (int64_t)ty * fd.tiles_x);
        const int y = ty * ROWS + wave;
        const int x0 = tx * TILE_COLS;
        const int H = fd.h, W = fd.w;
        if (y >= H) continue;      // wave-uniform; no barrier follows

        v4f acc[NB][PB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int p = 0; p < PB; ++p) acc[nb][p] = v4f{0.f, 0.f, 0.f, 0.f};

        if constexpr (P == DL_FP32) {
            constexpr int G = C / 16;
            const float *base = static_cast<const float *>(a.in) + fd.px_off * C;
            v4f bb[2][PB];
            auto load_b = [&](v4f *dst, int it) {
                const int tap = it / G, gg = it - (it / G) * G;
                const int yy = y + (tap / 3 - 1) * dd;
                const int dx = (tap % 3 - 1) * dd;
                const bool rok = (unsigned)yy < (unsigned)H;
                const float *rp = base + (int64_t)yy * W * C + gg * 16 + kq * 4;
#pragma unroll
                for (int p = 0; p < PB; ++p) {
                    const int xx = x0 + p * 16 + j + dx;
                    const bool ok = rok && (unsigned)xx < (unsigned)W;
                    dst[p] = ok ? *reinterpret_cast<const v4f *>(rp + (int64_t)xx * C) : v4f{0.f, 0.f, 0.f, 0.f};
                }
            };
            load_b(bb[0], 0);
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                if (it + 1 < NIT) load_b(bb[(it + 1) & 1], it + 1);
                v4f av[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) av[nb] = sW[(it * NB + nb) * 64 + lane];
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int p = 0; p < PB; ++p)
                            acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[nb][s], bb[it & 1][p][s],
                                                                              acc[nb][p], 0, 0, 0);
            }
        } else {
            constexpr int CH8 = KPlan<C, P>::CH8, NCH = KPlan<C, P>::NCH;
            const uint16_t *base = static_cast<const uint16_t *>(a.in) + fd.px_off * C;
            v4f bb[2][PB];      // 16 bytes = 8 bf16 per lane
            auto load_b = [&](v4f *dst, int it) {
                const int ch = it * 4 + kq;                 // this lane group's chunk
                const bool real = ch < NCH;
                const int tap = real ? ch / CH8 : 4;
                const int c0 = real ? (ch - tap * CH8) * 8 : 0;
                const int yy = y + (tap / 3 - 1) * dd;
                const int dx = (tap % 3 - 1) * dd;
                const bool rok = real && (unsigned)yy < (unsigned)H;
                const uint16_t *rp = base + (int64_t)yy * W * C + c0;
#pragma unroll
                for (int p = 0; p < PB; ++p) {
                    const int xx = x0 + p * 16 + j + dx;
                    const bool ok = rok && (unsigned)xx < (unsigned)W;
                    dst[p] = ok ? *reinterpret_cast<const v4f *>(rp + (int64_t)xx * C) : v4f{0.f, 0.f, 0.f, 0.f};
                }
            };
            load_b(bb[0], 0);
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                if (it + 1 < NIT) load_b(bb[(it + 1) & 1], it + 1);
                v4f av[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) av[nb] = sW[(it * NB + nb) * 64 + lane];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int p = 0; p < PB; ++p)
                        acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(v8bf, av[nb]), __builtin_bit_cast(v8bf, bb[it & 1][p]),
                            acc[nb][p], 0, 0, 0);
            }
        }

        // epilogue: D row = output channel 16 nb + 4 kq + r, column = pixel j
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int px = x0 + p * 16 + j;
            const bool ok = px < W;
            const int64_t pix = fd.px_off + (int64_t)y * W + px;
            float h0 = 0.f, h1 = 0.f, h2 = 0.f, h3 = 0.f, h4 = 0.f;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int oc = nb * 16 + kq * 4;
                v4f v = acc[nb][p];
                v[0] += sB[oc + 0]; v[1] += sB[oc + 1]; v[2] += sB[oc + 2]; v[3] += sB[oc + 3];
                if (RES && ok) v += Act<P>::load4(a.res, pix * C + oc);
                v = relu4(v);
                if (!HEAD) {
                    if (ok) Act<P>::store4(a.out, pix * C + oc, v);
                } else {
                    if (P != DL_FP32) {       // the head reads the stored (rounded) features
                        v[0] = __uint_as_float(bf16_rne(v[0]) << 16);
                        v[1] = __uint_as_float(bf16_rne(v[1]) << 16);
                        v[2] = __uint_as_float(bf16_rne(v[2]) << 16);
                        v[3] = __uint_as_float(bf16_rne(v[3]) << 16);
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        h0 += sH[0 * C + oc + r] * v[r];
                        h1 += sH[1 * C + oc + r] * v[r];
                        h2 += sH[2 * C + oc + r] * v[r];
                        h3 += sH[3 * C + oc + r] * v[r];
                        h4 += sH[4 * C + oc + r] * v[r];
                    }
                }
            }
            if (HEAD) {
                h0 += __shfl_xor(h0, 16); h0 += __shfl_xor(h0, 32);
                h1 += __shfl_xor(h1, 16); h1 += __shfl_xor(h1, 32);
                h2 += __shfl_xor(h2, 16); h2 += __shfl_xor(h2, 32);
                h3 += __shfl_xor(h3, 16); h3 += __shfl_xor(h3, 32);
                h4 += __shfl_xor(h4, 16); h4 += __shfl_xor(h4, 32);
                if (ok) {
                    const int64_t plane = (int64_t)H * W;
                    float *mp = a.maps + 5 * fd.px_off + (int64_t)y * W + px;
                    const float mine = kq == 0 ? h0 : kq == 1 ? h1 : kq == 2 ? h2 : h3;
                    mp[kq * plane] = mine + sH[5 * C + kq];
                    if (kq == 0) mp[4 * plane] = h4 + sH[5 * C + 4];
                }
            }
        }
    }
}

// ------------------------------------------------------------- launchers
template <int C, int ROWS, bool RES, bool HEAD, int P>
hipError_t launch_t(const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    auto kern = k_conv<C, ROWS, RES, HEAD, P>;
    constexpr size_t sh = conv_smem<C, P>();
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(ROWS * 64), sh, s, a, g);
    return hipGetLastError();
}

template <int C, int ROWS, int P>
hipError_t launch_rows(const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    if (a.head) return launch_t<C, ROWS, true, true, P>(a, g, grid, s);
    if (a.res) return launch_t<C, ROWS, true, false, P>(a, g, grid, s);
    return launch_t<C, ROWS, false, false, P>(a, g, grid, s);
}

template <int C, int P>
hipError_t launch_c(const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    switch (g.tile_rows) {
    case 4: return launch_rows<C, 4, P>(a, g, grid, s);
    case 8: return launch_rows<C, 8, P>(a, g, grid, s);
    case 16: return launch_rows<C, 16, P>(a, g, grid, s);
    default: return hipErrorInvalidValue;
    }
}

template <int C, int P>
hipError_t launch_cp(const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    return launch_c<C, P>(a, g, grid, s);
}

template <int C, int ROWS, int P>
int blocks_per_cu()
{
    int nb = 0;
    auto kern = k_conv<C, ROWS, true, false, P>;
    constexpr size_t sh = conv_smem<C, P>();
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, ROWS * 64, sh) != hipSuccess) nb = 1;
    return nb > 0 ? nb : 1;
}

template <int C, int P>
int bpc(int rows)
{
    switch (rows) {
    case 4: return blocks_per_cu<C, 4, P>();
    case 8: return blocks_per_cu<C, 8, P>();
    case 16: return blocks_per_cu<C, 16, P>();
    default: return 1;
    }
}

template <int P>
int bpc_c(int C, int rows)
{
    switch (C) {
    case 16: return bpc<16, P>(rows);
    case 32: return bpc<32, P>(rows);
    case 48: return bpc<48, P>(rows);
    case 64: return bpc<64, P>(rows);
    default: return 1;
    }
}

template <int P>
hipError_t launch_p(int C, const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    switch (C) {
    case 16: return launch_cp<16, P>(a, g, grid, s);
    case 32: return launch_cp<32, P>(a, g, grid, s);
    case 48: return launch_cp<48, P>(a, g, grid, s);
    case 64: return launch_cp<64, P>(a, g, grid, s);
    default: return hipErrorInvalidValue;
    }
}

uint16_t host_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace

size_t conv_packed_bytes(int C, int precision)
{
    const int NB = C / 16;
    if (precision == DL_FP32) return (size_t)9 * C * C * 4;
    const int nit = (9 * (C / 8) + 3) / 4;
    return (size_t)nit * NB * 64 * 16;
}

void pack_conv_weights(int C, int precision, const float *W, void *dst)
{
    const int NB = C / 16;
    if (precision == DL_FP32) {
        const int G = C / 16;
        float *o = static_cast<float *>(dst);
        for (int tap = 0; tap < 9; ++tap)
            for (int g = 0; g < G; ++g)
                for (int nb = 0; nb < NB; ++nb)
                    for (int lane = 0; lane < 64; ++lane)
                        for (int s = 0; s < 4; ++s) {
                            const int oc = nb * 16 + (lane & 15);
                            const int c = g * 16 + 4 * (lane >> 4) + s;
                            const int it = tap * G + g;
                            o[((size_t)(it * NB + nb) * 64 + lane) * 4 + s] = W[((size_t)oc * C + c) * 9 + tap];
                        }
        return;
    }
    // BF16: step m, block nb, lane (i, kq): 8 bf16 of chunk ch = 4 m + kq
    const int CH8 = C / 8, NCH = 9 * CH8, NIT = (NCH + 3) / 4;
    uint16_t *o = static_cast<uint16_t *>(dst);
    for (int m = 0; m < NIT; ++m)
        for (int nb = 0; nb < NB; ++nb)
            for (int lane = 0; lane < 64; ++lane) {
                const int oc = nb * 16 + (lane & 15);
                const int ch = 4 * m + (lane >> 4);
                for (int e = 0; e < 8; ++e) {
                    float v = 0.f;
                    if (ch < NCH) {
                        const int tap = ch / CH8, c = (ch % CH8) * 8 + e;
                        v = W[((size_t)oc * C + c) * 9 + tap];
                    }
                    o[((size_t)(m * NB + nb) * 64 + lane) * 8 + e] = host_bf16(v);
                }
            }
}

int conv_max_grid(int C, int precision, int tile_rows, int ncu)
{
    const int b = precision == DL_FP32 ? bpc_c<DL_FP32>(C, tile_rows) : bpc_c<DL_BF16>(C, tile_rows);
    return b * ncu;
}

hipError_t launch_conv(int C, int precision, const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    if (precision == DL_FP32) return launch_p<DL_FP32>(C, a, g, grid, s);
    if (precision == DL_BF16) return launch_p<DL_BF16>(C, a, g, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace dloc
