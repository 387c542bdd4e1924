// 3x3 dilated convolution layers as MFMA implicit GEMM (gfx950).
//
// Operation (paper Sec. 3.2.1, dilated convolution; Sec. 3.2, DECODE-style
// per-pixel head): for every output pixel p and output channel o
//     y[p][o] = b[o] + sum_{tap, c} W[o][c][tap] * x[p + d * off(tap)][c]
// with zero padding at the frame border, then optional residual add, ReLU and
// an optional fused 1x1 head (C -> 5 planar maps).
//
// Tiling.  A layer of dilation d works on phase tiles (see conv_tiles): a
// workgroup computes TR x TC output pixels spaced d apart, whose input is the
// (TR + 2) x (TC + 2) lattice points around them -- the same LDS footprint
// for every dilation.  The workgroup stages that input once into LDS (points
// padded so 16-byte reads of consecutive points hit distinct banks), then
// wave w computes lattice row w for all C output channels.  Workgroups are
// persistent; tiles are handed out XCD by XCD in contiguous ranges, and
// consecutive tiles are the d*d phases of one region, so they share L2 lines.
//
// GEMM view: M = output channels (blocks of 16), N = pixels (blocks of 16),
// K = 9 taps x C input channels.
//   FP32  v_mfma_f32_16x16x4_f32; lane group kq takes channels 16 g + 4 kq + s
//         (s = MFMA step), so one float4 feeds 4 steps.  Weights are read from
//         global memory (they stay in L1/L2), one K iteration ahead.
//   BF16  v_mfma_f32_16x16x32_bf16 (FP32 accumulation); K is cut into chunks
//         of 8 channels of one tap and lane group kq of step m takes chunk
//         4 m + kq (one 16-byte LDS read).  Weights live in LDS.
//   FP8   v_mfma_scale_f32_16x16x128_f8f6f4 with e4m3 operands (unit block
//         scales); lane group kq of step m takes chunks 16 m + 4 kq + 0..3.
//         Activations are stored in BF16; staging quantises them into LDS with
//         the frame's scale amax / 448 (round to nearest even, saturating);
//         weights carry a per-output-channel scale.  The epilogue multiplies
//         the FP32 accumulator by both scales and tracks the max of what it
//         stores, which sets the next layer's scale.
// K is padded with zero-weight chunks when 9 C is not a multiple of the MFMA's K.
#include "dloc_internal.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace dloc {

namespace {

constexpr int NXCD = 8;
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));

// smallest dword count >= dw that is 4 mod 8: 16-byte reads of consecutive
// points then fall into distinct LDS banks
constexpr int pad_dw(int dw) { return dw + ((4 - dw % 8) + 8) % 8; }
constexpr int align16(int b) { return (b + 15) / 16 * 16; }

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

__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float(bf16_rne(f) << 16); }

// OCP e4m3fn code of a finite float: round to nearest even, saturating at
// +-448.  Normal range: round the 23-bit mantissa to 3 bits; below 2^-6 the
// spacing is 2^-9 (subnormals), and 8 * 2^-9 is the smallest normal (code 8).
__device__ __forceinline__ uint32_t f32_to_e4m3(float x)
{
    const uint32_t s = (__float_as_uint(x) >> 24) & 0x80u;
    const float a = fabsf(x);
    if (!(a < 448.f)) return s | 0x7Eu;
    if (a < 0.015625f) return s | (uint32_t)__float2int_rn(a * 512.f);
    uint32_t ua = __float_as_uint(a);
    ua += 0x7FFFFu + ((ua >> 20) & 1u);
    const uint32_t code = (((ua >> 23) - 120u) << 3) | ((ua >> 20) & 7u);
    return s | (code > 0x7Eu ? 0x7Eu : code);
}

// storage of the activations in HBM: FP32, or BF16 (BF16 and FP8 forms)
template <int P> struct Store {
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
template <> struct Store<DL_FP32> {
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

// K plan and packed-weight bytes per precision
template <int C, int P> struct KPlan;
template <int C> struct KPlan<C, DL_FP32> {
    static constexpr int NIT = 9 * (C / 16);
    static constexpr int BYTES = 9 * C * C * 4;
    static constexpr int LDS_W = 0;               // weights stay in global memory
    static constexpr int LESZ = 4;                // LDS bytes per channel
};
template <int C> struct KPlan<C, DL_BF16> {
    static constexpr int CH8 = C / 8, NCH = 9 * CH8;
    static constexpr int NIT = (NCH + 3) / 4;
    static constexpr int BYTES = NIT * (C / 16) * 64 * 16;
    static constexpr int LDS_W = BYTES;
    static constexpr int LESZ = 2;
};
template <int C> struct KPlan<C, DL_FP8> {
    static constexpr int CH8 = C / 8, NCH = 9 * CH8;
    static constexpr int NIT = (NCH + 15) / 16;
    static constexpr int BYTES = NIT * (C / 16) * 64 * 32;
    static constexpr int LDS_W = BYTES;
    static constexpr int LESZ = 1;
};

// lattice columns per tile (TC; the rows, one wave each, are a template choice)
// and the waves per SIMD the register budget is sized for (MINW)
template <int P> struct TileShape;
template <> struct TileShape<DL_FP32> { static constexpr int TC = 32, MINW = 4; };
template <> struct TileShape<DL_BF16> { static constexpr int TC = 64, MINW = 2; };
template <> struct TileShape<DL_FP8> { static constexpr int TC = 64, MINW = 2; };

template <int C, int P, int TR_>
struct Lds {
    static constexpr int TR = TR_, TC = TileShape<P>::TC;
    static constexpr int PS = pad_dw(C * KPlan<C, P>::LESZ / 4) * 4;   // bytes per lattice point
    static constexpr int PW = TC + 2;
    static constexpr int NPT = (TR + 2) * PW;
    static constexpr int TBYTES = align16(NPT * PS);
    static constexpr int WOFF = TBYTES;
    static constexpr int BOFF = WOFF + KPlan<C, P>::LDS_W;            // bias [C]
    static constexpr int HOFF = BOFF + C * 4;                          // head [5C + 5]
    static constexpr int TOTAL = align16(HOFF + (5 * C + 5) * 4);
};

// --------------------------------------------------------------- kernel
template <int C, int P, int TR_, bool RES, bool HEAD>
__global__ void __launch_bounds__(TR_ * 64, TileShape<P>::MINW)
k_conv(ConvArgs a, Geometry geo)
{
    using L = Lds<C, P, TR_>;
    constexpr int TR = L::TR, TC = L::TC, PS = L::PS, PW = L::PW, NPT = L::NPT;
    constexpr int NB = C / 16, PB = TC / 16, NT = TR * 64;
    extern __shared__ v4f smem[];
    char *sT = reinterpret_cast<char *>(smem);
    float *sB = reinterpret_cast<float *>(sT + L::BOFF);
    float *sH = reinterpret_cast<float *>(sT + L::HOFF);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = lane & 15, kq = lane >> 4;
    const int dd = a.d, blk = a.blk;

    if constexpr (KPlan<C, P>::LDS_W > 0) {
        const v4f *gw = static_cast<const v4f *>(a.wpk);
        v4f *sW = reinterpret_cast<v4f *>(sT + L::WOFF);
        for (int i = tid; i < KPlan<C, P>::LDS_W / 16; i += NT) sW[i] = gw[i];
    }
    for (int i = tid; i < C; i += NT) sB[i] = a.bias[i];
    if (HEAD)
        for (int i = tid; i < 5 * C + 5; i += NT) sH[i] = a.head[i];

    const int64_t T = a.list ? (int64_t)*a.list_count : geo.tiles[blk];
    const int xcd = blockIdx.x % NXCD, slot = blockIdx.x / NXCD, nslot = gridDim.x / NXCD;
    const int64_t chunk = (T + NXCD - 1) / NXCD;
    const int64_t t0 = (int64_t)xcd * chunk;
    const int64_t t1 = t0 + chunk < T ? t0 + chunk : T;

    for (int64_t ti = t0 + slot; ti < t1; ti += nslot) {
        const int64_t t = a.list ? (int64_t)a.list[ti] : ti;
        const int f = find_frame(a.fd, geo.nf, t, [blk](const FrameDesc &d) { return d.tile_start[blk]; });
        const FrameDesc &fd = a.fd[f];      // read in place: tile_start is indexed by the block
        int Y0, X0;
        decode_tile(fd, t - fd.tile_start[blk], dd, TR, TC, Y0, X0);
        const int H = fd.h, W = fd.w;
        const int64_t px_off = fd.px_off;
        float qinv = 1.f, qscale = 1.f;          // FP8 activation quantisation
        if constexpr (P == DL_FP8) {
            const float amax = __uint_as_float(a.amax_in[f]);
            qinv = amax > 0.f ? 448.f / amax : 0.f;
            qscale = amax / 448.f;
        }

        __syncthreads();   // the previous tile's LDS reads are done (and weights staged)
        {
            constexpr int SESZ = Store<P>::ESZ;
            constexpr int SCH = C * SESZ / 16;   // 16-byte source chunks per point
            const char *src = static_cast<const char *>(a.in) + px_off * C * SESZ;
            for (int q = tid; q < NPT * SCH; q += NT) {
                const int pt = q / SCH, ch = q - (q / SCH) * SCH;
                const int ii = pt / PW - 1, jj = pt - (pt / PW) * PW - 1;
                const int y = Y0 + dd * ii, x = X0 + dd * jj;
                const bool ok = (unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W;
                v4f v = {0.f, 0.f, 0.f, 0.f};
                if (ok) v = *reinterpret_cast<const v4f *>(src + ((int64_t)y * W + x) * (C * SESZ) + ch * 16);
                if constexpr (P != DL_FP8) {
                    *reinterpret_cast<v4f *>(sT + pt * PS + ch * 16) = v;
                } else {
                    uint32_t q8[8];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const uint32_t w32 = __float_as_uint(v[e]);
                        q8[2 * e] = f32_to_e4m3(__uint_as_float(w32 << 16) * qinv);
                        q8[2 * e + 1] = f32_to_e4m3(__uint_as_float(w32 & 0xFFFF0000u) * qinv);
                    }
                    uint2 o;
                    o.x = q8[0] | (q8[1] << 8) | (q8[2] << 16) | (q8[3] << 24);
                    o.y = q8[4] | (q8[5] << 8) | (q8[6] << 16) | (q8[7] << 24);
                    *reinterpret_cast<uint2 *>(sT + pt * PS + ch * 8) = o;
                }
            }
        }
        __syncthreads();

        const int yo = Y0 + dd * wave;
        if (yo >= H) continue;       // this wave's lattice row is off the frame (barriers are at the loop top)

        v4f acc[NB][PB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int p = 0; p < PB; ++p) acc[nb][p] = v4f{0.f, 0.f, 0.f, 0.f};
        // LDS address of lattice point (row wave + u, column 16 p + j + v) for tap (u, v), u, v in 0..2
        auto pt_addr = [&](int p, int tap) { return sT + ((wave + tap / 3) * PW + 16 * p + j + tap % 3) * PS; };

        if constexpr (P == DL_FP32) {
            constexpr int G = C / 16, NIT = KPlan<C, P>::NIT;
            const v4f *gw = static_cast<const v4f *>(a.wpk);
            v4f awn[NB];                             // weights of the next K iteration
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) awn[nb] = gw[nb * 64 + lane];
#pragma unroll 1
            for (int tap = 0; tap < 9; ++tap) {
#pragma unroll
                for (int gg = 0; gg < G; ++gg) {
                    const int it = tap * G + gg;
                    v4f aw[NB];
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) aw[nb] = awn[nb];
                    if (it + 1 < NIT)
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) awn[nb] = gw[((it + 1) * NB + nb) * 64 + lane];
                    v4f bv[PB];
#pragma unroll
                    for (int p = 0; p < PB; ++p)
                        bv[p] = *reinterpret_cast<const v4f *>(pt_addr(p, tap) + (gg * 16 + kq * 4) * 4);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                            for (int p = 0; p < PB; ++p)
                                acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[nb][s], bv[p][s], acc[nb][p], 0, 0, 0);
                }
            }
        } else if constexpr (P == DL_BF16) {
            constexpr int CH8 = KPlan<C, P>::CH8, NCH = KPlan<C, P>::NCH, NIT = KPlan<C, P>::NIT;
            const char *sW = sT + L::WOFF;
#pragma unroll
            for (int m = 0; m < NIT; ++m) {
                const int ch = 4 * m + kq;
                const int tap = ch < NCH ? ch / CH8 : 4;          // padding chunks have zero weights
                const int c0 = ch < NCH ? (ch - (ch / CH8) * CH8) * 8 : 0;
                v4f av[NB], bv[PB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    av[nb] = *reinterpret_cast<const v4f *>(sW + ((m * NB + nb) * 64 + lane) * 16);
#pragma unroll
                for (int p = 0; p < PB; ++p) bv[p] = *reinterpret_cast<const v4f *>(pt_addr(p, tap) + c0 * 2);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int p = 0; p < PB; ++p)
                        acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(v8bf, av[nb]), __builtin_bit_cast(v8bf, bv[p]), acc[nb][p], 0, 0, 0);
            }
        } else {
            constexpr int CH8 = KPlan<C, P>::CH8, NCH = KPlan<C, P>::NCH, NIT = KPlan<C, P>::NIT;
            const char *sW = sT + L::WOFF;
#pragma unroll 1
            for (int m = 0; m < NIT; ++m) {
                v8i av[NB], bv[PB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const uint4 *pa = reinterpret_cast<const uint4 *>(sW + ((m * NB + nb) * 64 + lane) * 32);
                    const uint4 lo = pa[0], hi = pa[1];
                    av[nb] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
                }
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int ch = 16 * m + 4 * kq + s;
                    const int tap = ch < NCH ? ch / CH8 : 4;
                    const int c0 = ch < NCH ? (ch - (ch / CH8) * CH8) * 8 : 0;
#pragma unroll
                    for (int p = 0; p < PB; ++p) {
                        const uint2 u = *reinterpret_cast<const uint2 *>(pt_addr(p, tap) + c0);
                        bv[p][2 * s] = (int)u.x;
                        bv[p][2 * s + 1] = (int)u.y;
                    }
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int p = 0; p < PB; ++p)
                        acc[nb][p] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                            av[nb], bv[p], acc[nb][p], 0, 0, 0, 0x7F7F7F7F, 0, 0x7F7F7F7F);
            }
        }

        // epilogue: D row = output channel 16 nb + 4 kq + r, column = pixel j
        float wmax = 0.f;
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int xo = X0 + dd * (16 * p + j);
            const bool ok = xo < W;
            const int64_t pix = px_off + (int64_t)yo * W + xo;
            float h0 = 0.f, h1 = 0.f, h2 = 0.f, h3 = 0.f, h4 = 0.f;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int oc = nb * 16 + kq * 4;
                v4f v = acc[nb][p];
                if constexpr (P == DL_FP8) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] *= a.wscale[oc + r] * qscale;
                }
                v[0] += sB[oc + 0]; v[1] += sB[oc + 1]; v[2] += sB[oc + 2]; v[3] += sB[oc + 3];
                if (RES && ok) v += Store<P>::load4(a.res, pix * C + oc);
                v = relu4(v);
                if constexpr (P != DL_FP32) {        // what is stored (and what the head reads) is BF16
                    v[0] = bf16_round(v[0]); v[1] = bf16_round(v[1]);
                    v[2] = bf16_round(v[2]); v[3] = bf16_round(v[3]);
                }
                if (!HEAD) {
                    if (ok) {
                        Store<P>::store4(a.out, pix * C + oc, v);
                        wmax = fmaxf(wmax, fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])));
                    }
                } else {
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
                    float *mp = a.maps + 5 * px_off + (int64_t)yo * W + xo;
                    const float mine = kq == 0 ? h0 : kq == 1 ? h1 : kq == 2 ? h2 : h3;
                    mp[kq * plane] = mine + sH[5 * C + kq];
                    if (kq == 0) mp[4 * plane] = h4 + sH[5 * C + 4];
                }
            }
        }
        if (!HEAD && a.amax_out) {
            // ReLU outputs are >= 0, so float order equals unsigned order of the bits
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) wmax = fmaxf(wmax, __shfl_xor(wmax, o));
            if (lane == 0) atomicMax(a.amax_out + f, __float_as_uint(wmax));
        }
    }
}

// ------------------------------------------------------------- launchers
template <int C, int P, int TR, bool RES, bool HEAD>
hipError_t launch_t(const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    auto kern = k_conv<C, P, TR, RES, HEAD>;
    constexpr size_t sh = Lds<C, P, TR>::TOTAL;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(TR * 64), sh, s, a, g);
    return hipGetLastError();
}

template <int C, int P, int TR>
hipError_t launch_ct(const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    if (a.head) return launch_t<C, P, TR, true, true>(a, g, grid, s);
    if (a.res) return launch_t<C, P, TR, true, false>(a, g, grid, s);
    return launch_t<C, P, TR, false, false>(a, g, grid, s);
}

template <int C, int P>
hipError_t launch_cp(const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    if (g.tr == 4) return launch_ct<C, P, 4>(a, g, grid, s);
    if (g.tr == 8) return launch_ct<C, P, 8>(a, g, grid, s);
    return hipErrorInvalidValue;
}

template <int C, int P, int TR>
int blocks_per_cu()
{
    int nb = 0;
    auto kern = k_conv<C, P, TR, true, false>;
    constexpr size_t sh = Lds<C, P, TR>::TOTAL;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, TR * 64, sh) != hipSuccess) nb = 1;
    return nb > 0 ? nb : 1;
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

template <int P, int TR>
int bpc_pt(int C)
{
    switch (C) {
    case 16: return blocks_per_cu<16, P, TR>();
    case 32: return blocks_per_cu<32, P, TR>();
    case 48: return blocks_per_cu<48, P, TR>();
    case 64: return blocks_per_cu<64, P, TR>();
    default: return 1;
    }
}

template <int P>
int bpc_p(int C, int tr)
{
    return tr == 4 ? bpc_pt<P, 4>(C) : bpc_pt<P, 8>(C);
}

uint16_t host_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// host e4m3 code of x: nearest representable value (ties to the even
// mantissa), saturating at +-448; spacing 2^(e-3) for a in [2^e, 2^(e+1)),
// e >= -6 (subnormals share the spacing 2^-9)
uint8_t host_e4m3(float x)
{
    const uint8_t s = std::signbit(x) ? 0x80 : 0;
    const double a = std::fabs((double)x);
    if (a >= 448.0) return s | 0x7E;
    if (a == 0.0) return s;
    int e;
    (void)std::frexp(a, &e);             // a in [2^(e-1), 2^e)
    const int ex = e - 1 < -6 ? -6 : e - 1;
    const double q = std::ldexp(1.0, ex - 3);
    const double r = a / q;
    double n = std::floor(r);
    const double fr = r - n;
    if (fr > 0.5 || (fr == 0.5 && std::fmod(n, 2.0) != 0.0)) n += 1.0;
    const double val = n * q;            // rounded magnitude
    if (val >= 448.0) return s | 0x7E;
    if (val < 0.015625) return s | (uint8_t)std::lround(val * 512.0);
    int e2;
    const double fm = std::frexp(val, &e2);   // val = fm 2^e2, fm in [0.5, 1)
    const int mant = (int)std::lround((fm * 2.0 - 1.0) * 8.0);
    return s | (uint8_t)(((e2 - 1 + 7) << 3) | mant);
}

}  // namespace

void conv_tile_shape(int C, int precision, int rows, int *tr, int *tc)
{
    (void)C;
    *tr = rows == 4 ? 4 : 8;
    switch (precision) {
    case DL_FP32: *tc = TileShape<DL_FP32>::TC; break;
    case DL_BF16: *tc = TileShape<DL_BF16>::TC; break;
    default: *tc = TileShape<DL_FP8>::TC; break;
    }
}

size_t conv_packed_bytes(int C, int precision)
{
    const int NB = C / 16, NCH = 9 * (C / 8);
    if (precision == DL_FP32) return (size_t)9 * C * C * 4;
    if (precision == DL_BF16) return (size_t)((NCH + 3) / 4) * NB * 64 * 16;
    return (size_t)((NCH + 15) / 16) * NB * 64 * 32;
}

void pack_conv_weights(int C, int precision, const float *W, void *dst, float *scale)
{
    const int NB = C / 16;
    auto wt = [&](int oc, int c, int tap) { return W[((size_t)oc * C + c) * 9 + tap]; };
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
                            o[((size_t)((tap * G + g) * NB + nb) * 64 + lane) * 4 + s] = wt(oc, c, tap);
                        }
        return;
    }
    const int CH8 = C / 8, NCH = 9 * CH8;
    if (precision == DL_BF16) {
        // step m, block nb, lane (i, kq): 8 bf16 of chunk 4 m + kq
        const int NIT = (NCH + 3) / 4;
        uint16_t *o = static_cast<uint16_t *>(dst);
        for (int m = 0; m < NIT; ++m)
            for (int nb = 0; nb < NB; ++nb)
                for (int lane = 0; lane < 64; ++lane) {
                    const int oc = nb * 16 + (lane & 15), ch = 4 * m + (lane >> 4);
                    for (int e = 0; e < 8; ++e) {
                        const float v = ch < NCH ? wt(oc, (ch % CH8) * 8 + e, ch / CH8) : 0.f;
                        o[((size_t)(m * NB + nb) * 64 + lane) * 8 + e] = host_bf16(v);
                    }
                }
        return;
    }
    // FP8: per-output-channel scale s[o] = max|W[o]| / 448; codes of W * (448 / max|W[o]|);
    // step m, block nb, lane (i, kq): 32 bytes = chunks 16 m + 4 kq + 0..3
    std::vector<float> inv(C);
    for (int oc = 0; oc < C; ++oc) {
        float mx = 0.f;
        for (int k = 0; k < C * 9; ++k) mx = std::fmax(mx, std::fabs(W[(size_t)oc * C * 9 + k]));
        scale[oc] = mx > 0.f ? (float)((double)mx / 448.0) : 0.f;
        inv[oc] = mx > 0.f ? (float)(448.0 / (double)mx) : 0.f;
    }
    const int NIT = (NCH + 15) / 16;
    uint8_t *o = static_cast<uint8_t *>(dst);
    for (int m = 0; m < NIT; ++m)
        for (int nb = 0; nb < NB; ++nb)
            for (int lane = 0; lane < 64; ++lane) {
                const int oc = nb * 16 + (lane & 15);
                for (int e = 0; e < 32; ++e) {
                    const int ch = 16 * m + 4 * (lane >> 4) + e / 8;
                    const float v = ch < NCH ? wt(oc, (ch % CH8) * 8 + e % 8, ch / CH8) : 0.f;
                    o[((size_t)(m * NB + nb) * 64 + lane) * 32 + e] = host_e4m3(v * inv[oc]);
                }
            }
}

int conv_max_grid(int C, int precision, int tr, int ncu)
{
    int b = 1;
    if (precision == DL_FP32) b = bpc_p<DL_FP32>(C, tr);
    else if (precision == DL_BF16) b = bpc_p<DL_BF16>(C, tr);
    else b = bpc_p<DL_FP8>(C, tr);
    return b * ncu;
}

hipError_t launch_conv(int C, int precision, const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    if (precision == DL_FP32) return launch_p<DL_FP32>(C, a, g, grid, s);
    if (precision == DL_BF16) return launch_p<DL_BF16>(C, a, g, grid, s);
    if (precision == DL_FP8) return launch_p<DL_FP8>(C, a, g, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace dloc
