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
// for every dilation.  Activations feeding a dilation-d block are stored in
// the phase layout of d (dloc_internal.h: act_points), where those lattice
// points are contiguous rows of one dense sub-image, so a phase tile reads
// like a d = 1 tile; each block writes its output straight into the next
// block's layout.  The workgroup stages its input into LDS (points strided so
// the MFMA operand reads are free of bank conflicts), then wave w computes
// lattice row w for all C output channels.  Workgroups are persistent; tiles
// are handed out XCD by XCD in contiguous ranges, in an order that keeps
// vertically adjacent tiles close (see decode_tile), so the halo rows they
// share are read from L2.  The next tile's input is loaded into registers
// while the MFMAs run on the current one.
//
// GEMM view: M = output channels (blocks of 16), N = pixels (blocks of 16),
// K = 9 taps x C input channels.
//   FP32  v_mfma_f32_16x16x4_f32; lane group kq takes channels 16 g + 4 kq + s
//         (s = MFMA step), so one float4 feeds 4 steps.  Weights live in LDS
//         when they fit beside the tile (C <= 48 with 8-row tiles); otherwise
//         they are read from L2 one K iteration ahead.
//   BF16  v_mfma_f32_16x16x32_bf16 (FP32 accumulation); K is cut into chunks
//         of 8 channels of one tap and lane group kq of step m takes chunk
//         4 m + kq (one 16-byte LDS read).  Weights live in LDS.
//   FP8   v_mfma_scale_f32_16x16x128_f8f6f4 with e4m3 operands; K runs tap by
//         tap with each tap's channels padded to a multiple of 32, and lane
//         group kq of step m takes one 32-channel group of one tap (two
//         16-byte LDS reads).  Activations are stored as e4m3 codes with one
//         E8M0 scale byte per 32-channel group of each point (dloc_internal.h),
//         which is exactly the MFMA's per-lane block scale of the activation
//         operand; weights carry a per-output-channel scale applied in the
//         epilogue.  The epilogue takes each 32-channel group's max of the
//         FP32 outputs over the four lanes holding the pixel, and stores the
//         e4m3 codes of the FP32 values (scaled by the group's power of two)
//         and the scale bytes.
//   BF16X3 (split BF16) the BF16 MFMA on both halves of FP32 operands: the
//         tile is staged from FP32 activations as BF16 pairs (hi = bf16(v),
//         lo = bf16(v - hi); per point C hi values then C lo values), the
//         weights are packed as a hi block and a lo block, and each K chunk
//         takes three MFMAs, wh xh + wh xl + wl xh, into one FP32 accumulator.
//         Storage, residual, epilogue and fused head are those of FP32.
// K is padded with zero-weight chunks when 9 C is not a multiple of the MFMA's K.
// BF16 and FP8 pass each wave's output row (and residual) through LDS so they
// move in whole 16-byte lanes; every store is a buffer store whose offset is
// out of range for pixels off the frame, so the epilogue has no branches.
#include "dloc_internal.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace dloc {

namespace {

constexpr int NXCD = 8;
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// Buffer resource over nbytes at base (raw addressing: stride 0, offsets in
// bytes).  A store whose offset lies past nbytes is dropped by the hardware,
// which lets the epilogue store without a branch around pixels off the frame.
constexpr uint32_t BUF_DWORD3 = 0x00020000u;
constexpr int BUF_OOB = (int)0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(void *base, uint32_t nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)nbytes, (int)BUF_DWORD3);
}

// Dword stride of one lattice point in the LDS tile.  gfx950's LDS serves a
// 16-byte read (ds_read_b128) of the 64 lanes in groups whose banks collide
// unless the point stride is 8 mod 16 dwords; measured with rocprof's
// SQ_LDS_BANK_CONFLICT over the exact read and staging-write patterns of the
// FP32 and BF16 kernels (every C in 16..64: zero read conflicts at 8 mod 16,
// about 4 extra cycles per read at 4 or 12 mod 16, 12 or more at 0 mod 16).
constexpr int stride_8_mod_16(int dw) { return dw + ((8 - dw % 16) + 16) % 16; }
constexpr int align16(int b) { return (b + 15) / 16 * 16; }

__device__ __forceinline__ v4f relu4(v4f v)
{
    v4f r;
    r[0] = fmaxf(v[0], 0.f); r[1] = fmaxf(v[1], 0.f);
    r[2] = fmaxf(v[2], 0.f); r[3] = fmaxf(v[3], 0.f);
    return r;
}


// storage of the activations in HBM: FP32, BF16, or FP8 (e4m3 codes plus
// one scale byte per 32-channel group of a point, dloc_internal.h)
template <int P> struct Store {
    static constexpr int ESZ = 2;
    using Raw = uint2;                      // 4 BF16 values as loaded
    __device__ static Raw raw4(const void *base, int64_t idx)
    {
        return *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(base) + idx);
    }
    __device__ static v4f unpack(Raw u)
    {
        return v4f{__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xFFFF0000u),
                   __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xFFFF0000u)};
    }
    // 4 values (already BF16-exact) at byte offset off of a buffer resource
    __device__ static void bstore4(__amdgpu_buffer_rsrc_t rs, int off, v4f v)
    {
        v2u u;
        u[0] = (__float_as_uint(v[0]) >> 16) | (__float_as_uint(v[1]) & 0xFFFF0000u);
        u[1] = (__float_as_uint(v[2]) >> 16) | (__float_as_uint(v[3]) & 0xFFFF0000u);
        __builtin_amdgcn_raw_buffer_store_b64(u, rs, off, 0, 0);
    }
};
template <> struct Store<DL_FP8> {
    static constexpr int ESZ = 1;
    using Raw = uint2;                      // 4 codes and their group's scale byte
    __device__ static v4f unpack(Raw u) { return fp8_unpack4(u.x, fp8_scale_value(u.y)); }
};
template <> struct Store<DL_FP32> {
    static constexpr int ESZ = 4;
    using Raw = v4f;
    __device__ static Raw raw4(const void *base, int64_t idx)
    {
        return *reinterpret_cast<const v4f *>(static_cast<const float *>(base) + idx);
    }
    __device__ static v4f unpack(Raw u) { return u; }
    __device__ static void bstore4(__amdgpu_buffer_rsrc_t rs, int off, v4f v)
    {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u, v), rs, off, 0, 0);
    }
};

// split BF16 stores FP32 activations
template <> struct Store<DL_BF16X3> : Store<DL_FP32> {};

// K plan and packed-weight bytes per precision
template <int C, int P> struct KPlan;
template <int C> struct KPlan<C, DL_FP32> {
    static constexpr int NIT = 9 * (C / 16);
    static constexpr int BYTES = 9 * C * C * 4;
    static constexpr int LDS_W = BYTES;           // in LDS when the tile leaves room (see Lds)
    static constexpr int LESZ = 4;                // LDS bytes per channel
};
template <int C> struct KPlan<C, DL_BF16> {
    static constexpr int CH8 = C / 8, NCH = 9 * CH8;
    static constexpr int NIT = (NCH + 3) / 4;
    static constexpr int BYTES = NIT * (C / 16) * 64 * 16;
    static constexpr int LDS_W = BYTES;
    static constexpr int LESZ = 2;
};
template <int C> struct KPlan<C, DL_BF16X3> {
    // the BF16 K plan, with a hi and a lo block of weights
    static constexpr int CH8 = C / 8, NCH = 9 * CH8;
    static constexpr int NIT = (NCH + 3) / 4;
    static constexpr int HALF = NIT * (C / 16) * 64 * 16;
    static constexpr int BYTES = 2 * HALF;
    static constexpr int LDS_W = BYTES;
    static constexpr int LESZ = 4;                // hi and lo BF16 per channel
};
template <int C> struct KPlan<C, DL_FP8> {
    // K runs tap by tap, each tap's channels padded to CT (a multiple of 32):
    // K chunk g (32 channels) is half g % HPT of tap g / HPT, and lane group
    // kq of step m takes chunk 4 m + kq -- 32 consecutive bytes of one point
    static constexpr int CT = (C + 31) / 32 * 32, HPT = CT / 32, NG = 9 * HPT;
    static constexpr int NIT = (NG + 3) / 4;
    static constexpr int BYTES = NIT * (C / 16) * 64 * 32;
    static constexpr int LDS_W = BYTES;
    static constexpr int LESZ = 1;
};

// lattice columns per tile (TC; the rows, one wave each, are a template choice)
template <int P> struct TileShape;
template <> struct TileShape<DL_FP32> { static constexpr int TC = 32; };
template <> struct TileShape<DL_BF16> { static constexpr int TC = 64; };
template <> struct TileShape<DL_FP8> { static constexpr int TC = 64; };
template <> struct TileShape<DL_BF16X3> { static constexpr int TC = 32; };
// waves per SIMD the register budget is sized for: FP32 4-row tiles fit three
// workgroups per CU in LDS (one wave per SIMD each); every other shape is
// limited to one or two workgroups by LDS and gets the larger budget of two
// waves per SIMD
template <int P, int TR> constexpr int min_waves() { return P == DL_FP32 && TR == 4 ? 3 : 2; }

// NHL: head outputs the LDS holds weights for (5, or 10 with uncertainties)
template <int C, int P, int TR_, int NHL = 5>
struct Lds {
    static constexpr int TR = TR_, TC = TileShape<P>::TC;
    // bytes per point; FP8 points hold the tap's padded CT codes (the padding
    // is zeroed once, staging writes only the C real channels), then the
    // point's two group scale bytes at byte CT
    static constexpr int CT8 = (C + 31) / 32 * 32;
    static constexpr int PS = stride_8_mod_16(P == DL_FP8 ? CT8 / 4 + 1 : C * KPlan<C, P>::LESZ / 4) * 4;
    static constexpr int PW = TC + 2;
    static constexpr int NPT = (TR + 2) * PW;
    static constexpr int TBYTES = align16(NPT * PS);
    static constexpr int EXTRA = C * 4 + (NHL * C + NHL) * 4 + C * 4 + 64;  // bias, head, scales, alignment
    // FP32 keeps its weights in LDS when they fit beside the tile (C <= 48 at
    // 8 rows); otherwise each K iteration reads them from L2, one ahead
    static constexpr bool LDSW_FP32 = TBYTES + KPlan<C, P>::BYTES + EXTRA <= 160 * 1024;
    static constexpr int LDSW = P == DL_FP32 ? (LDSW_FP32 ? KPlan<C, P>::BYTES : 0) : KPlan<C, P>::LDS_W;
    static constexpr int WOFF = TBYTES;
    static constexpr int BOFF = WOFF + LDSW;                           // bias [C]
    static constexpr int HOFF = BOFF + C * 4;                          // head [NHL C + NHL]
    static constexpr int SOFF = HOFF + (NHL * C + NHL) * 4;            // FP8 weight scales [C]
    // BF16 and FP8 stage each wave's output row (TC pixels x C BF16 values or
    // e4m3 codes, pixel-major) so it leaves in whole 16-byte lanes; FP8 adds
    // the row's residual scales and output scales (2 bytes per pixel each)
    static constexpr int OPX = P == DL_FP8 ? C : C * 2;                // staging bytes per pixel
    static constexpr int RSOFF = TC * OPX;                             // FP8: residual scales
    static constexpr int OSOFF = RSOFF + TC * 2;                       // FP8: output scales
    static constexpr int OWAVE = P == DL_FP32 || P == DL_BF16X3 ? 0 : P == DL_FP8 ? align16(OSOFF + TC * 2) : TC * OPX;
    static constexpr int OOFF = align16(SOFF + C * 4);
    static constexpr int DOFF = align16(OOFF + TR * OWAVE);            // two decoded-tile slots
    static constexpr int TOTAL = DOFF + 2 * 64;
    static constexpr bool FITS = TOTAL <= 160 * 1024;   // else no kernel exists for this shape
};

// a decoded tile: origin (y0, x0) and size of its frame, where its input
// sits (point (ii, jj) of the tile is activation point a0 + ii rs + jj cs of
// the frame), and the frame's map and activation offsets
struct TileDec {
    int y0, x0, h, w, a0, rs, cs;
    int64_t px, act;
};

// --------------------------------------------------------------- kernel
// NH: outputs of the fused 1x1 head (0: no head, the layer's activations are
// stored; 5 or 10: the head's maps are stored instead)
template <int C, int P, int TR_, bool RES, int NH>
__global__ void __launch_bounds__(TR_ * 64, (min_waves<P, TR_>()))
k_conv(ConvArgs a, Geometry geo)
{
    constexpr bool HEAD = NH > 0;
    using L = Lds<C, P, TR_, (NH > 5 ? NH : 5)>;
    constexpr int TR = L::TR, TC = L::TC, PS = L::PS, PW = L::PW, NPT = L::NPT;
    constexpr int NB = C / 16, PB = TC / 16, NT = TR * 64;
    extern __shared__ v4f smem[];
    char *sT = reinterpret_cast<char *>(smem);
    float *sB = reinterpret_cast<float *>(sT + L::BOFF);
    float *sH = reinterpret_cast<float *>(sT + L::HOFF);
    float *sS = reinterpret_cast<float *>(sT + L::SOFF);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: keeps row state scalar
    const int j = lane & 15, kq = lane >> 4;
    const int dd = a.d, blk = a.blk;

    if constexpr (L::LDSW > 0) {
        const v4f *gw = static_cast<const v4f *>(a.wpk);
        v4f *sW = reinterpret_cast<v4f *>(sT + L::WOFF);
        for (int i = tid; i < L::LDSW / 16; i += NT) sW[i] = gw[i];
    }
    for (int i = tid; i < C; i += NT) sB[i] = a.bias[i];
    if (HEAD)
        for (int i = tid; i < NH * C + NH; i += NT) sH[i] = a.head[i];
    if constexpr (P == DL_FP8) {
        for (int i = tid; i < C; i += NT) sS[i] = a.wscale[i];
        // the channel padding of every point must read as e4m3 zero (never
        // written by staging, and uninitialised LDS may hold NaN codes)
        for (int i = tid; i < L::TBYTES / 16; i += NT) smem[i] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    // FP32: the weights of K iteration 0, read ahead of every tile (the last
    // iteration of a tile reads them for the next)
    constexpr bool GW = P == DL_FP32 && !L::LDSW_FP32;
    v4f awn[GW ? NB : 1];
    if constexpr (GW)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) awn[nb] = static_cast<const v4f *>(a.wpk)[nb * 64 + lane];

    const int64_t T = a.list ? (int64_t)ld_const(a.list_count)
                      : geo.dyn ? ld_const(geo.dyn + DYN_TILES + blk) : geo.tiles[blk];
    const int nfr = geo.dyn ? (int)ld_const(geo.dyn + DYN_NF) : geo.nf;
    const int xcd = blockIdx.x % NXCD, slot = blockIdx.x / NXCD, nslot = gridDim.x / NXCD;
    const int64_t chunk = (T + NXCD - 1) / NXCD;
    const int64_t t0 = (int64_t)xcd * chunk;
    const int64_t t1 = t0 + chunk < T ? t0 + chunk : T;

    // Staging is software-pipelined: the input of the workgroup's next tile is
    // loaded into registers (NPF 16-byte chunks per thread) while the MFMAs
    // run on the current one, and written to LDS after the next barrier.  The
    // loads are unconditional (off-frame points read zeros as out-of-range
    // buffer loads), so no branch separates them from the compute they overlap.
    constexpr int SESZ = Store<P>::ESZ;
    constexpr int SCH = C * SESZ / 16;       // 16-byte source chunks per point
    constexpr int NQ = NPT * SCH;
    constexpr int NPF = (NQ + NT - 1) / NT;
    v4f pf[NPF];
    // FP8: the two group scale bytes of each point, from the scale region
    // (byte total_act * C of the activation buffer)
    constexpr int NPS = P == DL_FP8 ? (NPT + NT - 1) / NT : 1;
    uint32_t psc[NPS];
    const int64_t sc_off = geo.total_act * C;
    // the prefetched tile: frame, origin, the frame fields the tile needs, and
    // where its input sits: point (ii, jj) of the tile, at pixel (Y0 + d ii,
    // X0 + d jj), is activation point A0 + ii RS + jj CS of the frame.  In the
    // phase layout of the tile's dilation that is row iy0 + ii, column
    // ix0 + jj of one dense sub-image (RS = its width, CS = 1); in plain NHWC,
    // RS = d w and CS = d.  A frame's activations span less than 2^31 bytes,
    // so offsets within the frame are 32-bit; loads go through a buffer
    // resource over the frame, and points off the frame take an out-of-range
    // offset, which reads as zero.
    TileDec n{};
    auto decode = [&](int64_t ti) {
        TileDec r;
        const int64_t t = a.list ? (int64_t)ld_const(a.list + ti) : ti;
        const int f = find_frame(a.fd, nfr, t, [blk](const FrameDesc &d) { return ld_const(&d.tile_start[blk]); });
        const FrameDesc *fd = a.fd + f;      // fields read in place: tile_start is indexed by the block
        r.h = ld_const(&fd->h);
        r.w = ld_const(&fd->w);
        r.px = ld_const(&fd->px_off);
        r.act = ld_const(&fd->act_off);
        decode_tile(r.h, r.w, t - ld_const(&fd->tile_start[blk]), dd, TR, TC, blk == geo.minor_blk, geo.strip, r.y0,
                    r.x0);
        if (a.in_phase) {
            const int hd = (r.h + dd - 1) / dd, wd = (r.w + dd - 1) / dd;
            const int py = r.y0 % dd, px = r.x0 % dd;
            r.a0 = ((py * dd + px) * hd + r.y0 / dd) * wd + r.x0 / dd;
            r.rs = wd;
            r.cs = 1;
        } else {
            r.a0 = r.y0 * r.w + r.x0;
            r.rs = dd * r.w;
            r.cs = dd;
        }
        return r;
    };
    // Wave 0 alone decodes tiles (the scalar unit is shared by the CU's
    // waves): it publishes the tile after next in one of two LDS slots from
    // inside its MFMA loop, and every wave picks it up after the next loop-top
    // barrier.  A slot is rewritten only after every wave has passed the
    // barrier that follows its last reading.
    int *sdec = reinterpret_cast<int *>(sT + L::DOFF);
    auto publish = [&](int sl, const TileDec &r) {
        if (lane == 0) {
            int4 *q = reinterpret_cast<int4 *>(sdec + 16 * sl);
            q[0] = int4{r.y0, r.x0, r.h, r.w};
            q[1] = int4{r.a0, r.rs, r.cs, 0};
            q[2] = int4{(int)(uint32_t)r.px, (int)(r.px >> 32), (int)(uint32_t)r.act, (int)(r.act >> 32)};
        }
    };
    auto pickup = [&](int sl) {
        const int4 *q = reinterpret_cast<const int4 *>(sdec + 16 * sl);
        const int4 u0 = q[0], u1 = q[1], u2 = q[2];
        TileDec r;
        r.y0 = __builtin_amdgcn_readfirstlane(u0.x);
        r.x0 = __builtin_amdgcn_readfirstlane(u0.y);
        r.h = __builtin_amdgcn_readfirstlane(u0.z);
        r.w = __builtin_amdgcn_readfirstlane(u0.w);
        r.a0 = __builtin_amdgcn_readfirstlane(u1.x);
        r.rs = __builtin_amdgcn_readfirstlane(u1.y);
        r.cs = __builtin_amdgcn_readfirstlane(u1.z);
        r.px = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(u2.x) |
               ((int64_t)__builtin_amdgcn_readfirstlane(u2.y) << 32);
        r.act = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(u2.z) |
                ((int64_t)__builtin_amdgcn_readfirstlane(u2.w) << 32);
        return r;
    };
    // the tile's input into registers: point (ii, jj) of the tile is
    // activation point a0 + ii rs + jj cs of the frame (off-frame points take
    // an out-of-range offset and read zero)
    auto issue = [&](const TileDec &r) {
        const __amdgpu_buffer_rsrc_t rin =
            buf_rsrc(const_cast<char *>(static_cast<const char *>(a.in)) + r.act * (C * SESZ), 0x7FFFFFFFu);
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            const int q0 = tid + k * NT;
            const int q = q0 < NQ ? q0 : NQ - 1;
            const int pt = q / SCH, ch = q - (q / SCH) * SCH;
            const int ii = pt / PW - 1, jj = pt - (pt / PW) * PW - 1;
            const int y = r.y0 + dd * ii, x = r.x0 + dd * jj;
            const bool ok = q0 < NQ && (unsigned)y < (unsigned)r.h && (unsigned)x < (unsigned)r.w;
            pf[k] = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(
                                                rin, ok ? (r.a0 + ii * r.rs + jj * r.cs) * (C * SESZ) + ch * 16 : BUF_OOB, 0, 0));
        }
        if constexpr (P == DL_FP8) {
            const __amdgpu_buffer_rsrc_t rsc =
                buf_rsrc(const_cast<char *>(static_cast<const char *>(a.in)) + sc_off + r.act * 2, 0x7FFFFFFFu);
#pragma unroll
            for (int k = 0; k < NPS; ++k) {
                const int pt0 = tid + k * NT;
                const int pt = pt0 < NPT ? pt0 : NPT - 1;
                const int ii = pt / PW - 1, jj = pt - (pt / PW) * PW - 1;
                const int y = r.y0 + dd * ii, x = r.x0 + dd * jj;
                const bool ok = pt0 < NPT && (unsigned)y < (unsigned)r.h && (unsigned)x < (unsigned)r.w;
                psc[k] = __builtin_amdgcn_raw_buffer_load_b16(rsc, ok ? (r.a0 + ii * r.rs + jj * r.cs) * 2 : BUF_OOB, 0, 0);
            }
        }
    };

    int64_t ti = t0 + slot;
    if (ti < t1) {
        n = decode(ti);
        issue(n);
        if (wave == 0) publish(0, decode(ti + nslot < t1 ? ti + nslot : ti));
    }
    // the first tile's data is waited for here, outside the loop: the
    // compiler's wait at the loop top then only has to cover the loop's own
    // path, where the previous tile's stores follow the loads
#pragma unroll
    for (int k = 0; k < NPF; ++k) asm volatile("" : : "v"(pf[k]));
#pragma unroll
    for (int k = 0; k < NPS; ++k) asm volatile("" : : "v"(psc[k]));
    for (int par = 0; ti < t1; ti += nslot, par ^= 1) {
        const int Y0 = n.y0, X0 = n.x0, H = n.h, W = n.w, A0 = n.a0, RS = n.rs, CS = n.cs;
        const int64_t px_off = n.px, act = n.act;

        __syncthreads();   // the previous tile's LDS reads are done (and weights staged)
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            const int q = tid + k * NT;
            if (q < NQ) {
                const int pt = q / SCH, ch = q - (q / SCH) * SCH;
                if constexpr (P == DL_BF16X3) {
                    // four FP32 channels -> their BF16 halves: hi at byte 8 ch of
                    // the point, lo at 2 C + 8 ch (v - hi is exact in FP32)
                    const v4f v = pf[k];
                    const uint32_t h01 = bf16_pack2(v[0], v[1]), h23 = bf16_pack2(v[2], v[3]);
                    const uint32_t l01 = bf16_pack2(v[0] - __uint_as_float(h01 << 16),
                                                    v[1] - __uint_as_float(h01 & 0xFFFF0000u));
                    const uint32_t l23 = bf16_pack2(v[2] - __uint_as_float(h23 << 16),
                                                    v[3] - __uint_as_float(h23 & 0xFFFF0000u));
                    *reinterpret_cast<uint2 *>(sT + pt * PS + ch * 8) = uint2{h01, h23};
                    *reinterpret_cast<uint2 *>(sT + pt * PS + 2 * C + ch * 8) = uint2{l01, l23};
                } else {
                    *reinterpret_cast<v4f *>(sT + pt * PS + ch * 16) = pf[k];
                }
            }
        }
        if constexpr (P == DL_FP8) {
#pragma unroll
            for (int k = 0; k < NPS; ++k) {
                const int pt = tid + k * NT;
                if (pt < NPT) *reinterpret_cast<uint16_t *>(sT + pt * PS + L::CT8) = (uint16_t)psc[k];
            }
        }
        __syncthreads();

        // The residual (block input) at this wave's output pixels, loaded
        // unconditionally from clamped addresses (values of pixels off the
        // frame are never stored).  BF16 and FP8 issue all these loads before
        // the next tile's, so waiting for them does not wait for the prefetch
        // (vector loads complete in order); FP32 has no registers to spare and
        // loads them in the epilogue, one pixel block at a time.
        const int yo = Y0 + dd * wave;
        // A wave whose lattice row is off the frame computes anyway (its LDS
        // rows hold zeros) and stores nothing: keeping the loop body free of
        // branches lets the compiler count the stores still in flight when it
        // waits for the next tile's loads, instead of waiting for everything.
        const bool row_ok = yo < H;
        // BF16/FP8 without the head: output (and residual) pass through this
        // wave's LDS staging row and move in whole 16-byte lanes.  The fused
        // head layer and FP32 with weights in LDS load the residual in the
        // MFMA layout before the next tile's input (EARLY_RES); FP32 with
        // weights in L2 has no registers to spare and loads it in the
        // epilogue, one pixel block at a time.
        constexpr bool F32IO = P == DL_FP32 || P == DL_BF16X3;      // FP32 activations in HBM
        constexpr bool STAGE = !F32IO && !HEAD;
        constexpr bool EARLY_RES = RES && (!F32IO ? HEAD : P == DL_BF16X3 || L::LDSW_FP32);
        constexpr int CPX = L::OPX / 16;                    // 16-byte chunks per staged pixel
        constexpr int NRC = STAGE ? TC * CPX / 64 : 1;      // chunks per lane
        static_assert(!STAGE || (TC * CPX) % 64 == 0, "staging chunks per lane");
        // this wave's output row: input-layout point of its lattice column c is
        // Ar + c CS (the residual sits there); frame-relative, < 2^31 bytes
        const int Ar = A0 + wave * RS;
        v4u rc[RES && STAGE ? NRC : 1];
        uint32_t rsc = 0;                                   // FP8: this lane's pixel's residual scales
        static_assert(P != DL_FP8 || TC == 64, "FP8 staging: one lane per pixel of the row");
        if constexpr (RES && STAGE) {
            const __amdgpu_buffer_rsrc_t rres =
                buf_rsrc(const_cast<char *>(static_cast<const char *>(a.res)) + act * L::OPX, 0x7FFFFFFFu);
#pragma unroll
            for (int i = 0; i < NRC; ++i) {
                const int q = lane + 64 * i, px = q / CPX, part = q - (q / CPX) * CPX;
                const int xo = X0 + dd * px;
                rc[i] = __builtin_amdgcn_raw_buffer_load_b128(
                    rres, row_ok && xo < W ? (Ar + px * CS) * L::OPX + part * 16 : BUF_OOB, 0, 0);
            }
            if constexpr (P == DL_FP8) {
                const __amdgpu_buffer_rsrc_t rrs =
                    buf_rsrc(const_cast<char *>(static_cast<const char *>(a.res)) + sc_off + act * 2, 0x7FFFFFFFu);
                const int xo = X0 + dd * lane;
                rsc = __builtin_amdgcn_raw_buffer_load_b16(rrs, row_ok && xo < W ? (Ar + lane * CS) * 2 : BUF_OOB, 0, 0);
            }
        }
        constexpr int RPB = EARLY_RES ? PB : 1;
        typename Store<P>::Raw rr[RES && !STAGE ? NB : 1][RPB];
        auto load_res = [&](int p0) {
#pragma unroll
            for (int pp = 0; pp < RPB; ++pp) {
                const int c = 16 * (p0 + pp) + j, xo = X0 + dd * c;
                const int64_t pix = act + (row_ok && xo < W ? Ar + c * CS : 0);   // off-frame: any valid point
                if constexpr (P == DL_FP8) {
                    const uint8_t *rb = static_cast<const uint8_t *>(a.res);
                    const uint32_t sc2 = *reinterpret_cast<const uint16_t *>(rb + sc_off + pix * 2);
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        rr[nb][pp] = uint2{*reinterpret_cast<const uint32_t *>(rb + pix * C + nb * 16 + kq * 4),
                                           (sc2 >> (8 * (nb >> 1))) & 0xFFu};
                } else {
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) rr[nb][pp] = Store<P>::raw4(a.res, pix * C + nb * 16 + kq * 4);
                }
            }
        };
        // FP32 with weights and tile in LDS and the register budget of two
        // waves per SIMD (see its MFMA loop below)
        constexpr bool PREF = P == DL_FP32 && !GW && min_waves<P, TR_>() == 2;
        // the residual (early forms) and the next tile's input.  Past the
        // last tile the current one is read again (and not used), so no branch
        // separates the residual loads from the prefetch and the wait for them
        // stays exact.  FP32 with weights in L2 (4-row tiles, no register room
        // for that) skips the read.  PREF issues these after the first K step's
        // MFMAs, so the matrix unit works while they go out; the other forms
        // issue them before their K loop.
        auto pre_loads = [&]() {
            if constexpr (EARLY_RES) load_res(0);
            __builtin_amdgcn_sched_barrier(0);   // residual loads stay ahead of the prefetch
            if constexpr (GW) {
                if (ti + nslot < t1) {
                    n = pickup(par);
                    issue(n);
                }
            } else {
                n = pickup(par);                 // the next tile, or this one again past the last
                issue(n);
            }
            // keep the scheduler from sinking these loads below the MFMAs they
            // are meant to overlap
            __builtin_amdgcn_sched_barrier(0);
        };
        if constexpr (!PREF) pre_loads();


        v4f acc[NB][PB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int p = 0; p < PB; ++p) acc[nb][p] = v4f{0.f, 0.f, 0.f, 0.f};
        // LDS address of lattice point (row wave + u, column 16 p + j + v) for tap (u, v), u, v in 0..2
        auto pt_addr = [&](int p, int tap) { return sT + ((wave + tap / 3) * PW + 16 * p + j + tap % 3) * PS; };
        // BF16 forms: byte offset, from the lane's tap-0 point, of K chunk
        // 4 m + kq (8 channels of one tap; chunk c is channels 8 (c mod CH8) ..
        // of tap c / CH8).  Step m (a constant once the K loop is unrolled)
        // starts at channel group r of tap tb; lane group kq's chunk is group
        // r + kq of that tap, or, when that reaches CH8, group r + kq - CH8 of
        // the next one (4 lane groups never span more than two taps, since
        // CH8 >= 2).  Chunks past the ninth tap carry zero weights and read
        // any in-tile point (the centre tap's).
        auto bf16_chunk_off = [&](int m) {
            constexpr int CH8 = KPlan<C, DL_BF16>::CH8;        // the same for both BF16 forms
            auto tap_off = [](int t) { return ((t / 3) * PW + t % 3) * PS; };
            const int tb = 4 * m / CH8, r = 4 * m - tb * CH8, tn = tb + 1 < 9 ? tb + 1 : 4;
            return kq * 16 + (kq >= CH8 - r ? tap_off(tn) + (r - CH8) * 16 : tap_off(tb) + r * 16);
        };

        // Wave 0 decodes the tile the next iteration prefetches (or that tile
        // again when it is the last) into the slot the next iteration reads.
        // Each form calls this once per iteration inside its MFMA loop, where
        // the other wave of the SIMD keeps the matrix unit busy while wave 0
        // runs scalar code and waits for its descriptor loads.
        auto ahead = [&]() {
            if (wave == 0 && ti + nslot < t1) {
                const int64_t t2 = ti + 2 * nslot;
                publish(par ^ 1, decode(t2 < t1 ? t2 : ti + nslot));
            }
        };
        // PREF: the operands of K step it + 1 are read while the MFMAs of step
        // it run (the reads past the last step fetch step 0 again and are not
        // used), so the MFMAs wait only for reads issued one step earlier
        if constexpr (PREF) {
            constexpr int G = C / 16, NIT = KPlan<C, P>::NIT;
            const v4f *sW = reinterpret_cast<const v4f *>(sT + L::WOFF);
            auto operands = [&](int it, v4f (&aw)[NB], v4f (&bv)[PB]) {
                const int tap = it / G, gg = it - (it / G) * G;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) aw[nb] = sW[(it * NB + nb) * 64 + lane];
#pragma unroll
                for (int p = 0; p < PB; ++p)
                    bv[p] = *reinterpret_cast<const v4f *>(pt_addr(p, tap) + (gg * 16 + kq * 4) * 4);
            };
            v4f aw[NB], bv[PB];
            operands(0, aw, bv);
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                v4f an[NB], bn[PB];
                operands(it + 1 < NIT ? it + 1 : 0, an, bn);
                __builtin_amdgcn_sched_barrier(0);   // issued before this step's MFMAs
                if (it == NIT / 2) ahead();
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int p = 0; p < PB; ++p)
                            acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[nb][s], bv[p][s], acc[nb][p], 0, 0, 0);
                if (it == 0) pre_loads();
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) aw[nb] = an[nb];
#pragma unroll
                for (int p = 0; p < PB; ++p) bv[p] = bn[p];
            }
        } else if constexpr (P == DL_FP32) {
            constexpr int G = C / 16, NIT = KPlan<C, P>::NIT;
            const v4f *gw = static_cast<const v4f *>(a.wpk);
            const v4f *sW = reinterpret_cast<const v4f *>(sT + L::WOFF);
#pragma unroll 1
            for (int tap = 0; tap < 9; ++tap) {
                if (tap == 4) ahead();
#pragma unroll
                for (int gg = 0; gg < G; ++gg) {
                    const int it = tap * G + gg;
                    v4f aw[NB];
                    if constexpr (GW) {             // weights from L2, one K step ahead
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) aw[nb] = awn[nb];
                        const int itn = it + 1 < NIT ? it + 1 : 0;
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) awn[nb] = gw[(itn * NB + nb) * 64 + lane];
                    } else {
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) aw[nb] = sW[(it * NB + nb) * 64 + lane];
                    }
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
            constexpr int NIT = KPlan<C, P>::NIT;
            const char *sW = sT + L::WOFF;
#pragma unroll
            for (int m = 0; m < NIT; ++m) {
                if (m == NIT / 2) ahead();
                const int co = bf16_chunk_off(m);
                v4f av[NB], bv[PB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    av[nb] = *reinterpret_cast<const v4f *>(sW + ((m * NB + nb) * 64 + lane) * 16);
#pragma unroll
                for (int p = 0; p < PB; ++p) bv[p] = *reinterpret_cast<const v4f *>(pt_addr(p, 0) + co);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int p = 0; p < PB; ++p)
                        acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(v8bf, av[nb]), __builtin_bit_cast(v8bf, bv[p]), acc[nb][p], 0, 0, 0);
            }
        } else if constexpr (P == DL_BF16X3) {
            // as BF16, with both halves of every operand; the operands of step
            // m + 1 are read while the MFMAs of step m run (past the last step
            // step 0 is read again and not used)
            constexpr int NIT = KPlan<C, P>::NIT;
            constexpr int HALF = KPlan<C, P>::HALF;
            const char *sW = sT + L::WOFF;
            auto operands = [&](int m, v4f (&ah)[NB], v4f (&al)[NB], v4f (&bh)[PB], v4f (&bl)[PB]) {
                const int co = bf16_chunk_off(m);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int wo = ((m * NB + nb) * 64 + lane) * 16;
                    ah[nb] = *reinterpret_cast<const v4f *>(sW + wo);
                    al[nb] = *reinterpret_cast<const v4f *>(sW + HALF + wo);
                }
#pragma unroll
                for (int p = 0; p < PB; ++p) {
                    const char *pa = pt_addr(p, 0) + co;
                    bh[p] = *reinterpret_cast<const v4f *>(pa);
                    bl[p] = *reinterpret_cast<const v4f *>(pa + 2 * C);
                }
            };
#pragma unroll
            for (int m = 0; m < NIT; ++m) {
                v4f ah[NB], al[NB], bh[PB], bl[PB];
                operands(m, ah, al, bh, bl);
                if (m == NIT / 2) ahead();
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int p = 0; p < PB; ++p) {
                        const v8bf wh = __builtin_bit_cast(v8bf, ah[nb]), wl = __builtin_bit_cast(v8bf, al[nb]);
                        const v8bf xh = __builtin_bit_cast(v8bf, bh[p]), xl = __builtin_bit_cast(v8bf, bl[p]);
                        acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xh, acc[nb][p], 0, 0, 0);
                        acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xl, acc[nb][p], 0, 0, 0);
                        acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, xh, acc[nb][p], 0, 0, 0);
                    }
            }
        } else {
            constexpr int HPT = KPlan<C, P>::HPT, NIT = KPlan<C, P>::NIT;
            const char *sW = sT + L::WOFF;
#pragma unroll 1
            for (int m = 0; m < NIT; ++m) {
                // The MFMA scales K in blocks of 32: block b of step m is K chunk
                // 4 m + b (half hf of tap t: one channel group of one point;
                // past the ninth tap the weights are zero and any point will
                // do).  Its values are half kq & 1 of lane groups {0, 1} (b
                // even) or {2, 3} (b odd), in bytes 0-15 (b < 2) or 16-31
                // (b >= 2), and its scale comes from lane group b.  So this
                // lane reads half kq & 1 of chunks 4 m + kq / 2 (low 16 bytes)
                // and 4 m + 2 + kq / 2 (high), and the scale of chunk 4 m + kq.
                // Chunk g is half g % HPT of tap g / HPT.  With HPT = 2 (48 or
                // 64 channels) this lane's chunks are halves kq / 2 of taps 2 m
                // and 2 m + 1 and its scale chunk is half kq & 1 of tap
                // 2 m + kq / 2; with HPT = 1 they are taps 4 m + kq / 2,
                // 4 m + 2 + kq / 2 and 4 m + kq.  A tap's point offset depends
                // on m alone (scalar); the lane adds a fixed part.
                auto tap_off = [&](int t) {
                    const int tc = t < 9 ? t : 4;
                    return ((tc / 3) * PW + tc % 3) * PS;
                };
                const int kh = kq >> 1, kl = kq & 1;
                int lo_off, hi_off, soff;
                if constexpr (HPT == 2) {
                    const int p0 = tap_off(2 * m), p1 = tap_off(2 * m + 1);
                    lo_off = p0 + kh * 32 + 16 * kl;
                    hi_off = p1 + kh * 32 + 16 * kl;
                    soff = (kh ? p1 : p0) + L::CT8 + kl;
                } else {
                    static_assert(HPT == 1, "FP8 taps hold one or two 32-channel groups");
                    const int p0 = tap_off(4 * m), p1 = tap_off(4 * m + 1);
                    const int p2 = tap_off(4 * m + 2), p3 = tap_off(4 * m + 3);
                    lo_off = (kh ? p1 : p0) + 16 * kl;
                    hi_off = (kh ? p3 : p2) + 16 * kl;
                    soff = (kq == 0 ? p0 : kq == 1 ? p1 : kq == 2 ? p2 : p3) + L::CT8;
                }
                v8i av[NB], bv[PB];
                int sb[PB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const v4u *pa = reinterpret_cast<const v4u *>(sW + ((m * NB + nb) * 64 + lane) * 32);
                    const v4u lo = pa[0], hi = pa[1];
                    av[nb] = v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
                }
#pragma unroll
                for (int p = 0; p < PB; ++p) {
                    const char *pt = sT + (wave * PW + 16 * p + j) * PS;
                    const v4u lo = *reinterpret_cast<const v4u *>(pt + lo_off);
                    const v4u hi = *reinterpret_cast<const v4u *>(pt + hi_off);
                    bv[p] = v8i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3], (int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
                    sb[p] = *reinterpret_cast<const uint8_t *>(sT + (wave * PW + 16 * p + j) * PS + soff);
                }
                // weights: unit block scales (their per-channel scale is applied
                // in the epilogue); activations: each lane's 32 K values are one
                // group of one point, scaled by that group's E8M0 byte
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int p = 0; p < PB; ++p)
                        acc[nb][p] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                            av[nb], bv[p], acc[nb][p], 0, 0, 0, 0x7F7F7F7F, 0, sb[p]);
            }
            ahead();                         // after the (not unrolled) K loop: no branch inside it
        }

        // epilogue: D row = output channel 16 nb + 4 kq + r, column = pixel j.
        // Stores go through a resource over this wave's output row; pixels
        // past the frame edge take an out-of-range offset and are dropped.
        constexpr int ESZ = Store<P>::ESZ;
        char *sO = sT + L::OOFF + wave * L::OWAVE;          // this wave's staging row
        if constexpr (RES && STAGE) {
#pragma unroll
            for (int i = 0; i < NRC; ++i) {
                const int q = lane + 64 * i, px = q / CPX, part = q - (q / CPX) * CPX;
                *reinterpret_cast<v4u *>(sO + px * L::OPX + part * 16) = rc[i];
            }
            if constexpr (P == DL_FP8) *reinterpret_cast<uint16_t *>(sO + L::RSOFF + lane * 2) = (uint16_t)rsc;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
        // output in phase layout lo = 2^out_shift (1: plain NHWC): pixel (y, x)
        // is point ((y mod lo) lo + x mod lo) hd wd + (y div lo) wd + x div lo
        // of the frame; pixels off the frame take an out-of-range offset
        const int osh = a.out_shift, om = (1 << osh) - 1;
        const int ohd = (H + om) >> osh, owd = (W + om) >> osh;
        const int osub = (yo & om) << osh, oiy = yo >> osh;
        auto out_point = [&](int xo) { return ((osub + (xo & om)) * ohd + oiy) * owd + (xo >> osh); };
        const __amdgpu_buffer_rsrc_t orow =
            buf_rsrc(HEAD ? nullptr : static_cast<char *>(a.out) + act * C * ESZ, HEAD ? 0u : 0x7FFFFFFFu);
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int xo = X0 + dd * (16 * p + j);
            const bool ok = xo < W;
            const int spx = 16 * p + j;                      // this lane's pixel in the staged row
            float hh[NH > 0 ? NH : 1];                        // head partial sums of this lane's channels
#pragma unroll
            for (int q = 0; q < (NH > 0 ? NH : 1); ++q) hh[q] = 0.f;
            v4f vs[P == DL_FP8 && STAGE ? NB : 1];           // FP8: quantised once all NB are known
            if constexpr (RES && !STAGE && !EARLY_RES) load_res(p);
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int oc = nb * 16 + kq * 4;
                v4f v = acc[nb][p];
                if constexpr (P == DL_FP8) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] *= sS[oc + r];
                }
                v[0] += sB[oc + 0]; v[1] += sB[oc + 1]; v[2] += sB[oc + 2]; v[3] += sB[oc + 3];
                uint2 *so = reinterpret_cast<uint2 *>(sO + spx * L::OPX + oc * 2);
                if constexpr (RES && STAGE && P == DL_FP8) {
                    const uint32_t codes = *reinterpret_cast<const uint32_t *>(sO + spx * L::OPX + oc);
                    const uint32_t sbr = *reinterpret_cast<const uint8_t *>(sO + L::RSOFF + spx * 2 + (oc >> 5));
                    v += fp8_unpack4(codes, fp8_scale_value(sbr));
                } else if constexpr (RES && STAGE) {
                    const uint2 u = *so;
                    v += v4f{__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xFFFF0000u),
                             __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xFFFF0000u)};
                } else if constexpr (RES) {
                    v += Store<P>::unpack(rr[nb][EARLY_RES ? p : 0]);
                }
                v = relu4(v);
                // BF16: what is stored, and what the head reads, is BF16
                uint2 pk{0u, 0u};
                if constexpr (P == DL_BF16) {
                    pk = uint2{bf16_pack2(v[0], v[1]), bf16_pack2(v[2], v[3])};
                    if constexpr (HEAD)
                        v = v4f{__uint_as_float(pk.x << 16), __uint_as_float(pk.x & 0xFFFF0000u),
                                __uint_as_float(pk.y << 16), __uint_as_float(pk.y & 0xFFFF0000u)};
                }
                if constexpr (STAGE && P == DL_FP8) {
                    vs[nb] = v;
                } else if constexpr (STAGE) {
                    *so = pk;
                } else if constexpr (!HEAD) {
                    Store<P>::bstore4(orow, ok && row_ok ? (out_point(xo) * C + oc) * ESZ : BUF_OOB, v);
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int q = 0; q < NH; ++q) hh[q] += sH[q * C + oc + r] * v[r];
                }
            }
            if constexpr (STAGE && P == DL_FP8) {
                // group g = channels 32 g .. 32 g + 31 = blocks nb = 2 g, 2 g + 1; its
                // max over the pixel's four lane groups sets the scale byte
                float gm[2] = {0.f, 0.f};
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    gm[nb >> 1] = fmaxf(gm[nb >> 1], fmaxf(fmaxf(vs[nb][0], vs[nb][1]), fmaxf(vs[nb][2], vs[nb][3])));
                uint32_t sbyte[2];
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    gm[g] = fmaxf(gm[g], __shfl_xor(gm[g], 16));
                    gm[g] = fmaxf(gm[g], __shfl_xor(gm[g], 32));
                    sbyte[g] = fp8_scale_byte(gm[g]);
                }
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const v4f v = vs[nb];
                    *reinterpret_cast<uint32_t *>(sO + spx * L::OPX + nb * 16 + kq * 4) =
                        fp8_pack4(v[0], v[1], v[2], v[3], fp8_scale_value(sbyte[nb >> 1]));
                }
                if (kq == 0) *reinterpret_cast<uint16_t *>(sO + L::OSOFF + spx * 2) = (uint16_t)(sbyte[0] | (sbyte[1] << 8));
            }
            if constexpr (HEAD) {
                // the four lane groups hold disjoint channel subsets of the pixel
#pragma unroll
                for (int q = 0; q < NH; ++q) {
                    hh[q] += __shfl_xor(hh[q], 16);
                    hh[q] += __shfl_xor(hh[q], 32);
                }
                if (ok && row_ok) {
                    const int64_t plane = (int64_t)H * W;
                    float *mp = a.maps + NH * px_off + (int64_t)yo * W + xo;
                    // lane group kq writes planes kq, kq + 4, kq + 8
#pragma unroll
                    for (int q = 0; q < NH; ++q)
                        if ((q & 3) == kq) mp[q * plane] = hh[q] + sH[NH * C + q];
                }
            }
        }
        if constexpr (STAGE) {
            // the staged row leaves in whole 16-byte lanes; pixels past the
            // frame edge (and rows off the frame) are dropped as out of range
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
            for (int i = 0; i < NRC; ++i) {
                const int q = lane + 64 * i, px = q / CPX, part = q - (q / CPX) * CPX;
                const int xo = X0 + dd * px;
                const v4u d = *reinterpret_cast<const v4u *>(sO + px * L::OPX + part * 16);
                __builtin_amdgcn_raw_buffer_store_b128(d, orow, row_ok && xo < W ? out_point(xo) * L::OPX + part * 16 : BUF_OOB,
                                                       0, 0);
            }
            if constexpr (P == DL_FP8) {            // one lane per pixel: its two scale bytes
                const __amdgpu_buffer_rsrc_t osc =
                    buf_rsrc(static_cast<char *>(a.out) + sc_off + act * 2, 0x7FFFFFFFu);
                const int xo = X0 + dd * lane;
                const uint32_t sc2 = *reinterpret_cast<const uint16_t *>(sO + L::OSOFF + lane * 2);
                __builtin_amdgcn_raw_buffer_store_b16((unsigned short)sc2, osc, row_ok && xo < W ? out_point(xo) * 2 : BUF_OOB, 0, 0);
            }
        }
    }
}

// ------------------------------------------------------------- launchers
template <int C, int P, int TR, bool RES, int NH>
hipError_t launch_t(const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    using L = Lds<C, P, TR, (NH > 5 ? NH : 5)>;
    if constexpr (!L::FITS) {
        return hipErrorInvalidValue;
    } else {
        auto kern = k_conv<C, P, TR, RES, NH>;
        constexpr size_t sh = L::TOTAL;
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
}

template <int C, int P, int TR>
hipError_t launch_ct(const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    if (a.head) return a.nh == 10 ? launch_t<C, P, TR, true, 10>(a, g, grid, s) : launch_t<C, P, TR, true, 5>(a, g, grid, s);
    if (a.res) return launch_t<C, P, TR, true, 0>(a, g, grid, s);
    return launch_t<C, P, TR, false, 0>(a, g, grid, s);
}

template <int C, int P>
hipError_t launch_cp(const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    if (a.tr == 4) return launch_ct<C, P, 4>(a, g, grid, s);
    if (a.tr == 8) return launch_ct<C, P, 8>(a, g, grid, s);
    return hipErrorInvalidValue;
}

template <int C, int P, int TR>
int blocks_per_cu()
{
    if constexpr (!Lds<C, P, TR>::FITS) {
        return 1;
    } else {
        int nb = 0;
        auto kern = k_conv<C, P, TR, true, 0>;
        constexpr size_t sh = Lds<C, P, TR>::TOTAL;
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)sh);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, TR * 64, sh) != hipSuccess) nb = 1;
        return nb > 0 ? nb : 1;
    }
}

template <int P, int NHL>
bool fits_pn(int C)
{
    switch (C) {
    case 16: return Lds<16, P, 4, NHL>::FITS && Lds<16, P, 8, NHL>::FITS;
    case 32: return Lds<32, P, 4, NHL>::FITS && Lds<32, P, 8, NHL>::FITS;
    case 48: return Lds<48, P, 4, NHL>::FITS && Lds<48, P, 8, NHL>::FITS;
    case 64: return Lds<64, P, 4, NHL>::FITS && Lds<64, P, 8, NHL>::FITS;
    default: return false;
    }
}

template <int P>
bool fits_p(int C, int nh)
{
    return nh == 10 ? fits_pn<P, 10>(C) : fits_pn<P, 5>(C);
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
    // FP32 defaults to 8 rows when its weights then fit in LDS (C <= 48)
    *tr = rows == 4 || (rows == 0 && precision == DL_FP32 && C > 48) ? 4 : 8;
    switch (precision) {
    case DL_FP32: *tc = TileShape<DL_FP32>::TC; break;
    case DL_BF16: *tc = TileShape<DL_BF16>::TC; break;
    case DL_BF16X3: *tc = TileShape<DL_BF16X3>::TC; break;
    default: *tc = TileShape<DL_FP8>::TC; break;
    }
}

bool conv_supported(int C, int precision, int nh)
{
    if (precision == DL_FP32) return fits_p<DL_FP32>(C, nh);
    if (precision == DL_BF16) return fits_p<DL_BF16>(C, nh);
    if (precision == DL_FP8) return fits_p<DL_FP8>(C, nh);
    if (precision == DL_BF16X3) return fits_p<DL_BF16X3>(C, nh);
    return false;
}

size_t conv_packed_bytes(int C, int precision)
{
    const int NB = C / 16, NCH = 9 * (C / 8);
    if (precision == DL_FP32) return (size_t)9 * C * C * 4;
    if (precision == DL_BF16) return (size_t)((NCH + 3) / 4) * NB * 64 * 16;
    if (precision == DL_BF16X3) return 2 * (size_t)((NCH + 3) / 4) * NB * 64 * 16;
    const int HPT = (C + 31) / 32;
    return (size_t)((9 * HPT + 3) / 4) * NB * 64 * 32;
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
    if (precision == DL_BF16 || precision == DL_BF16X3) {
        // step m, block nb, lane (i, kq): 8 bf16 of chunk 4 m + kq; split BF16
        // follows with a second block of the same layout holding the lo
        // halves bf16(w - hi)
        const int NIT = (NCH + 3) / 4;
        const size_t half = (size_t)NIT * NB * 64 * 8;
        uint16_t *o = static_cast<uint16_t *>(dst);
        for (int m = 0; m < NIT; ++m)
            for (int nb = 0; nb < NB; ++nb)
                for (int lane = 0; lane < 64; ++lane) {
                    const int oc = nb * 16 + (lane & 15), ch = 4 * m + (lane >> 4);
                    for (int e = 0; e < 8; ++e) {
                        const float v = ch < NCH ? wt(oc, (ch % CH8) * 8 + e, ch / CH8) : 0.f;
                        const size_t i = ((size_t)(m * NB + nb) * 64 + lane) * 8 + e;
                        const uint16_t hb = host_bf16(v);
                        o[i] = hb;
                        if (precision == DL_BF16X3) {
                            const uint32_t hu = (uint32_t)hb << 16;
                            float hf;
                            std::memcpy(&hf, &hu, 4);
                            o[half + i] = host_bf16(v - hf);
                        }
                    }
                }
        return;
    }
    // FP8: per-output-channel scale s[o] = max|W[o]| / 448; codes of W * (448 / max|W[o]|).
    // K chunk g (32 values) is channels 32 hf .. 32 hf + 31 of tap t = g / HPT,
    // hf = g mod HPT.  Step m, block nb, lane (i, kq): bytes 0-15 = 16-channel
    // half kq & 1 of chunk 4 m + kq / 2, bytes 16-31 = the same half of chunk
    // 4 m + 2 + kq / 2 (the MFMA's K order; see the kernel's FP8 loop)
    std::vector<float> inv(C);
    for (int oc = 0; oc < C; ++oc) {
        float mx = 0.f;
        for (int k = 0; k < C * 9; ++k) mx = std::fmax(mx, std::fabs(W[(size_t)oc * C * 9 + k]));
        scale[oc] = mx > 0.f ? (float)((double)mx / 448.0) : 0.f;
        inv[oc] = mx > 0.f ? (float)(448.0 / (double)mx) : 0.f;
    }
    const int HPT = (C + 31) / 32, NIT = (9 * HPT + 3) / 4;
    uint8_t *o = static_cast<uint8_t *>(dst);
    for (int m = 0; m < NIT; ++m)
        for (int nb = 0; nb < NB; ++nb)
            for (int lane = 0; lane < 64; ++lane) {
                // the MFMA's scale block b of step m is K chunk 4 m + b; its 32
                // values are half kq & 1 of lane groups {0, 1} (b even) or
                // {2, 3} (b odd), bytes 0-15 for b < 2 and 16-31 for b >= 2
                const int oc = nb * 16 + (lane & 15), kq = lane >> 4;
                for (int e = 0; e < 32; ++e) {
                    const int g = 4 * m + (e < 16 ? 0 : 2) + (kq >> 1), tap = g / HPT, hf = g % HPT;
                    const int c = hf * 32 + 16 * (kq & 1) + (e & 15);
                    const float v = tap < 9 && c < C ? wt(oc, c, tap) : 0.f;
                    o[((size_t)(m * NB + nb) * 64 + lane) * 32 + e] = host_e4m3(v * inv[oc]);
                }
            }
}

int conv_max_grid(int C, int precision, int tr, int ncu)
{
    int b = 1;
    if (precision == DL_FP32) b = bpc_p<DL_FP32>(C, tr);
    else if (precision == DL_BF16) b = bpc_p<DL_BF16>(C, tr);
    else if (precision == DL_BF16X3) b = bpc_p<DL_BF16X3>(C, tr);
    else b = bpc_p<DL_FP8>(C, tr);
    return b * ncu;
}

hipError_t launch_conv(int C, int precision, const ConvArgs &a, const Geometry &g, int grid, hipStream_t s)
{
    if (precision == DL_FP32) return launch_p<DL_FP32>(C, a, g, grid, s);
    if (precision == DL_BF16) return launch_p<DL_BF16>(C, a, g, grid, s);
    if (precision == DL_FP8) return launch_p<DL_FP8>(C, a, g, grid, s);
    if (precision == DL_BF16X3) return launch_p<DL_BF16X3>(C, a, g, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace dloc
