// Dense-connection dilated blocks (paper Sec. 3.2: DilatedLoc's blocks connect
// every layer to the outputs of all layers before it, as DenseNet does; Sec.
// 3.2.1: the convolutions are dilated; Sec. 4.1.2: one dilation per block,
// 2, 4, 8, 16).
//
// A block keeps its concatenation in one NHWC buffer of CT = C + L G channels
// per point: channels 0 .. C-1 hold the block input, layer i (3x3, dilation d)
// reads channels 0 .. C + i G - 1 and writes its G channels after them, and
// the 1x1 transition reads all CT channels and writes the next block's input
// into channels 0 .. C-1 of the other buffer.  FP32 throughout.
//
//   k_dstem   preprocessing + 3x3 conv 1 -> C + ReLU into channels 0 .. C-1
//   k_dconv   one dense layer (TAPS = 9) or transition (TAPS = 1) as MFMA
//             implicit GEMM (v_mfma_f32_16x16x4_f32): M = output channels
//             (NB blocks of 16), N = pixels, K = taps x input channels, the
//             input channels taken 16 at a time -- a group's tile and weights
//             are staged in LDS, the next group's tile is loaded into
//             registers while the MFMAs run on the current one
//   k_dhead   1x1 head C -> nh into planar maps
#include <algorithm>

#include "dloc_internal.h"

namespace dloc {

namespace {

constexpr int DXCD = 8;

// ---------------------------------------------------------------- stem
// one workgroup per global row; item = (pixel, 4 output channels)
template <int C>
__global__ void __launch_bounds__(256)
k_dstem(const FrameDesc *__restrict__ fdp, int nf, int64_t nrows, const int64_t *__restrict__ dyn,
        const float *__restrict__ w, const float *__restrict__ b, float offset, float scale, float *__restrict__ act,
        int cs)
{
    __shared__ float sw[C * 9], sb[C];
    for (int i = threadIdx.x; i < C * 9; i += 256) sw[i] = w[i];
    for (int i = threadIdx.x; i < C; i += 256) sb[i] = b[i];
    __syncthreads();
    if (dyn) {
        nf = (int)dyn[DYN_NF];
        nrows = dyn[DYN_ROWS];
    }
    const int64_t row = blockIdx.x;
    if (row >= nrows) return;
    const int f = find_frame(fdp, nf, row, [](const FrameDesc &d) { return d.row_start; });
    const FrameDesc fd = fdp[f];
    const int y = (int)(row - fd.row_start), H = fd.h, W = fd.w;
    constexpr int Q = C / 4;
    for (int idx = threadIdx.x; idx < W * Q; idx += 256) {
        const int x = idx / Q, q = idx - (idx / Q) * Q;
        float xin[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
            xin[t] = (unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W
                         ? ((float)fd.data[(int64_t)yy * fd.stride + xx] - offset) * scale
                         : 0.f;
        }
        v4f o;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 4 * q + r;
            float s = sb[c];
#pragma unroll
            for (int t = 0; t < 9; ++t) s += sw[c * 9 + t] * xin[t];
            o[r] = fmaxf(s, 0.f);
        }
        *reinterpret_cast<v4f *>(act + (fd.act_off + (int64_t)y * W + x) * cs + 4 * q) = o;
    }
}

// ---------------------------------------------------------------- head
// one workgroup per global row; a thread per pixel: nh dot products over the
// first C channels of its point
template <int C>
__global__ void __launch_bounds__(256)
k_dhead(const FrameDesc *__restrict__ fdp, int nf, int64_t nrows, const int64_t *__restrict__ dyn,
        const float *__restrict__ act, int cs, const float *__restrict__ head, int nh, float *__restrict__ maps)
{
    __shared__ float sh[16 * C + 16];
    for (int i = threadIdx.x; i < nh * C + nh; i += 256) sh[i] = head[i];
    __syncthreads();
    if (dyn) {
        nf = (int)dyn[DYN_NF];
        nrows = dyn[DYN_ROWS];
    }
    const int64_t row = blockIdx.x;
    if (row >= nrows) return;
    const int f = find_frame(fdp, nf, row, [](const FrameDesc &d) { return d.row_start; });
    const FrameDesc fd = fdp[f];
    const int y = (int)(row - fd.row_start), W = fd.w;
    const int64_t plane = (int64_t)fd.h * W;
    for (int x = threadIdx.x; x < W; x += 256) {
        const float *pt = act + (fd.act_off + (int64_t)y * W + x) * cs;
        float v[C];
#pragma unroll
        for (int c = 0; c < C; c += 4) {
            const v4f u = *reinterpret_cast<const v4f *>(pt + c);
            v[c] = u[0]; v[c + 1] = u[1]; v[c + 2] = u[2]; v[c + 3] = u[3];
        }
        float *mp = maps + (int64_t)nh * fd.px_off + (int64_t)y * W + x;
        for (int q = 0; q < nh; ++q) {
            float s = sh[nh * C + q];
#pragma unroll
            for (int c = 0; c < C; ++c) s += sh[q * C + c] * v[c];
            mp[q * plane] = s;
        }
    }
}

// ---------------------------------------------------------------- conv
constexpr int DTR = 8, DTC = 32, DPB = DTC / 16;
constexpr int DPS = 24;                  // LDS floats per point: 16 channels, stride 8 mod 16 dwords

template <int NB, int TAPS>
struct DLds {
    static constexpr int HALO = TAPS == 9 ? 1 : 0;
    static constexpr int PW = DTC + 2 * HALO, NPT = (DTR + 2 * HALO) * PW;
    static constexpr int TILE = NPT * DPS;                  // floats
    static constexpr int W = TAPS * NB * 64 * 4;             // floats of one group's weights
    static constexpr int NQ = NPT * 4;                       // 16-byte chunks of a group's tile
    static constexpr int NPF = (NQ + DTR * 64 - 1) / (DTR * 64);
    static constexpr int BYTES = (TILE + W + NB * 16) * 4 + 64;
};

template <int NB, int TAPS>
__global__ void __launch_bounds__(DTR * 64, 2)
k_dconv(DenseConvArgs a, Geometry geo)
{
    using L = DLds<NB, TAPS>;
    constexpr int HALO = L::HALO, PW = L::PW, NT = DTR * 64;
    extern __shared__ v4f dsm[];
    float *sT = reinterpret_cast<float *>(dsm);
    v4f *sW = reinterpret_cast<v4f *>(sT + L::TILE);
    float *sB = sT + L::TILE + L::W;
    int *sdec = reinterpret_cast<int *>(sB + NB * 16);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = lane & 15, kq = lane >> 4;
    const int dd = a.d, blk = a.blk, ngroups = a.cin / 16;
    for (int i = tid; i < NB * 16; i += NT) sB[i] = a.bias[i];

    const int64_t T = geo.dyn ? ld_const(geo.dyn + DYN_TILES + blk) : geo.tiles[blk];
    const int nfr = geo.dyn ? (int)ld_const(geo.dyn + DYN_NF) : geo.nf;
    const int xcd = blockIdx.x % DXCD, slot = blockIdx.x / DXCD, nslot = gridDim.x / DXCD;
    const int64_t chunk = (T + DXCD - 1) / DXCD;
    const int64_t t0 = (int64_t)xcd * chunk, t1 = min(T, t0 + chunk);

    for (int64_t ti = t0 + slot; ti < t1; ti += nslot) {
        // the tile: frame, origin of its phase lattice, frame size and offset
        __syncthreads();                 // the previous tile's LDS reads are done
        if (tid == 0) {
            const int f = find_frame(a.fd, nfr, ti, [blk](const FrameDesc &d) { return ld_const(&d.tile_start[blk]); });
            const FrameDesc *fd = a.fd + f;
            const int h = ld_const(&fd->h), w = ld_const(&fd->w);
            int Y0, X0;
            decode_tile(h, w, ti - ld_const(&fd->tile_start[blk]), dd, DTR, DTC, false, 8u, Y0, X0);
            const int64_t act = ld_const(&fd->act_off);
            sdec[0] = Y0;
            sdec[1] = X0;
            sdec[2] = h;
            sdec[3] = w;
            sdec[4] = (int)(uint32_t)act;
            sdec[5] = (int)(act >> 32);
        }
        __syncthreads();
        const int Y0 = __builtin_amdgcn_readfirstlane(sdec[0]), X0 = __builtin_amdgcn_readfirstlane(sdec[1]);
        const int H = __builtin_amdgcn_readfirstlane(sdec[2]), W = __builtin_amdgcn_readfirstlane(sdec[3]);
        const int64_t act = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(sdec[4]) |
                            ((int64_t)__builtin_amdgcn_readfirstlane(sdec[5]) << 32);
        const float *in = a.in + act * a.csi;

        // one input group's tile (16 channels of every tile point) into registers
        v4f pf[L::NPF];
        auto issue = [&](int g) {
#pragma unroll
            for (int k = 0; k < L::NPF; ++k) {
                const int q = tid + k * NT;
                const int pt = q / 4, c4 = q - (q / 4) * 4;
                const int ii = pt / PW - HALO, jj = pt - (pt / PW) * PW - HALO;
                const int y = Y0 + dd * ii, x = X0 + dd * jj;
                const bool ok = q < L::NQ && (unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W;
                pf[k] = ok ? *reinterpret_cast<const v4f *>(in + ((int64_t)y * W + x) * a.csi + g * 16 + c4 * 4)
                           : v4f{0.f, 0.f, 0.f, 0.f};
            }
        };
        issue(0);
        v4f acc[NB][DPB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int p = 0; p < DPB; ++p) acc[nb][p] = v4f{0.f, 0.f, 0.f, 0.f};
        for (int g = 0; g < ngroups; ++g) {
            __syncthreads();             // the previous group's LDS reads are done
#pragma unroll
            for (int k = 0; k < L::NPF; ++k) {
                const int q = tid + k * NT;
                if (q < L::NQ) *reinterpret_cast<v4f *>(sT + (q / 4) * DPS + (q % 4) * 4) = pf[k];
            }
            const v4f *gw = reinterpret_cast<const v4f *>(a.w) + (size_t)g * (L::W / 4);
            for (int i = tid; i < L::W / 4; i += NT) sW[i] = gw[i];
            __syncthreads();
            if (g + 1 < ngroups) issue(g + 1);   // in flight while the MFMAs run
#pragma unroll
            for (int tap = 0; tap < TAPS; ++tap) {
                const int u = TAPS == 9 ? tap / 3 : 0, v = TAPS == 9 ? tap % 3 : 0;
                v4f aw[NB], bv[DPB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) aw[nb] = sW[(tap * NB + nb) * 64 + lane];
#pragma unroll
                for (int p = 0; p < DPB; ++p)
                    bv[p] = *reinterpret_cast<const v4f *>(sT + ((wave + u) * PW + 16 * p + j + v) * DPS + kq * 4);
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int p = 0; p < DPB; ++p)
                            acc[nb][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[nb][s], bv[p][s], acc[nb][p], 0, 0, 0);
            }
        }
        // epilogue: lane (j, kq) holds output channels 16 nb + 4 kq + r of pixel j
        const int yo = Y0 + dd * wave;
#pragma unroll
        for (int p = 0; p < DPB; ++p) {
            const int xo = X0 + dd * (16 * p + j);
            if (yo >= H || xo >= W) continue;
            float *op = a.out + (act + (int64_t)yo * W + xo) * a.cso + a.co;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                v4f o = acc[nb][p];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float s = o[r] + sB[nb * 16 + 4 * kq + r];
                    o[r] = a.relu ? fmaxf(s, 0.f) : s;
                }
                *reinterpret_cast<v4f *>(op + nb * 16 + 4 * kq) = o;
            }
        }
    }
}

template <int NB, int TAPS>
hipError_t launch_dconv_t(const DenseConvArgs &a, const Geometry &g, int ncu, hipStream_t s)
{
    using L = DLds<NB, TAPS>;
    auto kern = k_dconv<NB, TAPS>;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, L::BYTES);
        if (e != hipSuccess) return e;
        attr = true;
    }
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, DTR * 64, L::BYTES) != hipSuccess || per < 1) per = 1;
    const int64_t tiles = g.dyn ? (int64_t)1 << 40 : g.tiles[a.blk];
    int grid = (int)std::min<int64_t>(tiles, (int64_t)per * ncu);
    grid = std::max(DXCD, grid / DXCD * DXCD);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(DTR * 64), L::BYTES, s, a, g);
    return hipGetLastError();
}

}  // namespace

int dense_tile_rows() { return DTR; }
int dense_tile_cols() { return DTC; }

hipError_t launch_dconv(int nb_out, int taps, const DenseConvArgs &a, const Geometry &g, int ncu, hipStream_t s)
{
    if (taps == 9 && nb_out == 1) return launch_dconv_t<1, 9>(a, g, ncu, s);
    if (taps == 9 && nb_out == 2) return launch_dconv_t<2, 9>(a, g, ncu, s);
    if (taps == 1 && nb_out == 1) return launch_dconv_t<1, 1>(a, g, ncu, s);
    if (taps == 1 && nb_out == 2) return launch_dconv_t<2, 1>(a, g, ncu, s);
    return hipErrorInvalidValue;
}

hipError_t launch_dstem(int C, const FrameDesc *fd, const Geometry &g, const float *w, const float *b, float offset,
                        float scale, float *act, int cs, hipStream_t s)
{
    const unsigned grid = (unsigned)g.total_rows;
    if (C == 32)
        hipLaunchKernelGGL(k_dstem<32>, dim3(grid), dim3(256), 0, s, fd, g.nf, g.total_rows, g.dyn, w, b, offset, scale,
                           act, cs);
    else if (C == 16)
        hipLaunchKernelGGL(k_dstem<16>, dim3(grid), dim3(256), 0, s, fd, g.nf, g.total_rows, g.dyn, w, b, offset, scale,
                           act, cs);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_dhead(int C, const FrameDesc *fd, const Geometry &g, const float *act, int cs, const float *head,
                        int nh, float *maps, hipStream_t s)
{
    const unsigned grid = (unsigned)g.total_rows;
    if (nh > 16) return hipErrorInvalidValue;
    if (C == 32)
        hipLaunchKernelGGL(k_dhead<32>, dim3(grid), dim3(256), 0, s, fd, g.nf, g.total_rows, g.dyn, act, cs, head, nh,
                           maps);
    else if (C == 16)
        hipLaunchKernelGGL(k_dhead<16>, dim3(grid), dim3(256), 0, s, fd, g.nf, g.total_rows, g.dyn, act, cs, head, nh,
                           maps);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// FP32 MFMA layout of one dense conv: input group g (16 channels), tap, output
// block nb, lane (i, kq) -> the 4 weights of output channel 16 nb + i and input
// channels 16 g + 4 kq + s, s = 0..3.  W is [cout][cin][taps] (taps = 9 or 1).
void pack_dense_weights(int cout, int cin, int taps, const float *W, float *dst)
{
    const int NB = cout / 16, G = cin / 16;
    for (int g = 0; g < G; ++g)
        for (int t = 0; t < taps; ++t)
            for (int nb = 0; nb < NB; ++nb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int s = 0; s < 4; ++s) {
                        const int oc = nb * 16 + (lane & 15), c = g * 16 + 4 * (lane >> 4) + s;
                        dst[((((size_t)g * taps + t) * NB + nb) * 64 + lane) * 4 + s] = W[((size_t)oc * cin + c) * taps + t];
                    }
}

}  // namespace dloc
