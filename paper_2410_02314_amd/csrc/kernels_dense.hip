// Dense-connection dilated blocks (paper Sec. 3.2: DilatedLoc's blocks connect
// every layer to the outputs of all layers before it, as DenseNet does; Sec.
// 3.2.1: the convolutions are dilated; Sec. 4.1.2: one dilation per block,
// 2, 4, 8, 16).
//
// A block keeps its concatenation in one NHWC buffer of CT = C + L G channels
// per point: channels 0 .. C-1 hold the block input, layer i (3x3, dilation d)
// reads channels 0 .. C + i G - 1 and writes its G channels after them.  The
// block's 1x1 transition (CT -> C) is fused into its last layer: that layer's
// own G outputs feed only the transition, so they never leave registers, and
// the transition writes the next block's input into channels 0 .. C-1 of the
// other buffer; in the last block the 1x1 head is fused after it as well.
// FP32 throughout.
//
//   k_dstem   preprocessing + 3x3 conv 1 -> C + ReLU into channels 0 .. C-1
//   k_dconv   one dense layer as MFMA implicit GEMM (v_mfma_f32_16x16x4_f32):
//             M = output channels (NB blocks of 16), N = pixels, K = 9 taps x
//             input channels taken 16 at a time -- a group's tile and weights
//             are staged in LDS, the next group's tile and weights are loaded
//             into registers while the MFMAs run on the current one.  FUSE = 1
//             adds the transition, FUSE = 2 the transition and the head.
//             TRAIN: the training passes' epilogue (optional bias, residual,
//             ReLU and mask); with FUSE = 1 it also stores the last layer's
//             own outputs, which the backward pass needs.
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

// ---------------------------------------------------------------- conv
constexpr int DTR = 8, DTC = 32, DPB = DTC / 16;
constexpr int DPS = 24;                  // LDS floats per point: 16 channels, stride 8 mod 16 dwords
constexpr int PW = DTC + 2, NPT = (DTR + 2) * PW;   // tile points with the one-point halo

// LDS of one workgroup (floats): the group's tile, the group's layer weights,
// [fused] the group's transition weights, the transition weights of the
// layer's own outputs, [head] the head weights; then the biases.
// FUSE: 0 the layer alone; 1 + the block's 1x1 transition; 2 + transition +
// head; 3 + head (on the layer's own outputs)
template <int NB, int NT, int FUSE>
struct DLds {
    static constexpr bool TR = FUSE == 1 || FUSE == 2, HD = FUSE >= 2;
    static constexpr int HK = FUSE == 3 ? NB : NT;           // head K groups (16 channels each)
    static constexpr int TILE = NPT * DPS;
    static constexpr int W = 9 * NB * 64 * 4;                // one group's layer weights
    static constexpr int WT = TR ? NT * 64 * 4 : 0;          // one group's transition weights
    static constexpr int WTL = TR ? NB * NT * 64 * 4 : 0;    // transition weights of the layer's outputs
    static constexpr int WH = HD ? HK * 64 * 4 : 0;          // head weights (16 rows, K = 16 HK)
    static constexpr int BIAS = NB * 16 + (TR ? NT * 16 : 0) + (HD ? 16 : 0);
    static constexpr int NQ = NPT * 4;                       // 16-byte chunks of a group's tile
    static constexpr int NPF = (NQ + DTR * 64 - 1) / (DTR * 64);
    static constexpr int NWF = (W / 4 + DTR * 64 - 1) / (DTR * 64);   // weight chunks per thread
    static constexpr int NTF = (WT / 4 + DTR * 64 - 1) / (DTR * 64);
    static constexpr int BYTES = (TILE + W + WT + WTL + WH + BIAS) * 4 + 64;
};

template <int NB, int NT, int FUSE, bool QUEUE, bool TRAIN>
__global__ void __launch_bounds__(DTR * 64)
k_dconv(DenseConvArgs a, Geometry geo)
{
    using L = DLds<NB, NT, FUSE>;
    constexpr bool TR = L::TR, HD = L::HD;
    constexpr int HK = L::HK;
    constexpr int NTH = DTR * 64;
    extern __shared__ v4f dsm[];
    float *sT = reinterpret_cast<float *>(dsm);
    v4f *sW = reinterpret_cast<v4f *>(sT + L::TILE);
    v4f *sWT = sW + L::W / 4;
    v4f *sWTL = sWT + L::WT / 4;
    v4f *sWH = sWTL + L::WTL / 4;
    float *sB = reinterpret_cast<float *>(sWH + L::WH / 4);
    float *sBT = sB + NB * 16;                   // [fused] transition bias
    float *sBH = sBT + (TR ? NT * 16 : 0);       // [head] head bias (nh of 16)
    int *sdec = reinterpret_cast<int *>(sB + L::BIAS);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int j = lane & 15, kq = lane >> 4;
    const int dd = a.d, blk = a.blk, ngroups = a.cin / 16;
    for (int i = tid; i < NB * 16; i += NTH) sB[i] = !TRAIN || a.bias ? a.bias[i] : 0.f;
    if constexpr (TR) {
        const v4f *wl = reinterpret_cast<const v4f *>(a.wt) + (size_t)ngroups * NT * 64;
        for (int i = tid; i < L::WTL / 4; i += NTH) sWTL[i] = wl[i];
        for (int i = tid; i < NT * 16; i += NTH) sBT[i] = a.bt[i];
    }
    if constexpr (HD) {
        for (int i = tid; i < L::WH / 4; i += NTH) sWH[i] = reinterpret_cast<const v4f *>(a.wh)[i];
        for (int i = tid; i < 16; i += NTH) sBH[i] = i < a.nh ? a.bh[i] : 0.f;
    }

    const int64_t T = geo.dyn ? ld_const(geo.dyn + DYN_TILES + blk) : geo.tiles[blk];
    const int nfr = geo.dyn ? (int)ld_const(geo.dyn + DYN_NF) : geo.nf;
    const int xcd = blockIdx.x % DXCD, slot = blockIdx.x / DXCD, nslot = gridDim.x / DXCD;
    const int64_t chunk = (T + DXCD - 1) / DXCD;
    const int64_t t0 = (int64_t)xcd * chunk, t1 = min(T, t0 + chunk);

    // tile schedule: static (tile t0 + slot, then every nslot-th of the XCD's
    // range), or (QUEUE) claimed from an atomic queue -- the XCD's, over its
    // range (queue_mode 1), or one over all tiles (2); a claim past the end
    // ends the workgroup
    const int64_t qb = a.queue_mode == 2 ? 0 : t0, qe = a.queue_mode == 2 ? T : t1;
    for (int64_t si = t0 + slot; QUEUE || si < t1; si += nslot) {
        // the tile: frame, origin of its phase lattice, frame size and offsets
        __syncthreads();                 // the previous tile's LDS reads are done
        if (tid == 0) {
            int64_t ti = si;
            bool valid = true;
            if constexpr (QUEUE) {
                ti = qb + (int64_t)atomicAdd(a.queue + (a.queue_mode == 1 ? xcd : 0), 1u);
                valid = ti < qe;
                sdec[8] = valid;
            }
            if (valid) {
                const int f = find_frame(a.fd, nfr, ti, [blk](const FrameDesc &d) { return ld_const(&d.tile_start[blk]); });
                const FrameDesc *fd = a.fd + f;
                const int h = ld_const(&fd->h), w = ld_const(&fd->w);
                int Y0, X0;
                decode_tile(h, w, ti - ld_const(&fd->tile_start[blk]), dd, DTR, DTC, false, 8u, Y0, X0);
                const int64_t act = ld_const(&fd->act_off), px = ld_const(&fd->px_off);
                sdec[0] = Y0;
                sdec[1] = X0;
                sdec[2] = h;
                sdec[3] = w;
                sdec[4] = (int)(uint32_t)act;
                sdec[5] = (int)(act >> 32);
                sdec[6] = (int)(uint32_t)px;
                sdec[7] = (int)(px >> 32);
            }
        }
        __syncthreads();
        if constexpr (QUEUE)
            if (!__builtin_amdgcn_readfirstlane(sdec[8])) break;   // uniform: every thread reads the same flag
        const int Y0 = __builtin_amdgcn_readfirstlane(sdec[0]), X0 = __builtin_amdgcn_readfirstlane(sdec[1]);
        const int H = __builtin_amdgcn_readfirstlane(sdec[2]), W = __builtin_amdgcn_readfirstlane(sdec[3]);
        const int64_t act = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(sdec[4]) |
                            ((int64_t)__builtin_amdgcn_readfirstlane(sdec[5]) << 32);
        const float *in = a.in + act * a.csi;

        // one input group's tile (16 channels of every tile point) and the
        // group's weights into registers
        v4f pf[L::NPF], wf[L::NWF], tf[L::NTF > 0 ? L::NTF : 1];
        auto issue = [&](int g) {
            const v4f *gw = reinterpret_cast<const v4f *>(a.w) + (size_t)g * (L::W / 4);
#pragma unroll
            for (int k = 0; k < L::NWF; ++k) {
                const int i = tid + k * NTH;
                if (i < L::W / 4) wf[k] = gw[i];
            }
            if constexpr (TR) {
                const v4f *tw = reinterpret_cast<const v4f *>(a.wt) + (size_t)g * (L::WT / 4);
#pragma unroll
                for (int k = 0; k < L::NTF; ++k) {
                    const int i = tid + k * NTH;
                    if (i < L::WT / 4) tf[k] = tw[i];
                }
            }
#pragma unroll
            for (int k = 0; k < L::NPF; ++k) {
                const int q = tid + k * NTH;
                const int pt = q / 4, c4 = q - (q / 4) * 4;
                const int ii = pt / PW - 1, jj = pt - (pt / PW) * PW - 1;
                const int y = Y0 + dd * ii, x = X0 + dd * jj;
                const bool ok = q < L::NQ && (unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W;
                pf[k] = ok ? *reinterpret_cast<const v4f *>(in + ((int64_t)y * W + x) * a.csi + g * 16 + c4 * 4)
                           : v4f{0.f, 0.f, 0.f, 0.f};
            }
        };
        issue(0);
        v4f acc[NB][DPB];
        v4f accT[TR ? NT : 1][DPB];      // [fused] transition accumulators
#pragma unroll
        for (int p = 0; p < DPB; ++p) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb][p] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int nt = 0; nt < (TR ? NT : 1); ++nt) accT[nt][p] = v4f{0.f, 0.f, 0.f, 0.f};
        }
        for (int g = 0; g < ngroups; ++g) {
            __syncthreads();             // the previous group's LDS reads are done
#pragma unroll
            for (int k = 0; k < L::NPF; ++k) {
                const int q = tid + k * NTH;
                if (q < L::NQ) *reinterpret_cast<v4f *>(sT + (q / 4) * DPS + (q % 4) * 4) = pf[k];
            }
#pragma unroll
            for (int k = 0; k < L::NWF; ++k) {
                const int i = tid + k * NTH;
                if (i < L::W / 4) sW[i] = wf[k];
            }
            if constexpr (TR) {
#pragma unroll
                for (int k = 0; k < L::NTF; ++k) {
                    const int i = tid + k * NTH;
                    if (i < L::WT / 4) sWT[i] = tf[k];
                }
            }
            __syncthreads();
            if (g + 1 < ngroups) issue(g + 1);   // in flight while the MFMAs run
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int u = tap / 3, v = tap % 3;
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
                if constexpr (TR) {
                    if (tap == 4) {      // the centre tap's operand is this group's 1x1 input
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) {
                            const v4f awt = sWT[nt * 64 + lane];
#pragma unroll
                            for (int s = 0; s < 4; ++s)
#pragma unroll
                                for (int p = 0; p < DPB; ++p)
                                    accT[nt][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(awt[s], bv[p][s], accT[nt][p], 0, 0, 0);
                        }
                    }
                }
            }
        }
        // epilogue: lane (j, kq) holds output channels 16 nb + 4 kq + r of pixel j
        const int yo = Y0 + dd * wave;
#pragma unroll
        for (int p = 0; p < DPB; ++p) {
            const int xo = X0 + dd * (16 * p + j);
            const bool inside = yo < H && xo < W;
            v4f o[NB];
            if constexpr (TRAIN) {
                // training passes: (acc + bias [+ res]) [ReLU] [times (mask > 0)],
                // res and mask read at the output point
                const int64_t pt = act + (int64_t)yo * W + xo;
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int c0 = nb * 16 + 4 * kq;
                    const v4f rv = a.res && inside ? *reinterpret_cast<const v4f *>(a.res + pt * a.rcs + c0)
                                                   : v4f{0.f, 0.f, 0.f, 0.f};
                    const v4f mv = a.mask && inside ? *reinterpret_cast<const v4f *>(a.mask + pt * a.mcs + c0)
                                                    : v4f{1.f, 1.f, 1.f, 1.f};
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float v = acc[nb][p][r] + sB[c0 + r] + rv[r];
                        if (a.relu) v = fmaxf(v, 0.f);
                        o[nb][r] = mv[r] > 0.f ? v : 0.f;
                    }
                }
            } else {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) o[nb][r] = fmaxf(acc[nb][p][r] + sB[nb * 16 + 4 * kq + r], 0.f);
                }
            }
            if constexpr (!TR && !HD) {
                if (inside) {
                    float *op = a.out + (act + (int64_t)yo * W + xo) * a.cso + a.co;
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) *reinterpret_cast<v4f *>(op + nb * 16 + 4 * kq) = o[nb];
                }
            } else {
                v4f hin[HK];                 // the head's input: transition or layer outputs
                if constexpr (TRAIN && TR) {
                    // training keeps the layer's own outputs too
                    if (inside) {
                        float *op = a.out + (act + (int64_t)yo * W + xo) * a.cso + a.co;
#pragma unroll
                        for (int nb = 0; nb < NB; ++nb) *reinterpret_cast<v4f *>(op + nb * 16 + 4 * kq) = o[nb];
                    }
                }
                if constexpr (TR) {
                    // the layer's outputs are the transition's last K groups: in the
                    // accumulator layout, lane (j, kq) element s is channel 4 kq + s
                    // of pixel j, which is the B operand's layout for K step s
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) {
                            const v4f awl = sWTL[(nb * NT + nt) * 64 + lane];
#pragma unroll
                            for (int s = 0; s < 4; ++s)
                                accT[nt][p] = __builtin_amdgcn_mfma_f32_16x16x4f32(awl[s], o[nb][s], accT[nt][p], 0, 0, 0);
                        }
                    v4f t[NT];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int r = 0; r < 4; ++r) t[nt][r] = fmaxf(accT[nt][p][r] + sBT[nt * 16 + 4 * kq + r], 0.f);
                    if constexpr (FUSE == 1) {
                        if (inside) {
                            float *op = a.tout + (act + (int64_t)yo * W + xo) * a.cst;
#pragma unroll
                            for (int nt = 0; nt < NT; ++nt) *reinterpret_cast<v4f *>(op + nt * 16 + 4 * kq) = t[nt];
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < HK; ++k) hin[k] = t[k];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < HK; ++k) hin[k] = o[k];
                }
                if constexpr (HD) {
                    // head: outputs q = 4 kq + r of pixel j, K = the head's 16 HK inputs
                    v4f hq = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int k = 0; k < HK; ++k) {
                        const v4f awh = sWH[k * 64 + lane];
#pragma unroll
                        for (int s = 0; s < 4; ++s) hq = __builtin_amdgcn_mfma_f32_16x16x4f32(awh[s], hin[k][s], hq, 0, 0, 0);
                    }
                    if (inside) {
                        const int64_t px = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane(sdec[6]) |
                                           ((int64_t)__builtin_amdgcn_readfirstlane(sdec[7]) << 32);
                        const int64_t plane = (int64_t)H * W;
                        float *mp = a.maps + a.nh * px + (int64_t)yo * W + xo;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int q = 4 * kq + r;
                            if (q < a.nh) mp[q * plane] = hq[r] + sBH[q];
                        }
                    }
                }
            }
        }
    }
}

template <int NB, int NT, int FUSE, bool QUEUE, bool TRAIN = false>
hipError_t launch_dconv_q(const DenseConvArgs &a, const Geometry &g, int ncu, hipStream_t s)
{
    using L = DLds<NB, NT, FUSE>;
    auto kern = k_dconv<NB, NT, FUSE, QUEUE, TRAIN>;
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

template <int NB, int NT, int FUSE>
hipError_t launch_dconv_t(const DenseConvArgs &a, const Geometry &g, int ncu, hipStream_t s)
{
    return a.queue ? launch_dconv_q<NB, NT, FUSE, true>(a, g, ncu, s) : launch_dconv_q<NB, NT, FUSE, false>(a, g, ncu, s);
}

template <int NB, int FUSE>
hipError_t launch_nt(int nt, const DenseConvArgs &a, const Geometry &g, int ncu, hipStream_t s)
{
    if (nt == 1) return launch_dconv_t<NB, 1, FUSE>(a, g, ncu, s);
    if (nt == 2) return launch_dconv_t<NB, 2, FUSE>(a, g, ncu, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- U-Net
// Levels of a frame: level l + 1 of an h x w level is ceil(h/2) x ceil(w/2);
// each level has its own frame descriptors (h, w, act_off), one per frame in
// the same order.  One thread per (destination point, 4 channels).

// 2 x 2 max pooling of C channels: src level -> dst (the next level); a
// window at an odd edge takes the pixels it has
__global__ void __launch_bounds__(256)
k_pool2(const FrameDesc *__restrict__ sfd, const FrameDesc *__restrict__ dfd, int nf, int64_t npts,
        const float *__restrict__ src, int scs, float *__restrict__ dst, int dcs, int C)
{
    const int Q = C / 4;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npts * Q; i += (int64_t)gridDim.x * 256) {
        const int64_t pt = i / Q;
        const int q = (int)(i - pt * Q);
        const int f = find_frame(dfd, nf, pt, [](const FrameDesc &d) { return d.act_off; });
        const FrameDesc D = dfd[f], Sd = sfd[f];
        const int64_t local = pt - D.act_off;
        const int y = (int)(local / D.w), x = (int)(local - (int64_t)y * D.w);
        v4f m = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int yy = 2 * y + dy, xx = 2 * x + dx;
                if (yy < Sd.h && xx < Sd.w) {
                    const v4f v = *reinterpret_cast<const v4f *>(src + (Sd.act_off + (int64_t)yy * Sd.w + xx) * scs + 4 * q);
#pragma unroll
                    for (int r = 0; r < 4; ++r) m[r] = fmaxf(m[r], v[r]);
                }
            }
        *reinterpret_cast<v4f *>(dst + pt * dcs + 4 * q) = m;
    }
}

// nearest upsampling of C channels: src level -> dst (the level above):
// dst(y, x) = src(y / 2, x / 2)
__global__ void __launch_bounds__(256)
k_up2(const FrameDesc *__restrict__ sfd, const FrameDesc *__restrict__ dfd, int nf, int64_t npts,
      const float *__restrict__ src, int scs, float *__restrict__ dst, int dcs, int C)
{
    const int Q = C / 4;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < npts * Q; i += (int64_t)gridDim.x * 256) {
        const int64_t pt = i / Q;
        const int q = (int)(i - pt * Q);
        const int f = find_frame(dfd, nf, pt, [](const FrameDesc &d) { return d.act_off; });
        const FrameDesc D = dfd[f], Sd = sfd[f];
        const int64_t local = pt - D.act_off;
        const int y = (int)(local / D.w), x = (int)(local - (int64_t)y * D.w);
        *reinterpret_cast<v4f *>(dst + pt * dcs + 4 * q) =
            *reinterpret_cast<const v4f *>(src + (Sd.act_off + (int64_t)(y / 2) * Sd.w + x / 2) * scs + 4 * q);
    }
}

}  // namespace

hipError_t launch_pool2(const FrameDesc *sfd, const FrameDesc *dfd, int nf, int64_t npts, const float *src, int scs,
                        float *dst, int dcs, int C, hipStream_t s)
{
    const int64_t n = npts * (C / 4);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
    hipLaunchKernelGGL(k_pool2, dim3(grid), dim3(256), 0, s, sfd, dfd, nf, npts, src, scs, dst, dcs, C);
    return hipGetLastError();
}

hipError_t launch_up2(const FrameDesc *sfd, const FrameDesc *dfd, int nf, int64_t npts, const float *src, int scs,
                      float *dst, int dcs, int C, hipStream_t s)
{
    const int64_t n = npts * (C / 4);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
    hipLaunchKernelGGL(k_up2, dim3(grid), dim3(256), 0, s, sfd, dfd, nf, npts, src, scs, dst, dcs, C);
    return hipGetLastError();
}

hipError_t launch_dconv_train(int nb_out, const DenseConvArgs &a, const Geometry &g, int ncu, hipStream_t s)
{
    switch (nb_out) {
    case 1: return launch_dconv_q<1, 1, 0, false, true>(a, g, ncu, s);
    case 2: return launch_dconv_q<2, 1, 0, false, true>(a, g, ncu, s);
    case 3: return launch_dconv_q<3, 1, 0, false, true>(a, g, ncu, s);
    case 4: return launch_dconv_q<4, 1, 0, false, true>(a, g, ncu, s);
    case 5: return launch_dconv_q<5, 1, 0, false, true>(a, g, ncu, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dconv_train_fused(int nt, const DenseConvArgs &a, const Geometry &g, int ncu, hipStream_t s)
{
    if (nt == 1) return launch_dconv_q<1, 1, 1, false, true>(a, g, ncu, s);
    if (nt == 2) return launch_dconv_q<1, 2, 1, false, true>(a, g, ncu, s);
    return hipErrorInvalidValue;
}

int dense_tile_rows() { return DTR; }
int dense_tile_cols() { return DTC; }

hipError_t launch_dconv(int nb_out, int fuse, int nt, const DenseConvArgs &a, const Geometry &g, int ncu, hipStream_t s)
{
    if (fuse == 0) {
        if (nb_out == 1) return launch_dconv_t<1, 1, 0>(a, g, ncu, s);
        if (nb_out == 2) return launch_dconv_t<2, 1, 0>(a, g, ncu, s);
        return hipErrorInvalidValue;
    }
    if (a.nh > 16) return hipErrorInvalidValue;
    if (fuse == 3) {             // layer + head (no transition)
        if (nb_out == 1) return launch_dconv_t<1, 1, 3>(a, g, ncu, s);
        if (nb_out == 2) return launch_dconv_t<2, 1, 3>(a, g, ncu, s);
        return hipErrorInvalidValue;
    }
    if (nb_out == 1) return fuse == 1 ? launch_nt<1, 1>(nt, a, g, ncu, s) : launch_nt<1, 2>(nt, a, g, ncu, s);
    if (nb_out == 2) return fuse == 1 ? launch_nt<2, 1>(nt, a, g, ncu, s) : launch_nt<2, 2>(nt, a, g, ncu, s);
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
