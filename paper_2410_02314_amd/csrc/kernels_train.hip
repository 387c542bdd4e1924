// Training of the localisation network (paper Sec. 3.3: DECODE's loss with a
// binary cross-entropy on the per-pixel detection probability added).  The
// residual network with the 10-output head, FP32, plain NHWC activations of C
// floats per point; a batch of n frames of h x w, frame f's points from f h w.
// The convolutions of the forward and backward passes run on the dense conv
// kernel (launch_dconv_train); this file holds the rest:
//
//   k_pack_conv     a 3x3 conv's weights from the flat parameters into the
//                   conv kernel's MFMA layout (optionally flipped and
//                   transposed: the weights of the transposed convolution)
//   k_head_fwd      1x1 head C -> 10 into planar maps
//   k_occupancy     the pixels holding a true emitter
//   k_pix_terms     per pixel: log p - sum_d log s_d - 2 log 2 pi, m_d, 1 / s_d
//   k_frame_stats   per frame: mu = sum p, v = sum p (1 - p) + eps, BCE sum
//                   (16 blocks per frame, then summed in order)
//   k_lse_part      per true emitter and pixel chunk of its frame: partial
//                   log-sum-exp of q_k = log p_k - log mu + sum_d log N(t_d;
//                   m_kd, s_kd^2) (one lane per emitter, the chunk's pixel terms
//                   in LDS, a running maximum)
//   k_lse_fin       per true emitter: the chunks combined in order
//   k_loss_grad     per pixel: d loss / d maps (10 planes)
//   k_loss_total    the batch means of the loss terms
//   k_head_grad_part head weight and bias gradient partials per pixel chunk
//   k_head_back     d loss / d (last block's pre-activation)
//   k_wgrad         3x3 weight and bias gradient partial sums per workgroup on
//                   MFMA: dW[co][ci][tap] = sum_p dy[p][co] x[p + off(tap)][ci]
//   k_sum_partials  fixed-order sums of per-workgroup partials
//   k_stem_grad_part stem weight and bias gradient partials per pixel chunk
//   k_pack_jobs, k_mask_slice, k_1x1_back, k_pool2_back, k_up2_back: the
//                   dense network's weight packs, ReLU masks of channel slices,
//                   the transition's input gradient, the U-Net's pooling and
//                   upsampling gradients
// Reductions run in a fixed order: the gradients do not depend on timing.
#include <algorithm>
#include <cmath>

#include "dloc_internal.h"

namespace dloc {

namespace {

constexpr float TWO_PI = 6.283185307179586f;

__device__ __forceinline__ float softplusf(float u) { return fmaxf(u, 0.f) + log1pf(expf(-fabsf(u))); }
__device__ __forceinline__ float sigmoidf(float u) { return 1.f / (1.f + expf(-u)); }

// block-wide sum of one float per thread (blockDim 256), fixed order
__device__ float block_sum(float v, float *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) sh[t] += sh[t + o];
        __syncthreads();
    }
    const float r = sh[0];
    __syncthreads();
    return r;
}

__device__ float block_max(float v, float *sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) sh[t] = fmaxf(sh[t], sh[t + o]);
        __syncthreads();
    }
    const float r = sh[0];
    __syncthreads();
    return r;
}

// Packs count square 3x3 convolutions (C -> C) into the conv kernel's MFMA
// layout, each twice: pack (i, fl) at dst + (2 i + fl) 9 C^2, from the flat
// weights at W + i src_stride.  Within a pack,
// dst[(((g 9 + t) NB + nb) 64 + lane) 4 + s] = Wp[16 nb + (lane & 15)][16 g + 4 (lane >> 4) + s][t]
// with Wp = W [C][C][9] (fl = 0), or Wp[o][c][t] = W[c][o][8 - t] (fl = 1: the
// transposed convolution).
__global__ void __launch_bounds__(256)
k_pack_conv(const float *__restrict__ W0, int64_t src_stride, int count, int C, float *__restrict__ dst)
{
    const int n = C * C * 9;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)count * 2 * n) return;
    const int pk = (int)(e / n), i = (int)(e - (int64_t)pk * n);
    const int fl = pk & 1;
    const float *W = W0 + (pk >> 1) * src_stride;
    const int NB = C / 16;
    const int s = i & 3, lane = (i >> 2) & 63;
    const int rest = i >> 8;                 // ((g 9 + t) NB + nb)
    const int nb = rest % NB, gt = rest / NB;
    const int t = gt % 9, g = gt / 9;
    const int o = nb * 16 + (lane & 15), c = g * 16 + 4 * (lane >> 4) + s;
    dst[e] = fl ? W[((size_t)c * C + o) * 9 + (8 - t)] : W[((size_t)o * C + c) * 9 + t];
}

// Packs of any 3x3 or 1x1 conv weights into the conv kernel's MFMA layout,
// one job each (see PackJob): element i of job j is
// dst[j.dst + i] = Wp[row0 + 16 nb + (lane & 15)][16 g + 4 (lane >> 4) + s][t]
// for i = (((g taps + t) NB + nb) 64 + lane) 4 + s, NB = nrows / 16, where Wp
// is the job's weights W = params + src ([cout][cin][taps]) or, flipped, the
// transposed convolution's Wp[o][c][t] = W[c][o][taps - 1 - t].
__global__ void __launch_bounds__(256)
k_pack_jobs(const PackJob *__restrict__ jobs, int njobs, int64_t total, const float *__restrict__ params,
            float *__restrict__ dst)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].start <= e) lo = mid; else hi = mid - 1;
    }
    const PackJob J = jobs[lo];
    const int i = (int)(e - J.start);
    if (i >= J.nrows * (J.flip ? J.cout : J.cin) * J.taps) return;   // the padding before the next job
    const int NB = J.nrows / 16;
    const int s = i & 3, lane = (i >> 2) & 63, rest = i >> 8;
    const int nb = rest % NB, gt = rest / NB;
    const int t = gt % J.taps, g = gt / J.taps;
    const int o = J.row0 + nb * 16 + (lane & 15), c = g * 16 + 4 * (lane >> 4) + s;
    const float *W = params + J.src;
    dst[J.dst + i] = J.flip ? W[((size_t)c * J.cin + o) * J.taps + (J.taps - 1 - t)]
                            : W[((size_t)o * J.cin + c) * J.taps + t];
}

// dst[p][c] = src[p][so + c] where m[p][mo + c] > 0, else 0, for c < nc (a
// multiple of 4); points of scs, mcs and dcs floats; a thread per four channels
__global__ void __launch_bounds__(256)
k_mask_slice(const float *__restrict__ src, int scs, int so, const float *__restrict__ m, int mcs, int mo, int nc,
             int64_t npx, float *__restrict__ dst, int dcs)
{
    const int q4 = nc / 4;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= npx * q4) return;
    const int64_t p = i / q4;
    const int c = (int)(i - p * q4) * 4;
    const float4 v = *reinterpret_cast<const float4 *>(src + p * scs + so + c);
    const float4 k = *reinterpret_cast<const float4 *>(m + p * mcs + mo + c);
    *reinterpret_cast<float4 *>(dst + p * dcs + c) =
        make_float4(k.x > 0.f ? v.x : 0.f, k.y > 0.f ? v.y : 0.f, k.z > 0.f ? v.z : 0.f, k.w > 0.f ? v.w : 0.f);
}

// The 1x1 transition's input gradient: out[p][c] = sum_o Wt[o][c] g[p][o] for
// c < ct (Wt [C][ct] from the flat weights, staged in LDS; g: points of C
// floats; out: points of ct floats, ct a multiple of 16), a GEMM on
// v_mfma_f32_16x16x4_f32: a wave takes 16 points at a time, rows = points,
// columns = 16 output channels, K = the C gradient channels with lane (i, kq)
// giving g[point i][(C / 4) kq + s] at K step s (one or two 16-byte loads per
// lane).  The output: lane (j, kq) holds channel j of points 4 kq + r.
template <int C>
__global__ void __launch_bounds__(256)
k_1x1_back(const float *__restrict__ g, const float *__restrict__ Wt, int ct, int64_t npx, float *__restrict__ out)
{
    constexpr int KS = C / 4;                  // K steps
    extern __shared__ float sWt[];
    for (int i = threadIdx.x; i < C * ct; i += 256) sWt[i] = Wt[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, i = lane & 15, kq = lane >> 4;
    const int64_t ngrp = (npx + 15) / 16;
    for (int64_t grp = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); grp < ngrp; grp += (int64_t)gridDim.x * 4) {
        const int64_t p = grp * 16 + i;
        float av[KS];
#pragma unroll
        for (int k = 0; k < KS / 4; ++k) {
            const float4 v = p < npx ? *reinterpret_cast<const float4 *>(g + p * C + KS * kq + 4 * k)
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
            av[4 * k] = v.x;
            av[4 * k + 1] = v.y;
            av[4 * k + 2] = v.z;
            av[4 * k + 3] = v.w;
        }
        for (int cb = 0; cb < ct / 16; ++cb) {
            v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int st = 0; st < KS; ++st)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[st], sWt[(KS * kq + st) * ct + cb * 16 + i], acc, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t q = grp * 16 + 4 * kq + r;
                if (q < npx) out[q * ct + cb * 16 + i] = acc[r];
            }
        }
    }
}

// U-Net backward over a batch of n uniform frames of h x w at the fine level
// (the coarse level is ceil(h/2) x ceil(w/2); frame f's points from f h w and
// f h2 w2).  A thread per (coarse point, four channels).
//
// k_pool2_back: the 2 x 2 max pooling's gradient.  Each window's argmax is
// taken again from the pooling's input a (points of acs floats, channels
// 0 .. C-1): the first maximum in the window's raster order among its pixels
// inside the frame; g (coarse, points of gcs floats) is added there into out
// (fine, points of ocs floats).  Windows do not overlap, so no point is
// written twice.
__global__ void __launch_bounds__(256)
k_pool2_back(const float *__restrict__ a, int acs, const float *__restrict__ g, int gcs, float *__restrict__ out,
             int ocs, int n, int h, int w, int C)
{
    const int h2 = (h + 1) / 2, w2 = (w + 1) / 2, q4 = C / 4;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)n * h2 * w2 * q4) return;
    const int64_t pc = i / q4;
    const int c = (int)(i - pc * q4) * 4;
    const int f = (int)(pc / ((int64_t)h2 * w2)), k = (int)(pc - (int64_t)f * h2 * w2);
    const int y2 = k / w2, x2 = k - y2 * w2;
    const int64_t base = (int64_t)f * h * w;
    float m[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    const int64_t first = base + (int64_t)(2 * y2) * w + 2 * x2;   // inside the frame for every window
    int64_t at[4] = {first, first, first, first};
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const int y = 2 * y2 + dy, x = 2 * x2 + dx;
            if (y < h && x < w) {
                const int64_t pt = base + (int64_t)y * w + x;
                const float4 v = *reinterpret_cast<const float4 *>(a + pt * acs + c);
                const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (vv[r] > m[r]) {
                        m[r] = vv[r];
                        at[r] = pt;
                    }
            }
        }
    const float4 gv = *reinterpret_cast<const float4 *>(g + pc * gcs + c);
    const float gg[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) out[at[r] * ocs + c + r] += gg[r];
}

// k_up2_back: the nearest upsampling's gradient: out (coarse, points of ocs
// floats) = the sum of g (fine, points of gcs floats) over the (up to) four
// fine pixels each coarse pixel fills, in raster order.
__global__ void __launch_bounds__(256)
k_up2_back(const float *__restrict__ g, int gcs, float *__restrict__ out, int ocs, int n, int h, int w, int C)
{
    const int h2 = (h + 1) / 2, w2 = (w + 1) / 2, q4 = C / 4;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)n * h2 * w2 * q4) return;
    const int64_t pc = i / q4;
    const int c = (int)(i - pc * q4) * 4;
    const int f = (int)(pc / ((int64_t)h2 * w2)), k = (int)(pc - (int64_t)f * h2 * w2);
    const int y2 = k / w2, x2 = k - y2 * w2;
    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            const int y = 2 * y2 + dy, x = 2 * x2 + dx;
            if (y < h && x < w) {
                const float4 v = *reinterpret_cast<const float4 *>(g + ((int64_t)f * h * w + (int64_t)y * w + x) * gcs + c);
                sum.x += v.x;
                sum.y += v.y;
                sum.z += v.z;
                sum.w += v.w;
            }
        }
    *reinterpret_cast<float4 *>(out + pc * ocs + c) = sum;
}

template <int C>
__global__ void __launch_bounds__(256)
k_head_fwd(const float *__restrict__ act, const float *__restrict__ hw, const float *__restrict__ hb, int64_t npx,
           int64_t hwpx, float *__restrict__ maps)
{
    __shared__ float sw[10 * C + 10];
    for (int i = threadIdx.x; i < 10 * C + 10; i += 256) sw[i] = i < 10 * C ? hw[i] : hb[i - 10 * C];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= npx) return;
    const int64_t f = p / hwpx, k = p - f * hwpx;
    float v[C];
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = act[p * C + c];
    for (int q = 0; q < 10; ++q) {
        float s = sw[10 * C + q];
#pragma unroll
        for (int c = 0; c < C; ++c) s += sw[q * C + c] * v[c];
        maps[(f * 10 + q) * hwpx + k] = s;
    }
}

// frame of emitter e: the largest f with toff[f] <= e (toff[0] = 0, increasing)
__device__ int find_frame_off(const int32_t *toff, int n, int e)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (toff[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// occupancy of every pixel (1 where a true emitter lies), from the truth list
__global__ void __launch_bounds__(256)
k_occupancy(const dl_truth *__restrict__ tr, const int32_t *__restrict__ toff, int n, int ntruth, int h, int w,
            uint8_t *__restrict__ occ)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= ntruth) return;
    const int f = find_frame_off(toff, n, e);
    const int row = (int)floorf(tr[e].y), col = (int)floorf(tr[e].x);
    if ((unsigned)row < (unsigned)h && (unsigned)col < (unsigned)w) occ[((int64_t)f * h + row) * w + col] = 1;
}

__global__ void __launch_bounds__(256) k_zero_u8(uint8_t *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

// Per pixel, what the mixture terms need, planar over the batch's pixels:
// term[0] = log p - sum_d log s_d - 2 log(2 pi), term[1 + d] = m_d,
// term[5 + d] = 1 / s_d (d = x, y, z, N in the units of the targets; s_d =
// softplus(u_d) + DL_SIGMA_FLOOR)
__global__ void __launch_bounds__(256)
k_pix_terms(const float *__restrict__ maps, int n, int h, int w, float *__restrict__ term)
{
    const int64_t P = (int64_t)h * w, np = (int64_t)n * P;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= np) return;
    const int64_t f = i / P, k = i - f * P;
    const int row = (int)(k / w), col = (int)(k - (int64_t)row * w);
    const float *M = maps + f * 10 * P;
    float c = -softplusf(-M[k]) - 2.f * logf(TWO_PI);
    term[np + i] = col + 0.5f + M[P + k];
    term[2 * np + i] = row + 0.5f + M[2 * P + k];
    term[3 * np + i] = M[3 * P + k];
    term[4 * np + i] = M[4 * P + k];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const float sd = softplusf(M[(5 + d) * P + k]) + DL_SIGMA_FLOOR;
        c -= logf(sd);
        term[(5 + d) * np + i] = 1.f / sd;
    }
    term[i] = c;
}

constexpr int STAT_CHUNKS = 16;   // blocks per frame for the frame statistics

// partial[f][chunk] = {sum p, sum p (1 - p), sum softplus(l) - y l}
__global__ void __launch_bounds__(256)
k_frame_stats(const float *__restrict__ maps, int h, int w, const uint8_t *__restrict__ occ, float *__restrict__ partial)
{
    __shared__ float sh[256];
    const int f = blockIdx.x / STAT_CHUNKS, ch = blockIdx.x % STAT_CHUNKS;
    const int64_t P = (int64_t)h * w;
    const float *L = maps + (int64_t)f * 10 * P;
    const uint8_t *Y = occ + (int64_t)f * P;
    float mu = 0.f, v = 0.f, b = 0.f;
    for (int64_t k = (int64_t)ch * 256 + threadIdx.x; k < P; k += STAT_CHUNKS * 256) {
        const float l = L[k], p = sigmoidf(l);
        mu += p;
        v += p * (1.f - p);
        b += softplusf(l) - (Y[k] ? l : 0.f);
    }
    mu = block_sum(mu, sh);
    v = block_sum(v, sh);
    b = block_sum(b, sh);
    if (threadIdx.x == 0) {
        float *o = partial + 3 * (size_t)blockIdx.x;
        o[0] = mu;
        o[1] = v;
        o[2] = b;
    }
}

// stats[f] = {mu, v + eps, bce sum}: the chunks summed in order
__global__ void __launch_bounds__(256)
k_frame_stats_sum(const float *__restrict__ partial, int n, float eps, float *__restrict__ stats)
{
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (f >= n) return;
    float a[3] = {0.f, 0.f, 0.f};
    for (int c = 0; c < STAT_CHUNKS; ++c)
        for (int q = 0; q < 3; ++q) a[q] += partial[3 * ((size_t)f * STAT_CHUNKS + c) + q];
    stats[3 * f] = a[0];
    stats[3 * f + 1] = a[1] + eps;
    stats[3 * f + 2] = a[2];
}

// The localisation term's log-sum-exp over a frame's pixels, per true emitter,
// is computed in base 2 (q' = q log2 e): a pixel's q' is
//   q'_k = log2e term0_k - (log2e / 2) sum_d ((t_d - m_kd) / s_kd)^2.
constexpr float LOG2E = 1.4426950408889634f;
constexpr float LN2 = 0.6931471805599453f;
constexpr int LSE_MAX_CHUNKS = 64;   // pixel chunks per frame whose partials are combined per emitter
constexpr int EM_STRIDE = 8;         // floats of an emitter's constants

// Emitter constants em[e] = {t_x, t_y, t_z, t_N, lse2_e, -, -, -}: the targets
// in the maps' units and log2 sum_k 2^(q'_k) over the emitter's frame.
__device__ __forceinline__ void target_of(const dl_truth &t, float izs, float ips, float (&tv)[4])
{
    tv[0] = t.x;
    tv[1] = t.y;
    tv[2] = t.z_nm * izs;
    tv[3] = t.photons * ips;
}

// the pixel chunks of the log-sum-exp: chunk c of a frame covers the 256-pixel
// groups [c spc, c spc + spc), spc = ceil(ceil(P / 256) / LSE_MAX_CHUNKS)
__host__ __device__ __forceinline__ int lse_groups_per_chunk(int64_t P)
{
    const int64_t g = (P + 255) / 256;
    return (int)((g + LSE_MAX_CHUNKS - 1) / LSE_MAX_CHUNKS);
}
__host__ __device__ __forceinline__ int lse_chunks(int64_t P)
{
    const int64_t g = (P + 255) / 256, spc = lse_groups_per_chunk(P);
    return (int)((g + spc - 1) / spc);
}

// Partial log-sum-exp of every true emitter of frame f over one pixel chunk:
// one lane per emitter, the chunk's pixel terms staged in LDS 256 at a time
// and read by all lanes at once; a running (max, sum of 2^(q' - max)) per lane
// updated eight pixels at a time.  part[(e nch + c) 2 + {0, 1}] = (max, sum).
__global__ void __launch_bounds__(256)
k_lse_part(const float *__restrict__ term, int n, int h, int w, const dl_truth *__restrict__ tr,
           const int32_t *__restrict__ toff, float izs, float ips, float *__restrict__ part)
{
    __shared__ __align__(16) float4 sa[256], sb[256];
    __shared__ float sc[256];
    const int64_t P = (int64_t)h * w, np = (int64_t)n * P;
    const int nch = lse_chunks(P), spc = lse_groups_per_chunk(P);
    const int f = blockIdx.x / nch, c = blockIdx.x - f * nch;
    const int e0 = toff[f], e1 = toff[f + 1];
    const int t = threadIdx.x;
    const int64_t k0 = (int64_t)c * spc * 256, k1 = std::min<int64_t>(P, k0 + (int64_t)spc * 256);
    const float hz = -0.5f * LOG2E;
    for (int eg = e0; eg < e1; eg += 256) {
        const int e = eg + t;
        float tv[4] = {0.f, 0.f, 0.f, 0.f};
        if (e < e1) target_of(tr[e], izs, ips, tv);
        float m = -3.0e38f, s = 0.f;
        for (int64_t kb = k0; kb < k1; kb += 256) {
            __syncthreads();
            {
                const int64_t k = kb + t;
                if (k < k1) {
                    const int64_t i = (int64_t)f * P + k;
                    sa[t] = make_float4(term[i] * LOG2E, term[np + i], term[2 * np + i], term[3 * np + i]);
                    sb[t] = make_float4(term[4 * np + i], term[5 * np + i], term[6 * np + i], term[7 * np + i]);
                    sc[t] = term[8 * np + i];
                } else {                      // past the frame: q' = -inf
                    sa[t] = make_float4(-INFINITY, 0.f, 0.f, 0.f);
                    sb[t] = make_float4(0.f, 0.f, 0.f, 0.f);
                    sc[t] = 0.f;
                }
            }
            __syncthreads();
            if (e >= e1) continue;
            for (int j0 = 0; j0 < 256; j0 += 8) {
                float q[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float4 A = sa[j0 + j], B = sb[j0 + j];
                    const float zx = (tv[0] - A.y) * B.y, zy = (tv[1] - A.z) * B.z;
                    const float zz = (tv[2] - A.w) * B.w, zn = (tv[3] - B.x) * sc[j0 + j];
                    q[j] = fmaf(hz, zx * zx + zy * zy + zz * zz + zn * zn, A.x);
                }
                float mx = q[0];
#pragma unroll
                for (int j = 1; j < 8; ++j) mx = fmaxf(mx, q[j]);
                const float mn = fmaxf(m, mx);
                float a = s * __builtin_amdgcn_exp2f(m - mn);
#pragma unroll
                for (int j = 0; j < 8; ++j) a += __builtin_amdgcn_exp2f(q[j] - mn);
                s = a;
                m = mn;
            }
        }
        if (e < e1) {
            part[((size_t)e * nch + c) * 2] = m;
            part[((size_t)e * nch + c) * 2 + 1] = s;
        }
    }
}

// Per emitter (a wave each, lane c holding chunk c): the chunks' partials
// combined by a fixed butterfly; lse[e] = the localisation log-sum-exp
// (natural log, with -log mu), em[e] its constants.
__global__ void __launch_bounds__(256)
k_lse_fin(int n, int h, int w, const dl_truth *__restrict__ tr, const int32_t *__restrict__ toff, int ntruth,
          const float *__restrict__ stats, float izs, float ips, const float *__restrict__ part, float *__restrict__ lse,
          float *__restrict__ em)
{
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (e >= ntruth) return;
    const int nch = lse_chunks((int64_t)h * w);
    const float *pp = part + (size_t)e * nch * 2;
    const float m = lane < nch ? pp[2 * lane] : -3.0e38f;
    float M = m;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) M = fmaxf(M, __shfl_xor(M, o));
    float S = lane < nch ? pp[2 * lane + 1] * exp2f(m - M) : 0.f;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) S += __shfl_xor(S, o);
    if (lane != 0) return;
    const int f = find_frame_off(toff, n, e);
    const float l2 = M + log2f(S);
    lse[e] = l2 * LN2 - logf(stats[3 * f]);
    float tv[4];
    target_of(tr[e], izs, ips, tv);
    float *o = em + (size_t)e * EM_STRIDE;
    o[0] = tv[0];
    o[1] = tv[1];
    o[2] = tv[2];
    o[3] = tv[3];
    o[4] = l2;
    o[5] = o[6] = o[7] = 0.f;
}

// d (batch mean loss) / d maps: workgroup (f, chunk) takes 256 pixels of frame
// f, one per thread; the frame's emitters are the same for the whole
// workgroup, so their constants are read once per wave.  r_ek = 2^(q'_ek -
// lse2_e) is pixel k's responsibility for emitter e; with R = sum_e r_ek, Z_d =
// sum_e r z_d, Z2_d = sum_e r z_d^2 (z_d = (t_d - m_kd) / s_kd):
//   d/dl   = (p - y) / P + p(1-p) (dmu + (1 - 2p) dv) - (1 - p) R + E p (1-p) / mu
//   d/dm_d = -Z_d / s_d,   d/du_d = -(Z2_d - R) sigmoid(u_d) / s_d
__global__ void __launch_bounds__(256)
k_loss_grad(const float *__restrict__ maps, const float *__restrict__ term, const uint8_t *__restrict__ occ, int n,
            int h, int w, const int32_t *__restrict__ toff, const float *__restrict__ stats,
            const float *__restrict__ em, float *__restrict__ gm)
{
    const int P = h * w, np = n * P;
    const int cpf = (P + 255) / 256;
    const int f = blockIdx.x / cpf, k = (blockIdx.x - f * cpf) * 256 + threadIdx.x;
    if (k >= P) return;
    const int i = f * P + k;
    const float *M = maps + (size_t)f * 10 * P;
    float *G = gm + (size_t)f * 10 * P;
    const float inv_n = 1.f / (float)n;
    const int e0 = toff[f], e1 = toff[f + 1];
    const float E = (float)(e1 - e0);
    const float mu = stats[3 * f], v = stats[3 * f + 1];
    const float l = M[k], p = sigmoidf(l), pq = p * (1.f - p);
    // cross-entropy and count
    float gl = (p - (occ[i] ? 1.f : 0.f)) / (float)P;
    const float dmu = -(E - mu) / v, dv = 0.5f / v - (E - mu) * (E - mu) / (2.f * v * v);
    gl += pq * (dmu + (1.f - 2.f * p) * dv);
    // localisation
    float mv[4], is[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        mv[d] = term[(size_t)(1 + d) * np + i];
        is[d] = term[(size_t)(5 + d) * np + i];
    }
    const float q0 = term[i] * LOG2E, hz = -0.5f * LOG2E;
    float R = 0.f, Z[4] = {0.f, 0.f, 0.f, 0.f}, Z2[4] = {0.f, 0.f, 0.f, 0.f};
    for (int e = e0; e < e1; ++e) {
        const float *c = em + (size_t)e * EM_STRIDE;
        float z[4], zz[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            z[d] = (c[d] - mv[d]) * is[d];
            zz[d] = z[d] * z[d];
        }
        const float r = __builtin_amdgcn_exp2f(fmaf(hz, zz[0] + zz[1] + zz[2] + zz[3], q0) - c[4]);
        R += r;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            Z[d] = fmaf(r, z[d], Z[d]);
            Z2[d] = fmaf(r, zz[d], Z2[d]);
        }
    }
    gl += -(1.f - p) * R + E * pq / mu;
    G[k] = gl * inv_n;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        G[(1 + d) * P + k] = -Z[d] * is[d] * inv_n;
        G[(5 + d) * P + k] = -(Z2[d] - R) * is[d] * sigmoidf(M[(5 + d) * P + k]) * inv_n;
    }
    G[9 * P + k] = 0.f;
}

// loss[4] = batch means of {total, bce, count, loc}
__global__ void __launch_bounds__(256)
k_loss_total(int n, int h, int w, const int32_t *__restrict__ toff, int ntruth, const float *__restrict__ stats,
             const float *__restrict__ lse, float *__restrict__ loss)
{
    __shared__ float sh[256];
    const float P = (float)h * (float)w;
    float b = 0.f, c = 0.f, l = 0.f;
    for (int f = threadIdx.x; f < n; f += 256) {
        const float mu = stats[3 * f], v = stats[3 * f + 1];
        const float E = (float)(toff[f + 1] - toff[f]);
        b += stats[3 * f + 2] / P;
        c += 0.5f * logf(TWO_PI * v) + (E - mu) * (E - mu) / (2.f * v);
    }
    for (int e = threadIdx.x; e < ntruth; e += 256) l -= lse[e];
    b = block_sum(b, sh);
    c = block_sum(c, sh);
    l = block_sum(l, sh);
    if (threadIdx.x == 0) {
        loss[0] = (b + c + l) / n;
        loss[1] = b / n;
        loss[2] = c / n;
        loss[3] = l / n;
    }
}

constexpr int GCHUNK = 256;   // pixels per workgroup of the head and stem gradient partials

// Head gradient partials: workgroup b sums over pixels [b GCHUNK, b GCHUNK +
// GCHUNK) of the batch; part[b][q C + c] = sum gm[q][p] a[p][c], part[b][10 C +
// q] = sum gm[q][p].  The chunk's map gradients are staged in LDS (one pixel
// per thread); thread (slot, c) then sums channel c over every (256 / C)-th
// pixel, and the slots are added in order.
template <int C>
__global__ void __launch_bounds__(256)
k_head_grad_part(const float *__restrict__ gm, const float *__restrict__ act, int npx, int hwpx,
                 float *__restrict__ part)
{
    constexpr int NS = 256 / C, NO = 10 * C + 10;
    __shared__ float sg[10][GCHUNK];
    __shared__ float red[NS][NO];
    const int t = threadIdx.x, p0 = blockIdx.x * GCHUNK, np = min(GCHUNK, npx - p0);
    if (t < np) {
        const int p = p0 + t, f = p / hwpx, k = p - f * hwpx;
#pragma unroll
        for (int q = 0; q < 10; ++q) sg[q][t] = gm[((size_t)f * 10 + q) * hwpx + k];
    }
    __syncthreads();
    const int sl = t / C, c = t - sl * C;
    float acc[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, bacc = 0.f;
    for (int j = sl; j < np; j += NS) {
        const float a = act[(size_t)(p0 + j) * C + c];
#pragma unroll
        for (int q = 0; q < 10; ++q) acc[q] = fmaf(sg[q][j], a, acc[q]);
        if (c < 10) bacc += sg[c][j];
    }
#pragma unroll
    for (int q = 0; q < 10; ++q) red[sl][q * C + c] = acc[q];
    if (c < 10) red[sl][10 * C + c] = bacc;
    __syncthreads();
    for (int o = t; o < NO; o += 256) {
        float v = 0.f;
        for (int k = 0; k < NS; ++k) v += red[k][o];
        part[(size_t)blockIdx.x * NO + o] = v;
    }
}

// du[p][c] = (sum_q W[q][c] gm[q][p]) where a[p][c] > 0, else 0: a thread per
// (pixel, four channels), so a wave reads and writes 64 / (C / 4) whole points
template <int C>
__global__ void __launch_bounds__(256)
k_head_back(const float *__restrict__ gm, const float *__restrict__ hw, const float *__restrict__ act, int npx,
            int hwpx, float *__restrict__ du)
{
    constexpr int QT = C / 4;
    __shared__ float sw[10 * C];
    for (int i = threadIdx.x; i < 10 * C; i += 256) sw[i] = hw[i];
    __syncthreads();
    const int gid = blockIdx.x * 256 + threadIdx.x;
    const int p = gid / QT, c0 = (gid - p * QT) * 4;
    if (p >= npx) return;
    const int f = p / hwpx, k = p - f * hwpx;
    float g[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) g[q] = gm[((size_t)f * 10 + q) * hwpx + k];
    const float4 a = *reinterpret_cast<const float4 *>(act + (size_t)p * C + c0);
    float v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 10; ++q) s += sw[q * C + c0 + j] * g[q];
        v[j] = s;
    }
    *reinterpret_cast<float4 *>(du + (size_t)p * C + c0) =
        make_float4(a.x > 0.f ? v[0] : 0.f, a.y > 0.f ? v[1] : 0.f, a.z > 0.f ? v[2] : 0.f, a.w > 0.f ? v[3] : 0.f);
}

typedef float v16f __attribute__((ext_vector_type(16)));

// The weight gradient's matrix instruction per channel count.  In both, lane l
// gives channel l % C of pixel l / C to both operands (A = dy: rows are output
// channels; B = x: columns are input channels), so K = 64 / C pixels per
// instruction; C = 32 takes v_mfma_f32_32x32x2f32 (twice the arithmetic per
// operand of the 16 x 16 x 4 form), C = 16 v_mfma_f32_16x16x4f32.  The
// accumulator's registers come in groups of four rows of one column (l % C):
// row0(l, g) is the first row of group g.
template <int C> struct WgMma;
template <> struct WgMma<32> {
    typedef v16f acc_t;
    static constexpr int NG = 4;
    __device__ static acc_t mma(float a, float b, const acc_t &c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row0(int l, int g) { return 8 * g + 4 * (l >> 5); }
};
template <> struct WgMma<16> {
    typedef v4f acc_t;
    static constexpr int NG = 1;
    __device__ static acc_t mma(float a, float b, const acc_t &c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row0(int l, int) { return 4 * (l >> 4); }
};

constexpr int WG_WAVES = 8;
constexpr uint32_t BUF_FLAGS = 0x00020000u;   // raw buffer, 32-bit words
constexpr int BUF_OOB = (int)0x80000000u;      // an offset past any buffer: reads zero

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float *base, uint32_t nbytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, (int)nbytes, (int)BUF_FLAGS);
}

// Weight gradient of a 3x3 (TAPS = 9) or 1x1 (TAPS = 1) conv at dilation d
// over NHWC tensors: dW[co][ci][tap] = sum_p dy[p][co] x[p + off(tap)][ci]
// (zero off the frame), db[co] = sum_p dy[p][co], for CO output channels (dy:
// points of dcs floats) and CI input channels (x: points of xcs floats,
// channels 0 .. CI-1), CI a multiple of CO.  Workgroup (b, cb) takes input
// channels [cb CO, cb CO + CO).
//
// Work unit: a column segment (sps steps of 64 / CO pixels) of a chain of K
// output rows of one frame spaced by the dilation (y, y + d, .., y + (K-1) d;
// K = 4 for 3x3, 1 for 1x1); chain c's segments are units c nseg .. c nseg +
// nseg - 1, and a wave takes cpw consecutive units.  Output row j's tap row u reads input row y + (j + u - 1)
// d, so the chain's K rows need only K + 2 input rows per step (not 3 K), and
// all of them add into the same nine accumulators.  Per step: K dy loads, 3 (K
// + 2) x loads, 9 K matrix instructions.  A frame's chains: blocks of K d rows
// by residue mod d.  Every operand is a buffer load: a row off the frame is a
// buffer of no bytes and a column off the frame an offset past the buffer,
// both of which read zero, so the loads carry no branch; the next step's
// loads are issued before this step's matrix instructions.  The eight waves'
// sums are added in order through LDS, one group of output rows at a time
// (each wave only stores its accumulators, so they go to LDS without passing
// through vector registers), and written in the weights' own order:
// part[b][(co CI + ci) TAPS + tap]; pb[b][co] (cb = 0).
template <int CO, int TAPS>
__global__ void __launch_bounds__(64 * WG_WAVES)
k_wgrad(const float *__restrict__ dy, int dcs, const float *__restrict__ x, int xcs, int CI, int n, int h, int w,
        int d, int nseg, int sps, int cpw, float *__restrict__ part, float *__restrict__ pb)
{
    using M = WgMma<CO>;
    constexpr int PX = 64 / CO;
    constexpr int GR = CO / M::NG;             // output rows per group (8 or 16)
    constexpr int TSR = CO * GR + 4;           // LDS floats per (wave, tap), padded against bank conflicts
    constexpr int NU = TAPS == 9 ? 3 : 1;      // tap rows (and columns)
    constexpr int K = TAPS == 9 ? 4 : 1;       // output rows per chain
    constexpr int XR = K + NU - 1;             // input rows per chain
    __shared__ __align__(16) float red[WG_WAVES * TAPS * TSR];
    __shared__ float sb[WG_WAVES][CO];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ch = lane % CO, kp = lane / CO;
    const int cb = blockIdx.y, xch = cb * CO + ch;
    const int de = TAPS == 9 ? d : 1;                    // row spacing within a chain
    const int nres = min(de, h), nblk = (h + K * de - 1) / (K * de);
    const int cpf = nblk * nres;                         // chains per frame
    const int nun = n * cpf * nseg;                      // units
    const int u0 = (blockIdx.x * WG_WAVES + wave) * cpw, u1 = min(nun, u0 + cpw);
    const int steps = (w + PX - 1) / PX;
    const uint32_t dbytes = (uint32_t)w * dcs * 4, xbytes = (uint32_t)w * xcs * 4;
    typename M::acc_t acc[TAPS];
#pragma unroll
    for (int t = 0; t < TAPS; ++t) acc[t] = typename M::acc_t{};
    float bsum = 0.f;
    __amdgpu_buffer_rsrc_t rd[K], rx[XR];
    int u = u0, q = 0, qend = 0;
    auto set_unit = [&]() {
        const int c = u / nseg, sg = u - c * nseg;
        q = sg * sps;
        qend = min(steps, q + sps);
        const int f = c / cpf, cc = c - f * cpf;
        const int y0 = (cc / nres) * K * de + cc % nres;
        const float *fx = x + (size_t)f * h * w * xcs, *fd = dy + (size_t)f * h * w * dcs;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int y = y0 + j * de;
            rd[j] = row_rsrc(fd + (size_t)(y < h ? y : 0) * w * dcs, y < h ? dbytes : 0u);
        }
#pragma unroll
        for (int j = 0; j < XR; ++j) {
            const int y = y0 + (j - (NU - 1) / 2) * de;       // input row j: output row j - 1 (3x3) or j (1x1)
            const bool ok = (unsigned)y < (unsigned)h;
            rx[j] = row_rsrc(fx + (size_t)(ok ? y : 0) * w * xcs, ok ? xbytes : 0u);
        }
    };
    // loads of step (u, q), then on to the step after it; past the last unit
    // the dy rows become buffers of no bytes, so further steps add zeros
    auto load_next = [&](float (&a)[K], float (&b)[XR][NU]) {
        const int xx = q * PX + kp;
        const int oa = xx < w ? (xx * dcs + ch) * 4 : BUF_OOB;
#pragma unroll
        for (int j = 0; j < K; ++j) a[j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rd[j], oa, 0, 0));
#pragma unroll
        for (int v = 0; v < NU; ++v) {
            const int xs = TAPS == 9 ? xx + d * (v - 1) : xx;
            const int o = (unsigned)xs < (unsigned)w ? (xs * xcs + xch) * 4 : BUF_OOB;
#pragma unroll
            for (int j = 0; j < XR; ++j)
                b[j][v] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx[j], o, 0, 0));
        }
        if (++q == qend) {
            if (u + 1 < u1) {
                ++u;
                set_unit();
            } else {
#pragma unroll
                for (int j = 0; j < K; ++j) rd[j] = row_rsrc(dy, 0u);
            }
        }
    };
    auto step = [&](const float (&a)[K], const float (&b)[XR][NU]) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            bsum += a[j];
#pragma unroll
            for (int u = 0; u < NU; ++u)
#pragma unroll
                for (int v = 0; v < NU; ++v) acc[NU * u + v] = M::mma(a[j], b[j + u][v], acc[NU * u + v]);
        }
    };
    if (u0 < u1) {
        const int total = (u1 - u0) * sps;           // at least the units' steps (a short last segment adds zeros)
        set_unit();
        float a0[K], b0[XR][NU], a1[K], b1[XR][NU];
        load_next(a0, b0);
        for (int it = 0; it < total; it += 2) {   // an odd total ends with a step of zeros
            load_next(a1, b1);
            step(a0, b0);
            load_next(a0, b0);
            step(a1, b1);
        }
    }
    // the bias: the K pixel groups of channel ch
#pragma unroll
    for (int o = CO; o < 64; o <<= 1) bsum += __shfl_xor(bsum, o);
    if (lane < CO) sb[wave][lane] = bsum;
    // per group of GR output rows: every wave stores its accumulators, then the
    // waves' values are added in order; LDS [wave][tap][ci][row in group]
    float *P = part + (size_t)blockIdx.x * CO * CI * TAPS;
#pragma unroll
    for (int g = 0; g < M::NG; ++g) {
#pragma unroll
        for (int t = 0; t < TAPS; ++t) {
            float4 *dst = reinterpret_cast<float4 *>(red + (wave * TAPS + t) * TSR + ch * GR + M::row0(lane, g) - g * GR);
            *dst = make_float4(acc[t][4 * g], acc[t][4 * g + 1], acc[t][4 * g + 2], acc[t][4 * g + 3]);
        }
        __syncthreads();
        for (int j = threadIdx.x; j < GR * CO * TAPS; j += 64 * WG_WAVES) {
            const int t = j % TAPS, ci = (j / TAPS) % CO, r = j / (TAPS * CO);
            float v = 0.f;
#pragma unroll
            for (int k = 0; k < WG_WAVES; ++k) v += red[(k * TAPS + t) * TSR + ci * GR + r];
            P[((size_t)(g * GR + r) * CI + cb * CO + ci) * TAPS + t] = v;
        }
        __syncthreads();
    }
    if (cb == 0 && threadIdx.x < CO) {
        float v = 0.f;
        for (int k = 0; k < WG_WAVES; ++k) v += sb[k][threadIdx.x];
        pb[(size_t)blockIdx.x * CO + threadIdx.x] = v;
    }
}

// Sums over nb partials of two arrays at once (ma values of pa and mb of pb
// per partial), in two fixed-order stages: groups of G = ceil(nb / ng)
// partials into mid[g][ma + mb], then the ng groups into oa and ob.  Each
// thread adds its terms in order, eight loads in flight at a time.
__device__ __forceinline__ float ordered_sum(const float *__restrict__ src, size_t stride, int cnt)
{
    float s = 0.f;
    int b = 0;
    for (; b + 8 <= cnt; b += 8) {
        float v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = src[(size_t)(b + k) * stride];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; b < cnt; ++b) s += src[(size_t)b * stride];
    return s;
}

__global__ void __launch_bounds__(256)
k_sum_partials_grouped(const float *__restrict__ pa, int ma, const float *__restrict__ pbb, int mb, int nb, int ng,
                       float *__restrict__ mid)
{
    const int m = ma + mb;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)ng * m) return;
    const int g = (int)(idx / m), j = (int)(idx - (int64_t)g * m);
    const int G = (nb + ng - 1) / ng;
    const int b0 = g * G, b1 = min(nb, b0 + G);
    const int stride = j < ma ? ma : mb;
    const float *src = (j < ma ? pa + j : pbb + (j - ma)) + (size_t)b0 * stride;
    mid[idx] = ordered_sum(src, stride, b1 - b0);
}

__global__ void __launch_bounds__(256)
k_sum_partials(const float *__restrict__ mid, int ng, int ma, int mb, float *__restrict__ oa, float *__restrict__ ob)
{
    const int m = ma + mb;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const float s = ordered_sum(mid + j, m, ng);
    if (j < ma) oa[j] = s;
    else ob[j - ma] = s;
}

// Stem gradient partials over pixels [b GCHUNK, b GCHUNK + GCHUNK): part[b][c 9 +
// tap] = sum ds[p][c] x(p + off(tap)), part[b][9 C + c] = sum ds[p][c].  The
// chunk's nine preprocessed inputs per pixel are staged in LDS (one pixel per
// thread); thread (slot, c) sums channel c over every (256 / C)-th pixel, and
// the slots are added in order.
template <int C>
__global__ void __launch_bounds__(256)
k_stem_grad_part(const float *__restrict__ ds, const uint16_t *__restrict__ frames, int n, int h, int w,
                 float offset, float scale, float *__restrict__ part)
{
    constexpr int NS = 256 / C, NO = 10 * C;
    __shared__ float sx[9][GCHUNK];
    __shared__ float red[NS][NO];
    const int hw = h * w, P = n * hw;
    const int t = threadIdx.x, p0 = blockIdx.x * GCHUNK, np = min(GCHUNK, P - p0);
    if (t < np) {
        const int p = p0 + t, f = p / hw, k = p - f * hw, y = k / w, xx = k - y * w;
        const uint16_t *F = frames + (size_t)f * hw;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int yy = y + tap / 3 - 1, xs = xx + tap % 3 - 1;
            sx[tap][t] = (unsigned)yy < (unsigned)h && (unsigned)xs < (unsigned)w
                             ? ((float)F[yy * w + xs] - offset) * scale : 0.f;
        }
    }
    __syncthreads();
    const int sl = t / C, c = t - sl * C;
    float acc[10] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int j = sl; j < np; j += NS) {
        const float g = ds[(size_t)(p0 + j) * C + c];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) acc[tap] = fmaf(g, sx[tap][j], acc[tap]);
        acc[9] += g;
    }
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) red[sl][c * 9 + tap] = acc[tap];
    red[sl][9 * C + c] = acc[9];
    __syncthreads();
    for (int o = t; o < NO; o += 256) {
        float v = 0.f;
        for (int k = 0; k < NS; ++k) v += red[k][o];
        part[(size_t)blockIdx.x * NO + o] = v;
    }
}

// the sums over nb partials of ma values (into oa) and mb values (into ob) in
// two fixed-order stages; mid holds 32 (ma + mb) floats
void reduce_partials(const float *pa, int ma, float *oa, const float *pbb, int mb, float *ob, int nb, float *mid,
                     hipStream_t s)
{
    const int ng = std::min(32, nb), m = ma + mb;
    hipLaunchKernelGGL(k_sum_partials_grouped, dim3((unsigned)(((int64_t)ng * m + 255) / 256)), dim3(256), 0, s, pa,
                       ma, pbb, mb, nb, ng, mid);
    hipLaunchKernelGGL(k_sum_partials, dim3((m + 255) / 256), dim3(256), 0, s, mid, ng, ma, mb, oa, ob);
}

}  // namespace

hipError_t launch_pack_jobs(const PackJob *jobs, int njobs, int64_t total, const float *params, float *dst,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_jobs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, jobs, njobs, total, params,
                       dst);
    return hipGetLastError();
}

hipError_t launch_mask_slice(const float *src, int scs, int so, const float *m, int mcs, int mo, int nc, int64_t npx,
                             float *dst, int dcs, hipStream_t s)
{
    if (nc % 4) return hipErrorInvalidValue;
    const int64_t n = npx * (nc / 4);
    hipLaunchKernelGGL(k_mask_slice, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, scs, so, m, mcs, mo, nc, npx,
                       dst, dcs);
    return hipGetLastError();
}

hipError_t launch_1x1_back(int C, const float *g, const float *Wt, int ct, int64_t npx, float *out, hipStream_t s)
{
    if (ct % 16) return hipErrorInvalidValue;
    const int64_t groups = (npx + 15) / 16;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((groups + 3) / 4, 4096));
    const size_t lds = (size_t)C * ct * 4;
    if (C == 32)
        hipLaunchKernelGGL(k_1x1_back<32>, dim3(grid), dim3(256), lds, s, g, Wt, ct, npx, out);
    else if (C == 16)
        hipLaunchKernelGGL(k_1x1_back<16>, dim3(grid), dim3(256), lds, s, g, Wt, ct, npx, out);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_pool2_back(const float *a, int acs, const float *g, int gcs, float *out, int ocs, int n, int h, int w,
                             int C, hipStream_t s)
{
    if (C % 4) return hipErrorInvalidValue;
    const int64_t m = (int64_t)n * ((h + 1) / 2) * ((w + 1) / 2) * (C / 4);
    hipLaunchKernelGGL(k_pool2_back, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a, acs, g, gcs, out, ocs, n, h,
                       w, C);
    return hipGetLastError();
}

hipError_t launch_up2_back(const float *g, int gcs, float *out, int ocs, int n, int h, int w, int C, hipStream_t s)
{
    if (C % 4) return hipErrorInvalidValue;
    const int64_t m = (int64_t)n * ((h + 1) / 2) * ((w + 1) / 2) * (C / 4);
    hipLaunchKernelGGL(k_up2_back, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, g, gcs, out, ocs, n, h, w, C);
    return hipGetLastError();
}

hipError_t launch_pack_convs(const float *W0, int64_t src_stride, int count, int C, float *dst, hipStream_t s)
{
    const int64_t n = (int64_t)count * 2 * C * C * 9;
    hipLaunchKernelGGL(k_pack_conv, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W0, src_stride, count, C, dst);
    return hipGetLastError();
}

int64_t train_lse_floats(int h, int w, int ntruth)
{
    const int64_t e = std::max(ntruth, 1);
    return e * (1 + EM_STRIDE + 2 * (int64_t)lse_chunks((int64_t)h * w));
}

hipError_t launch_train_loss(int C, const float *act, const float *hw, const float *hb, int n, int h, int w,
                             const dl_truth *tr, const int32_t *toff, int ntruth, float zs, float ps, float *maps,
                             float *stats, float *lse, float *gm, float *loss, float *term, uint8_t *occ,
                             hipStream_t s)
{
    const int64_t hwpx = (int64_t)h * w, npx = (int64_t)n * hwpx;
    const unsigned gp = (unsigned)((npx + 255) / 256);
    if (C == 32)
        hipLaunchKernelGGL(k_head_fwd<32>, dim3(gp), dim3(256), 0, s, act, hw, hb, npx, hwpx, maps);
    else if (C == 16)
        hipLaunchKernelGGL(k_head_fwd<16>, dim3(gp), dim3(256), 0, s, act, hw, hb, npx, hwpx, maps);
    else
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u8, dim3((unsigned)std::min<int64_t>(gp, 4096)), dim3(256), 0, s, occ, npx);
    if (ntruth > 0)
        hipLaunchKernelGGL(k_occupancy, dim3((ntruth + 255) / 256), dim3(256), 0, s, tr, toff, n, ntruth, h, w, occ);
    hipLaunchKernelGGL(k_pix_terms, dim3(gp), dim3(256), 0, s, maps, n, h, w, term);
    // the stats' partials sit past the pixel terms until the per-frame sums are taken
    float *partial = term + 9 * npx;
    hipLaunchKernelGGL(k_frame_stats, dim3(n * STAT_CHUNKS), dim3(256), 0, s, maps, h, w, occ, partial);
    hipLaunchKernelGGL(k_frame_stats_sum, dim3((n + 255) / 256), dim3(256), 0, s, partial, n, 1e-4f, stats);
    // lse: [ntruth] log-sum-exps, then [ntruth][EM_STRIDE] emitter constants,
    // then [ntruth][chunks][2] partials
    const float izs = 1.f / zs, ips = 1.f / ps;
    float *em = lse + std::max(ntruth, 1);
    float *lpart = em + (size_t)std::max(ntruth, 1) * EM_STRIDE;
    if (ntruth > 0) {
        hipLaunchKernelGGL(k_lse_part, dim3((unsigned)(n * lse_chunks(hwpx))), dim3(256), 0, s, term, n, h, w, tr, toff,
                           izs, ips, lpart);
        hipLaunchKernelGGL(k_lse_fin, dim3((ntruth + 3) / 4), dim3(256), 0, s, n, h, w, tr, toff, ntruth, stats,
                           izs, ips, lpart, lse, em);
    }
    hipLaunchKernelGGL(k_loss_grad, dim3((unsigned)(n * ((hwpx + 255) / 256))), dim3(256), 0, s, maps, term, occ, n,
                       h, w, toff, stats, em, gm);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, n, h, w, toff, ntruth, stats, lse, loss);
    return hipGetLastError();
}

int grad_chunks(int64_t npx) { return (int)((npx + GCHUNK - 1) / GCHUNK); }

hipError_t launch_head_backward(int C, const float *gm, const float *act, const float *hw, int n, int h, int w,
                                float *gwb, float *part, float *mid, float *du, hipStream_t s)
{
    const int64_t hwpx = (int64_t)h * w, npx = (int64_t)n * hwpx;
    const int nb = grad_chunks(npx);
    if (C == 32) {
        hipLaunchKernelGGL(k_head_grad_part<32>, dim3(nb), dim3(256), 0, s, gm, act, (int)npx, (int)hwpx, part);
        hipLaunchKernelGGL(k_head_back<32>, dim3((unsigned)((npx * 8 + 255) / 256)), dim3(256), 0, s, gm, hw, act,
                           (int)npx, (int)hwpx, du);
    } else if (C == 16) {
        hipLaunchKernelGGL(k_head_grad_part<16>, dim3(nb), dim3(256), 0, s, gm, act, (int)npx, (int)hwpx, part);
        hipLaunchKernelGGL(k_head_back<16>, dim3((unsigned)((npx * 4 + 255) / 256)), dim3(256), 0, s, gm, hw, act,
                           (int)npx, (int)hwpx, du);
    } else {
        return hipErrorInvalidValue;
    }
    reduce_partials(part, 10 * C + 10, gwb, nullptr, 0, nullptr, nb, mid, s);   // head.w then head.b, as in the blob
    return hipGetLastError();
}

// rows per workgroup: WG_WAVES waves of rpw rows each, rpw the smallest that
// keeps the batch within 2048 waves (two per SIMD with the 9 x 16 accumulator
// registers of C = 32); the weight gradient runs at most ceil(n h / this)
// workgroups, which sizes its partial buffers
int wgrad_rows_per_block(int n, int h) { return WG_WAVES * std::max(1, (n * h + 2047) / 2048); }

hipError_t launch_wgrad_ex(int CO, int taps, const float *dy, int dcs, const float *x, int xcs, int CI, int n, int h,
                           int w, int d, float *part, float *pb, float *tmp, float *gW, float *gb, hipStream_t s)
{
    if (!(CO == 16 || CO == 32) || !(taps == 1 || taps == 9) || CI < CO || CI % CO || d < 1) return hipErrorInvalidValue;
    // the kernel's chains (see k_wgrad); their waves are spread over at most
    // the workgroups the partial buffer was sized for
    const int K = taps == 9 ? 4 : 1, de = taps == 9 ? d : 1;
    const int64_t nch = (int64_t)n * ((h + K * de - 1) / (K * de)) * std::min(de, h);
    // column segments: enough units for about 2048 waves
    const int steps = (w + 64 / CO - 1) / (64 / CO);
    int nseg = (int)std::min<int64_t>(steps, std::max<int64_t>(1, (2048 + nch - 1) / nch));
    const int sps = (steps + nseg - 1) / nseg;
    nseg = (steps + sps - 1) / sps;
    const int64_t nun = nch * nseg;
    const int R = wgrad_rows_per_block(n, h);
    const int64_t nblk_max = ((int64_t)n * h + R - 1) / R;
    const int cpw = (int)std::max<int64_t>({1, (nun + 2047) / 2048, (nun + WG_WAVES * nblk_max - 1) / (WG_WAVES * nblk_max)});
    const dim3 grid((unsigned)((nun + (int64_t)WG_WAVES * cpw - 1) / ((int64_t)WG_WAVES * cpw)), CI / CO);
    if (CO == 32 && taps == 9)
        hipLaunchKernelGGL((k_wgrad<32, 9>), grid, dim3(64 * WG_WAVES), 0, s, dy, dcs, x, xcs, CI, n, h, w, d, nseg,
                           sps, cpw, part, pb);
    else if (CO == 32)
        hipLaunchKernelGGL((k_wgrad<32, 1>), grid, dim3(64 * WG_WAVES), 0, s, dy, dcs, x, xcs, CI, n, h, w, d, nseg,
                           sps, cpw, part, pb);
    else if (taps == 9)
        hipLaunchKernelGGL((k_wgrad<16, 9>), grid, dim3(64 * WG_WAVES), 0, s, dy, dcs, x, xcs, CI, n, h, w, d, nseg,
                           sps, cpw, part, pb);
    else
        hipLaunchKernelGGL((k_wgrad<16, 1>), grid, dim3(64 * WG_WAVES), 0, s, dy, dcs, x, xcs, CI, n, h, w, d, nseg,
                           sps, cpw, part, pb);
    reduce_partials(part, CO * CI * taps, gW, pb, CO, gb, (int)grid.x, tmp, s);
    return hipGetLastError();
}

hipError_t launch_wgrad(int C, const float *dy, const float *x, int n, int h, int w, int d, float *part, float *pb,
                        float *tmp, float *gW, float *gb, hipStream_t s)
{
    return launch_wgrad_ex(C, 9, dy, C, x, C, C, n, h, w, d, part, pb, tmp, gW, gb, s);
}

hipError_t launch_stem_grad(const float *ds, const uint16_t *frames, int n, int h, int w, float offset, float scale,
                            int C, float *gwb, float *part, float *mid, hipStream_t s)
{
    const int nb = grad_chunks((int64_t)n * h * w);
    if (C == 32)
        hipLaunchKernelGGL(k_stem_grad_part<32>, dim3(nb), dim3(256), 0, s, ds, frames, n, h, w, offset, scale, part);
    else if (C == 16)
        hipLaunchKernelGGL(k_stem_grad_part<16>, dim3(nb), dim3(256), 0, s, ds, frames, n, h, w, offset, scale, part);
    else
        return hipErrorInvalidValue;
    reduce_partials(part, 10 * C, gwb, nullptr, 0, nullptr, nb, mid, s);   // stem.w then stem.b, as in the blob
    return hipGetLastError();
}

}  // namespace dloc
