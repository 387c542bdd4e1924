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
//   k_loc_lse       per true emitter: log-sum-exp over its frame's pixels of
//                   q_k = log p_k - log mu + sum_d log N(t_d; m_kd, s_kd^2), one
//                   pass with a running maximum
//   k_loss_grad     per pixel: d loss / d maps (10 planes)
//   k_loss_total    the batch means of the loss terms
//   k_head_grad_part head weight and bias gradient partials per pixel chunk
//   k_head_back     d loss / d (last block's pre-activation)
//   k_wgrad         3x3 weight gradient partial sums per workgroup on MFMA:
//                   dW[co][ci][tap] = sum_p dy[p][co] x[p + off(tap)][ci]
//   k_sum_partials  fixed-order sums of per-workgroup partials
//   k_stem_grad_part stem weight and bias gradient partials per pixel chunk
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

// dst[(((g 9 + t) NB + nb) 64 + lane) 4 + s] = Wp[16 nb + (lane & 15)][16 g + 4 (lane >> 4) + s][t]
// with Wp = W [cout][cin][9], or (flip) Wp[o][c][t] = W[c][o][8 - t]
__global__ void __launch_bounds__(256)
k_pack_conv(const float *__restrict__ W, int cout, int cin, int flip, float *__restrict__ dst)
{
    const int n = cout * cin * 9;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int NB = cout / 16;
    const int s = i & 3, lane = (i >> 2) & 63;
    const int rest = i >> 8;                 // ((g 9 + t) NB + nb)
    const int nb = rest % NB, gt = rest / NB;
    const int t = gt % 9, g = gt / 9;
    const int o = nb * 16 + (lane & 15), c = g * 16 + 4 * (lane >> 4) + s;
    dst[i] = flip ? W[((size_t)c * cout + o) * 9 + (8 - t)] : W[((size_t)o * cin + c) * 9 + t];
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
// term[5 + d] = 1 / s_d (d = x, y, z, N in the units of the targets)
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
        const float sd = softplusf(M[(5 + d) * P + k]);
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

// q of emitter target tv at pixel i, from the pixel terms (without -log mu)
__device__ __forceinline__ float mix_q(const float *__restrict__ term, int64_t np, int64_t i, const float (&tv)[4])
{
    float q = term[i], z2 = 0.f;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const float z = (tv[d] - term[(1 + d) * np + i]) * term[(5 + d) * np + i];
        z2 += z * z;
    }
    return q - 0.5f * z2;
}

// lse[e] = log sum_k exp(q_ek) - log mu over emitter e's frame, one pass with
// a running maximum per thread, then (max, sum) pairs combined in a fixed order
__global__ void __launch_bounds__(256)
k_loc_lse(const float *__restrict__ term, int n, int h, int w, const dl_truth *__restrict__ tr,
          const int32_t *__restrict__ toff, const float *__restrict__ stats, float zs, float ps, float *__restrict__ lse)
{
    __shared__ float smx[256], ssm[256];
    const int e = blockIdx.x;
    const int f = find_frame_off(toff, n, e);
    const int64_t P = (int64_t)h * w, np = (int64_t)n * P, base = (int64_t)f * P;
    const dl_truth t = tr[e];
    const float tv[4] = {t.x, t.y, t.z_nm / zs, t.photons / ps};
    float mx = -INFINITY, sm = 0.f;
    for (int64_t k = threadIdx.x; k < P; k += 256) {
        const float q = mix_q(term, np, base + k, tv);
        if (q > mx) {
            sm = sm * expf(mx - q) + 1.f;
            mx = q;
        } else {
            sm += expf(q - mx);
        }
    }
    const int tid = threadIdx.x;
    smx[tid] = mx;
    ssm[tid] = sm;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            const float m1 = smx[tid], m2 = smx[tid + o];
            const float m = fmaxf(m1, m2);
            ssm[tid] = (m1 == -INFINITY ? 0.f : ssm[tid] * expf(m1 - m)) + (m2 == -INFINITY ? 0.f : ssm[tid + o] * expf(m2 - m));
            smx[tid] = m;
        }
        __syncthreads();
    }
    if (tid == 0) lse[e] = smx[0] + logf(ssm[0]) - logf(stats[3 * f]);
}

// d (batch mean loss) / d maps, one thread per pixel of the batch
__global__ void __launch_bounds__(256)
k_loss_grad(const float *__restrict__ maps, const float *__restrict__ term, const uint8_t *__restrict__ occ, int n,
            int h, int w, const dl_truth *__restrict__ tr, const int32_t *__restrict__ toff,
            const float *__restrict__ stats, const float *__restrict__ lse, float zs, float ps, float *__restrict__ gm)
{
    const int64_t P = (int64_t)h * w, np = (int64_t)n * P;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= np) return;
    const int f = (int)(i / P);
    const int64_t k = i - (int64_t)f * P;
    const float *M = maps + (int64_t)f * 10 * P;
    float *G = gm + (int64_t)f * 10 * P;
    const float inv_n = 1.f / (float)n;
    const int e0 = toff[f], e1 = toff[f + 1];
    const float E = (float)(e1 - e0);
    const float mu = stats[3 * f], v = stats[3 * f + 1];
    const float l = M[k], p = sigmoidf(l), pq = p * (1.f - p);
    // cross-entropy and count
    float gl = (p - (occ[i] ? 1.f : 0.f)) / (float)P;
    const float dmu = -(E - mu) / v, dv = 0.5f / v - (E - mu) * (E - mu) / (2.f * v * v);
    gl += pq * (dmu + (1.f - 2.f * p) * dv);
    // localisation: this pixel's responsibility for each emitter of its frame
    float g[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float mv[4], is[4], sg[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        mv[d] = term[(1 + d) * np + i];
        is[d] = term[(5 + d) * np + i];
        sg[d] = sigmoidf(M[(5 + d) * P + k]);
    }
    const float logmu = logf(mu);
    for (int e = e0; e < e1; ++e) {
        const dl_truth t = tr[e];
        const float tv[4] = {t.x, t.y, t.z_nm / zs, t.photons / ps};
        const float r = expf(mix_q(term, np, i, tv) - logmu - lse[e]);
        gl += -r * (1.f - p) + pq / mu;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const float dm = tv[d] - mv[d], z = dm * is[d];
            g[d] += -r * dm * is[d] * is[d];
            g[4 + d] += -r * (z * z - 1.f) * is[d] * sg[d];
        }
    }
    G[k] = gl * inv_n;
#pragma unroll
    for (int d = 0; d < 8; ++d) G[(1 + d) * P + k] = g[d] * inv_n;
    G[9 * P + k] = 0.f;
}

// loss[4] = batch means of {total, bce, count, loc}
__global__ void __launch_bounds__(256)
k_loss_total(int n, int h, int w, const int32_t *__restrict__ toff, const float *__restrict__ stats,
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
        for (int e = toff[f]; e < toff[f + 1]; ++e) l -= lse[e];
    }
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

// head gradient partials: workgroup b sums over pixels [b GCHUNK, b GCHUNK + GCHUNK);
// part[b][q C + c] = sum gm[q][p] a[p][c], part[b][10 C + q] = sum gm[q][p]
template <int C>
__global__ void __launch_bounds__(256)
k_head_grad_part(const float *__restrict__ gm, const float *__restrict__ act, int64_t npx, int64_t hwpx,
                 float *__restrict__ part)
{
    const int t = threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.x * GCHUNK, p1 = min(npx, p0 + GCHUNK);
    float *P = part + (size_t)blockIdx.x * (10 * C + 10);
    for (int o = t; o < 10 * (C + 1); o += 256) {
        const int q = o / (C + 1), c = o - q * (C + 1);
        float s = 0.f;
        for (int64_t p = p0; p < p1; ++p) {
            const int64_t f = p / hwpx, k = p - f * hwpx;
            const float g = gm[(f * 10 + q) * hwpx + k];
            s += c < C ? g * act[p * C + c] : g;
        }
        if (c < C) P[q * C + c] = s;
        else P[10 * C + q] = s;
    }
}

// du[p][c] = (sum_q W[q][c] gm[q][p]) where a[p][c] > 0, else 0
template <int C>
__global__ void __launch_bounds__(256)
k_head_back(const float *__restrict__ gm, const float *__restrict__ hw, const float *__restrict__ act, int64_t npx,
            int64_t hwpx, float *__restrict__ du)
{
    __shared__ float sw[10 * C];
    for (int i = threadIdx.x; i < 10 * C; i += 256) sw[i] = hw[i];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= npx) return;
    const int64_t f = p / hwpx, k = p - f * hwpx;
    float g[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) g[q] = gm[(f * 10 + q) * hwpx + k];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 10; ++q) s += sw[q * C + c] * g[q];
        du[p * C + c] = act[p * C + c] > 0.f ? s : 0.f;
    }
}

// Weight gradient of a 3x3 conv at dilation d over NHWC tensors of C floats
// per point (C = 16 CB): workgroup b takes rows [b R, b R + R) of the batch
// (a frame's rows are consecutive), wave w the (co block, ci block) pair
// w % (CB CB) for all 9 taps; v_mfma_f32_16x16x4_f32 with K = 4 pixels:
// lane (i, kq) gives dy[pixel kq][co 16 cb + i] and x[pixel kq + off][ci 16 cb2 + i].
// part[b][tap][co][ci] (+ part of the bias: pb[b][co]).
template <int CB>
__global__ void __launch_bounds__(256)
k_wgrad(const float *__restrict__ dy, const float *__restrict__ x, int n, int h, int w, int d, int R,
        float *__restrict__ part, float *__restrict__ pb)
{
    constexpr int C = 16 * CB;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kq = lane >> 4;
    const int64_t rows = (int64_t)n * h;
    const int64_t r0 = (int64_t)blockIdx.x * R, r1 = std::min<int64_t>(rows, r0 + R);
    float *P = part + (size_t)blockIdx.x * 9 * C * C;
    for (int pair = wave; pair < CB * CB; pair += 4) {
        const int cb = pair / CB, cb2 = pair % CB;
        v4f acc[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
        float bsum = 0.f;
        for (int64_t gr = r0; gr < r1; ++gr) {
            const int f = (int)(gr / h), y = (int)(gr - (int64_t)f * h);
            const int64_t base = (int64_t)f * h * w;
            for (int x0 = 0; x0 < w; x0 += 4) {
                const int xx = x0 + kq;
                const bool in = xx < w;
                const float a = in ? dy[(base + (int64_t)y * w + xx) * C + 16 * cb + i] : 0.f;
                bsum += a;
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const int ys = y + d * (t / 3 - 1), xs = xx + d * (t % 3 - 1);
                    const bool ok = in && (unsigned)ys < (unsigned)h && (unsigned)xs < (unsigned)w;
                    const float b = ok ? x[(base + (int64_t)ys * w + xs) * C + 16 * cb2 + i] : 0.f;
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
                }
            }
        }
        // lane (j, kq) holds D[co 4 kq + r][ci j]
#pragma unroll
        for (int t = 0; t < 9; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int co = 16 * cb + 4 * kq + r, ci = 16 * cb2 + i;
                P[((size_t)t * C + co) * C + ci] = acc[t][r];
            }
        if (cb2 == 0) {
            // the bias: each lane summed dy of channel 16 cb + i over its pixels kq
            bsum += __shfl_xor(bsum, 16);
            bsum += __shfl_xor(bsum, 32);
            if (kq == 0) pb[(size_t)blockIdx.x * C + 16 * cb + i] = bsum;
        }
    }
}

// out[j] = sum_b part[b][j] (b in order), j < m
__global__ void __launch_bounds__(256)
k_sum_partials(const float *__restrict__ part, int nb, int m, float *__restrict__ out)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * m + j];
    out[j] = s;
}

// first stage of the same sum for many partials: out[g][j] = sum over
// b in [g G, g G + G) of part[b][j], G = ceil(nb / ng)
__global__ void __launch_bounds__(256)
k_sum_partials_grouped(const float *__restrict__ part, int nb, int m, int ng, float *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)ng * m) return;
    const int g = (int)(idx / m), j = (int)(idx - (int64_t)g * m);
    const int G = (nb + ng - 1) / ng;
    const int b0 = g * G, b1 = min(nb, b0 + G);
    float s = 0.f;
    for (int b = b0; b < b1; ++b) s += part[(size_t)b * m + j];
    out[idx] = s;
}

// dW[co][ci][tap] <- part sums laid out [tap][co][ci]
__global__ void __launch_bounds__(256)
k_wgrad_layout(const float *__restrict__ t_co_ci, int C, float *__restrict__ W)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= 9 * C * C) return;
    const int t = j % 9, rest = j / 9, ci = rest % C, co = rest / C;
    W[j] = t_co_ci[((size_t)t * C + co) * C + ci];
}

// stem gradient partials over pixels [b GCHUNK, b GCHUNK + GCHUNK):
// part[b][c 9 + tap] = sum ds[p][c] x(p + off(tap)), part[b][9 C + c] = sum ds[p][c]
__global__ void __launch_bounds__(256)
k_stem_grad_part(const float *__restrict__ ds, const uint16_t *__restrict__ frames, int n, int h, int w,
                 float offset, float scale, int C, float *__restrict__ part)
{
    const int64_t hw = (int64_t)h * w, P = (int64_t)n * hw;
    const int64_t p0 = (int64_t)blockIdx.x * GCHUNK, p1 = min(P, p0 + GCHUNK);
    float *O = part + (size_t)blockIdx.x * 10 * C;
    for (int o = threadIdx.x; o < 10 * C; o += 256) {
        const int c = o % C, t = o / C;             // consecutive threads: consecutive channels
        float s = 0.f;
        for (int64_t p = p0; p < p1; ++p) {
            const float g = ds[p * C + c];
            if (t == 9) {
                s += g;
                continue;
            }
            const int64_t f = p / hw, k = p - f * hw;
            const int y = (int)(k / w) + t / 3 - 1, xx = (int)(k % w) + t % 3 - 1;
            if ((unsigned)y < (unsigned)h && (unsigned)xx < (unsigned)w)
                s += g * (((float)frames[(f * h + y) * w + xx] - offset) * scale);
        }
        if (t < 9) O[c * 9 + t] = s;
        else O[9 * C + c] = s;
    }
}

// the sum over nb partials of m values in two fixed-order stages (groups, then
// the groups' sums); mid holds 32 m floats
void reduce_partials(const float *part, int nb, int m, float *mid, float *out, hipStream_t s)
{
    const int ng = std::min(32, nb);
    hipLaunchKernelGGL(k_sum_partials_grouped, dim3((unsigned)(((int64_t)ng * m + 255) / 256)), dim3(256), 0, s, part,
                       nb, m, ng, mid);
    hipLaunchKernelGGL(k_sum_partials, dim3((m + 255) / 256), dim3(256), 0, s, mid, ng, m, out);
}

}  // namespace

hipError_t launch_pack_conv(const float *W, int cout, int cin, int flip, float *dst, hipStream_t s)
{
    const int n = cout * cin * 9;
    hipLaunchKernelGGL(k_pack_conv, dim3((n + 255) / 256), dim3(256), 0, s, W, cout, cin, flip, dst);
    return hipGetLastError();
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
    // the stats' partials sit in lse's place until the per-frame sums are taken
    float *partial = term + 9 * npx;
    hipLaunchKernelGGL(k_frame_stats, dim3(n * STAT_CHUNKS), dim3(256), 0, s, maps, h, w, occ, partial);
    hipLaunchKernelGGL(k_frame_stats_sum, dim3((n + 255) / 256), dim3(256), 0, s, partial, n, 1e-4f, stats);
    if (ntruth > 0)
        hipLaunchKernelGGL(k_loc_lse, dim3(ntruth), dim3(256), 0, s, term, n, h, w, tr, toff, stats, zs, ps, lse);
    hipLaunchKernelGGL(k_loss_grad, dim3(gp), dim3(256), 0, s, maps, term, occ, n, h, w, tr, toff, stats, lse, zs, ps,
                       gm);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(256), 0, s, n, h, w, toff, stats, lse, loss);
    return hipGetLastError();
}

int grad_chunks(int64_t npx) { return (int)((npx + GCHUNK - 1) / GCHUNK); }

hipError_t launch_head_backward(int C, const float *gm, const float *act, const float *hw, int n, int h, int w,
                                float *gwb, float *part, float *mid, float *du, hipStream_t s)
{
    const int64_t hwpx = (int64_t)h * w, npx = (int64_t)n * hwpx;
    const unsigned gp = (unsigned)((npx + 255) / 256);
    const int nb = grad_chunks(npx);
    if (C == 32) {
        hipLaunchKernelGGL(k_head_grad_part<32>, dim3(nb), dim3(256), 0, s, gm, act, npx, hwpx, part);
        hipLaunchKernelGGL(k_head_back<32>, dim3(gp), dim3(256), 0, s, gm, hw, act, npx, hwpx, du);
    } else if (C == 16) {
        hipLaunchKernelGGL(k_head_grad_part<16>, dim3(nb), dim3(256), 0, s, gm, act, npx, hwpx, part);
        hipLaunchKernelGGL(k_head_back<16>, dim3(gp), dim3(256), 0, s, gm, hw, act, npx, hwpx, du);
    } else {
        return hipErrorInvalidValue;
    }
    reduce_partials(part, nb, 10 * C + 10, mid, gwb, s);   // head.w then head.b, as in the blob
    return hipGetLastError();
}

// about 1024 workgroups: four waves each, so enough waves per SIMD to hide the
// operand loads' latency
int wgrad_rows_per_block(int n, int h) { return std::max(1, (n * h + 1023) / 1024); }

hipError_t launch_wgrad(int C, const float *dy, const float *x, int n, int h, int w, int d, float *part, float *pb,
                        float *tmp, float *gW, float *gb, hipStream_t s)
{
    const int R = wgrad_rows_per_block(n, h);
    const int nblk = (n * h + R - 1) / R;
    if (C == 32)
        hipLaunchKernelGGL(k_wgrad<2>, dim3(nblk), dim3(256), 0, s, dy, x, n, h, w, d, R, part, pb);
    else if (C == 16)
        hipLaunchKernelGGL(k_wgrad<1>, dim3(nblk), dim3(256), 0, s, dy, x, n, h, w, d, R, part, pb);
    else
        return hipErrorInvalidValue;
    const int m = 9 * C * C;
    float *mid = tmp + m;
    reduce_partials(part, nblk, m, mid, tmp, s);
    hipLaunchKernelGGL(k_wgrad_layout, dim3((m + 255) / 256), dim3(256), 0, s, tmp, C, gW);
    reduce_partials(pb, nblk, C, mid, gb, s);
    return hipGetLastError();
}

hipError_t launch_stem_grad(const float *ds, const uint16_t *frames, int n, int h, int w, float offset, float scale,
                            int C, float *gwb, float *part, float *mid, hipStream_t s)
{
    const int nb = grad_chunks((int64_t)n * h * w);
    hipLaunchKernelGGL(k_stem_grad_part, dim3(nb), dim3(256), 0, s, ds, frames, n, h, w, offset, scale, C, part);
    reduce_partials(part, nb, 10 * C, mid, gwb, s);           // stem.w then stem.b, as in the blob
    return hipGetLastError();
}

}  // namespace dloc
