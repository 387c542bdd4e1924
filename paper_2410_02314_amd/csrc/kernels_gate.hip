// Tile-occupancy gate: inference and training kernels (FP32, VALU + LDS).
//
// Per 256 x 256 tile of preprocessed input x:
//   p  = mean of 4x4 blocks of x                  (64 x 64)
//   z1 = conv3x3(p; W1, b1), pad 1, 1 -> 8;   h1 = ReLU(z1)
//   z2 = conv3x3(h1; W2, b2), pad 1, 8 -> 8;  h2 = ReLU(z2)
//   m  = max over pixels of h2 (8);           g  = fw . m + fb   (logit)
// The global pool is a max (a single emitter-like spot decides that a tile is
// occupied); its gradient goes to the first pixel in raster order that
// attains the max.  Training loss is binary cross-entropy on g (paper
// Sec. 3.3), so dL/dg = (sigmoid(g) - y) / batch.  Parameters theta[673] in
// the order W1[8][1][3][3], b1[8], W2[8][8][3][3], b2[8], fw[8], fb[1].
//
// One workgroup per tile keeps p (padded 66 x 66) and h1 (8 x 64 x 64) in LDS
// (~150 KB).  Backward: dz2[o] is k[o] = dg fw[o] [m[o] > 0] at the argmax
// a[o] and zero elsewhere, so dW2[o][c][tap] = k[o] h1[c][a[o] + tap], and dz1
// (written over h1 in place) is nonzero only around the eight argmaxes.  Every
// reduction has a fixed order (shuffle butterflies, fixed per-thread loops,
// per-tile partial gradients summed tile by tile), so gradients are bitwise
// reproducible.
#include "dloc_internal.h"

namespace dloc {

namespace {

constexpr int GT = 256;          // gate tile side (input pixels)
constexpr int GPOOL = 4;
constexpr int GP = GT / GPOOL;   // 64: pooled side
constexpr int GPP = GP + 2;      // padded pooled side
constexpr int GC = 8;
constexpr int NPARAM = 673;
constexpr int NPIX = GP * GP;    // 4096

__device__ __forceinline__ float wave_sum(float v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// --------------------------------------------------------------- pooling
// grid: one workgroup per tile (frame-major, then tile row, tile column).
__global__ void __launch_bounds__(256)
k_gate_pool(const uint16_t *__restrict__ frames, int n, int h, int w, float offset, float scale,
            const float2 *__restrict__ cam, float *__restrict__ pooled)
{
    const int tiles_x = w / GT, tiles_y = h / GT;
    const int tile = blockIdx.x;
    const int f = tile / (tiles_x * tiles_y);
    const int r = tile - f * tiles_x * tiles_y;
    const int ty = r / tiles_x, tx = r - (r / tiles_x) * tiles_x;
    const uint16_t *src = frames + (int64_t)f * h * w + (int64_t)(ty * GT) * w + tx * GT;
    float *dst = pooled + (int64_t)tile * NPIX;
    for (int q = threadIdx.x; q < NPIX; q += 256) {
        const int i = q / GP, j = q - (q / GP) * GP;
        float s = 0.f;
#pragma unroll
        for (int u = 0; u < GPOOL; ++u)
#pragma unroll
            for (int v = 0; v < GPOOL; ++v) {
                const int64_t q2 = (int64_t)(i * GPOOL + u) * w + j * GPOOL + v;
                const float adu = (float)src[q2];
                if (cam) {               // sCMOS: this pixel's offset and gain
                    const float2 cm = cam[(int64_t)(ty * GT) * w + tx * GT + q2];
                    s += (adu - cm.x) * cm.y;
                } else {
                    s += (adu - offset) * scale;
                }
            }
        dst[q] = s * (1.f / (GPOOL * GPOOL));
    }
}

struct GateSmem {
    float P[GPP * GPP];           // padded pooled tile
    float H1[GC * NPIX];          // h1, later dz1
    float th[NPARAM + 3];
    float red[GC * 4];            // per-wave maxima
    int redi[GC * 4];             // and where they are
    float m[GC];
    int am[GC];                   // argmax of each channel (first in raster order)
};

// (value, index) pairs: the larger value wins, a tie goes to the smaller index
__device__ __forceinline__ void max_first(float &v, int &i, float v2, int i2)
{
    if (v2 > v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
    }
}

// Forward (and backward when BWD): logits[tile]; gpart[tile][673] holds the
// tile's gradient of dlogit[tile] * g with respect to theta.
template <bool BWD>
__global__ void __launch_bounds__(256)
k_gate(const float *__restrict__ pooled, int ntiles, const float *__restrict__ theta,
       float *__restrict__ logits, const float *__restrict__ dlogits, float *__restrict__ gpart)
{
    extern __shared__ float4 gsm_raw[];
    GateSmem &S = *reinterpret_cast<GateSmem *>(gsm_raw);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = blockIdx.x;
    for (int k = tid; k < NPARAM; k += 256) S.th[k] = theta[k];
    const float *src = pooled + (int64_t)tile * NPIX;
    for (int q = tid; q < GPP * GPP; q += 256) {
        const int i = q / GPP - 1, j = q - (q / GPP) * GPP - 1;
        S.P[q] = (i >= 0 && i < GP && j >= 0 && j < GP) ? src[i * GP + j] : 0.f;
    }
    __syncthreads();
    const float *W1 = S.th, *B1 = S.th + 72, *W2 = S.th + 80, *B2 = S.th + 656, *FW = S.th + 664;
    const float FB = S.th[672];

    // conv1 + ReLU
    for (int q = tid; q < NPIX; q += 256) {
        const int i = q / GP, j = q - (q / GP) * GP;
        float pv[9];
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
            for (int v = 0; v < 3; ++v) pv[u * 3 + v] = S.P[(i + u) * GPP + j + v];
#pragma unroll
        for (int o = 0; o < GC; ++o) {
            float z = B1[o];
#pragma unroll
            for (int t = 0; t < 9; ++t) z += W1[o * 9 + t] * pv[t];
            S.H1[o * NPIX + q] = fmaxf(z, 0.f);
        }
    }
    __syncthreads();

    // conv2 + ReLU, channel maxima of h2 and their first positions
    float mv[GC];
    int mi[GC];
#pragma unroll
    for (int o = 0; o < GC; ++o) {
        mv[o] = -1.f;                 // below every ReLU output: the first pixel always enters
        mi[o] = 0;
    }
    for (int k = 0; k < NPIX / 256; ++k) {
        const int q = tid + 256 * k;
        const int i = q / GP, j = q - (q / GP) * GP;
        float z[GC];
#pragma unroll
        for (int o = 0; o < GC; ++o) z[o] = B2[o];
        for (int c = 0; c < GC; ++c) {
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const int ii = i + u - 1;
                if (ii < 0 || ii >= GP) continue;
#pragma unroll
                for (int v = 0; v < 3; ++v) {
                    const int jj = j + v - 1;
                    if (jj < 0 || jj >= GP) continue;
                    const float hv = S.H1[c * NPIX + ii * GP + jj];
#pragma unroll
                    for (int o = 0; o < GC; ++o) z[o] += W2[(o * GC + c) * 9 + u * 3 + v] * hv;
                }
            }
        }
#pragma unroll
        for (int o = 0; o < GC; ++o) {
            const float h = fmaxf(z[o], 0.f);
            if (h > mv[o]) {          // q grows with k: the first maximum is kept
                mv[o] = h;
                mi[o] = q;
            }
        }
    }
#pragma unroll
    for (int o = 0; o < GC; ++o) {
        float v = mv[o];
        int ix = mi[o];
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) max_first(v, ix, __shfl_xor(v, sh), __shfl_xor(ix, sh));
        if (lane == 0) {
            S.red[o * 4 + wave] = v;
            S.redi[o * 4 + wave] = ix;
        }
    }
    __syncthreads();
    if (tid < GC) {
        float v = S.red[tid * 4];
        int ix = S.redi[tid * 4];
        for (int w = 1; w < 4; ++w) max_first(v, ix, S.red[tid * 4 + w], S.redi[tid * 4 + w]);
        S.m[tid] = v;
        S.am[tid] = ix;
    }
    __syncthreads();
    if (tid == 0) {
        float g = FB;
        for (int o = 0; o < GC; ++o) g += FW[o] * S.m[o];
        logits[tile] = g;
    }
    if (!BWD) return;

    // ----------------------------------------------------------- backward
    // k[o] = dg fw[o] where z2 > 0 at the argmax (m[o] > 0), else 0
    const float dg = dlogits[tile];
    float *gp = gpart + (int64_t)tile * NPARAM;
    if (tid < GC) {
        gp[664 + tid] = dg * S.m[tid];
        gp[656 + tid] = S.m[tid] > 0.f ? dg * FW[tid] : 0.f;
    }
    if (tid == 0) gp[672] = dg;
    // dW2[o][c][tap] = k[o] h1[c][a[o] + tap] (zero outside the tile)
    for (int e = tid; e < GC * GC * 9; e += 256) {
        const int o = e / (GC * 9), c = (e / 9) % GC, t = e % 9;
        const int ai = S.am[o] / GP, aj = S.am[o] % GP;
        const int ii = ai + t / 3 - 1, jj = aj + t % 3 - 1;
        const float ko = S.m[o] > 0.f ? dg * FW[o] : 0.f;
        const float hv = ii >= 0 && ii < GP && jj >= 0 && jj < GP ? S.H1[c * NPIX + ii * GP + jj] : 0.f;
        gp[80 + e] = ko * hv;
    }
    __syncthreads();
    // dz1[c][q] = [h1 > 0] sum_o k[o] W2[o][c][q - a[o] + 1], in place over h1
    for (int q = tid; q < NPIX; q += 256) {
        const int i = q / GP, j = q - (q / GP) * GP;
        float dh[GC];
#pragma unroll
        for (int c = 0; c < GC; ++c) dh[c] = 0.f;
        for (int o = 0; o < GC; ++o) {
            const int u = i - S.am[o] / GP + 1, v = j - S.am[o] % GP + 1;
            if (u < 0 || u > 2 || v < 0 || v > 2 || !(S.m[o] > 0.f)) continue;
            const float ko = dg * FW[o];
#pragma unroll
            for (int c = 0; c < GC; ++c) dh[c] += ko * W2[(o * GC + c) * 9 + u * 3 + v];
        }
#pragma unroll
        for (int c = 0; c < GC; ++c) {
            const float hv = S.H1[c * NPIX + q];
            S.H1[c * NPIX + q] = hv > 0.f ? dh[c] : 0.f;
        }
    }
    __syncthreads();
    // dW1[o][tap] = sum_q dz1[o][q] p[q + tap], db1[o] = sum_q dz1[o][q]
    {
        const int o = tid >> 5, sl = tid & 31;
        float s[10];
#pragma unroll
        for (int t = 0; t < 10; ++t) s[t] = 0.f;
        for (int q = sl; q < NPIX; q += 32) {
            const float dz = S.H1[o * NPIX + q];
            const int i = q / GP, j = q - (q / GP) * GP;
#pragma unroll
            for (int u = 0; u < 3; ++u)
#pragma unroll
                for (int v = 0; v < 3; ++v) s[u * 3 + v] += dz * S.P[(i + u) * GPP + j + v];
            s[9] += dz;
        }
#pragma unroll
        for (int t = 0; t < 10; ++t) {
            float v = s[t];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            v += __shfl_xor(v, 8);
            v += __shfl_xor(v, 16);
            if (sl == 0) {
                if (t < 9) gp[o * 9 + t] = v;
                else gp[72 + o] = v;
            }
        }
    }
}

// sum of per-tile partial gradients in tile order (deterministic)
__global__ void __launch_bounds__(256)
k_gate_reduce(const float *__restrict__ gpart, int ntiles, float *__restrict__ grad)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= NPARAM) return;
    float s = 0.f;
    for (int t = 0; t < ntiles; ++t) s += gpart[(int64_t)t * NPARAM + k];
    grad[k] = s;
}

// BCE with logits, mean over n: loss and dL/dg (single workgroup, fixed order)
__global__ void __launch_bounds__(1024)
k_gate_bce(const float *__restrict__ g, const float *__restrict__ y, int n, float *__restrict__ loss,
           float *__restrict__ dg)
{
    __shared__ float sh[16];
    const int tid = threadIdx.x;
    float s = 0.f;
    for (int b = tid; b < n; b += 1024) {
        const float gb = g[b], yb = y[b];
        s += fmaxf(gb, 0.f) - gb * yb + log1pf(expf(-fabsf(gb)));
        if (dg) dg[b] = (1.f / (1.f + expf(-gb)) - yb) / (float)n;
    }
    s = wave_sum(s);
    if ((tid & 63) == 0) sh[tid >> 6] = s;
    __syncthreads();
    if (tid == 0 && loss) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += sh[k];
        *loss = t / (float)n;
    }
}

__global__ void __launch_bounds__(256)
k_adam(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v, const float *__restrict__ grad,
       int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const float gk = grad[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    theta[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

}  // namespace

size_t gate_smem_bytes() { return sizeof(GateSmem); }

hipError_t launch_gate_pool(const uint16_t *frames, int n, int h, int w, float offset, float scale,
                            const float2 *cam, float *pooled, hipStream_t s)
{
    const int nt = n * (h / GT) * (w / GT);
    hipLaunchKernelGGL(k_gate_pool, dim3(nt), dim3(256), 0, s, frames, n, h, w, offset, scale, cam, pooled);
    return hipGetLastError();
}

hipError_t launch_gate(const float *pooled, int ntiles, const float *theta, float *logits,
                       const float *dlogits, float *gpart, hipStream_t s)
{
    const size_t sh = sizeof(GateSmem);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_gate<false>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_gate<true>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
        if (e != hipSuccess) return e;
        attr = true;
    }
    if (dlogits)
        hipLaunchKernelGGL(k_gate<true>, dim3(ntiles), dim3(256), sh, s, pooled, ntiles, theta, logits, dlogits, gpart);
    else
        hipLaunchKernelGGL(k_gate<false>, dim3(ntiles), dim3(256), sh, s, pooled, ntiles, theta, logits, dlogits, gpart);
    return hipGetLastError();
}

hipError_t launch_gate_reduce(const float *gpart, int ntiles, float *grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_gate_reduce, dim3((NPARAM + 255) / 256), dim3(256), 0, s, gpart, ntiles, grad);
    return hipGetLastError();
}

hipError_t launch_gate_bce(const float *g, const float *y, int n, float *loss, float *dg, hipStream_t s)
{
    hipLaunchKernelGGL(k_gate_bce, dim3(1), dim3(1024), 0, s, g, y, n, loss, dg);
    return hipGetLastError();
}

hipError_t launch_adam(float *theta, float *m, float *v, const float *grad, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s)
{
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, theta, m, v, grad, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace dloc
