/*
 * oracle.c -- plain FP64 CPU reference of the localization path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; it exists so the tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the HIP library against an
 * obviously correct, slow definition.  It shares no code with the HIP path.
 *
 * What is computed (paper Sec. 2.2: the network runs on the preloaded frames
 * and post-processing stays on the device; Sec. 3.2: a dilated-convolution
 * network whose per-pixel output is a detection probability plus sub-pixel
 * offsets, as in DECODE; Sec. 3.2.1: dilated 3x3 convolutions):
 *
 *   x      = (ADU - offset) * gain * in_scale                       preprocessing
 *            (scalar gain/offset, or per-pixel sCMOS maps)
 *   a      = ReLU(conv_1(x; stem))                                  stem, 1 -> C
 *   per block k with dilation d_k:
 *     t    = ReLU(conv_dk(a; W_k1, b_k1))
 *     a    = ReLU(a + conv_dk(t; W_k2, b_k2))                       residual block
 *   maps   = head(a), 1x1, C -> 5: logit, dx, dy, dz, photons
 *            (C -> 10: then the raw uncertainties of x, y, z and photons and
 *            the background, Sec. 3.2's per-pixel position uncertainty)
 *
 * conv_d is a cross-correlation with taps spaced d pixels apart and zero
 * "same" padding applied at the true frame border at every layer:
 *   y[o][i][j] = b[o] + sum_c sum_{u,v in -1..1} W[o][c][u+1][v+1] * x[c][i+d*u][j+d*v]
 *
 * Every multiply and add is done in double precision in the plain loop order
 * written below (no blocking, no reordering).  Parallelism (OpenMP) is only
 * over independent output rows/channels and never changes an output's
 * summation order.
 *
 * Emulation modes (quant = 1: BF16, quant = 2: FP8 e4m3) round the stored
 * activations and block-convolution weights the way the reduced-precision
 * forms store them; products and sums stay in double.  FP8 stores every
 * activation tensor that a block convolution reads as e4m3 codes with one
 * power-of-two scale per 32-channel group of each pixel (the last block's
 * output goes to the head unrounded); the block-convolution weights carry one
 * scale per output channel.  quant = 3 (split BF16) stores activations in
 * FP32 and forms each product of a block convolution from BF16 halves:
 * v = hi + lo with hi = bf16(v), lo = bf16(v - hi) for the FP32 activation and
 * the weight alike, and w * x is taken as wh xh + wh xl + wl xh (the wl xl
 * term is left out); bias, residual and ReLU are exact, stem and head as in
 * the other modes.
 *
 * Pins (tests/test_oracle_*.py): delta input reproduces the kernel weights;
 * linearity; constant field; torch-CPU float64 conv2d(dilation=d); residual
 * special cases; positive homogeneity of a bias-free net; locality (crop with
 * receptive-radius margin == whole frame); NMS brute force on tiny frames;
 * BF16/e4m3 rounding against torch casts; gate gradients against central
 * differences and torch autograd; Adam against torch.optim.Adam.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR (-1)

/* ---------------------------------------------------------------- rounding */

/* float64 -> bfloat16 -> float64, round to nearest even (via the float32 value
 * the reduced-precision path starts from). NaN is not expected. */
double or_round_bf16(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    u &= 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* OCP e4m3fn value nearest to v (ties to even mantissa), saturating at +-448.
 * Finite e4m3fn values: subnormals m * 2^-9 (m = 1..7), normals
 * (1 + m/8) * 2^(e-7) for e = 1..15 (m <= 6 when e = 15). */
double or_round_e4m3(double v)
{
    double a = fabs(v);
    double s = v < 0 ? -1.0 : 1.0;
    if (a >= 448.0) return s * 448.0;
    if (a == 0.0) return 0.0 * s;
    int e;
    frexp(a, &e);              /* a = f * 2^e, f in [0.5, 1) -> a in [2^(e-1), 2^e) */
    int ex = e - 1;            /* a in [2^ex, 2^(ex+1)) */
    if (ex < -6) ex = -6;      /* subnormal range shares the quantum 2^-9 */
    double q = ldexp(1.0, ex - 3);   /* spacing of representable values */
    double r = a / q;                /* exact: scaling by a power of two */
    double fl = floor(r);
    double frac = r - fl;
    double n;
    if (frac > 0.5) n = fl + 1.0;
    else if (frac < 0.5) n = fl;
    else n = (fmod(fl, 2.0) == 0.0) ? fl : fl + 1.0;
    double out = n * q;
    if (out > 448.0) out = 448.0;
    return s * out;
}

static double store_round(double v, int quant)
{
    if (quant == 1) return or_round_bf16(v);
    if (quant == 3) return (double)(float)v;   /* split BF16 stores FP32 */
    return v;   /* FP8 storage is applied per tensor (or_store_fp8_groups) */
}

/* Split of an FP32 value into its BF16 halves: hi = bf16(v), lo = bf16(v - hi)
 * (v - hi is exact in FP32: hi is v rounded to 8 significant bits).
 * n values in place: v -> hi, and lo into lo[]. */
void or_split_bf16(double *v, double *lo, long n)
{
    for (long k = 0; k < n; ++k) {
        double f = (double)(float)v[k];
        double hi = or_round_bf16(f);
        lo[k] = or_round_bf16(f - hi);
        v[k] = hi;
    }
}



/* Exponent k of the FP8 group scale 2^k: the smallest k with amax <= 448 2^k,
 * kept to normal float scales (k in -126..127, E8M0 byte k + 127 in 1..254);
 * amax = 0 gives k = -126. */
int or_fp8_group_exp(double amax)
{
    if (!(amax > 0.0)) return -126;
    int e;
    double f = 2.0 * frexp(amax, &e);     /* amax = f 2^(e-1), f in [1, 2) */
    int k = (e - 1) - (f <= 1.75 ? 8 : 7);
    if (k < -126) k = -126;
    if (k > 127) k = 127;
    return k;
}

/* FP8 storage of a planar [C][hw] tensor: each pixel's channels are cut into
 * groups of 32 (the last may be shorter); a value v of a group with largest
 * magnitude amax is stored as e4m3(v / 2^k) 2^k with k = or_fp8_group_exp(amax). */
void or_store_fp8_groups(double *a, int C, long hw)
{
    for (long p = 0; p < hw; ++p)
        for (int c0 = 0; c0 < C; c0 += 32) {
            int c1 = c0 + 32 < C ? c0 + 32 : C;
            double amax = 0.0;
            for (int c = c0; c < c1; ++c) {
                double v = a[(long)c * hw + p];
                if (fabs(v) > amax) amax = fabs(v);
            }
            int k = or_fp8_group_exp(amax);
            for (int c = c0; c < c1; ++c) {
                double v = a[(long)c * hw + p];
                a[(long)c * hw + p] = ldexp(or_round_e4m3(ldexp(v, -k)), k);
            }
        }
}

/* ------------------------------------------------------------ preprocessing */

void or_preprocess(const uint16_t *F, long npx, double gain, double offset,
                   double in_scale, double *x)
{
    for (long p = 0; p < npx; ++p)
        x[p] = ((double)F[p] - offset) * gain * in_scale;
}

/* sCMOS cameras: every pixel has its own offset (ADU) and gain (photons per
 * ADU); gain[p] and offset[p] replace the scalars in the same formula. */
void or_preprocess_maps(const uint16_t *F, long npx, const double *gain, const double *offset,
                        double in_scale, double *x)
{
    for (long p = 0; p < npx; ++p)
        x[p] = ((double)F[p] - offset[p]) * gain[p] * in_scale;
}

/* ------------------------------------------------------------- convolution */

/* One 3x3 dilated convolution, planar [cin][h][w] -> [cout][h][w], zero padding
 * outside the frame.  W is [cout][cin][3][3], b is [cout] (may be NULL). */
void or_conv3x3(const double *in, int cin, int h, int w, const double *W,
                const double *b, int cout, int d, double *out)
{
    long hw = (long)h * w;
#pragma omp parallel for schedule(static)
    for (int o = 0; o < cout; ++o) {
        double *y = out + (long)o * hw;
        for (long p = 0; p < hw; ++p) y[p] = b ? b[o] : 0.0;
        for (int c = 0; c < cin; ++c) {
            const double *xc = in + (long)c * hw;
            for (int u = -1; u <= 1; ++u) {
                for (int v = -1; v <= 1; ++v) {
                    double wt = W[(((long)o * cin + c) * 3 + (u + 1)) * 3 + (v + 1)];
                    for (int i = 0; i < h; ++i) {
                        int ii = i + d * u;
                        if (ii < 0 || ii >= h) continue;
                        int j0 = 0, j1 = w;           /* j + d*v inside [0, w) */
                        if (d * v < 0) j0 = -d * v;
                        if (d * v > 0) j1 = w - d * v;
                        double *yr = y + (long)i * w;
                        const double *xr = xc + (long)ii * w + d * v;
                        for (int j = j0; j < j1; ++j) yr[j] += wt * xr[j];
                    }
                }
            }
        }
    }
}

/* Block convolution of the split-BF16 form: y = b + sum (Wh xh + Wh xl + Wl xh)
 * over the same terms as or_conv3x3, with x and W split by or_split_bf16.
 * Written as three convolutions of the halves (every product of two BF16
 * values is exact in double).  tmp: scratch of cout * h * w doubles. */
static int conv3x3_split3(const double *in, int cin, int h, int w, const double *W, const double *b, int cout,
                          int d, double *out)
{
    long hw = (long)h * w, nin = (long)cin * hw, nw = (long)cout * cin * 9;
    double *xh = malloc(sizeof(double) * nin), *xl = malloc(sizeof(double) * nin);
    double *wh = malloc(sizeof(double) * nw), *wl = malloc(sizeof(double) * nw);
    double *tmp = malloc(sizeof(double) * (long)cout * hw);
    if (!xh || !xl || !wh || !wl || !tmp) {
        free(xh); free(xl); free(wh); free(wl); free(tmp);
        return OR_ERR;
    }
    memcpy(xh, in, sizeof(double) * nin);
    or_split_bf16(xh, xl, nin);
    memcpy(wh, W, sizeof(double) * nw);
    or_split_bf16(wh, wl, nw);
    or_conv3x3(xh, cin, h, w, wh, b, cout, d, out);          /* b + Wh xh */
    or_conv3x3(xl, cin, h, w, wh, NULL, cout, d, tmp);       /* Wh xl */
    for (long k = 0; k < (long)cout * hw; ++k) out[k] += tmp[k];
    or_conv3x3(xh, cin, h, w, wl, NULL, cout, d, tmp);       /* Wl xh */
    for (long k = 0; k < (long)cout * hw; ++k) out[k] += tmp[k];
    free(xh); free(xl); free(wh); free(wl); free(tmp);
    return OR_OK;
}

/* -------------------------------------------------------------- the network */

/* Parameters arrive as the FP32 blob tensors in order:
 *   stem.w [C][1][3][3], stem.b [C],
 *   per block: w1 [C][C][3][3], b1 [C], w2 [C][C][3][3], b2 [C],
 *   head.w [5][C], head.b [5]
 * quant: 0 = exact FP64, 1 = BF16 emulation, 2 = FP8 emulation. */
static void promote(const float *src, long n, double *dst)
{
    for (long i = 0; i < n; ++i) dst[i] = (double)src[i];
}

/* per-output-channel e4m3 weight quantisation: ws[o] = max|W[o]| / 448 (FP32),
 * Wq = e4m3(W * fl32(448 / max|W[o]|)) * ws[o], i.e. the dequantised value.
 * W is [cout][per_out], quantised in place. */
void or_quant_weights_fp8(double *W, int cout, long per_out)
{
    for (int o = 0; o < cout; ++o) {
        double *wo = W + (long)o * per_out;
        double mx = 0.0;
        for (long k = 0; k < per_out; ++k) if (fabs(wo[k]) > mx) mx = fabs(wo[k]);
        if (mx == 0.0) continue;
        float inv = (float)(448.0 / mx);
        float ws = (float)(mx / 448.0);
        for (long k = 0; k < per_out; ++k) {
            float sc = (float)wo[k] * inv;
            wo[k] = or_round_e4m3((double)sc) * (double)ws;
        }
    }
}

/* The network on the preprocessed input x [h][w]; nh head outputs. */
static int net_maps_from_input(const double *x, int h, int w, const float *params, int C, int nblocks,
                               const int *dil, int quant, int nh, double *maps /* [nh][h][w] */)
{
    if (h <= 0 || w <= 0 || C <= 0 || nblocks < 0 || quant < 0 || quant > 3) return OR_ERR;
    if (nh != 5 && nh != 10) return OR_ERR;
    long hw = (long)h * w;
    long nconv = (long)C * C * 9;
    double *a = malloc(sizeof(double) * hw * C);
    double *t = malloc(sizeof(double) * hw * C);
    double *u = malloc(sizeof(double) * hw * C);
    double *Wd = malloc(sizeof(double) * nconv);
    double *bd = malloc(sizeof(double) * (C > nh ? C : nh));
    if (!a || !t || !u || !Wd || !bd) {
        free(a); free(t); free(u); free(Wd); free(bd);
        return OR_ERR;
    }
    const float *p = params;

    /* stem: 1 -> C, dilation 1, FP32-exact weights in every mode */
    promote(p, (long)C * 9, Wd); p += (long)C * 9;
    promote(p, C, bd); p += C;
    or_conv3x3(x, 1, h, w, Wd, bd, C, 1, a);
    for (long k = 0; k < hw * C; ++k) a[k] = store_round(a[k] > 0 ? a[k] : 0.0, quant);
    if (quant == 2 && nblocks > 0) or_store_fp8_groups(a, C, hw);

    for (int blk = 0; blk < nblocks; ++blk) {
        int d = dil[blk];
        /* t = ReLU(conv_d(a; W1, b1)) */
        promote(p, nconv, Wd); p += nconv;
        promote(p, C, bd); p += C;
        if (quant == 1) for (long k = 0; k < nconv; ++k) Wd[k] = or_round_bf16(Wd[k]);
        if (quant == 2) or_quant_weights_fp8(Wd, C, (long)C * 9);
        if (quant == 3) {
            if (conv3x3_split3(a, C, h, w, Wd, bd, C, d, t) != OR_OK) goto fail;
        } else {
            or_conv3x3(a, C, h, w, Wd, bd, C, d, t);
        }
        for (long k = 0; k < hw * C; ++k) t[k] = store_round(t[k] > 0 ? t[k] : 0.0, quant);
        if (quant == 2) or_store_fp8_groups(t, C, hw);
        /* a = ReLU(a + conv_d(t; W2, b2)) */
        promote(p, nconv, Wd); p += nconv;
        promote(p, C, bd); p += C;
        if (quant == 1) for (long k = 0; k < nconv; ++k) Wd[k] = or_round_bf16(Wd[k]);
        if (quant == 2) or_quant_weights_fp8(Wd, C, (long)C * 9);
        if (quant == 3) {
            if (conv3x3_split3(t, C, h, w, Wd, bd, C, d, u) != OR_OK) goto fail;
        } else {
            or_conv3x3(t, C, h, w, Wd, bd, C, d, u);
        }
        for (long k = 0; k < hw * C; ++k) {
            double s = a[k] + u[k];
            a[k] = store_round(s > 0 ? s : 0.0, quant);
        }
        /* FP8: the last block's output feeds the head directly */
        if (quant == 2 && blk + 1 < nblocks) or_store_fp8_groups(a, C, hw);
    }

    /* head: 1x1, C -> nh, FP32 weights in every mode */
    promote(p, (long)nh * C, Wd); p += (long)nh * C;
    promote(p, nh, bd); p += nh;
#pragma omp parallel for schedule(static)
    for (int q = 0; q < nh; ++q) {
        double *m = maps + (long)q * hw;
        for (long k = 0; k < hw; ++k) m[k] = bd[q];
        for (int c = 0; c < C; ++c) {
            double wt = Wd[q * C + c];
            const double *ac = a + (long)c * hw;
            for (long k = 0; k < hw; ++k) m[k] += wt * ac[k];
        }
    }
    free(a); free(t); free(u); free(Wd); free(bd);
    return OR_OK;
fail:
    free(a); free(t); free(u); free(Wd); free(bd);
    return OR_ERR;
}

int or_net_maps(const uint16_t *F, int h, int w, double gain, double offset,
                double in_scale, const float *params, int C, int nblocks,
                const int *dil, int quant, int nh, double *maps /* [nh][h][w] */)
{
    if (h <= 0 || w <= 0) return OR_ERR;
    double *x = malloc(sizeof(double) * (long)h * w);
    if (!x) return OR_ERR;
    or_preprocess(F, (long)h * w, gain, offset, in_scale, x);
    int rc = net_maps_from_input(x, h, w, params, C, nblocks, dil, quant, nh, maps);
    free(x);
    return rc;
}

/* As or_net_maps with per-pixel camera maps gain [h][w] and offset [h][w]. */
int or_net_maps_cam(const uint16_t *F, int h, int w, const double *gain, const double *offset,
                    double in_scale, const float *params, int C, int nblocks,
                    const int *dil, int quant, int nh, double *maps /* [nh][h][w] */)
{
    if (h <= 0 || w <= 0) return OR_ERR;
    double *x = malloc(sizeof(double) * (long)h * w);
    if (!x) return OR_ERR;
    or_preprocess_maps(F, (long)h * w, gain, offset, in_scale, x);
    int rc = net_maps_from_input(x, h, w, params, C, nblocks, dil, quant, nh, maps);
    free(x);
    return rc;
}

/* ------------------------------------------------ dense-connection network */

/* The dense-connection dilated network (paper Sec. 3.2 / 3.2.1: dense
 * connections let each layer use the outputs of all layers before it in its
 * block; Sec. 4.1.2: dilations 2, 4, 8, 16), on the preprocessed input x:
 *   a      = ReLU(conv_1(x; stem))                                   1 -> C
 *   per block k at dilation d_k, on the block input a (C channels):
 *     cat  = [a]
 *     for i in 0 .. L-1:  y_i = ReLU(conv_dk(cat; W_ki, b_ki)),      cat = [cat, y_i]
 *                         (C + i G -> G channels)
 *     a    = ReLU(W_kt . cat + b_kt)                                  1x1, C + L G -> C
 *   maps   = head(a), 1x1, C -> nh
 * Parameters in blob order: stem w [C][1][3][3], b [C]; per block: per layer
 * w [G][C + i G][3][3], b [G]; transition w [C][C + L G], b [C]; head w
 * [nh][C], b [nh].  The concatenation is kept planar: channel c of cat is
 * plane c, so layer i reads planes 0 .. C + i G - 1 and writes the next G. */
static void pointwise(const double *in, int cin, long hw, const double *W, const double *b, int cout, int relu,
                      double *out)
{
#pragma omp parallel for schedule(static)
    for (int o = 0; o < cout; ++o) {
        double *y = out + (long)o * hw;
        for (long p = 0; p < hw; ++p) y[p] = b[o];
        for (int c = 0; c < cin; ++c) {
            const double wt = W[(long)o * cin + c];
            const double *xc = in + (long)c * hw;
            for (long p = 0; p < hw; ++p) y[p] += wt * xc[p];
        }
        if (relu)
            for (long p = 0; p < hw; ++p) y[p] = y[p] > 0 ? y[p] : 0.0;
    }
}

/* The fine-grained stage read as a two-stage U-Net (paper Sec. 3.2: after
 * feature extraction a two-stage U-Net refines the features; its sizes are
 * not given -- the reading here): on the extractor's output a0 (C channels),
 *   p1 = pool(a0),  d1 = ReLU(conv_1(p1))          level 1, C -> C
 *   p2 = pool(d1),  d2 = ReLU(conv_1(p2))          level 2, C -> C
 *   u1 = ReLU(conv_1([d1, up(d2)]))                level 1, 2C -> C
 *   u0 = ReLU(conv_1([a0, up(u1)]))                level 0, 2C -> C
 * and the head reads u0.  Level l + 1 of an h x w level is ceil(h/2) x
 * ceil(w/2); pool = max over the 2 x 2 window's pixels inside the level
 * (windows at an odd edge hold fewer); up = nearest: up(v)[y][x] = v[y/2][x/2].
 * [u, v] concatenates channels, u first.  Convolutions zero-pad at each
 * level's border. */
static void pool2(const double *in, int C, int h, int w, double *out)
{
    const int h2 = (h + 1) / 2, w2 = (w + 1) / 2;
    for (int c = 0; c < C; ++c)
        for (int y = 0; y < h2; ++y)
            for (int x = 0; x < w2; ++x) {
                double m = -INFINITY;
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        const int yy = 2 * y + dy, xx = 2 * x + dx;
                        if (yy < h && xx < w && in[((long)c * h + yy) * w + xx] > m) m = in[((long)c * h + yy) * w + xx];
                    }
                out[((long)c * h2 + y) * w2 + x] = m;
            }
}

/* out [C][h][w] = nearest upsampling of in [C][ceil(h/2)][ceil(w/2)] */
static void up2(const double *in, int C, int h, int w, double *out)
{
    const int h2 = (h + 1) / 2, w2 = (w + 1) / 2;
    for (int c = 0; c < C; ++c)
        for (int y = 0; y < h; ++y)
            for (int x = 0; x < w; ++x) out[((long)c * h + y) * w + x] = in[((long)c * h2 + y / 2) * w2 + x / 2];
}

static void relu_inplace(double *v, long n)
{
    for (long k = 0; k < n; ++k) v[k] = v[k] > 0 ? v[k] : 0.0;
}

/* the U-Net stage on a0 [C][h][w] -> u0 [C][h][w]; p points at its
 * parameters (d1 w, b; d2 w, b; u1 w, b; u0 w, b); returns the parameters
 * after them, or NULL when memory runs out */
static const float *unet_stage(const double *a0, int C, int h, int w, const float *p, double *u0)
{
    const int h1 = (h + 1) / 2, w1 = (w + 1) / 2, h2 = (h1 + 1) / 2, w2 = (w1 + 1) / 2;
    const long n0 = (long)h * w, n1 = (long)h1 * w1, n2 = (long)h2 * w2;
    double *p1 = malloc(sizeof(double) * C * n1), *c1 = malloc(sizeof(double) * 2 * C * n1);
    double *p2 = malloc(sizeof(double) * C * n2), *d2 = malloc(sizeof(double) * C * n2);
    double *u1 = malloc(sizeof(double) * C * n1), *c0 = malloc(sizeof(double) * 2 * C * n0);
    double *Wd = malloc(sizeof(double) * (long)C * 2 * C * 9), *bd = malloc(sizeof(double) * C);
    const float *ret = NULL;
    if (!p1 || !c1 || !p2 || !d2 || !u1 || !c0 || !Wd || !bd) goto done;
    /* down: d1 goes to the first half of c1, d2 to p2's partner */
    pool2(a0, C, h, w, p1);
    promote(p, (long)C * C * 9, Wd); p += (long)C * C * 9;
    promote(p, C, bd); p += C;
    or_conv3x3(p1, C, h1, w1, Wd, bd, C, 1, c1);
    relu_inplace(c1, C * n1);
    pool2(c1, C, h1, w1, p2);
    promote(p, (long)C * C * 9, Wd); p += (long)C * C * 9;
    promote(p, C, bd); p += C;
    or_conv3x3(p2, C, h2, w2, Wd, bd, C, 1, d2);
    relu_inplace(d2, C * n2);
    /* up: c1 = [d1, up(d2)], c0 = [a0, up(u1)] */
    up2(d2, C, h1, w1, c1 + C * n1);
    promote(p, (long)C * 2 * C * 9, Wd); p += (long)C * 2 * C * 9;
    promote(p, C, bd); p += C;
    or_conv3x3(c1, 2 * C, h1, w1, Wd, bd, C, 1, u1);
    relu_inplace(u1, C * n1);
    memcpy(c0, a0, sizeof(double) * C * n0);
    up2(u1, C, h, w, c0 + C * n0);
    promote(p, (long)C * 2 * C * 9, Wd); p += (long)C * 2 * C * 9;
    promote(p, C, bd); p += C;
    or_conv3x3(c0, 2 * C, h, w, Wd, bd, C, 1, u0);
    relu_inplace(u0, C * n0);
    ret = p;
done:
    free(p1); free(c1); free(p2); free(d2); free(u1); free(c0); free(Wd); free(bd);
    return ret;
}

static int dense_maps_from_input(const double *x, int h, int w, const float *params, int C, int nblocks, int L,
                                 int G, const int *dil, int unet, int nh, double *maps)
{
    if (h <= 0 || w <= 0 || C <= 0 || G <= 0 || L < 0 || nblocks < 0 || nh <= 0 || !(unet == 0 || unet == 2))
        return OR_ERR;
    const long hw = (long)h * w;
    const int CT = C + L * G;
    double *cat = malloc(sizeof(double) * hw * CT);
    double *Wd = malloc(sizeof(double) * (long)CT * 9 * (G > C ? G : C));
    double *bd = malloc(sizeof(double) * (CT > nh ? CT : nh));
    if (!cat || !Wd || !bd) {
        free(cat); free(Wd); free(bd);
        return OR_ERR;
    }
    const float *p = params;
    promote(p, (long)C * 9, Wd); p += (long)C * 9;
    promote(p, C, bd); p += C;
    or_conv3x3(x, 1, h, w, Wd, bd, C, 1, cat);
    for (long k = 0; k < hw * C; ++k) cat[k] = cat[k] > 0 ? cat[k] : 0.0;
    for (int blk = 0; blk < nblocks; ++blk) {
        for (int i = 0; i < L; ++i) {
            const int cin = C + i * G;
            promote(p, (long)G * cin * 9, Wd); p += (long)G * cin * 9;
            promote(p, G, bd); p += G;
            double *y = cat + (long)cin * hw;
            or_conv3x3(cat, cin, h, w, Wd, bd, G, dil[blk], y);
            for (long k = 0; k < hw * G; ++k) y[k] = y[k] > 0 ? y[k] : 0.0;
        }
        promote(p, (long)C * CT, Wd); p += (long)C * CT;
        promote(p, C, bd); p += C;
        /* the transition's output becomes the next block's input (planes 0 .. C-1) */
        double *t = malloc(sizeof(double) * hw * C);
        if (!t) {
            free(cat); free(Wd); free(bd);
            return OR_ERR;
        }
        pointwise(cat, CT, hw, Wd, bd, C, 1, t);
        memcpy(cat, t, sizeof(double) * hw * C);
        free(t);
    }
    if (unet) {
        double *u0 = malloc(sizeof(double) * hw * C);
        if (!u0 || !(p = unet_stage(cat, C, h, w, p, u0))) {
            free(u0); free(cat); free(Wd); free(bd);
            return OR_ERR;
        }
        memcpy(cat, u0, sizeof(double) * hw * C);
        free(u0);
    }
    promote(p, (long)nh * C, Wd); p += (long)nh * C;
    promote(p, nh, bd); p += nh;
    pointwise(cat, C, hw, Wd, bd, nh, 0, maps);
    free(cat); free(Wd); free(bd);
    return OR_OK;
}

/* unet: 0 (the head reads the extractor's output) or 2 (the two-stage U-Net
 * above runs first; its parameters follow the blocks') */
int or_dense_maps(const uint16_t *F, int h, int w, double gain, double offset, double in_scale, const float *params,
                  int C, int nblocks, int L, int G, const int *dil, int unet, int nh, double *maps)
{
    if (h <= 0 || w <= 0) return OR_ERR;
    double *x = malloc(sizeof(double) * (long)h * w);
    if (!x) return OR_ERR;
    or_preprocess(F, (long)h * w, gain, offset, in_scale, x);
    int rc = dense_maps_from_input(x, h, w, params, C, nblocks, L, G, dil, unet, nh, maps);
    free(x);
    return rc;
}

/* --------------------------------------------------------------- detection */

/* Pixel (i, j) is detected iff logit > tau and it beats every in-frame
 * 8-neighbour in the order (value, then smaller raster index). */
void or_detect(const double *logit, int h, int w, double tau, uint8_t *det)
{
    for (int i = 0; i < h; ++i) {
        for (int j = 0; j < w; ++j) {
            long idx = (long)i * w + j;
            double v = logit[idx];
            int keep = v > tau;
            for (int di = -1; di <= 1 && keep; ++di) {
                for (int dj = -1; dj <= 1 && keep; ++dj) {
                    if (di == 0 && dj == 0) continue;
                    int ii = i + di, jj = j + dj;
                    if (ii < 0 || ii >= h || jj < 0 || jj >= w) continue;
                    long nidx = (long)ii * w + jj;
                    double nv = logit[nidx];
                    if (!(v > nv || (v == nv && idx < nidx))) keep = 0;
                }
            }
            det[idx] = (uint8_t)keep;
        }
    }
}

/* ------------------------------------------------------------- tile gate */

/* Gate network on one pooled 64x64 tile p (mean of 4x4 input blocks):
 *   z1 = conv(p; g1.w, g1.b)  (1 -> 8, 3x3, pad 1), h1 = ReLU(z1)
 *   z2 = conv(h1; g2.w, g2.b) (8 -> 8),            h2 = ReLU(z2)
 *   m  = max over pixels of h2,   g = fc.w . m + fc.b
 * The global pool is a max: a tile holds a detection as soon as one place in
 * it looks like an emitter, which a mean over 4096 pixels dilutes away.  Its
 * gradient goes to the first pixel in raster order that attains the max.
 * Gate parameters (673) in order: g1.w[8][1][3][3] g1.b[8] g2.w[8][8][3][3]
 * g2.b[8] fc.w[8] fc.b[1]. */
#define GC 8
void or_gate_pool(const double *x, int th, int tw, int pool, double *p)
{
    int ph = th / pool, pw = tw / pool;
    for (int i = 0; i < ph; ++i)
        for (int j = 0; j < pw; ++j) {
            double s = 0.0;
            for (int u = 0; u < pool; ++u)
                for (int v = 0; v < pool; ++v) s += x[(long)(i * pool + u) * tw + j * pool + v];
            p[(long)i * pw + j] = s / (double)(pool * pool);
        }
}

static void gate_forward_one(const double *p, int ph, int pw, const double *th,
                             double *z1, double *h1, double *z2, double *h2,
                             double *m, long *am, double *g)
{
    const double *w1 = th, *b1 = th + 72, *w2 = th + 80, *b2 = th + 656, *fw = th + 664, *fb = th + 672;
    long hw = (long)ph * pw;
    or_conv3x3(p, 1, ph, pw, w1, b1, GC, 1, z1);
    for (long k = 0; k < GC * hw; ++k) h1[k] = z1[k] > 0 ? z1[k] : 0.0;
    or_conv3x3(h1, GC, ph, pw, w2, b2, GC, 1, z2);
    for (long k = 0; k < GC * hw; ++k) h2[k] = z2[k] > 0 ? z2[k] : 0.0;
    double gg = fb[0];
    for (int c = 0; c < GC; ++c) {
        long a = 0;
        for (long k = 1; k < hw; ++k)
            if (h2[(long)c * hw + k] > h2[(long)c * hw + a]) a = k;
        am[c] = a;
        m[c] = h2[(long)c * hw + a];
        gg += fw[c] * m[c];
    }
    *g = gg;
}

/* Forward for n pooled tiles [n][ph][pw]; params theta[673] (double). */
void or_gate_forward(const double *pooled, int n, int ph, int pw, const double *theta, double *g)
{
    long hw = (long)ph * pw;
#pragma omp parallel
    {
        double *z1 = malloc(sizeof(double) * GC * hw), *h1 = malloc(sizeof(double) * GC * hw);
        double *z2 = malloc(sizeof(double) * GC * hw), *h2 = malloc(sizeof(double) * GC * hw);
        double m[GC];
        long am[GC];
#pragma omp for schedule(static)
        for (int b = 0; b < n; ++b)
            gate_forward_one(pooled + (long)b * hw, ph, pw, theta, z1, h1, z2, h2, m, am, &g[b]);
        free(z1); free(h1); free(z2); free(h2);
    }
}

/* Binary cross-entropy with logits, mean over the batch (paper Sec. 3.3):
 *   L = -(1/n) sum_b [ y_b ln s(g_b) + (1 - y_b) ln(1 - s(g_b)) ]
 * written in the overflow-free form max(g,0) - g*y + ln(1 + e^-|g|).
 * dL/dg_b = (s(g_b) - y_b) / n. */
double or_bce(const double *g, const double *y, int n, double *dg)
{
    double L = 0.0;
    for (int b = 0; b < n; ++b) {
        double gb = g[b];
        L += (gb > 0 ? gb : 0.0) - gb * y[b] + log1p(exp(-fabs(gb)));
        if (dg) dg[b] = (1.0 / (1.0 + exp(-gb)) - y[b]) / (double)n;
    }
    return L / (double)n;
}

/* Backward: gradient of sum_b dg[b] * g_b with respect to theta (673), summed
 * over the batch; ReLU'(z) = 1 for z > 0 else 0. */
void or_gate_backward(const double *pooled, int n, int ph, int pw, const double *theta,
                      const double *dg, double *grad)
{
    long hw = (long)ph * pw;
    const double *w2 = theta + 80, *fw = theta + 664;
    memset(grad, 0, sizeof(double) * 673);
    double *z1 = malloc(sizeof(double) * GC * hw), *h1 = malloc(sizeof(double) * GC * hw);
    double *z2 = malloc(sizeof(double) * GC * hw), *h2 = malloc(sizeof(double) * GC * hw);
    double *dz2 = malloc(sizeof(double) * GC * hw), *dz1 = malloc(sizeof(double) * GC * hw);
    double m[GC], g;
    long am[GC];
    for (int b = 0; b < n; ++b) {
        const double *p = pooled + (long)b * hw;
        gate_forward_one(p, ph, pw, theta, z1, h1, z2, h2, m, am, &g);
        double d = dg[b];
        /* linear layer */
        for (int c = 0; c < GC; ++c) grad[664 + c] += d * m[c];
        grad[672] += d;
        /* max pool (to its first maximising pixel) + ReLU */
        for (int c = 0; c < GC; ++c)
            for (long k = 0; k < hw; ++k)
                dz2[(long)c * hw + k] = k == am[c] && z2[(long)c * hw + k] > 0 ? d * fw[c] : 0.0;
        /* conv2: dW2, db2, dh1 */
        for (int o = 0; o < GC; ++o) {
            for (long k = 0; k < hw; ++k) grad[656 + o] += dz2[(long)o * hw + k];
            for (int c = 0; c < GC; ++c)
                for (int u = -1; u <= 1; ++u)
                    for (int v = -1; v <= 1; ++v) {
                        double s = 0.0;
                        for (int i = 0; i < ph; ++i) {
                            int ii = i + u;
                            if (ii < 0 || ii >= ph) continue;
                            for (int j = 0; j < pw; ++j) {
                                int jj = j + v;
                                if (jj < 0 || jj >= pw) continue;
                                s += dz2[(long)o * hw + (long)i * pw + j] * h1[(long)c * hw + (long)ii * pw + jj];
                            }
                        }
                        grad[80 + ((o * GC + c) * 3 + (u + 1)) * 3 + (v + 1)] += s;
                    }
        }
        /* dh1[c][ii][jj] = sum_o sum_uv W2[o][c][u][v] dz2[o][ii-u][jj-v]; then ReLU */
        for (int c = 0; c < GC; ++c)
            for (int ii = 0; ii < ph; ++ii)
                for (int jj = 0; jj < pw; ++jj) {
                    double s = 0.0;
                    for (int o = 0; o < GC; ++o)
                        for (int u = -1; u <= 1; ++u)
                            for (int v = -1; v <= 1; ++v) {
                                int i = ii - u, j = jj - v;
                                if (i < 0 || i >= ph || j < 0 || j >= pw) continue;
                                s += w2[((o * GC + c) * 3 + (u + 1)) * 3 + (v + 1)] * dz2[(long)o * hw + (long)i * pw + j];
                            }
                    long k = (long)c * hw + (long)ii * pw + jj;
                    dz1[k] = z1[k] > 0 ? s : 0.0;
                }
        /* conv1: dW1, db1 */
        for (int o = 0; o < GC; ++o) {
            for (long k = 0; k < hw; ++k) grad[72 + o] += dz1[(long)o * hw + k];
            for (int u = -1; u <= 1; ++u)
                for (int v = -1; v <= 1; ++v) {
                    double s = 0.0;
                    for (int i = 0; i < ph; ++i) {
                        int ii = i + u;
                        if (ii < 0 || ii >= ph) continue;
                        for (int j = 0; j < pw; ++j) {
                            int jj = j + v;
                            if (jj < 0 || jj >= pw) continue;
                            s += dz1[(long)o * hw + (long)i * pw + j] * p[(long)ii * pw + jj];
                        }
                    }
                    grad[(o * 3 + (u + 1)) * 3 + (v + 1)] += s;
                }
        }
    }
    free(z1); free(h1); free(z2); free(h2); free(dz2); free(dz1);
}

/* Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); t counts from 1. */
void or_adam_step(double *theta, double *m, double *v, const double *grad, int n, int t,
                  double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int k = 0; k < n; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * grad[k];
        v[k] = b2 * v[k] + (1.0 - b2) * grad[k] * grad[k];
        theta[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
    }
}
