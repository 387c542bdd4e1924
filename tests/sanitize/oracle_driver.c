/* Runs every oracle routine once on small seeded inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py).
 * Exit status 0 = every call returned and every output is finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double or_round_bf16(double v);
double or_round_e4m3(double v);
void or_split_bf16(double *v, double *lo, long n);
int or_fp8_group_exp(double amax);
void or_store_fp8_groups(double *a, int C, long hw);
void or_preprocess(const uint16_t *F, long npx, double gain, double offset, double in_scale, double *x);
void or_preprocess_maps(const uint16_t *F, long npx, const double *gain, const double *offset, double in_scale,
                        double *x);
void or_conv3x3(const double *in, int cin, int h, int w, const double *W, const double *b, int cout, int d,
                double *out);
void or_quant_weights_fp8(double *W, int cout, long per_out);
int or_net_maps(const uint16_t *F, int h, int w, double gain, double offset, double in_scale, const float *params,
                int C, int nblocks, const int *dil, int quant, int nh, double *maps);
int or_net_maps_cam(const uint16_t *F, int h, int w, const double *gain, const double *offset, double in_scale,
                    const float *params, int C, int nblocks, const int *dil, int quant, int nh, double *maps);
int or_dense_maps(const uint16_t *F, int h, int w, double gain, double offset, double in_scale, const float *params,
                  int C, int nblocks, int L, int G, const int *dil, int unet, int nh, double *maps);
void or_detect(const double *logit, int h, int w, double tau, uint8_t *det);
void or_gate_pool(const double *x, int th, int tw, int pool, double *p);
void or_gate_forward(const double *pooled, int n, int ph, int pw, const double *theta, double *g);
double or_bce(const double *g, const double *y, int n, double *dg);
void or_gate_backward(const double *pooled, int n, int ph, int pw, const double *theta, const double *dg,
                      double *grad);
void or_adam_step(double *theta, double *m, double *v, const double *grad, int n, int t, double lr, double b1,
                  double b2, double eps);

static uint64_t state = 88172645463325252ull;
static double urand(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0;
}

static int finite_all(const double *p, long n)
{
    for (long i = 0; i < n; ++i)
        if (!isfinite(p[i])) return 0;
    return 1;
}

#define CHECK(cond)                                                       \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

int main(void)
{
    enum { H = 13, W = 17, C = 16, NB = 2, NH = 10 };
    const int dil[NB] = {1, 3};
    uint16_t F[H * W];
    for (int i = 0; i < H * W; ++i) F[i] = (uint16_t)(90 + 40 * urand());
    /* blob tensors in order: stem w, b; per block w1, b1, w2, b2; head w, b */
    long np = (long)C * 9 + C + (long)NB * 2 * ((long)C * C * 9 + C) + (long)NH * C + NH;
    float *params = malloc(sizeof(float) * np);
    for (long i = 0; i < np; ++i) params[i] = (float)(urand() - 0.5);
    double *maps = malloc(sizeof(double) * NH * H * W);
    double gain[H * W], offset[H * W];
    for (int i = 0; i < H * W; ++i) {
        gain[i] = 0.5 + 0.01 * urand();
        offset[i] = 100.0 + urand();
    }
    for (int q = 0; q <= 3; ++q) {
        CHECK(or_net_maps(F, H, W, 0.5, 100.0, 0.01, params, C, NB, dil, q, NH, maps) == 0);
        CHECK(finite_all(maps, (long)NH * H * W));
        CHECK(or_net_maps_cam(F, H, W, gain, offset, 0.01, params, C, NB, dil, q, NH, maps) == 0);
        CHECK(finite_all(maps, (long)NH * H * W));
    }
    CHECK(or_net_maps(F, H, W, 0.5, 100.0, 0.01, params, C, NB, dil, 4, NH, maps) != 0);   /* bad mode */
    {
        /* dense-connection net, 2 blocks of 2 layers of growth 16, with and
         * without the two-stage U-Net, on an odd-sized frame */
        enum { DL = 2, DG = 16, CT = C + DL * DG };
        long nd = (long)C * 9 + C + (long)NH * C + NH + 4L * C + 2L * C * C * 9 + 2L * C * 2 * C * 9;
        for (int i = 0; i < DL; ++i) nd += NB * ((long)DG * (C + i * DG) * 9 + DG);
        nd += NB * ((long)C * CT + C);
        float *pd = malloc(sizeof(float) * nd);
        for (long i = 0; i < nd; ++i) pd[i] = (float)(0.3 * (urand() - 0.5));
        for (int unet = 0; unet <= 2; unet += 2) {
            CHECK(or_dense_maps(F, H, W, 0.5, 100.0, 0.01, pd, C, NB, DL, DG, dil, unet, NH, maps) == 0);
            CHECK(finite_all(maps, (long)NH * H * W));
        }
        CHECK(or_dense_maps(F, H, W, 0.5, 100.0, 0.01, pd, C, NB, DL, DG, dil, 1, NH, maps) != 0);   /* bad U-Net */
        free(pd);
    }
    uint8_t det[H * W];
    or_detect(maps, H, W, -0.5, det);
    double x[H * W], lo[H * W];
    or_preprocess(F, H * W, 0.5, 100.0, 0.01, x);
    or_preprocess_maps(F, H * W, gain, offset, 0.01, x);
    memcpy(lo, x, sizeof x);
    or_split_bf16(x, lo, H * W);
    CHECK(isfinite(or_round_bf16(3.14159)) && isfinite(or_round_e4m3(1000.0)) && or_fp8_group_exp(0.0) == -126);
    double *a = malloc(sizeof(double) * C * H * W), *y = malloc(sizeof(double) * C * H * W);
    double *Wd = malloc(sizeof(double) * C * C * 9), bd[C];
    for (long i = 0; i < (long)C * H * W; ++i) a[i] = urand();
    for (long i = 0; i < (long)C * C * 9; ++i) Wd[i] = urand() - 0.5;
    for (int i = 0; i < C; ++i) bd[i] = urand();
    or_conv3x3(a, C, H, W, Wd, bd, C, 2, y);
    or_store_fp8_groups(y, C, (long)H * W);
    or_quant_weights_fp8(Wd, C, (long)C * 9);
    CHECK(finite_all(y, (long)C * H * W) && finite_all(Wd, (long)C * C * 9));
    /* gate: two 32 x 32 tiles pooled 4x4 -> 8 x 8 */
    enum { GT = 32, NT = 2, PP = GT / 4 };
    double tile[GT * GT], pooled[NT * PP * PP], theta[673], g[NT], yl[NT] = {0.0, 1.0}, dg[NT], grad[673];
    double m[673] = {0}, v[673] = {0};
    for (int i = 0; i < GT * GT; ++i) tile[i] = urand();
    or_gate_pool(tile, GT, GT, 4, pooled);
    or_gate_pool(tile, GT, GT, 4, pooled + PP * PP);
    for (int i = 0; i < 673; ++i) theta[i] = 0.2 * (urand() - 0.5);
    or_gate_forward(pooled, NT, PP, PP, theta, g);
    double L = or_bce(g, yl, NT, dg);
    or_gate_backward(pooled, NT, PP, PP, theta, dg, grad);
    or_adam_step(theta, m, v, grad, 673, 1, 1e-3, 0.9, 0.999, 1e-8);
    CHECK(isfinite(L) && finite_all(grad, 673) && finite_all(theta, 673));
    free(params); free(maps); free(a); free(y); free(Wd);
    printf("oracle driver ok\n");
    return 0;
}
