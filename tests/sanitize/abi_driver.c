/* Exercises the host-side paths of the C ABI that need no GPU -- weights
 * parsing and validation, config checks, refusals of bad arguments, error
 * text -- for a build of libdloc whose host code carries AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  argv[1]: a valid
 * weights blob.  Exit status 0 = every call answered as documented. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dloc.h"

#define CHECK(cond)                                                       \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    fseek(f, 0, SEEK_END);
    long nb = ftell(f);
    fseek(f, 0, SEEK_SET);
    unsigned char *blob = malloc((size_t)nb);
    if (fread(blob, 1, (size_t)nb, f) != (size_t)nb) return 2;
    fclose(f);

    CHECK(dl_abi_version() == DL_ABI_VERSION);
    dl_config cfg;
    CHECK(dl_default_config(&cfg) == DL_OK && cfg.precision == DL_FP32);
    CHECK(dl_default_config(NULL) == DL_ERR_INVALID_ARG);
    dl_net_info info;
    CHECK(dl_inspect_weights(blob, (size_t)nb, &info) == DL_OK && info.nparams > 0);
    /* every truncation of the blob is refused without reading past it */
    for (long k = 0; k < nb; k += nb / 61 + 1) {
        unsigned char *cut = malloc((size_t)(k ? k : 1));
        memcpy(cut, blob, (size_t)k);
        CHECK(dl_inspect_weights(cut, (size_t)k, &info) == DL_ERR_BAD_WEIGHTS);
        free(cut);
    }
    unsigned char *bad = malloc((size_t)nb);
    memcpy(bad, blob, (size_t)nb);
    bad[0] = 'X';
    CHECK(dl_inspect_weights(bad, (size_t)nb, &info) == DL_ERR_BAD_WEIGHTS);
    CHECK(strlen(dl_last_error(NULL)) > 0);
    free(bad);
    CHECK(dl_inspect_weights(NULL, 64, &info) == DL_ERR_INVALID_ARG);
    CHECK(dl_inspect_weights(blob, (size_t)nb, NULL) == DL_ERR_INVALID_ARG);
    /* bad configs are refused before any device call */
    dl_net *net = NULL;
    dl_config c = cfg;
    c.precision = 9;
    CHECK(dl_create_net(blob, (size_t)nb, &c, &net) == DL_ERR_INVALID_ARG && net == NULL);
    c = cfg;
    c.threshold = 1.5f;
    CHECK(dl_create_net(blob, (size_t)nb, &c, &net) == DL_ERR_INVALID_ARG);
    c = cfg;
    c.tile_w = 48;
    CHECK(dl_create_net(blob, (size_t)nb, &c, &net) == DL_ERR_UNSUPPORTED);
    c = cfg;
    c.reserved[2] = 1;
    CHECK(dl_create_net(blob, (size_t)nb, &c, &net) == DL_ERR_INVALID_ARG);
    CHECK(dl_create_net(blob, (size_t)nb, NULL, NULL) == DL_ERR_INVALID_ARG);
    /* calls on a NULL handle */
    dl_emitter e[4];
    size_t cnt = 0;
    uint16_t frame[64] = {0};
    CHECK(dl_localize(NULL, frame, 1, 8, 8, e, 4, &cnt) == DL_ERR_INVALID_ARG);
    CHECK(dl_localize_maps(NULL, frame, 1, 8, 8, NULL) == DL_ERR_INVALID_ARG);
    CHECK(dl_localize_rois(NULL, NULL, 1, e, 4, &cnt) == DL_ERR_INVALID_ARG);
    CHECK(dl_set_config(NULL, &cfg) == DL_ERR_INVALID_ARG);
    CHECK(dl_set_camera_maps(NULL, NULL, NULL, 0, 0) == DL_ERR_INVALID_ARG);
    CHECK(dl_profile_enable(NULL, 1) == DL_ERR_INVALID_ARG);
    CHECK(dl_gate_keep_map(NULL, NULL, NULL, 0, &cnt) == DL_ERR_INVALID_ARG);
    double rate;
    CHECK(dl_measure_rate(99, 0, 1, &rate) == DL_ERR_INVALID_ARG);
    dl_destroy_net(NULL);
    dl_host_free(NULL);
    free(blob);
    printf("abi driver ok\n");
    return 0;
}
