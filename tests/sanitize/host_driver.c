/*
 * Sanitizer driver for the host side of the C ABI (test infrastructure):
 * every call below checks arguments or touches host memory only, so it runs
 * without a GPU.  Built with AddressSanitizer and UndefinedBehaviorSanitizer
 * (host code of the library instrumented too); exit status 0 when every
 * check passes.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/spgemm.h"

static int fails = 0;
#define EXPECT(cond)                                                  \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++fails;                                                  \
        }                                                             \
    } while (0)

int main(int argc, char **argv) {
    const char *dir = argc > 1 ? argv[1] : ".";
    for (int s = 0; s <= 12; ++s) EXPECT(spgemm_status_string((spgemm_status)s) != NULL);
    EXPECT(strcmp(spgemm_status_string((spgemm_status)99), "unknown status") == 0);

    /* descriptors: device pointers are never dereferenced by the size query */
    int64_t fake_rp = 0;
    spgemm_csr A = {10, 5, 0, &fake_rp, NULL, NULL}, B = {5, 7, 0, &fake_rp, NULL, NULL};
    spgemm_options o = {SPGEMM_SIZER_EXACT, 0, NULL, NULL};
    size_t bytes = 0;
    EXPECT(spgemm_plan_workspace_size(&A, &B, &o, NULL) == SPGEMM_E_NULL);
    EXPECT(spgemm_plan_workspace_size(&A, &B, &o, &bytes) == SPGEMM_OK && bytes > 0);
    B.rows = 6;
    EXPECT(spgemm_plan_workspace_size(&A, &B, &o, &bytes) == SPGEMM_E_DIM);
    B.rows = 5;
    A.rows = -1;
    EXPECT(spgemm_plan_workspace_size(&A, &B, &o, &bytes) == SPGEMM_E_DIM);
    A.rows = 10;
    B.cols = (int64_t)1 << 31;
    EXPECT(spgemm_plan_workspace_size(&A, &B, &o, &bytes) == SPGEMM_E_INDEX_OVERFLOW);
    B.cols = 7;
    A.nnz = 3;
    EXPECT(spgemm_plan_workspace_size(&A, &B, &o, &bytes) == SPGEMM_E_NULL);
    A.nnz = 0;
    EXPECT(spgemm_plan_create(&A, &B, NULL, NULL, 0, NULL, NULL, NULL) == SPGEMM_E_NULL);
    EXPECT(spgemm_symbolic(NULL, NULL, 0, NULL, NULL, NULL) == SPGEMM_E_NULL);
    EXPECT(spgemm_numeric(NULL, NULL, 0, NULL, NULL, NULL, NULL, NULL, 0, NULL, NULL) == SPGEMM_E_NULL);
    EXPECT(spgemm_numeric_static(NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, NULL) == SPGEMM_E_NULL);
    EXPECT(spgemm_compute_only(NULL, NULL, NULL, NULL, NULL, NULL) == SPGEMM_E_NULL);
    EXPECT(spgemm_numeric_static_limit() == ((size_t)64 << 20));
    EXPECT(spgemm_transpose_scratch(&A) > 0);

    /* batched plan: descriptors only */
    spgemm_csr As[3] = {{4, 3, 0, &fake_rp, NULL, NULL}, {2, 2, 0, &fake_rp, NULL, NULL}, {0, 5, 0, &fake_rp, NULL, NULL}};
    spgemm_csr Bs[3] = {{3, 4, 0, &fake_rp, NULL, NULL}, {2, 9, 0, &fake_rp, NULL, NULL}, {5, 1, 0, &fake_rp, NULL, NULL}};
    int64_t base[4];
    spgemm_batch *batch = NULL;
    EXPECT(spgemm_batched_plan(3, As, Bs, &o, base, &bytes, &batch) == SPGEMM_OK && batch && bytes > 0);
    EXPECT(base[0] == 0 && base[1] == 5 && base[2] == 8 && base[3] == 9);
    spgemm_batched_destroy(batch);
    Bs[1].rows = 3;
    batch = NULL;
    EXPECT(spgemm_batched_plan(3, As, Bs, &o, base, &bytes, &batch) == SPGEMM_E_DIM && !batch);
    EXPECT(spgemm_batched_plan(-1, As, Bs, &o, base, &bytes, &batch) == SPGEMM_E_INVALID);

    /* models: validation, accessors, a save/load round trip and bad files */
    float theta[1217], mu[3] = {1, 2, 3}, sd[3] = {1, 1, 2}, th2[1217], mu2[3], sd2[3];
    for (int i = 0; i < 1217; ++i) theta[i] = (float)((i % 17) - 8) / 16.0f;
    spgemm_model *m = NULL, *m2 = NULL;
    EXPECT(spgemm_model_create(theta, mu, sd, &m) == SPGEMM_OK && m);
    EXPECT(spgemm_model_get(m, th2, mu2, sd2) == SPGEMM_OK);
    EXPECT(memcmp(th2, theta, sizeof(theta)) == 0 && memcmp(mu2, mu, sizeof(mu)) == 0);
    char path[1024];
    snprintf(path, sizeof(path), "%s/model.bin", dir);
    EXPECT(spgemm_model_save(m, path) == SPGEMM_OK);
    EXPECT(spgemm_model_load(path, &m2) == SPGEMM_OK && m2);
    EXPECT(spgemm_model_get(m2, th2, mu2, sd2) == SPGEMM_OK && memcmp(th2, theta, sizeof(theta)) == 0 &&
           memcmp(sd2, sd, sizeof(sd)) == 0);
    spgemm_model_destroy(m2);
    m2 = NULL;
    /* a truncated copy and a missing file are refused */
    FILE *f = fopen(path, "rb");
    char buf[4096];
    size_t got = f ? fread(buf, 1, sizeof(buf), f) : 0;
    if (f) fclose(f);
    char tpath[1100];
    snprintf(tpath, sizeof(tpath), "%s/truncated.bin", dir);
    f = fopen(tpath, "wb");
    if (f) {
        fwrite(buf, 1, got / 2, f);
        fclose(f);
    }
    EXPECT(spgemm_model_load(tpath, &m2) != SPGEMM_OK && !m2);
    snprintf(tpath, sizeof(tpath), "%s/missing.bin", dir);
    EXPECT(spgemm_model_load(tpath, &m2) == SPGEMM_E_IO && !m2);
    theta[5] = NAN;
    EXPECT(spgemm_model_create(theta, mu, sd, &m2) == SPGEMM_E_INVALID && !m2);
    theta[5] = 0.0f;
    sd[1] = 0.0f;
    EXPECT(spgemm_model_create(theta, mu, sd, &m2) == SPGEMM_E_INVALID && !m2);
    spgemm_model_destroy(m);
    EXPECT(spgemm_model_stats_scratch(1000) > 0 && spgemm_model_grad_scratch(1000) > 0);
    EXPECT(spgemm_model_train_scratch(1000, 256) > 0 && spgemm_model_device_bytes() > 0);
    printf(fails ? "host driver: %d checks failed\n" : "host driver: ok\n", fails);
    return fails ? 1 : 0;
}
