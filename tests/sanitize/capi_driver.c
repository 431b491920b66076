/* Calls every entry point of the C ABI (include/nnls.h) with invalid arguments, and the host-only
 * sizing functions with valid ones, against a build of the library whose host code carries
 * AddressSanitizer and UndefinedBehaviorSanitizer.  Every call here is refused or answered on
 * the host before any HIP call, so the driver runs without a GPU; the device pointers are never
 * dereferenced.  Exit status 0 when every return code is the documented one. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/nnls.h"

static int failures = 0;
#define EXPECT(call, want)                                                            \
    do {                                                                              \
        long long got_ = (long long)(call);                                           \
        if (got_ != (long long)(want)) {                                              \
            fprintf(stderr, "FAIL line %d: %s = %lld, want %lld\n", __LINE__, #call,  \
                    got_, (long long)(want));                                         \
            ++failures;                                                               \
        }                                                                             \
    } while (0)

int main(int argc, char** argv)
{
    void* F = (void*)0x1000; /* never dereferenced */
    const size_t big = (size_t)1 << 40;
    const char* dir = argc > 1 ? argv[1] : "/tmp";
    char path[4096];

    /* workspace sizing (host arithmetic only) */
    if (nnls_workspace_bytes(NNLS_OP_PREPARE, 1000, 100, 1, NNLS_GRAM_BF16X3, NNLS_F32) == 0) ++failures;
    if (nnls_workspace_bytes(NNLS_OP_REFINE, 1000, 100, 7, 0, NNLS_F32) == 0) ++failures;
    if (nnls_workspace_bytes(NNLS_OP_SCALES, 1000, 100, 0, 0, NNLS_F64) == 0) ++failures;
    if (nnls_workspace_bytes(NNLS_OP_GRAM, 20000, 5000, 1, NNLS_GRAM_BF16X3, NNLS_F32) == 0) ++failures;
    EXPECT(nnls_workspace_bytes(NNLS_OP_SOLVE, 0, 0, 3, 0, NNLS_F32), 0);
    EXPECT(nnls_workspace_bytes(99, 10, 10, 3, 0, NNLS_F32), 0);

    /* prepare and its pieces */
    EXPECT(nnls_prepare(0, 10, 2, F, 10, F, 2, NNLS_GRAM_BF16X3, NNLS_F32, F, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_prepare(100, 10, 2, F, 5, F, 2, NNLS_GRAM_BF16X3, NNLS_F32, F, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_prepare(100, 10, 2, F, 10, NULL, 2, NNLS_GRAM_BF16X3, NNLS_F32, F, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_prepare(100, 10, 2, F, 10, F, 2, NNLS_GRAM_BF16X3, NNLS_F64, F, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_prepare(100, 10, 2, F, 10, F, 2, 7, NNLS_F32, F, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_prepare(100, 10, 2, F, 10, F, 2, NNLS_GRAM_BF16X3, NNLS_F32, F, F, F, F, 0, NULL), NNLS_E_WORKSPACE);
    EXPECT(nnls_prepare_split(100, 10, 2, NULL, 10, F, 2, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_prepare_product(100, 10, 2, NULL, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_column_scales(10, 10, F, 9, NNLS_F32, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_column_scales(10, 10, F, 10, NNLS_F32, F, F, 0, NULL), NNLS_E_WORKSPACE);
    EXPECT(nnls_gram(10, 10, 1, NULL, 10, F, 1, NNLS_GRAM_BF16X3, NNLS_F32, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_gram(10, 10, 1, F, 10, F, 1, NNLS_GRAM_FP64, NNLS_F32, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_gram_rescaled(10, 10, 1, F, 10, F, 1, NNLS_GRAM_BF16X3, NNLS_F32, NULL, F, F, F, big, NULL), NNLS_E_ARG);

    /* solve (the argument checks come before the workspace check) */
    EXPECT(nnls_solve(0, 2, NNLS_F32, F, F, NULL, 1e-5, 0, NULL, F, F, F, F, NULL, NULL, 0, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_solve(10, 0, NNLS_F32, F, F, NULL, 1e-5, 0, NULL, F, F, F, F, NULL, NULL, 0, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_solve(10, 2, 3, F, F, NULL, 1e-5, 0, NULL, F, F, F, F, NULL, NULL, 0, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_solve(10, 2, NNLS_F32, NULL, F, NULL, 1e-5, 0, NULL, F, F, F, F, NULL, NULL, 0, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_solve(10, 2, NNLS_F32, F, F, NULL, -1.0, 0, NULL, F, F, F, F, NULL, NULL, 0, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_solve(10, 2, NNLS_F32, F, F, NULL, 1e-5, -1, NULL, F, F, F, F, NULL, NULL, 0, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_solve(10, 2, NNLS_F32, F, F, NULL, 1e-5, 0, NULL, F, F, F, F, NULL, F, 0, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_solve(10, 2, NNLS_F32, F, F, NULL, 1e-5, 0, NULL, F, F, F, F, NULL, NULL, -1, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_solve_noalloc(0, 3, NNLS_F32, F, F, NULL, 1e-5, 0, NULL, F, F, F, F, NULL, NULL, 0, NULL), NNLS_E_ARG);
    EXPECT(nnls_solve_noalloc(10, 3, 9, F, F, NULL, 1e-5, 0, NULL, F, F, F, F, NULL, NULL, 0, NULL), NNLS_E_ARG);

    /* refine */
    EXPECT(nnls_refine(0, 10, 2, F, 10, F, 2, NNLS_F32, F, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_refine(50, 10, 2, F, 9, F, 2, NNLS_F32, F, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_refine(50, 10, 2, F, 10, F, 2, NNLS_F32, F, NULL, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_refine(50, 10, 2, F, 10, F, 2, NNLS_F32, F, F, F, F, 8, NULL), NNLS_E_WORKSPACE);
    EXPECT(nnls_refine(50, 10, 2, F, 10, F, 2, NNLS_F32, F, F, NULL, F, 8, NULL), NNLS_E_WORKSPACE);

    /* batched: sizing of valid descriptors, then rejected plans */
    {
        enum { NP = 300 };
        nnls_problem_desc* d = (nnls_problem_desc*)calloc(NP, sizeof(nnls_problem_desc));
        int64_t oA = 0, ob = 0, oQ = 0, oq = 0;
        for (int i = 0; i < NP; ++i) {
            d[i].n = 1 + (i * 37) % 1024;
            d[i].d = 3 * d[i].n;
            d[i].offA = oA;
            d[i].offB = ob;
            d[i].offQ = oQ;
            d[i].offq = oq;
            d[i].offX = oq;
            oA += d[i].d * d[i].n;
            ob += d[i].d;
            oQ += d[i].n * d[i].n;
            oq += d[i].n;
        }
        if (nnls_batched_workspace_bytes(d, NP) == 0) ++failures;
        EXPECT(nnls_batched_workspace_bytes(NULL, 2), 0);
        nnls_plan* plan = NULL;
        EXPECT(nnls_batched_plan_create(d, 0, 1e-5, 0, NULL, F, F, F, F, F, F, F, F, F, NULL, F, big, F, &plan), NNLS_E_ARG);
        EXPECT(nnls_batched_plan_create(d, NP, -1.0, 0, NULL, F, F, F, F, F, F, F, F, F, NULL, F, big, F, &plan), NNLS_E_ARG);
        EXPECT(nnls_batched_plan_create(d, NP, 1e-5, 0, NULL, F, F, F, F, F, F, F, F, F, NULL, F, big, NULL, &plan), NNLS_E_ARG);
        EXPECT(nnls_batched_plan_create(d, NP, 1e-5, 0, NULL, F, NULL, F, F, F, F, F, F, F, NULL, F, big, F, &plan), NNLS_E_ARG);
        EXPECT(nnls_batched_plan_create(d, NP, 1e-5, 0, NULL, F, F, F, F, F, F, F, F, F, NULL, F, 16, F, &plan), NNLS_E_WORKSPACE);
        d[7].n = 2000;
        d[7].d = 3000;
        EXPECT(nnls_batched_plan_create(d, NP, 1e-5, 0, NULL, F, F, F, F, F, F, F, F, F, NULL, F, big, F, &plan), NNLS_E_UNSUPPORTED);
        d[7].d = 0;
        EXPECT(nnls_batched_plan_create(d, NP, 1e-5, 0, NULL, F, F, F, F, F, F, F, F, F, NULL, F, big, F, &plan), NNLS_E_ARG);
        EXPECT(nnls_batched_plan_launch(NULL, NULL), NNLS_E_ARG);
        nnls_batched_plan_destroy(NULL);
        free(d);
    }

    /* autotune */
    {
        int64_t shapes[4] = {300, 100, 900, 300};
        int64_t bad[2] = {300, 0};
        int64_t huge[2] = {3000, 2000};
        snprintf(path, sizeof(path), "%s/tune.json", dir);
        EXPECT(nnls_autotune(NULL, NNLS_TUNE_BATCHED, shapes, 2, NULL), NNLS_E_ARG);
        EXPECT(nnls_autotune(path, 7, shapes, 2, NULL), NNLS_E_ARG);
        EXPECT(nnls_autotune(path, NNLS_TUNE_BATCHED, NULL, 2, NULL), NNLS_E_ARG);
        EXPECT(nnls_autotune(path, NNLS_TUNE_BATCHED, bad, 1, NULL), NNLS_E_ARG);
        EXPECT(nnls_autotune(path, NNLS_TUNE_BATCHED, huge, 1, NULL), NNLS_E_UNSUPPORTED);
    }

    /* network and warm start */
    EXPECT(nnls_mlp_param_count(), 256 * 1024 + 1024 + 1024 * 1024 + 1024 + 1024 * 256 + 256);
    EXPECT(nnls_mlp_forward(65, F, F, F, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_mlp_forward(64, F, F, F, F, 16, NULL), NNLS_E_WORKSPACE);
    EXPECT(nnls_mlp_gradients(64, F, F, NULL, 0.01f, NULL, NULL, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_mlp_train_step(64, F, F, F, 1e-3f, 0, 0.01f, NULL, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_mlp_reset_state(NULL, NULL), NNLS_E_ARG);
    EXPECT(nnls_mlp_fit_input(10, F, F, F, 8, NULL), NNLS_E_WORKSPACE);
    EXPECT(nnls_mlp_inputs(128, 4, F, NULL, F, NULL, NULL), NNLS_E_UNSUPPORTED);
    EXPECT(nnls_warm_start(256, 4, F, F, F, F, NULL, F, big, NULL), NNLS_E_ARG);
    EXPECT(nnls_warm_start(256, 4, F, F, F, F, F, F, 16, NULL), NNLS_E_WORKSPACE);

    /* checkpoints: files checked before any device copy */
    {
        int64_t step = -1;
        snprintf(path, sizeof(path), "%s/missing.ckpt", dir);
        EXPECT(nnls_mlp_load(F, &step, path, NULL), NNLS_E_IO);
        snprintf(path, sizeof(path), "%s/short.ckpt", dir);
        FILE* f = fopen(path, "wb");
        if (f) {
            fwrite("NNLSCKP1", 1, 8, f);
            fclose(f);
        }
        EXPECT(nnls_mlp_load(F, &step, path, NULL), NNLS_E_IO);
        EXPECT(step, -1);
        EXPECT(nnls_mlp_load(NULL, &step, path, NULL), NNLS_E_ARG);
        EXPECT(nnls_mlp_save(F, -1, path, NULL), NNLS_E_ARG);
        snprintf(path, sizeof(path), "%s/no/such/dir/x.ckpt", dir);
        EXPECT(nnls_mlp_save(F, 0, path, NULL), NNLS_E_IO);
    }

    /* helpers */
    EXPECT(nnls_transpose(5, 6, F, 5, F, 5, NULL), NNLS_E_ARG);
    EXPECT(nnls_rescale_start(3, 3, NULL, F, F, NULL), NNLS_E_ARG);
    if (!nnls_version() || !strlen(nnls_version())) ++failures;

    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("C ABI sanitizer driver: all checks passed\n");
    return 0;
}
