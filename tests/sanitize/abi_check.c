/* Host-side checks of the library's argument and workspace-layout code under
 * AddressSanitizer and UndefinedBehaviorSanitizer (host code only; no GPU is used:
 * every call here returns before a device call, or its first device call fails).
 * Prints "ok" and returns 0 when every return code is the expected one. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "nbody.h"

static int fails = 0;
#define EXPECT(cond)                                                             \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond);  \
            ++fails;                                                             \
        }                                                                        \
    } while (0)

static nb_params params(int64_t n, int precision, int flags, int64_t slots)
{
    nb_params p;
    memset(&p, 0, sizeof p);
    p.n = n;
    p.eps = 1e-4;
    p.eta = 0.45;
    p.eta_init = 0.01;
    p.dt_max_log2 = -3;
    p.dt_min_log2 = -40;
    p.precision = precision;
    p.flags = flags;
    p.partial_slots = slots;
    return p;
}

static nb_batch_params bparams(int64_t cap, int jobs, int precision)
{
    nb_batch_params p;
    memset(&p, 0, sizeof p);
    p.capacity = cap;
    p.max_jobs = jobs;
    p.precision = precision;
    p.eps = 1e-4;
    p.eta = 0.45;
    p.eta_init = 0.01;
    p.dt_max_log2 = -3;
    p.dt_min_log2 = -40;
    return p;
}

int main(void)
{
    /* workspace sizes over the range of n, both precisions, with and without the
     * crackle start and with explicit partial-sum capacities */
    const int64_t ns[] = {1, 2, 3, 767, 768, 769, 8191, 8192, 9001, 65535, 65536, 65537,
                          1 << 20, (int64_t)1 << 25, (int64_t)1 << 30};
    for (size_t k = 0; k < sizeof ns / sizeof ns[0]; ++k)
        for (int prec = 0; prec < 2; ++prec)
            for (int flags = 0; flags < 2; ++flags)
                for (int64_t slots = 0; slots <= (int64_t)1 << 24; slots += (int64_t)1 << 22) {
                    nb_params p = params(ns[k], prec, flags, slots);
                    size_t b = 0;
                    EXPECT(nb_workspace_bytes(&p, &b) == NB_OK);
                    EXPECT(b > 0 && b % 256 == 0);
                    if (slots > 0) {
                        /* an explicit capacity: at least its partial sums */
                        EXPECT(b >= (size_t)slots * 80);
                    }
                }
    /* invalid parameters */
    {
        size_t b = 0;
        nb_params p = params(0, 0, 0, 0);
        EXPECT(nb_workspace_bytes(&p, &b) == NB_ERR_ARG);
        p = params(((int64_t)1 << 30) + 1, 0, 0, 0);
        EXPECT(nb_workspace_bytes(&p, &b) == NB_ERR_ARG);
        p = params(100, 0, 0, 0);
        p.eps = -1.0;
        EXPECT(nb_workspace_bytes(&p, &b) == NB_ERR_ARG);
        p = params(100, 0, 0, 0);
        p.dt_max_log2 = 30;  /* 70 levels */
        EXPECT(nb_workspace_bytes(&p, &b) == NB_ERR_ARG);
        EXPECT(nb_workspace_bytes(NULL, &b) == NB_ERR_ARG);
        p = params(100, 0, 0, 0);
        EXPECT(nb_workspace_bytes(&p, NULL) == NB_ERR_ARG);
    }
    /* context creation: argument checks, then the layout over a (never touched)
     * aligned address, then the first device call, which fails without a GPU */
    {
        nb_params p = params(5000, 0, 1, 0);
        size_t b = 0;
        EXPECT(nb_workspace_bytes(&p, &b) == NB_OK);
        nb_ctx *c = (nb_ctx *)0x1;
        EXPECT(nb_create(&p, NULL, b, &c) == NB_ERR_ARG && c == NULL);
        EXPECT(nb_create(&p, (void *)(uintptr_t)0x10010, b, &c) == NB_ERR_ARG);  /* unaligned */
        EXPECT(nb_create(&p, (void *)(uintptr_t)0x100000, b - 256, &c) == NB_ERR_SPACE);
        const nb_status s = nb_create(&p, (void *)(uintptr_t)0x100000, b, &c);
        EXPECT(s == NB_ERR_DEVICE || s == NB_OK);
        if (s == NB_OK)
            nb_destroy(c);
        nb_destroy(NULL);
    }
    /* the allocation-free evaluation's argument checks */
    {
        double d = 0.0;
        int32_t i = 0;
        EXPECT(nb_evaluate_static(0, &d, &d, &d, &d, 0.0, &i, 1, &d, NULL) == NB_ERR_ARG);
        EXPECT(nb_evaluate_static(10, &d, &d, &d, &d, -1.0, &i, 1, &d, NULL) == NB_ERR_ARG);
        EXPECT(nb_evaluate_static(10, &d, &d, &d, &d, 0.0, &i, 11, &d, NULL) == NB_ERR_ARG);
        EXPECT(nb_evaluate_static(10, NULL, &d, &d, &d, 0.0, &i, 1, &d, NULL) == NB_ERR_ARG);
        EXPECT(nb_evaluate_static(10, &d, &d, &d, &d, 0.0, &i, 0, &d, NULL) == NB_OK);
    }
    /* batch workspaces over capacities, job counts and work-split settings */
    {
        const int64_t caps[] = {1, 100, 65536, (int64_t)1 << 26, (int64_t)1 << 30};
        const int jobs[] = {1, 64, 65536};
        for (size_t k = 0; k < sizeof caps / sizeof caps[0]; ++k)
            for (size_t q = 0; q < sizeof jobs / sizeof jobs[0]; ++q)
                for (int prec = 0; prec < 2; ++prec) {
                    nb_batch_params p = bparams(caps[k], jobs[q], prec);
                    size_t b = 0;
                    EXPECT(nb_batch_workspace_bytes(&p, &b) == NB_OK);
                    EXPECT(b > 0 && b % 256 == 0);
                    p.items_per_job = 16384;
                    p.jchunk = 256;
                    p.chunk_tile = 64;
                    p.chunk_wide = 64;
                    p.chunk_direct = 64;
                    EXPECT(nb_batch_workspace_bytes(&p, &b) == NB_OK);
                }
        size_t b = 0;
        nb_batch_params p = bparams(0, 4, 0);
        EXPECT(nb_batch_workspace_bytes(&p, &b) == NB_ERR_ARG);
        p = bparams(100, 0, 0);
        EXPECT(nb_batch_workspace_bytes(&p, &b) == NB_ERR_ARG);
        p = bparams(100, 4, 0);
        p.jchunk = 65;  /* not a multiple of 64 */
        EXPECT(nb_batch_workspace_bytes(&p, &b) == NB_ERR_ARG);
        p = bparams(100, 4, 0);
        p.items_per_job = 16385;
        EXPECT(nb_batch_workspace_bytes(&p, &b) == NB_ERR_ARG);
        p = bparams(5000, 8, 0);
        EXPECT(nb_batch_workspace_bytes(&p, &b) == NB_OK);
        nb_batch *bt = NULL;
        EXPECT(nb_batch_create(&p, NULL, b, &bt) == NB_ERR_ARG);
        EXPECT(nb_batch_create(&p, (void *)(uintptr_t)0x100000, b - 256, &bt) == NB_ERR_SPACE);
        const nb_status s = nb_batch_create(&p, (void *)(uintptr_t)0x100000, b, &bt);
        EXPECT(s == NB_ERR_DEVICE || s == NB_OK);
        if (s == NB_OK)
            nb_batch_destroy(bt);
        nb_batch_destroy(NULL);
    }
    if (fails)
        return 1;
    printf("ok\n");
    return 0;
}
