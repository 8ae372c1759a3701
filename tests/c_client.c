/*
 * A plain C99 client of liblbfluct: no Python, no torch.  It owns the device memory and
 * the stream, as the header's conventions say a caller does, and exercises the C ABI end to
 * end: size the workspace, allocate it, initialise the replicas, advance them, read their
 * moments, check the documented error returns, release everything.
 *
 *   c_client PARAMS PRECISION STEPS OUT
 *
 * PARAMS holds n_rep lb_params structures back to back (the file size fixes n_rep).  The
 * state is advanced in two lb_step calls (STEPS/2, then the rest).  OUT receives, per
 * replica, the nine FP64 moment planes [9][ny][nx] followed by the six FP64 totals; then
 * the status flags (uint32) and the time step (int64).  Exit status 0 on success; any
 * failure prints the call and the library's message and exits with 1.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "lbfluct.h"

static int lb_fail(const char *call, lb_status s)
{
    fprintf(stderr, "c_client: %s: %s (%d)\n", call, lb_strerror(s), (int)s);
    return 1;
}

static int hip_fail(const char *call, hipError_t e)
{
    fprintf(stderr, "c_client: %s: %s\n", call, hipGetErrorString(e));
    return 1;
}

#define LB_TRY(call)                                        \
    do {                                                    \
        lb_status s_ = (call);                              \
        if (s_ != LB_OK) { rc = lb_fail(#call, s_); goto out; } \
    } while (0)

#define HIP_TRY(call)                                       \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) { rc = hip_fail(#call, e_); goto out; } \
    } while (0)

#define EXPECT(call, want)                                  \
    do {                                                    \
        lb_status s_ = (call);                              \
        if (s_ != (want)) {                                 \
            fprintf(stderr, "c_client: %s returned %d, expected %d\n", #call, (int)s_, (int)(want)); \
            rc = 1; goto out;                               \
        }                                                   \
    } while (0)

int main(int argc, char **argv)
{
    int rc = 0;
    FILE *fp = NULL, *fo = NULL;
    lb_params *p = NULL;
    double *h_m9 = NULL;
    void *d_ws = NULL;
    double *d_m9 = NULL;
    hipStream_t stream = NULL;
    lb_handle *h = NULL;
    long fsize;
    int32_t n_rep, precision, r;
    int64_t steps, first, step_now = 0;
    size_t bytes = 0, max_nodes = 0;
    double totals[6];
    uint32_t flags = 0;

    if (argc != 5) {
        fprintf(stderr, "usage: c_client PARAMS PRECISION STEPS OUT\n");
        return 2;
    }
    precision = (int32_t)atoi(argv[2]);
    steps = (int64_t)atoll(argv[3]);

    fp = fopen(argv[1], "rb");
    if (!fp || fseek(fp, 0, SEEK_END) != 0 || (fsize = ftell(fp)) <= 0 ||
        fsize % (long)sizeof(lb_params) != 0 || fseek(fp, 0, SEEK_SET) != 0) {
        fprintf(stderr, "c_client: cannot read a whole number of lb_params from %s\n", argv[1]);
        rc = 1;
        goto out;
    }
    n_rep = (int32_t)(fsize / (long)sizeof(lb_params));
    p = (lb_params *)malloc((size_t)fsize);
    if (!p || fread(p, sizeof(lb_params), (size_t)n_rep, fp) != (size_t)n_rep) {
        fprintf(stderr, "c_client: short read of %s\n", argv[1]);
        rc = 1;
        goto out;
    }
    for (r = 0; r < n_rep; ++r) {
        size_t nodes = (size_t)p[r].nx * (size_t)p[r].ny;
        if (nodes > max_nodes) max_nodes = nodes;
    }

    LB_TRY(lb_workspace_size(p, n_rep, precision, 0, &bytes));
    HIP_TRY(hipMalloc(&d_ws, bytes));
    HIP_TRY(hipMalloc((void **)&d_m9, 9 * max_nodes * sizeof(double)));
    HIP_TRY(hipStreamCreate(&stream));

    /* a workspace one byte short is refused before anything is written */
    EXPECT(lb_init(p, n_rep, precision, 0, d_ws, bytes - 1, stream, &h), LB_ENOMEM);
    LB_TRY(lb_init(p, n_rep, precision, 0, d_ws, bytes, stream, &h));

    first = steps / 2;
    LB_TRY(lb_step(h, first));
    LB_TRY(lb_step(h, steps - first));

    /* documented error returns: a replica index out of range, negative steps, and the
       structure factor without the feature it needs */
    EXPECT(lb_moments(h, n_rep, NULL, totals), LB_EINVAL);
    EXPECT(lb_step(h, -1), LB_EINVAL);
    EXPECT(lb_structure_factor(h, LB_SK_SAMPLE, -1, NULL, NULL), LB_ESTATE);

    fo = fopen(argv[4], "wb");
    if (!fo) {
        fprintf(stderr, "c_client: cannot open %s\n", argv[4]);
        rc = 1;
        goto out;
    }
    h_m9 = (double *)malloc(9 * max_nodes * sizeof(double));
    if (!h_m9) {
        rc = 1;
        goto out;
    }
    for (r = 0; r < n_rep; ++r) {
        size_t n9 = 9 * (size_t)p[r].nx * (size_t)p[r].ny;
        LB_TRY(lb_moments(h, r, d_m9, totals));
        HIP_TRY(hipMemcpy(h_m9, d_m9, n9 * sizeof(double), hipMemcpyDeviceToHost));
        if (fwrite(h_m9, sizeof(double), n9, fo) != n9 || fwrite(totals, sizeof(double), 6, fo) != 6) {
            rc = 1;
            goto out;
        }
    }
    LB_TRY(lb_status_flags(h, &flags, &step_now));
    if (fwrite(&flags, sizeof flags, 1, fo) != 1 || fwrite(&step_now, sizeof step_now, 1, fo) != 1) {
        rc = 1;
        goto out;
    }

out:
    if (h) lb_free(h);
    if (stream) hipStreamDestroy(stream);
    if (d_m9) hipFree(d_m9);
    if (d_ws) hipFree(d_ws);
    if (fo && fclose(fo) != 0) rc = 1;
    if (fp) fclose(fp);
    free(h_m9);
    free(p);
    return rc;
}
