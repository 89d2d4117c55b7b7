/*
 * pnce_c_client.c -- a plain C caller of libpnce.so (test infrastructure):
 * reads complex64 frames from a file, runs one correlator call through the
 * C ABI, writes the CIRs to a file. No Python or PyTorch involved.
 *
 * usage: pnce_c_client N T L R batch precision feedback spacing in.bin out.bin
 * Exit status: 0 on success; 2 for usage or I/O errors; 3 for a HIP error;
 * otherwise 10 - (the failing pnce status).
 */
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

#include "pnce.h"

static int check(pnce_status st, const char *what)
{
    if (st < 0) {
        fprintf(stderr, "%s: %s (%s)\n", what, pnce_status_string(st), pnce_last_error());
        return 10 - st;
    }
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 11) {
        fprintf(stderr, "usage: %s N T L R batch precision feedback spacing in.bin out.bin\n",
                argv[0]);
        return 2;
    }
    const int N = atoi(argv[1]), T = atoi(argv[2]), L = atoi(argv[3]), R = atoi(argv[4]);
    const int B = atoi(argv[5]), prec = atoi(argv[6]), spacing = atoi(argv[8]);
    const unsigned feedback = (unsigned)strtoul(argv[7], NULL, 0);
    const size_t ny = (size_t)B * R * N * 8, nh = (size_t)B * R * T * L * 8;
    void *hy = malloc(ny), *hh = malloc(nh);
    FILE *f = fopen(argv[9], "rb");
    if (!hy || !hh || !f || fread(hy, 1, ny, f) != ny) {
        fprintf(stderr, "cannot read %s\n", argv[9]);
        return 2;
    }
    fclose(f);

    pnce_plan *plan = NULL;
    int rc = check(pnce_create_ex(&plan, N, T, L, R, feedback, spacing), "pnce_create_ex");
    if (rc)
        return rc;
    void *dy = NULL, *dh = NULL;
    hipStream_t s;
    if (hipStreamCreate(&s) != hipSuccess || hipMalloc(&dy, ny) != hipSuccess ||
        hipMalloc(&dh, nh) != hipSuccess ||
        hipMemcpyAsync(dy, hy, ny, hipMemcpyHostToDevice, s) != hipSuccess)
        return 3;
    rc = check(pnce_estimate(plan, s, dy, dh, B, prec, 1.0 / N, NULL, 0.0), "pnce_estimate");
    if (rc)
        return rc;
    if (hipMemcpyAsync(hh, dh, nh, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return 3;
    f = fopen(argv[10], "wb");
    if (!f || fwrite(hh, 1, nh, f) != nh) {
        fprintf(stderr, "cannot write %s\n", argv[10]);
        return 2;
    }
    fclose(f);
    rc = check(pnce_destroy(plan), "pnce_destroy");
    (void)hipFree(dy);
    (void)hipFree(dh);
    (void)hipStreamDestroy(s);
    free(hy);
    free(hh);
    return rc;
}
