/*
 * pnce_c_client.c -- a plain C caller of libpnce.so (test infrastructure):
 * reads complex64 input from a file, runs one operation through the C ABI,
 * writes the complex64 result to a file. No Python or PyTorch involved.
 *
 * usage: pnce_c_client N T L R batch precision feedback spacing in.bin out.bin [op]
 *   op = estimate       (default) in: Y [batch][R][N], out: H [batch][R][T*L]
 *        adjoint        in: G [batch][R][T*L], out: A = G P^T / N [batch][R][N]
 *        packed:FMT     pnce_pack to format FMT (1 bf16, 2 f16, 3 e4m3), then
 *                       pnce_estimate_packed; in: Y, out: H
 *        packedws:FMT   the same with pnce_pack_ws and a workspace of
 *                       PNCE_PACK_WORK_BYTES(batch) bytes
 *        refine:STEPS   FP32-accurate estimate, then STEPS refinement steps;
 *                       in: Y, out: the refined H
 *        refinena:STEPS the same with pnce_refine_noalloc (no workspace)
 *        host:CHUNK:CP  pnce_estimate_host from page-locked host memory in
 *                       chunks of CHUNK frames on a second stream; in: raw
 *                       blocks [batch][R][CP + N], out: H
 * Exit status: 0 on success; 2 for usage or I/O errors; 3 for a HIP error;
 * otherwise 10 - (the failing pnce status).
 */
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

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
    if (argc != 11 && argc != 12) {
        fprintf(stderr,
                "usage: %s N T L R batch precision feedback spacing in.bin out.bin [op]\n",
                argv[0]);
        return 2;
    }
    const int N = atoi(argv[1]), T = atoi(argv[2]), L = atoi(argv[3]), R = atoi(argv[4]);
    const int B = atoi(argv[5]), prec = atoi(argv[6]), spacing = atoi(argv[8]);
    const unsigned feedback = (unsigned)strtoul(argv[7], NULL, 0);
    const char *op = argc == 12 ? argv[11] : "estimate";
    const int adjoint = strcmp(op, "adjoint") == 0;
    const int ws = strncmp(op, "packedws:", 9) == 0;
    const int fmt = strncmp(op, "packed:", 7) == 0 ? atoi(op + 7) : (ws ? atoi(op + 9) : 0);
    const int noalloc = strncmp(op, "refinena:", 9) == 0;
    const int steps = strncmp(op, "refine:", 7) == 0 ? atoi(op + 7)
                      : noalloc                        ? atoi(op + 9)
                                                       : -1;
    int chunk = 0, cp = 0;
    const int from_host = strncmp(op, "host:", 5) == 0;
    if (from_host && (sscanf(op + 5, "%d:%d", &chunk, &cp) != 2 || cp < 0)) {
        fprintf(stderr, "bad op %s\n", op);
        return 2;
    }
    if (!adjoint && !fmt && steps < 0 && !from_host && strcmp(op, "estimate") != 0) {
        fprintf(stderr, "unknown op %s\n", op);
        return 2;
    }
    const size_t ny = (size_t)B * R * (N + cp) * 8, nh = (size_t)B * R * T * L * 8;
    const size_t nin = adjoint ? nh : ny, nout = adjoint ? ny : nh;
    void *hin = NULL, *hout = malloc(nout);
    if (from_host) {
        if (hipHostMalloc(&hin, nin, hipHostMallocDefault) != hipSuccess)
            return 3;
    } else {
        hin = malloc(nin);
    }
    FILE *f = fopen(argv[9], "rb");
    if (!hin || !hout || !f || fread(hin, 1, nin, f) != nin) {
        fprintf(stderr, "cannot read %s\n", argv[9]);
        return 2;
    }
    fclose(f);

    pnce_plan *plan = NULL;
    int rc = check(pnce_create_ex(&plan, N, T, L, R, feedback, spacing), "pnce_create_ex");
    if (rc)
        return rc;
    /* codes of pnce_pack: [batch][R][2][N+1], 1 byte each for e4m3, else 2 */
    const size_t nq = (size_t)B * R * 2 * (N + 1) * (fmt == 3 ? 1 : 2);
    void *din = NULL, *dout = NULL, *dq = NULL, *dwork = NULL;
    float *dscale = NULL;
    hipStream_t s, cs = NULL;
    const int per = chunk < B ? chunk : B;
    const size_t nstage = from_host ? PNCE_HOST_STAGING_BYTES(R, N, cp, per, prec) : 0;
    if (hipStreamCreate(&s) != hipSuccess || hipMalloc(&din, from_host ? nstage : nin) != hipSuccess ||
        (from_host && hipStreamCreate(&cs) != hipSuccess) ||
        hipMalloc(&dout, nout) != hipSuccess ||
        (fmt && (hipMalloc(&dq, nq) != hipSuccess ||
                 hipMalloc((void **)&dscale, (size_t)B * sizeof(float)) != hipSuccess)) ||
        (steps > 0 && !noalloc && hipMalloc(&dwork, ny) != hipSuccess) ||
        (ws && hipMalloc(&dwork, PNCE_PACK_WORK_BYTES(B)) != hipSuccess) ||
        (!from_host && hipMemcpyAsync(din, hin, nin, hipMemcpyHostToDevice, s) != hipSuccess))
        return 3;
    if (from_host) {
        rc = check(pnce_estimate_host(plan, s, cs, hin, cp, dout, B, chunk, prec, din, nstage),
                   "pnce_estimate_host");
    } else if (adjoint) {
        rc = check(pnce_adjoint(plan, s, din, dout, NULL, B, prec, 1.0 / N, 0.0), "pnce_adjoint");
    } else if (fmt) {
        rc = ws ? check(pnce_pack_ws(plan, s, din, 0, dq, dscale, B, fmt, dwork,
                                     PNCE_PACK_WORK_BYTES(B)),
                        "pnce_pack_ws")
                : check(pnce_pack(plan, s, din, dq, dscale, B, fmt), "pnce_pack");
        if (!rc)
            rc = check(pnce_estimate_packed(plan, s, dq, dscale, dout, B, fmt, 0.0),
                       "pnce_estimate_packed");
    } else if (steps >= 0) {
        rc = check(pnce_estimate(plan, s, din, dout, B, PNCE_PREC_F32S, 1.0 / N, NULL, 0.0),
                   "pnce_estimate");
        if (!rc)
            rc = noalloc ? check(pnce_refine_noalloc(plan, s, din, dout, B, steps),
                                 "pnce_refine_noalloc")
                         : check(pnce_refine(plan, s, din, dout, dwork, B, steps), "pnce_refine");
    } else {
        rc = check(pnce_estimate(plan, s, din, dout, B, prec, 1.0 / N, NULL, 0.0),
                   "pnce_estimate");
    }
    if (rc)
        return rc;
    if (hipMemcpyAsync(hout, dout, nout, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return 3;
    f = fopen(argv[10], "wb");
    if (!f || fwrite(hout, 1, nout, f) != nout) {
        fprintf(stderr, "cannot write %s\n", argv[10]);
        return 2;
    }
    fclose(f);
    rc = check(pnce_destroy(plan), "pnce_destroy");
    (void)hipFree(din);
    (void)hipFree(dout);
    (void)hipFree(dq);
    (void)hipFree(dscale);
    (void)hipFree(dwork);
    (void)hipStreamDestroy(s);
    if (cs)
        (void)hipStreamDestroy(cs);
    if (from_host)
        (void)hipHostFree(hin);
    else
        free(hin);
    free(hout);
    return rc;
}
