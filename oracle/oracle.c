/*
 * oracle.c -- plain FP64 reference for PN-sequence correlation channel
 * estimation (arXiv 2206.05506).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library. It shares no code,
 * header, table or helper with the GPU library; the product never calls it.
 *
 * Every routine is the textbook definition written out as direct loops in
 * double precision (complex numbers are interleaved re/im double pairs),
 * with no blocking, no fusion and no reordering of the sums: a reader can
 * check each loop against the cited equation by eye.
 */
#include <stddef.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/*
 * Feedback taps of one primitive polynomial per degree d (exponents below d,
 * the polynomial being x^d + sum x^tap). Section II-A (Eq. 1) needs a
 * two-level circular autocorrelation, which holds for maximal-length
 * sequences; the paper does not name a polynomial, so this choice is a
 * convention, listed in the design notes.
 */
static const int oracle_taps[17][5] = {
    /* d=0,1 unused */ {-1}, {-1},
    /* 2  */ {1, 0, -1},
    /* 3  */ {1, 0, -1},
    /* 4  */ {1, 0, -1},
    /* 5  */ {2, 0, -1},
    /* 6  */ {1, 0, -1},
    /* 7  */ {1, 0, -1},
    /* 8  */ {4, 3, 2, 0, -1},
    /* 9  */ {4, 0, -1},
    /* 10 */ {3, 0, -1},
    /* 11 */ {2, 0, -1},
    /* 12 */ {6, 4, 1, 0, -1},
    /* 13 */ {4, 3, 1, 0, -1},
    /* 14 */ {10, 6, 1, 0, -1},
    /* 15 */ {1, 0, -1},
    /* 16 */ {12, 3, 1, 0, -1},
};

/*
 * m-sequence of length N = 2^d - 1 (Section II-A, Eq. 1).
 * Bits follow the linear recurrence b[n+d] = XOR over taps i of b[n+i],
 * started from b[0..d-1] = 1,0,...,0. A bit 0 is sent as +1 and a bit 1 as
 * -1 (the paper transmits a real sequence). Returns N, or -1 for d outside
 * [2, 16]. s must hold N entries.
 */
int oracle_mseq(int d, signed char *s)
{
    if (d < 2 || d > 16)
        return -1;
    int N = (1 << d) - 1;
    unsigned char b[1 << 16];
    memset(b, 0, sizeof(b));
    b[0] = 1;
    for (int n = 0; n + d < N; ++n) {
        unsigned char x = 0;
        for (int j = 0; oracle_taps[d][j] >= 0; ++j)
            x ^= b[n + oracle_taps[d][j]];
        b[n + d] = x;
    }
    for (int n = 0; n < N; ++n)
        s[n] = b[n] ? -1 : 1;
    return N;
}

/*
 * m-sequence of Section II-A from any feedback polynomial: the same
 * recurrence and start as oracle_mseq, with the taps given as a mask (bit i
 * set for each exponent i < d of x^d + sum x^i). Different primitive
 * polynomials of one degree give the distinct sequences that neighbouring
 * cells may use (Section II-B). Returns N when the bits repeat with period
 * exactly N = 2^d - 1 (the polynomial is primitive: maximal length), 0 when
 * they do not (s is then unspecified), -1 for d outside [2, 16] or a mask
 * with a bit at or above d. s must hold N entries.
 */
int oracle_mseq_mask(int d, unsigned mask, signed char *s)
{
    if (d < 2 || d > 16 || (mask >> d) != 0)
        return -1;
    int N = (1 << d) - 1;
    unsigned char b[(1 << 16) + 16];
    memset(b, 0, sizeof(b));
    b[0] = 1;
    for (int n = 0; n < N; ++n) {
        unsigned char x = 0;
        for (int i = 0; i < d; ++i)
            if ((mask >> i) & 1u)
                x ^= b[n + i];
        b[n + d] = x;
    }
    /* the d-bit window at n equals the start window 1,0,...,0 first at n = N */
    for (int n = 1; n <= N; ++n) {
        int same = 1;
        for (int i = 0; i < d && same; ++i)
            same = b[n + i] == b[i];
        if (same && n < N)
            return 0;
        if (!same && n == N)
            return 0;
    }
    for (int n = 0; n < N; ++n)
        s[n] = b[n] ? -1 : 1;
    return N;
}

/* (a mod N) in [0, N) for any integer a. */
static int oracle_mod(long a, int N)
{
    long m = a % N;
    return (int)(m < 0 ? m + N : m);
}

/*
 * Correlator of Eq. 3 / Eq. 10, restricted to the K = T*L lags that the
 * multiplexed transmitters occupy (Section II-B); output column k holds lag
 * lag[k] (k itself for adjacent blocks of L lags, Eq. 8's shifts otherwise):
 *
 *   H[b][r][k] = (1/N) * sum_{n=0}^{N-1} Y[b][r][n] * s[(n - lag[k]) mod N]
 *
 * Y: [B][R][N] complex, H: [B][R][K] complex. The sum runs in natural n order
 * and the 1/N is applied once at the end.
 */
void oracle_correlate(const double *Y, const signed char *s, int N,
                      const int *lag, int K, long B, int R, double *H)
{
    long rows = B * (long)R;
#pragma omp parallel for schedule(static)
    for (long row = 0; row < rows; ++row) {
        const double *y = Y + 2 * row * (long)N;
        double *h = H + 2 * row * (long)K;
        for (int k = 0; k < K; ++k) {
            double re = 0.0, im = 0.0;
            for (int n = 0; n < N; ++n) {
                double p = (double)s[oracle_mod((long)n - lag[k], N)];
                re += y[2 * n] * p;
                im += y[2 * n + 1] * p;
            }
            h[2 * k] = re / N;
            h[2 * k + 1] = im / N;
        }
    }
}

/*
 * Adjoint (transpose) of the correlator: a circular convolution of the
 * lag-domain input with the sequence,
 *
 *   A[b][r][n] = (1/N) * sum_{k=0}^{K-1} G[b][r][k] * s[(n - lag[k]) mod N]
 *
 * G: [B][R][K] complex, A: [B][R][N] complex. With G the stacked CIRs and the
 * 1/N removed this is the noiseless multiplexed receive model of Eq. 9.
 */
void oracle_adjoint(const double *G, const signed char *s, int N,
                    const int *lag, int K, long B, int R, double *A)
{
    long rows = B * (long)R;
#pragma omp parallel for schedule(static)
    for (long row = 0; row < rows; ++row) {
        const double *g = G + 2 * row * (long)K;
        double *a = A + 2 * row * (long)N;
        for (int n = 0; n < N; ++n) {
            double re = 0.0, im = 0.0;
            for (int k = 0; k < K; ++k) {
                double p = (double)s[oracle_mod((long)n - lag[k], N)];
                re += g[2 * k] * p;
                im += g[2 * k + 1] * p;
            }
            a[2 * n] = re / N;
            a[2 * n + 1] = im / N;
        }
    }
}

/* Threads for later parallel regions (n <= 0 leaves the setting). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of OpenMP threads a parallel region of this library will use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
