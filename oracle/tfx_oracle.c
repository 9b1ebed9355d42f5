/*
 * tfx_oracle.c -- FP64 CPU oracle for the multichannel FIR / IIR-SOS filter
 * chain.  TEST INFRASTRUCTURE ONLY: the HIP library never includes, links or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.
 *
 * What is computed (the paper, Sec. 3 "Design principles and core features",
 * names FIR filters and the generic coefficient-driven lfilter, applied to
 * multichannel [channels x samples] tensors and chained in pipe order; it
 * gives no equations, so the textbook definitions are written out here):
 *
 *   FIR   y[c,n] = sum_{k=0}^{min(M-1,n)} h[k] * x[c,n-k]          (causal,
 *         zero history, output length N, true convolution: h[0] weights the
 *         current sample)
 *   SOS   one second-order section in transposed direct form II, rows
 *         [b0 b1 b2 a1 a2] (a0 == 1 after normalisation):
 *             y[n]  = b0*x[n] + s1
 *             s1    = b1*x[n] - a1*y[n] + s2
 *             s2    = b2*x[n] - a2*y[n]
 *         i.e. H(z) = (b0 + b1 z^-1 + b2 z^-2) / (1 + a1 z^-1 + a2 z^-2);
 *         a cascade applies the sections in array order.
 *   Adjoint (for a scalar loss with upstream gradient g = dL/dy):
 *     FIR   gx[n] = sum_k h[k] g[n+k]  (n+k < N);  gh[k] = sum_{c,n} g[c,n] x[c,n-k]
 *     SOS   v = reverse-time all-pole recursion  v[n] = g[n] - a1 v[n+1] - a2 v[n+2];
 *           gb_i = sum_n v[n] x[n-i];  ga_i = -sum_n v[n] y[n-i];
 *           gx[n] = sum_i b_i v[n+i]
 *
 * Everything is double precision, one channel at a time, in the plain
 * per-sample order of the definitions above.  OpenMP is used only to run
 * independent channels on different cores; no blocking, fusion or
 * reordering is done inside a channel.
 */
#define _POSIX_C_SOURCE 199309L
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* Wall time of the filtering loops of the last oracle_fir / oracle_fir_at /
 * oracle_sos call, from the monotonic (steady) clock: what the CPU baseline
 * reports, without the Python-side promotion and copies. */
static double g_last_seconds = 0.0;

static double steady_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

double oracle_last_seconds(void) { return g_last_seconds; }

/* Threads the parallel loops over channels may use. */
int oracle_threads(void) { return omp_get_max_threads(); }

/* FIR: plain per-sample direct convolution (definition above). */
void oracle_fir(const double *x, double *y, int64_t C, int64_t N,
                const double *h, int64_t M)
{
    const double t0 = steady_seconds();
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < C; ++c) {
        const double *xc = x + c * N;
        double *yc = y + c * N;
        for (int64_t n = 0; n < N; ++n) {
            int64_t kmax = (M - 1 < n) ? (M - 1) : n;
            double acc = 0.0;
            for (int64_t k = 0; k <= kmax; ++k)
                acc += h[k] * xc[n - k];
            yc[n] = acc;
        }
    }
    g_last_seconds = steady_seconds() - t0;
}

/* FIR evaluated only at the listed output positions pos[0..P) of every
 * channel: out[c*P + p] = y[c, pos[p]].  Same definition, for full-size
 * spot checks where the whole convolution would take too long. */
void oracle_fir_at(const double *x, int64_t C, int64_t N, const double *h,
                   int64_t M, const int64_t *pos, int64_t P, double *out)
{
    const double t0 = steady_seconds();
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < C; ++c) {
        const double *xc = x + c * N;
        for (int64_t p = 0; p < P; ++p) {
            int64_t n = pos[p];
            int64_t kmax = (M - 1 < n) ? (M - 1) : n;
            double acc = 0.0;
            for (int64_t k = 0; k <= kmax; ++k)
                acc += h[k] * xc[n - k];
            out[c * P + p] = acc;
        }
    }
    g_last_seconds = steady_seconds() - t0;
}

/* One section in transposed direct form II over one channel, starting from
 * state (s1, s2) and leaving the final state there.  x and y may alias. */
static void tdf2_section(const double *x, double *y, int64_t N,
                         const double *coef, double *s1p, double *s2p)
{
    const double b0 = coef[0], b1 = coef[1], b2 = coef[2];
    const double a1 = coef[3], a2 = coef[4];
    double s1 = *s1p, s2 = *s2p;
    for (int64_t n = 0; n < N; ++n) {
        double xn = x[n];
        double yn = b0 * xn + s1;
        s1 = b1 * xn - a1 * yn + s2;
        s2 = b2 * xn - a2 * yn;
        y[n] = yn;
    }
    *s1p = s1;
    *s2p = s2;
}

/* Cascade of S sections (sos: S rows of [b0 b1 b2 a1 a2]).
 * state_in / state_out: NULL or [C][S][2] = (s1, s2) of every section,
 * the TDF-II delay registers before the first / after the last sample.
 * y may alias x. */
void oracle_sos(const double *x, double *y, int64_t C, int64_t N,
                const double *sos, int64_t S, const double *state_in,
                double *state_out)
{
    const double t0 = steady_seconds();
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < C; ++c) {
        const double *xc = x + c * N;
        double *yc = y + c * N;
        if (yc != xc)
            memcpy(yc, xc, (size_t)N * sizeof(double));
        for (int64_t s = 0; s < S; ++s) {
            double s1 = 0.0, s2 = 0.0;
            if (state_in) {
                s1 = state_in[(c * S + s) * 2 + 0];
                s2 = state_in[(c * S + s) * 2 + 1];
            }
            tdf2_section(yc, yc, N, sos + 5 * s, &s1, &s2);
            if (state_out) {
                state_out[(c * S + s) * 2 + 0] = s1;
                state_out[(c * S + s) * 2 + 1] = s2;
            }
        }
    }
    g_last_seconds = steady_seconds() - t0;
}

/* FIR adjoint.  g, x: [C][N].  gx: NULL or [C][N]; gh: NULL or [M]
 * (summed over all channels). */
void oracle_fir_backward(const double *g, const double *x, const double *h,
                         int64_t M, int64_t C, int64_t N, double *gx,
                         double *gh)
{
    if (gx) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = 0; c < C; ++c) {
            const double *gc = g + c * N;
            double *gxc = gx + c * N;
            for (int64_t n = 0; n < N; ++n) {
                double acc = 0.0;
                for (int64_t k = 0; k < M && n + k < N; ++k)
                    acc += h[k] * gc[n + k];
                gxc[n] = acc;
            }
        }
    }
    if (gh) {
        /* per-channel partial sums, then a fixed-order sum over channels */
        double *part = (double *)calloc((size_t)(C * M), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = 0; c < C; ++c) {
            const double *gc = g + c * N;
            const double *xc = x + c * N;
            for (int64_t k = 0; k < M; ++k) {
                double acc = 0.0;
                for (int64_t n = k; n < N; ++n)
                    acc += gc[n] * xc[n - k];
                part[c * M + k] = acc;
            }
        }
        for (int64_t k = 0; k < M; ++k) {
            double acc = 0.0;
            for (int64_t c = 0; c < C; ++c)
                acc += part[c * M + k];
            gh[k] = acc;
        }
        free(part);
    }
}

/* SOS-cascade adjoint, zero initial state.  g, x: [C][N].  gx: NULL or
 * [C][N] (may alias g); gsos: NULL or [S][5] (summed over channels), in the
 * same [b0 b1 b2 a1 a2] order as the coefficients.  The section signals are
 * recomputed here by a plain forward pass and kept in full. */
void oracle_sos_backward(const double *g, const double *x, const double *sos,
                         int64_t S, int64_t C, int64_t N, double *gx,
                         double *gsos)
{
    double *part = (double *)calloc((size_t)(C * S * 5 + 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < C; ++c) {
        /* sig[s] = input of section s; sig[S] = cascade output */
        double *sig = (double *)malloc((size_t)((S + 1) * N) * sizeof(double));
        double *v = (double *)malloc((size_t)N * sizeof(double));
        double *gcur = (double *)malloc((size_t)N * sizeof(double));
        memcpy(sig, x + c * N, (size_t)N * sizeof(double));
        for (int64_t s = 0; s < S; ++s) {
            double s1 = 0.0, s2 = 0.0;
            tdf2_section(sig + s * N, sig + (s + 1) * N, N, sos + 5 * s, &s1, &s2);
        }
        memcpy(gcur, g + c * N, (size_t)N * sizeof(double));
        for (int64_t s = S - 1; s >= 0; --s) {
            const double *co = sos + 5 * s;
            const double *xs = sig + s * N;
            const double *ys = sig + (s + 1) * N;
            const double a1 = co[3], a2 = co[4];
            /* v[n] = g[n] - a1 v[n+1] - a2 v[n+2], run backwards in time */
            for (int64_t n = N - 1; n >= 0; --n) {
                double vn = gcur[n];
                if (n + 1 < N) vn -= a1 * v[n + 1];
                if (n + 2 < N) vn -= a2 * v[n + 2];
                v[n] = vn;
            }
            double *pc = part + (c * S + s) * 5;
            for (int64_t i = 0; i < 3; ++i) {
                double acc = 0.0;
                for (int64_t n = i; n < N; ++n)
                    acc += v[n] * xs[n - i];
                pc[i] = acc;
            }
            for (int64_t i = 1; i < 3; ++i) {
                double acc = 0.0;
                for (int64_t n = i; n < N; ++n)
                    acc += v[n] * ys[n - i];
                pc[2 + i] = -acc;
            }
            /* gradient w.r.t. this section's input */
            for (int64_t n = 0; n < N; ++n) {
                double acc = co[0] * v[n];
                if (n + 1 < N) acc += co[1] * v[n + 1];
                if (n + 2 < N) acc += co[2] * v[n + 2];
                gcur[n] = acc;
            }
        }
        if (gx)
            memcpy(gx + c * N, gcur, (size_t)N * sizeof(double));
        free(sig);
        free(v);
        free(gcur);
    }
    if (gsos) {
        for (int64_t j = 0; j < S * 5; ++j) {
            double acc = 0.0;
            for (int64_t c = 0; c < C; ++c)
                acc += part[c * S * 5 + j];
            gsos[j] = acc;
        }
    }
    free(part);
}
