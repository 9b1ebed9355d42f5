// tfx_stft.hip -- short-time Fourier transform and its inverse, the FFT /
// STFT functions on the roadmap of Sec. 5.
//
// Each frame is an n_fft-point DFT (n_fft = 2^LOG2N, 16 .. 4096).  Two frames
// of the same channel travel through one complex FFT (frame t as the real part,
// frame t+1 as the imaginary part) and are separated afterwards by the
// conjugate symmetry of real-signal spectra, so the transform costs half a
// complex FFT per frame.  The FFT is a self-sorting (Stockham) mixed-radix
// transform in LDS: one pass of radix 2^(LOG2N mod 4) (or 16) without
// twiddles, then radix-16 passes, each butterfly held in registers (16-point
// DFTs as 4 x 4), so a 4096-point transform takes three trips through LDS.
// The LDS rows carry one float2 of padding per 16 so the strided stores of
// the early passes spread over the banks.  Base twiddles of each radix-16
// pass sit contiguously in LDS (computed once per workgroup in FP64) and
// their powers come from a product tree.  A workgroup transforms 4096 complex
// values per batch (G = 4096 / n_fft rows), one radix-16 butterfly per lane.
//
// Work units are dealt to the eight XCDs in contiguous ranges (the
// dispatcher places workgroup b on XCD b % 8), so that neighbouring units --
// overlapping input frames, shared boundary frames -- go through one L2.
//
// The inverse is one kernel: each unit is a segment of one channel's output.
// It inverts the frames touching the segment (the same FFT on the conjugated
// two-frame spectrum), adds each windowed frame into an LDS accumulator in
// frame order (fixed summation order, no atomics), and divides every sample by
// its summed squared window (weighted overlap-add).  Frames straddling two
// segments are inverted by both.
#include <hip/hip_runtime.h>

#include <cmath>

#include "tfx_internal.h"

namespace tfx {
namespace {

constexpr int SWG = 256;
constexpr int TOTMIN = 4096;  // complex values per workgroup transform batch (radix-16 passes: 1 butterfly per lane)

// LDS index with one float2 of padding after every 16: the strided Stockham
// stores of the first passes then spread over the banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

template <int LOG2N>
struct Shape {
    static constexpr int N = 1 << LOG2N;
    static constexpr int G = N >= TOTMIN ? 1 : TOTMIN / N;  // transforms per batch
    static constexpr int TOT = G * N;
    static constexpr int F = N / 2 + 1;
    static constexpr int R0 = (LOG2N % 4) ? (1 << (LOG2N % 4)) : 16;  // radix of the first pass
    static constexpr int NP = LOG2N / 4 + ((LOG2N % 4) ? 1 : 0);      // passes
    // base twiddles of the radix-16 passes after the first: pass p >= 1 has
    // sub-transform length R0 * 16^(p-1) and as many table entries
    static constexpr int TWN = N > R0 ? (N - R0) / 15 : 1;
    static constexpr int LDS_BUF = TOT + TOT / 16;
};

struct StftArgs {
    const float *x;       // [C][ldx] signal (forward)
    int64_t ldx, nx;      // row stride and length of the signal
    const float *win;     // window of wl samples at offset wleft in the frame (NULL = ones)
    int32_t wl, wleft;
    int32_t hop, off;     // frame step; left padding (n_fft/2 when centred, else 0)
    float scale;          // forward: 1 or n_fft^-1/2; inverse: (1 or n_fft^1/2) / n_fft
    int64_t T;            // frames per channel
    int64_t P;            // forward: frame pairs per channel, ceil(T/2)
    int64_t pairs;        // forward: C * P
    int64_t units;        // work units (forward: batches of G pairs; inverse: output segments)
    float2 *spec;         // [C][T][n_fft/2+1] (forward output / inverse input)
    // inverse
    int64_t C, L, total, ldy, nseg;
    float *y;
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // -i a

__device__ __forceinline__ float window_at(const StftArgs &a, int n) {
    const int j = n - a.wleft;
    if (j < 0 || j >= a.wl) return 0.f;
    return a.win ? a.win[j] : 1.f;
}

// forward DFTs of 2, 4, 8 and 16 points in registers
__device__ __forceinline__ void dft2(float2 &a, float2 &b) {
    const float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

__device__ __forceinline__ void dft4(float2 &a, float2 &b, float2 &c, float2 &d) {
    const float2 s02 = cadd(a, c), d02 = csub(a, c), s13 = cadd(b, d), d13 = csub(b, d);
    a = cadd(s02, s13);
    c = csub(s02, s13);
    b = cadd(d02, mul_mi(d13));
    d = csub(d02, mul_mi(d13));
}

constexpr float C8 = 0.70710678118654752f;  // cos(pi/4)
constexpr float C16 = 0.92387953251128674f; // cos(pi/8)
constexpr float S16 = 0.38268343236508977f; // sin(pi/8)

// v[n] -> V[k]: index n = 2 n1 + n2, k = k1 + 4 k2
__device__ __forceinline__ void dft8(float2 *v) {
    dft4(v[0], v[2], v[4], v[6]);
    dft4(v[1], v[3], v[5], v[7]);
    // twiddles W8^(n2 k1) on the n2 = 1 row: k1 = 1, 2, 3
    v[3] = make_float2(C8 * (v[3].x + v[3].y), C8 * (v[3].y - v[3].x));
    v[5] = mul_mi(v[5]);
    v[7] = make_float2(C8 * (v[7].y - v[7].x), -C8 * (v[7].x + v[7].y));
    float2 y[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        float2 a = v[2 * k1], b = v[2 * k1 + 1];
        dft2(a, b);
        y[k1] = a;
        y[k1 + 4] = b;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = y[k];
}

// v[n] -> V[k]: index n = 4 n1 + n2, k = k1 + 4 k2
__device__ __forceinline__ void dft16(float2 *v) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
    // element (n1 -> k1, n2) now sits at v[4 k1 + n2]; multiply by W16^(n2 k1)
    const float2 w1 = make_float2(C16, -S16), w2 = make_float2(C8, -C8), w3 = make_float2(S16, -C16);
    const float2 w6 = make_float2(-C8, -C8), w9 = make_float2(-C16, S16);
    v[5] = cmul(v[5], w1);
    v[6] = cmul(v[6], w2);
    v[7] = cmul(v[7], w3);
    v[9] = cmul(v[9], w2);
    v[10] = mul_mi(v[10]);
    v[11] = cmul(v[11], w6);
    v[13] = cmul(v[13], w3);
    v[14] = cmul(v[14], w6);
    v[15] = cmul(v[15], w9);
    float2 y[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        float2 a = v[4 * k1], b = v[4 * k1 + 1], c = v[4 * k1 + 2], d = v[4 * k1 + 3];
        dft4(a, b, c, d);
        y[k1] = a;
        y[k1 + 4] = b;
        y[k1 + 8] = c;
        y[k1 + 12] = d;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = y[k];
}

template <int R>
__device__ __forceinline__ void dft_r(float2 *v) {
    if constexpr (R == 2) dft2(v[0], v[1]);
    else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8(v);
    else dft16(v);
}

// Powers w^r, r = 1..15, of the base twiddle w by a product tree (each
// power is at most four products from w).
__device__ __forceinline__ void twiddle16(float2 *v, float2 w1) {
    const float2 w2 = cmul(w1, w1), w3 = cmul(w2, w1), w4 = cmul(w2, w2);
    const float2 w5 = cmul(w4, w1), w6 = cmul(w4, w2), w7 = cmul(w4, w3), w8 = cmul(w4, w4);
    v[1] = cmul(v[1], w1);
    v[2] = cmul(v[2], w2);
    v[3] = cmul(v[3], w3);
    v[4] = cmul(v[4], w4);
    v[5] = cmul(v[5], w5);
    v[6] = cmul(v[6], w6);
    v[7] = cmul(v[7], w7);
    v[8] = cmul(v[8], w8);
    v[9] = cmul(v[9], cmul(w8, w1));
    v[10] = cmul(v[10], cmul(w8, w2));
    v[11] = cmul(v[11], cmul(w8, w3));
    v[12] = cmul(v[12], cmul(w8, w4));
    v[13] = cmul(v[13], cmul(w8, w5));
    v[14] = cmul(v[14], cmul(w8, w6));
    v[15] = cmul(v[15], cmul(w8, w7));
}

// One self-sorting pass: radix R over sub-transforms of length NS, on the G
// rows of N points in buf (padded).  tw = base twiddles exp(-2 pi i k/(NS R)).
template <int LOG2N, int R, int NS>
__device__ __forceinline__ void fft_pass(float2 *buf, const float2 *tw, int tid) {
    constexpr int N = 1 << LOG2N, TOT = Shape<LOG2N>::TOT, M = N / R, NB = TOT / R / SWG;
    static_assert(NB >= 1, "every lane holds at least one butterfly");
    static_assert(NS == 1 || R == 16, "twiddled passes are radix 16");
    float2 v[NB][R];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = tid + q * SWG, g = i / M, j = i - g * M;
        if constexpr (M % 16 == 0) {  // r * M keeps the padding phase: one pad per butterfly
            const int b = pad(g * N + j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[b + r * (M + M / 16)];
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[pad(g * N + j + r * M)];
        }
        if constexpr (NS > 1) twiddle16(v[q], tw[j & (NS - 1)]);
        dft_r<R>(v[q]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int i = tid + q * SWG, g = i / M, j = i - g * M;
        const int o = g * N + (j / NS) * NS * R + (j & (NS - 1));
        if constexpr (NS % 16 == 0) {
            const int b = pad(o);
#pragma unroll
            for (int r = 0; r < R; ++r) buf[b + r * (NS + NS / 16)] = v[q][r];
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[pad(o + r * NS)] = v[q][r];
        }
    }
    __syncthreads();
}

// In-place forward DFT of the G rows; entry and exit with the workgroup in step.
template <int LOG2N>
__device__ __forceinline__ void fft_rows(float2 *buf, const float2 *tw, int tid) {
    using S = Shape<LOG2N>;
    fft_pass<LOG2N, S::R0, 1>(buf, tw, tid);
    if constexpr (S::NP > 1) fft_pass<LOG2N, 16, S::R0>(buf, tw, tid);
    if constexpr (S::NP > 2) fft_pass<LOG2N, 16, S::R0 * 16>(buf, tw + S::R0, tid);
}

// Base twiddles of the radix-16 passes: pass with sub-transform length ns
// at offset ns - R0 (R0, R0 + 16 R0, ...: the tables follow one another),
// entry k = exp(-2 pi i k / (16 ns)), in FP64 then rounded.
template <int LOG2N>
__device__ __forceinline__ void fill_twiddles(float2 *tw, int tid) {
    using S = Shape<LOG2N>;
    for (int ns = S::R0, base = 0; ns * 16 <= S::N; base += ns, ns *= 16) {
        for (int k = tid; k < ns; k += SWG) {
            double sn, cs;
            sincospi(2.0 * (double)k / (16.0 * (double)ns), &sn, &cs);
            tw[base + k] = make_float2((float)cs, (float)-sn);
        }
    }
}

// Units of this workgroup: XCD b % 8 owns a contiguous range of units, which
// its workgroups take in turn.
struct UnitRange {
    int64_t first, end, step;
};

__device__ __forceinline__ UnitRange unit_range(int64_t units) {
    const int64_t per_xcd = (units + 7) / 8;
    const int64_t xcd = blockIdx.x & 7, k = gridDim.x >> 3;
    const int64_t lo = xcd * per_xcd;
    const int64_t hi = lo + per_xcd < units ? lo + per_xcd : units;
    return UnitRange{lo + (int64_t)(blockIdx.x >> 3), hi, k};
}

// a wave-uniform 64-bit value moved to scalar registers
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t reflect(int64_t q, int64_t n) {
    return q < 0 ? -q : (q >= n ? 2 * (n - 1) - q : q);
}

template <int LOG2N>
__global__ __launch_bounds__(SWG, LOG2N == 4 ? 3 : 4) void stft_kernel(StftArgs a) {
    using S = Shape<LOG2N>;
    constexpr int N = S::N, G = S::G, TOT = S::TOT, F = S::F;
    __shared__ float2 buf[S::LDS_BUF];
    __shared__ float2 tw[S::TWN];
    // per row of the batch: input row start c*ldx, frame offset t*hop - off,
    // spectrum offset (c*T + t)*F, flags (1 valid, 2 second frame, 4 reflect)
    __shared__ int64_t rin[G], rof[G], rout[G];
    __shared__ int rfl[G];
    const int tid = threadIdx.x;
    fill_twiddles<LOG2N>(tw, tid);
    constexpr int QPR = N >= SWG ? N / SWG : 1;  // frame samples per lane and row
    float wq[QPR];                               // the window at those samples
#pragma unroll
    for (int m = 0; m < QPR; ++m) wq[m] = window_at(a, (tid + m * SWG) & (N - 1));
    const UnitRange ur = unit_range(a.units);
    for (int64_t u = ur.first; u < ur.end; u += ur.step) {
        __syncthreads();  // previous unit's reads of buf / rows are done; twiddles visible
        for (int g = tid; g < G; g += SWG) {
            const int64_t p = u * G + g;
            int fl = 0;
            if (p < a.pairs) {
                const int64_t c = p / a.P, t = 2 * (p - c * a.P);
                const int64_t o = t * a.hop - a.off;
                const bool two = t + 1 < a.T;
                const int64_t last = o + (two ? a.hop : 0) + N;  // one past the last sample read
                fl = 1 | (two ? 2 : 0) | ((o < 0 || last > a.nx) ? 4 : 0);
                rin[g] = c * a.ldx;
                rof[g] = o;
                rout[g] = (c * a.T + t) * F;
            }
            rfl[g] = fl;
        }
        __syncthreads();
        if constexpr (LOG2N >= 8) {
            // each lane reads samples n = tid + 256 m of every row: the row's
            // bookkeeping is uniform, and all loads are issued before the
            // first LDS store
            float2 v[G][QPR];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int fl = __builtin_amdgcn_readfirstlane(rfl[g]);
#pragma unroll
                for (int m = 0; m < QPR; ++m) v[g][m] = make_float2(0.f, 0.f);
                if ((fl & 5) == 1) {  // both frames inside the signal
                    const float *xr = a.x + uniform64(rin[g] + rof[g]);
#pragma unroll
                    for (int m = 0; m < QPR; ++m) v[g][m].x = xr[tid + m * SWG];
                    if (fl & 2) {
#pragma unroll
                        for (int m = 0; m < QPR; ++m) v[g][m].y = xr[tid + m * SWG + a.hop];
                    }
                } else if (fl & 1) {  // reflected padding at a signal end
                    const float *xc = a.x + rin[g];
                    const int64_t o = rof[g];
#pragma unroll
                    for (int m = 0; m < QPR; ++m) {
                        v[g][m].x = xc[reflect(o + tid + m * SWG, a.nx)];
                        if (fl & 2) v[g][m].y = xc[reflect(o + a.hop + tid + m * SWG, a.nx)];
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int m = 0; m < QPR; ++m)
                    buf[pad(g * N + tid + m * SWG)] = make_float2(wq[m] * v[g][m].x, wq[m] * v[g][m].y);
        } else {
            for (int i = tid; i < TOT; i += SWG) {
                const int g = i >> LOG2N, n = i & (N - 1);
                const int fl = rfl[g];
                const float w = window_at(a, n);
                float2 v = make_float2(0.f, 0.f);
                if (fl & 1) {
                    const float *xc = a.x + rin[g];
                    v.x = w * xc[reflect(rof[g] + n, a.nx)];
                    if (fl & 2) v.y = w * xc[reflect(rof[g] + a.hop + n, a.nx)];
                }
                buf[pad(i)] = v;
            }
        }
        __syncthreads();
        fft_rows<LOG2N>(buf, tw, tid);
        const float h = 0.5f * a.scale;
        for (int i = tid; i < G * F; i += SWG) {
            const int g = i / F, k = i - g * F;
            const int fl = rfl[g];
            if (!(fl & 1)) continue;
            const float2 z = buf[pad(g * N + k)], zm = buf[pad(g * N + ((N - k) & (N - 1)))];
            float2 *out = a.spec + rout[g] + k;
            out[0] = make_float2(h * (z.x + zm.x), h * (z.y - zm.y));
            if (fl & 2) out[F] = make_float2(h * (z.y + zm.y), h * (zm.x - z.x));
        }
    }
}

constexpr int ENV_TAB = 512;  // hops up to this length use the periodic envelope table

// Output samples per unit of the inverse and resident workgroups per CU:
// longer segments recompute fewer boundary frames (a fraction
// (n_fft - hop) / LEN of the frames is inverted twice) but take more LDS.
// Chosen by measurement on the 8 x 5.76 M signal at hop = n_fft / 4.
template <int LOG2N>
struct Seg {
    static constexpr int LEN = LOG2N >= 11 ? 8192 : (LOG2N >= 9 ? 2048 : 4096);
    static constexpr int PER_CU = LOG2N >= 11 ? 2 : 3;
};

// Inverse: each unit is a segment of one channel's output.  The frames that
// touch the segment are inverted G pairs at a time (two real frames per
// complex FFT), windowed and added into an LDS accumulator one frame after
// the other (fixed order); each sample is then divided by its summed squared
// window.
template <int LOG2N>
__global__ __launch_bounds__(SWG, Seg<LOG2N>::PER_CU) void istft_kernel(StftArgs a) {
    using S = Shape<LOG2N>;
    constexpr int N = S::N, G = S::G, F = S::F, SEG = Seg<LOG2N>::LEN;
    constexpr int NW = N >= SWG ? N / SWG : 1;  // frame samples per lane in the overlap-add
    __shared__ float2 buf[S::LDS_BUF];
    __shared__ float2 tw[S::TWN];
    __shared__ float acc[SEG];
    __shared__ float env_period[ENV_TAB];
    const int tid = threadIdx.x;
    fill_twiddles<LOG2N>(tw, tid);
    // summed squared window of a sample covered by every frame that can reach
    // it: periodic in the sample index with period hop
    const bool periodic = a.hop <= ENV_TAB;
    if (periodic) {
        for (int r = tid; r < a.hop; r += SWG) {
            float e = 0.f;
            for (int n = r; n < N; n += a.hop) {
                const float w = window_at(a, n);
                e += w * w;
            }
            env_period[r] = e;
        }
    }
    float wq[NW];  // window x scale at this lane's frame samples n = tid + q * SWG
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        const int n = tid + q * SWG;
        wq[q] = n < N ? window_at(a, n) * a.scale : 0.f;
    }
    const UnitRange ur = unit_range(a.units);
    for (int64_t u = ur.first; u < ur.end; u += ur.step) {
        const int64_t c = u / a.nseg, s0 = (u - c * a.nseg) * SEG;
        const int64_t s1 = s0 + SEG < a.L ? s0 + SEG : a.L;
        const int64_t p0 = s0 + a.off;
        const int64_t p1 = s1 + a.off < a.total ? s1 + a.off : a.total;  // covered padded samples [p0, p1)
        const int len = p0 < p1 ? (int)(p1 - p0) : 0;
        __syncthreads();  // previous unit done with acc and buf; tables visible
        for (int i = tid; i < SEG; i += SWG) acc[i] = 0.f;
        int64_t tlo = 0, thi = -1;
        if (len > 0) {
            tlo = p0 >= N ? (p0 - N) / a.hop + 1 : 0;
            thi = (p1 - 1) / a.hop;
            thi = thi < a.T - 1 ? thi : a.T - 1;
        }
        for (int64_t tb = tlo; tb <= thi; tb += 2 * G) {
            __syncthreads();  // acc cleared / previous batch's reads of buf done
            // conj of Z = Xa + i Xb over the full circle (Hermitian extension of
            // both real frames; the imaginary parts of bins 0 and N/2 are dropped).
            // Row g holds frames tb + 2g and tb + 2g + 1, at sb + i + g F.
            const float2 *sb = a.spec + (c * a.T + tb) * F;
            const int nfr = (int)(thi - tb + 1);  // frames left in this channel's range
            constexpr int NL = (G * F + SWG - 1) / SWG;
            float2 xa[NL], xb[NL];
#pragma unroll
            for (int q = 0; q < NL; ++q) {  // loads first
                const int i = tid + q * SWG, g = i / F;
                xa[q] = make_float2(0.f, 0.f);
                xb[q] = xa[q];
                if (i < G * F && 2 * g < nfr) {
                    const float2 *in = sb + i + g * F;
                    xa[q] = in[0];
                    if (2 * g + 1 < nfr) xb[q] = in[F];
                }
            }
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int i = tid + q * SWG, g = i / F, k = i - g * F;
                if (i >= G * F) break;
                if (k == 0 || k == N / 2) {
                    xa[q].y = 0.f;
                    xb[q].y = 0.f;
                }
                buf[pad(g * N + k)] = make_float2(xa[q].x - xb[q].y, -(xa[q].y + xb[q].x));
                if (k > 0 && k < N / 2)
                    buf[pad(g * N + N - k)] = make_float2(xa[q].x + xb[q].y, xa[q].y - xb[q].x);
            }
            __syncthreads();
            fft_rows<LOG2N>(buf, tw, tid);
            // frame tb + f is the real (f even) or negated imaginary (f odd) part of row f / 2
            for (int f = 0; f < 2 * G && f < nfr; ++f) {
                const int q0 = (int)((tb + f) * a.hop - p0);  // segment offset of the frame's first sample
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    const int n = tid + q * SWG, at = q0 + n;
                    if (n < N && (unsigned)at < (unsigned)len) {
                        const float2 z = buf[pad((f >> 1) * N + n)];
                        acc[at] += wq[q] * ((f & 1) ? -z.y : z.x);
                    }
                }
                __syncthreads();
            }
        }
        float *yc = a.y + c * a.ldy;
        const int64_t pq = p0 / a.hop;  // frame index of p0 + i is pq + (pr + i) / hop
        const uint32_t pr = (uint32_t)(p0 - pq * a.hop);
        for (int i = tid; i < s1 - s0; i += SWG) {
            float out = 0.f;
            if (i < len) {
                const int64_t p = p0 + i;
                const uint32_t d = (pr + (uint32_t)i) / (uint32_t)a.hop;
                const int64_t th = pq + d;  // last frame starting at or before p
                float env;
                if (periodic && p >= N - a.hop && th <= a.T - 1) {
                    env = env_period[pr + (uint32_t)i - d * (uint32_t)a.hop];
                } else {
                    env = 0.f;
                    for (int64_t t = th < a.T - 1 ? th : a.T - 1; t >= 0 && p - t * a.hop < N; --t) {
                        const float w = window_at(a, (int)(p - t * a.hop));
                        env += w * w;
                    }
                }
                out = env > 1e-11f ? acc[i] / env : 0.f;
            }
            yc[s0 + i] = out;
        }
    }
}

#define TFX_STFT_SWITCH(KERNEL, LOG2N, GRID, ST, ARGS)                                           \
    switch (LOG2N) {                                                                              \
    case 4: hipLaunchKernelGGL(KERNEL<4>, GRID, dim3(SWG), 0, ST, ARGS); break;                  \
    case 5: hipLaunchKernelGGL(KERNEL<5>, GRID, dim3(SWG), 0, ST, ARGS); break;                  \
    case 6: hipLaunchKernelGGL(KERNEL<6>, GRID, dim3(SWG), 0, ST, ARGS); break;                  \
    case 7: hipLaunchKernelGGL(KERNEL<7>, GRID, dim3(SWG), 0, ST, ARGS); break;                  \
    case 8: hipLaunchKernelGGL(KERNEL<8>, GRID, dim3(SWG), 0, ST, ARGS); break;                  \
    case 9: hipLaunchKernelGGL(KERNEL<9>, GRID, dim3(SWG), 0, ST, ARGS); break;                  \
    case 10: hipLaunchKernelGGL(KERNEL<10>, GRID, dim3(SWG), 0, ST, ARGS); break;                \
    case 11: hipLaunchKernelGGL(KERNEL<11>, GRID, dim3(SWG), 0, ST, ARGS); break;                \
    case 12: hipLaunchKernelGGL(KERNEL<12>, GRID, dim3(SWG), 0, ST, ARGS); break;                \
    default: return hipErrorInvalidValue;                                                         \
    }

StftArgs make_args(const StftPlan &sp) {
    StftArgs a{};
    const int N = 1 << sp.log2n;
    a.x = sp.x;
    a.ldx = sp.ldx;
    a.nx = sp.nx;
    a.win = sp.win;
    a.wl = sp.win_length;
    a.wleft = (N - sp.win_length) / 2;
    a.hop = sp.hop;
    a.off = sp.center ? N / 2 : 0;
    a.T = sp.T;
    a.C = sp.C;
    return a;
}

int batch_of(int log2n) { return (1 << log2n) >= TOTMIN ? 1 : TOTMIN >> log2n; }
int seg_of(int log2n) { return log2n >= 11 ? 8192 : (log2n >= 9 ? 2048 : 4096); }

dim3 unit_grid(int64_t units, int per_cu) {
    // enough workgroups for per_cu resident per CU, in eight equal XCD shares
    const int64_t per_xcd = (units + 7) / 8;
    const int64_t cap = 32 * (int64_t)per_cu;
    const int64_t k = per_xcd < cap ? per_xcd : cap;
    return dim3((unsigned)(8 * (k > 0 ? k : 1)));
}

}  // namespace

hipError_t launch_stft(const StftPlan &sp) {
    StftArgs a = make_args(sp);
    const int G = batch_of(sp.log2n);
    a.P = (sp.T + 1) / 2;
    a.pairs = sp.C * a.P;
    a.units = (a.pairs + G - 1) / G;
    if (a.units == 0) return hipSuccess;
    a.scale = sp.normalized ? (float)(1.0 / std::sqrt((double)(1 << sp.log2n))) : 1.f;
    a.spec = reinterpret_cast<float2 *>(sp.spec);
    TFX_STFT_SWITCH(stft_kernel, sp.log2n, unit_grid(a.units, 4), sp.stream, a);
    return hipGetLastError();
}

hipError_t launch_istft(const StftPlan &sp) {
    const int N = 1 << sp.log2n;
    StftArgs a = make_args(sp);
    if (sp.length == 0) return hipSuccess;
    a.scale = (float)((sp.normalized ? std::sqrt((double)N) : 1.0) / (double)N);
    a.spec = reinterpret_cast<float2 *>(const_cast<float *>(sp.spec_in));
    a.L = sp.length;
    a.total = (int64_t)N + (int64_t)sp.hop * (sp.T - 1);
    a.ldy = sp.ldy;
    a.y = sp.y;
    const int seg = seg_of(sp.log2n);
    a.nseg = (sp.length + seg - 1) / seg;
    a.units = sp.C * a.nseg;
    TFX_STFT_SWITCH(istft_kernel, sp.log2n, unit_grid(a.units, sp.log2n >= 11 ? 2 : 3), sp.stream, a);
    return hipGetLastError();
}

}  // namespace tfx
