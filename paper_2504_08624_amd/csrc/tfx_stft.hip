// tfx_stft.hip -- short-time Fourier transform and its inverse, the FFT /
// STFT functions on the roadmap of Sec. 5.
//
// Each frame is an n_fft-point DFT (n_fft = 2^LOG2N, 16 .. 4096).  Two frames
// of the same channel travel through one complex FFT (frame t as the real part,
// frame t+1 as the imaginary part) and are separated afterwards by the
// conjugate symmetry of real-signal spectra, so the transform costs half a
// complex FFT per frame.  The FFT is a self-sorting (Stockham) radix-4
// transform in LDS, with one radix-2 pass first when LOG2N is odd; twiddles
// w^m, m < n_fft/4, sit in an LDS table computed once per workgroup in FP64,
// and w^2m, w^3m are formed by complex products.  Small transforms are packed
// G to a workgroup so that every pass keeps all 256 lanes busy.
//
// Work is split into units of G frame pairs; the units are dealt to the eight
// XCDs in contiguous ranges (the dispatcher places workgroup b on XCD b % 8),
// so that the overlapping input of neighbouring frames is read through one L2.
//
// The inverse runs the same FFT on the conjugated two-frame spectrum, writes
// the windowed frames to a workspace, and a second kernel forms every output
// sample as the sum of the frames covering it divided by the summed squared
// window (weighted overlap-add, gathered per output sample, so no atomics and
// a fixed summation order).
#include <hip/hip_runtime.h>

#include <cmath>

#include "tfx_internal.h"

namespace tfx {
namespace {

constexpr int SWG = 256;

struct StftArgs {
    const float *x;       // [C][ldx] signal (forward) -- unused by the inverse
    int64_t ldx, nx;      // row stride and length of the signal
    const float *win;     // window of wl samples at offset wleft in the frame (NULL = ones)
    int32_t wl, wleft;
    int32_t hop, off;     // frame step; left padding (n_fft/2 when centred, else 0)
    float scale;          // spectrum scale (1 or n_fft^-1/2); inverse: its reciprocal / n_fft
    int64_t T;            // frames per channel
    int64_t P;            // frame pairs per channel, ceil(T/2)
    int64_t pairs;        // C * P
    int64_t units;        // ceil(pairs / G)
    float2 *spec;         // [C][T][n_fft/2+1] (forward output / inverse input)
    float *frames;        // inverse only: [C][T][n_fft] windowed frames
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ float window_at(const StftArgs &a, int n) {
    const int j = n - a.wleft;
    if (j < 0 || j >= a.wl) return 0.f;
    return a.win ? a.win[j] : 1.f;
}

// In-place forward DFT of G independent N-point rows of buf (N = 2^LOG2N,
// TOT = G * N complex values).  Entry and exit with the workgroup in step.
template <int LOG2N, int TOT>
__device__ __forceinline__ void fft_rows(float2 *buf, const float2 *tw, int tid) {
    constexpr int N = 1 << LOG2N;
    if constexpr (LOG2N & 1) {  // radix-2 pass with sub-transform length 1: no twiddles
        constexpr int NB = TOT / 2 / SWG;
        float2 v0[NB], v1[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int i = tid + q * SWG, g = i >> (LOG2N - 1), j = i & (N / 2 - 1);
            v0[q] = buf[g * N + j];
            v1[q] = buf[g * N + j + N / 2];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int i = tid + q * SWG, g = i >> (LOG2N - 1), j = i & (N / 2 - 1);
            buf[g * N + 2 * j] = make_float2(v0[q].x + v1[q].x, v0[q].y + v1[q].y);
            buf[g * N + 2 * j + 1] = make_float2(v0[q].x - v1[q].x, v0[q].y - v1[q].y);
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = (LOG2N & 1); s < LOG2N; s += 2) {  // radix-4 passes, sub-transform length 2^s
        constexpr int NB = TOT / 4 / SWG;
        float2 y[NB][4];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int i = tid + q * SWG, g = i >> (LOG2N - 2), j = i & (N / 4 - 1);
            float2 v0 = buf[g * N + j], v1 = buf[g * N + j + N / 4];
            float2 v2 = buf[g * N + j + N / 2], v3 = buf[g * N + j + 3 * N / 4];
            if (s > 0) {
                const int k = j & ((1 << s) - 1);
                const float2 w1 = tw[k << (LOG2N - 2 - s)];
                const float2 w2 = cmul(w1, w1), w3 = cmul(w1, w2);
                v1 = cmul(v1, w1);
                v2 = cmul(v2, w2);
                v3 = cmul(v3, w3);
            }
            const float2 s02 = make_float2(v0.x + v2.x, v0.y + v2.y), d02 = make_float2(v0.x - v2.x, v0.y - v2.y);
            const float2 s13 = make_float2(v1.x + v3.x, v1.y + v3.y), d13 = make_float2(v1.x - v3.x, v1.y - v3.y);
            y[q][0] = make_float2(s02.x + s13.x, s02.y + s13.y);
            y[q][1] = make_float2(d02.x + d13.y, d02.y - d13.x);  // d02 - i d13
            y[q][2] = make_float2(s02.x - s13.x, s02.y - s13.y);
            y[q][3] = make_float2(d02.x - d13.y, d02.y + d13.x);  // d02 + i d13
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int i = tid + q * SWG, g = i >> (LOG2N - 2), j = i & (N / 4 - 1);
            const int k = j & ((1 << s) - 1);
            const int o = g * N + ((j >> s) << (s + 2)) + k;
#pragma unroll
            for (int r = 0; r < 4; ++r) buf[o + (r << s)] = y[q][r];
        }
        __syncthreads();
    }
}

// Twiddle table w^m = exp(-2 pi i m / N), m < N/4, in FP64 then rounded.
template <int LOG2N>
__device__ __forceinline__ void fill_twiddles(float2 *tw, int tid) {
    constexpr int N = 1 << LOG2N;
    for (int m = tid; m < N / 4; m += SWG) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)N, &sn, &cs);
        tw[m] = make_float2((float)cs, (float)-sn);
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

template <int LOG2N>
__global__ __launch_bounds__(SWG) void stft_kernel(StftArgs a) {
    constexpr int N = 1 << LOG2N, G = N >= 1024 ? 1 : 1024 / N, TOT = G * N, F = N / 2 + 1;
    __shared__ float2 buf[TOT];
    __shared__ float2 tw[N / 4];
    __shared__ int64_t row[G], frame[G];
    const int tid = threadIdx.x;
    fill_twiddles<LOG2N>(tw, tid);
    const UnitRange ur = unit_range(a.units);
    for (int64_t u = ur.first; u < ur.end; u += ur.step) {
        __syncthreads();  // previous unit's reads of buf / row are done; twiddles visible
        if (tid < G) {
            const int64_t p = u * G + tid;
            const int64_t c = p < a.pairs ? p / a.P : -1;
            row[tid] = c;
            frame[tid] = c < 0 ? 0 : 2 * (p - c * a.P);
        }
        __syncthreads();
        for (int i = tid; i < TOT; i += SWG) {
            const int g = i >> LOG2N, n = i & (N - 1);
            const int64_t c = row[g], t = frame[g];
            float2 v = make_float2(0.f, 0.f);
            const float w = window_at(a, n);
            if (c >= 0 && w != 0.f) {
                const float *xc = a.x + c * a.ldx;
                int64_t q = t * a.hop + n - a.off;
                q = q < 0 ? -q : (q >= a.nx ? 2 * (a.nx - 1) - q : q);
                v.x = w * xc[q];
                if (t + 1 < a.T) {
                    int64_t q1 = (t + 1) * a.hop + n - a.off;
                    q1 = q1 < 0 ? -q1 : (q1 >= a.nx ? 2 * (a.nx - 1) - q1 : q1);
                    v.y = w * xc[q1];
                }
            }
            buf[i] = v;
        }
        __syncthreads();
        fft_rows<LOG2N, TOT>(buf, tw, tid);
        const float h = 0.5f * a.scale;
        for (int i = tid; i < G * F; i += SWG) {
            const int g = i / F, k = i - g * F;
            const int64_t c = row[g], t = frame[g];
            if (c < 0) continue;
            const float2 z = buf[g * N + k], zm = buf[g * N + ((N - k) & (N - 1))];
            float2 *out = a.spec + (c * a.T + t) * F + k;
            out[0] = make_float2(h * (z.x + zm.x), h * (z.y - zm.y));
            if (t + 1 < a.T) out[F] = make_float2(h * (z.y + zm.y), h * (zm.x - z.x));
        }
    }
}

template <int LOG2N>
__global__ __launch_bounds__(SWG) void istft_frames_kernel(StftArgs a) {
    constexpr int N = 1 << LOG2N, G = N >= 1024 ? 1 : 1024 / N, TOT = G * N, F = N / 2 + 1;
    __shared__ float2 buf[TOT];
    __shared__ float2 tw[N / 4];
    __shared__ int64_t row[G], frame[G];
    const int tid = threadIdx.x;
    fill_twiddles<LOG2N>(tw, tid);
    const UnitRange ur = unit_range(a.units);
    for (int64_t u = ur.first; u < ur.end; u += ur.step) {
        __syncthreads();
        if (tid < G) {
            const int64_t p = u * G + tid;
            const int64_t c = p < a.pairs ? p / a.P : -1;
            row[tid] = c;
            frame[tid] = c < 0 ? 0 : 2 * (p - c * a.P);
        }
        __syncthreads();
        // conj of Z = Xa + i Xb over the full circle (Hermitian extension of
        // both real frames; the imaginary parts of bins 0 and N/2 are dropped)
        for (int i = tid; i < G * F; i += SWG) {
            const int g = i / F, k = i - g * F;
            const int64_t c = row[g], t = frame[g];
            float2 xa = make_float2(0.f, 0.f), xb = xa;
            if (c >= 0) {
                const float2 *in = a.spec + (c * a.T + t) * F + k;
                xa = in[0];
                if (t + 1 < a.T) xb = in[F];
            }
            if (k == 0 || k == N / 2) {
                xa.y = 0.f;
                xb.y = 0.f;
            }
            buf[g * N + k] = make_float2(xa.x - xb.y, -(xa.y + xb.x));
            if (k > 0 && k < N / 2) buf[g * N + N - k] = make_float2(xa.x + xb.y, xa.y - xb.x);
        }
        __syncthreads();
        fft_rows<LOG2N, TOT>(buf, tw, tid);
        for (int i = tid; i < TOT; i += SWG) {
            const int g = i >> LOG2N, n = i & (N - 1);
            const int64_t c = row[g], t = frame[g];
            if (c < 0) continue;
            const float w = window_at(a, n) * a.scale;
            const float2 z = buf[i];
            float *out = a.frames + (c * a.T + t) * N + n;
            out[0] = w * z.x;
            if (t + 1 < a.T) out[N] = -w * z.y;
        }
    }
}

struct OlaArgs {
    const float *frames;  // [C][T][n_fft]
    const float *win;
    int32_t wl, wleft, n_fft, hop;
    int64_t T, C, L, off, total, ldy;
    float *y;
};

__global__ __launch_bounds__(SWG) void istft_ola_kernel(OlaArgs a) {
    const int64_t s = (int64_t)blockIdx.x * SWG + threadIdx.x;
    if (s >= a.L) return;
    const int64_t p = s + a.off;
    const int N = a.n_fft;
    int64_t tlo = 0, thi = -1;
    float env = 0.f;
    if (p < a.total) {
        thi = p / a.hop;
        thi = thi < a.T - 1 ? thi : a.T - 1;
        tlo = p >= N ? (p - N) / a.hop + 1 : 0;
        for (int64_t t = tlo; t <= thi; ++t) {
            const int j = (int)(p - t * a.hop) - a.wleft;
            const float w = (j >= 0 && j < a.wl) ? (a.win ? a.win[j] : 1.f) : 0.f;
            env += w * w;
        }
    }
    const bool ok = env > 1e-11f;
    for (int64_t c = blockIdx.y; c < a.C; c += gridDim.y) {
        float acc = 0.f;
        const float *fc = a.frames + c * a.T * N;
        for (int64_t t = tlo; t <= thi; ++t) acc += fc[t * N + (p - t * a.hop)];
        a.y[c * a.ldy + s] = ok ? acc / env : 0.f;
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
    const int log2n = sp.log2n, N = 1 << log2n;
    const int G = N >= 1024 ? 1 : 1024 / N;
    a.x = sp.x;
    a.ldx = sp.ldx;
    a.nx = sp.nx;
    a.win = sp.win;
    a.wl = sp.win_length;
    a.wleft = (N - sp.win_length) / 2;
    a.hop = sp.hop;
    a.off = sp.center ? N / 2 : 0;
    a.T = sp.T;
    a.P = (sp.T + 1) / 2;
    a.pairs = sp.C * a.P;
    a.units = (a.pairs + G - 1) / G;
    return a;
}

dim3 unit_grid(int64_t units) {
    // 8 workgroups per CU at most are resident; more only queue
    const int64_t per_xcd = (units + 7) / 8;
    const int64_t k = per_xcd < 256 ? per_xcd : 256;
    return dim3((unsigned)(8 * (k > 0 ? k : 1)));
}

}  // namespace

hipError_t launch_stft(const StftPlan &sp) {
    StftArgs a = make_args(sp);
    if (a.units == 0) return hipSuccess;
    a.scale = sp.normalized ? (float)(1.0 / std::sqrt((double)(1 << sp.log2n))) : 1.f;
    a.spec = reinterpret_cast<float2 *>(sp.spec);
    TFX_STFT_SWITCH(stft_kernel, sp.log2n, unit_grid(a.units), sp.stream, a);
    return hipGetLastError();
}

hipError_t launch_istft(const StftPlan &sp) {
    const int N = 1 << sp.log2n;
    StftArgs a = make_args(sp);
    if (sp.length == 0) return hipSuccess;
    a.scale = (float)((sp.normalized ? std::sqrt((double)N) : 1.0) / (double)N);
    a.spec = reinterpret_cast<float2 *>(const_cast<float *>(sp.spec_in));
    a.frames = sp.frames;
    TFX_STFT_SWITCH(istft_frames_kernel, sp.log2n, unit_grid(a.units), sp.stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    OlaArgs o{};
    o.frames = sp.frames;
    o.win = sp.win;
    o.wl = sp.win_length;
    o.wleft = (N - sp.win_length) / 2;
    o.n_fft = N;
    o.hop = sp.hop;
    o.T = sp.T;
    o.C = sp.C;
    o.L = sp.length;
    o.off = sp.center ? N / 2 : 0;
    o.total = (int64_t)N + (int64_t)sp.hop * (sp.T - 1);
    o.ldy = sp.ldy;
    o.y = sp.y;
    const int64_t nb = (sp.length + SWG - 1) / SWG;
    dim3 grid((unsigned)nb, (unsigned)(sp.C < 65535 ? sp.C : 65535));
    hipLaunchKernelGGL(istft_ola_kernel, grid, dim3(SWG), 0, sp.stream, o);
    return hipGetLastError();
}

}  // namespace tfx
