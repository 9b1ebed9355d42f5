// tfx_fft16k.hip -- overlap-save FIR with one 16384-point FFT per block, for
// long filters (1025 < M <= 8193 taps).
//
// The block of a channel pair is the complex signal z = x_a + i x_b over
// 16384 samples (the taps are real, so the two channels' outputs come back
// separated in the real and imaginary parts).  Convolution: the block starts
// 8192 samples before the tile it produces, and the last 8192 outputs of the
// circular convolution are the tile (M - 1 <= 8192, so none of them wraps).
// Correlation (the FIR adjoint, gx[n] = sum_k h[k] g[n+k]): the block starts
// at the tile, the spectrum is conjugated, and the first 8192 outputs are
// the tile.  Per 8192 x 2 outputs: one forward and one inverse transform
// (2 x 5 N log2 N flops) and the spectrum product, against one forward
// transform per 1025-tap partition in the 4096-point form.
//
// The transform: 16384 = 16 x 16 x 16 x 4.  With n = 1024 a + 64 b + 4 d + e
// and k = k1 + 16 k2 + 256 k3 + 4096 k4, W = e^{-2 pi i / 16384}:
//   pass A  (over a, lane t = 64 b + 4 d + e):  16-point DFT, then * W^(t k1)
//   pass B  (over b, lane (k1, c = 4 d + e)):   16-point DFT, then * W^(16 c k2)
//   pass C  (over d, lane (k1, k2, e)):         16-point DFT, then * W^(256 e k3)
//   pass D  (over e, lane (k1, k2, q)):         four 4-point DFTs (k3 = 4 q + r)
// Each of the 1024 lanes holds 16 values; the three exchanges go through one
// LDS array of 16384 complex values (re and im planes, 128 KB).  Exchange B->C
// and C->D rotate the 4-element groups of a 64-element row by the row index
// k2, which makes every access pattern free of bank conflicts (checked on the
// CPU for 64 banks per wave and 32 per half-wave, and for the 16-byte reads
// of pass D).  The inverse runs the passes backwards with conjugate twiddles
// and ends in pass A's layout.  The spectrum product is done in registers in
// pass D's lane order, in which the tap spectrum is stored: it is computed by
// this same forward transform from the zero-padded taps (fp32) and scaled by
// 1/16384.
#include <hip/hip_runtime.h>

#include "tfx_device.h"
#include "tfx_internal.h"

namespace tfx {

namespace {

constexpr int NB = FFT16_POINTS;  // 16384
constexpr int HOPB = FFT16_HOP;   // 8192 outputs per block
constexpr int WGB = 1024;         // lanes per workgroup
// twiddle regions (float2): TWA [1024][16], TWB [64][16], TWC [4][16]
constexpr int TWA_OFF = 0, TWB_OFF = 16384, TWC_OFF = 16384 + 1024;

// twiddle_row with the table loads in groups of two 16-byte loads (a
// compiler barrier between groups), so at most four twiddles sit in
// registers beside the 32 data values.
template <bool CONJ>
__device__ __forceinline__ void twiddle_row_lean(float (&zr)[16], float (&zi)[16], const float2 *row) {
    const float4 *r4 = reinterpret_cast<const float4 *>(row);
#pragma unroll
    for (int g = 0; g < 8; g += 2) {
        const float4 w0 = r4[g], w1 = r4[g + 1];
        if (g > 0) cmul_tw<CONJ>(zr[2 * g], zi[2 * g], make_float2(w0.x, w0.y));
        cmul_tw<CONJ>(zr[2 * g + 1], zi[2 * g + 1], make_float2(w0.z, w0.w));
        cmul_tw<CONJ>(zr[2 * g + 2], zi[2 * g + 2], make_float2(w1.x, w1.y));
        cmul_tw<CONJ>(zr[2 * g + 3], zi[2 * g + 3], make_float2(w1.z, w1.w));
        asm volatile("" ::: "memory");
    }
}

// Base of the imaginary plane, 64 KB into the LDS array.  The offset is
// passed through an empty asm so it stays a register value: folded into the
// addresses as a constant, offsets past 64 KB do not fit the 16-bit offset
// field of the LDS instructions, and every access to the plane would need
// an address register of its own (about twenty live registers).
__device__ __forceinline__ float *imag_plane(float *lds) {
    int off = NB;
    asm volatile("" : "+s"(off));
    return lds + off;
}

// Forward transform.  In: lane t holds z[1024 a + t] in zr/zi[a].  Out: lane
// L = 64 k1 + 4 k2 + q holds Z[k1 + 16 k2 + 256 (4 q + r) + 4096 k4] in
// zr/zi[4 r + k4].  Ends with every lane past its last LDS read only after
// the caller's next barrier.
__device__ __forceinline__ void fft16k_forward(float (&zr)[16], float (&zi)[16], float *Lr, float *Li,
                                               const float2 *tw, int L) {
    const int k1 = L >> 6, c = L & 63, d = c >> 2, e = c & 3;  // pass B lane
    const int k2 = (L >> 2) & 15, q = L & 3;                    // passes C (e = L & 3) and D
    // pass A
    dft16<-1>(zr, zi);
    twiddle_row_lean<false>(zr, zi, tw + TWA_OFF + 16 * L);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        Lr[1024 * j + L] = zr[j];
        Li[1024 * j + L] = zi[j];
    }
    __syncthreads();
    // pass B
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        zr[b] = Lr[1024 * k1 + 64 * b + c];
        zi[b] = Li[1024 * k1 + 64 * b + c];
    }
    dft16<-1>(zr, zi);
    twiddle_row_lean<false>(zr, zi, tw + TWB_OFF + 16 * c);
    __syncthreads();
    {
        // element (k1, k2 = j, d, e) at 1024 k1 + 64 j + 4 ((d + j) & 15) + e
        const int w0 = 1024 * k1 + 4 * d + e;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int ad = (j >= 16 - d ? w0 - 64 : w0) + 68 * j;
            Lr[ad] = zr[j];
            Li[ad] = zi[j];
        }
    }
    __syncthreads();
    // pass C: lane (k1, k2, e); element (k1, k2, j, e) at rowc + 4 ((j + k2) & 15)
    const int ec = L & 3, rc = 1024 * k1 + 64 * k2 + 4 * k2 + ec;
#pragma unroll
    for (int j = 0; j < 16; ++j) {  // j = d
        const int ad = (j >= 16 - k2 ? rc - 64 : rc) + 4 * j;
        zr[j] = Lr[ad];
        zi[j] = Li[ad];
    }
    dft16<-1>(zr, zi);
    twiddle_row_lean<false>(zr, zi, tw + TWC_OFF + 16 * ec);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) {  // j = k3
        const int ad = (j >= 16 - k2 ? rc - 64 : rc) + 4 * j;
        Lr[ad] = zr[j];
        Li[ad] = zi[j];
    }
    __syncthreads();
    // pass D: lane (k1, k2, q) reads (k3 = 4 q + r, e = 0..3) as 16-byte groups
    const int rowd = 1024 * k1 + 64 * k2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ad = rowd + 4 * ((4 * q + r + k2) & 15);
        const float4 vr = *reinterpret_cast<const float4 *>(Lr + ad);
        const float4 vi = *reinterpret_cast<const float4 *>(Li + ad);
        zr[4 * r] = vr.x; zr[4 * r + 1] = vr.y; zr[4 * r + 2] = vr.z; zr[4 * r + 3] = vr.w;
        zi[4 * r] = vi.x; zi[4 * r + 1] = vi.y; zi[4 * r + 2] = vi.z; zi[4 * r + 3] = vi.w;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        dft4<-1>(zr[4 * r], zi[4 * r], zr[4 * r + 1], zi[4 * r + 1], zr[4 * r + 2], zi[4 * r + 2], zr[4 * r + 3],
                 zi[4 * r + 3]);
}

// Inverse of fft16k_forward without the 1/16384 factor: from its output
// layout back to its input layout.  Begins with a barrier before its first
// LDS write.
__device__ __forceinline__ void fft16k_inverse(float (&zr)[16], float (&zi)[16], float *Lr, float *Li,
                                               const float2 *tw, int L) {
    const int k1 = L >> 6, c = L & 63, d = c >> 2, e = c & 3;
    const int k2 = (L >> 2) & 15, q = L & 3;
    const int rowd = 1024 * k1 + 64 * k2;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        dft4<1>(zr[4 * r], zi[4 * r], zr[4 * r + 1], zi[4 * r + 1], zr[4 * r + 2], zi[4 * r + 2], zr[4 * r + 3],
                zi[4 * r + 3]);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ad = rowd + 4 * ((4 * q + r + k2) & 15);
        *reinterpret_cast<float4 *>(Lr + ad) = make_float4(zr[4 * r], zr[4 * r + 1], zr[4 * r + 2], zr[4 * r + 3]);
        *reinterpret_cast<float4 *>(Li + ad) = make_float4(zi[4 * r], zi[4 * r + 1], zi[4 * r + 2], zi[4 * r + 3]);
    }
    __syncthreads();
    // pass C inverse: lane (k1, k2, e) over k3
    const int ec = L & 3, rc = rowd + 4 * k2 + ec;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int ad = (j >= 16 - k2 ? rc - 64 : rc) + 4 * j;
        zr[j] = Lr[ad];
        zi[j] = Li[ad];
    }
    twiddle_row_lean<true>(zr, zi, tw + TWC_OFF + 16 * ec);
    dft16<1>(zr, zi);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) {  // j = d
        const int ad = (j >= 16 - k2 ? rc - 64 : rc) + 4 * j;
        Lr[ad] = zr[j];
        Li[ad] = zi[j];
    }
    __syncthreads();
    // pass B inverse: lane (k1, c) over k2
    {
        const int w0 = 1024 * k1 + 4 * d + e;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int ad = (j >= 16 - d ? w0 - 64 : w0) + 68 * j;
            zr[j] = Lr[ad];
            zi[j] = Li[ad];
        }
    }
    twiddle_row_lean<true>(zr, zi, tw + TWB_OFF + 16 * c);
    dft16<1>(zr, zi);
    __syncthreads();
#pragma unroll
    for (int b = 0; b < 16; ++b) {
        Lr[1024 * k1 + 64 * b + c] = zr[b];
        Li[1024 * k1 + 64 * b + c] = zi[b];
    }
    __syncthreads();
    // pass A inverse: lane t over k1
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        zr[j] = Lr[1024 * j + L];
        zi[j] = Li[1024 * j + L];
    }
    twiddle_row_lean<true>(zr, zi, tw + TWA_OFF + 16 * L);
    dft16<1>(zr, zi);
}

struct F16Args {
    const float *x;
    float *y;
    int64_t C, N, ldx, ldy;
    int64_t ntiles, nblocks;
    const float2 *tw;
    const float2 *hs;   // [1024][16] tap spectrum / 16384 in pass D's lane order
    const float *hist;  // streaming: [C][hlen] inputs before the block (convolution only), or null
    int64_t hlen;
    int32_t correlate;
};

// Block id -> (pair, tile), tile-major within a pair; the blocks of one XCD
// (hardware id i runs on XCD i mod 8) take one contiguous range of logical
// blocks, so neighbouring tiles, which share half their input, are read
// through the same L2.
__device__ __forceinline__ int64_t xcd_block(int64_t i, int64_t nb) {
    const int64_t x = i & 7, per = nb >> 3, rem = nb & 7;
    return x * per + (x < rem ? x : rem) + (i >> 3);
}

__global__ __launch_bounds__(WGB, 1) void fir16k_kernel(F16Args a) {
    __shared__ float lds[2 * NB];
    float *Lr = lds, *Li = imag_plane(lds);
    const int t = threadIdx.x;
    const int64_t lb = xcd_block(blockIdx.x, a.nblocks);
    const int64_t pair = lb / a.ntiles, tile = lb - pair * a.ntiles;
    const int64_t ca = 2 * pair, cb = ca + 1;
    const bool has_b = cb < a.C;
    const float *xa = a.x + ca * a.ldx, *xb = has_b ? a.x + cb * a.ldx : nullptr;
    const int64_t n0 = tile * HOPB;
    const int64_t base = a.correlate ? n0 : n0 - HOPB;
    float zr[16], zi[16];
    if (base >= 0 && base + NB <= a.N) {
        const float *pa = xa + base + t;
#pragma unroll
        for (int q = 0; q < 16; ++q) zr[q] = pa[1024 * q];
        if (has_b) {
            const float *pb = xb + base + t;
#pragma unroll
            for (int q = 0; q < 16; ++q) zi[q] = pb[1024 * q];
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) zi[q] = 0.f;
        }
    } else {
        const float *ha = a.hist ? a.hist + ca * a.hlen : nullptr;
        const float *hb = (a.hist && has_b) ? a.hist + cb * a.hlen : nullptr;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int64_t n = base + 1024 * q + t;
            const bool in = n >= 0 && n < a.N;
            const bool inh = n < 0 && n >= -a.hlen;
            zr[q] = in ? xa[n] : ((inh && ha) ? ha[a.hlen + n] : 0.f);
            zi[q] = (in && has_b) ? xb[n] : ((inh && hb) ? hb[a.hlen + n] : 0.f);
        }
    }
    fft16k_forward(zr, zi, Lr, Li, a.tw, t);
    {
        const float sg = a.correlate ? -1.f : 1.f;
        const float4 *h4 = reinterpret_cast<const float4 *>(a.hs + 16 * t);
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
            const float4 p = h4[2 * g4], r = h4[2 * g4 + 1];
            const float2 w[4] = {make_float2(p.x, sg * p.y), make_float2(p.z, sg * p.w), make_float2(r.x, sg * r.y),
                                 make_float2(r.z, sg * r.w)};
#pragma unroll
            for (int u = 0; u < 4; ++u) cmul_tw<false>(zr[4 * g4 + u], zi[4 * g4 + u], w[u]);
            asm volatile("" ::: "memory");  // at most four bins' spectra in registers at a time
        }
    }
    fft16k_inverse(zr, zi, Lr, Li, a.tw, t);
    // rows 8..15 of the block (convolution) or 0..7 (correlation) are the tile
    const int q0 = a.correlate ? 0 : 8;
    float *ya = a.y + ca * a.ldy, *yb = has_b ? a.y + cb * a.ldy : nullptr;
    if (n0 + HOPB <= a.N) {
#pragma unroll
        for (int q = 0; q < 8; ++q) ya[n0 + 1024 * q + t] = zr[q0 + q];
        if (has_b) {
#pragma unroll
            for (int q = 0; q < 8; ++q) yb[n0 + 1024 * q + t] = zi[q0 + q];
        }
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t n = n0 + 1024 * q + t;
            if (n < a.N) {
                ya[n] = zr[q0 + q];
                if (has_b) yb[n] = zi[q0 + q];
            }
        }
    }
}

// Twiddle tables in fp32 from sincospi of exact arguments (2 m / 16384):
//   TWA[t][k] = W^(t k), TWB[c][k] = W^(16 c k), TWC[e][k] = W^(256 e k).
__global__ void fft16k_twiddle_kernel(float2 *tw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int m;
    if (i < TWB_OFF) m = ((i >> 4) * (i & 15)) & (NB - 1);
    else if (i < TWC_OFF) m = (16 * ((i - TWB_OFF) >> 4) * (i & 15)) & (NB - 1);
    else if (i < TWC_OFF + 64) m = (256 * ((i - TWC_OFF) >> 4) * (i & 15)) & (NB - 1);
    else return;
    float s, c;
    sincospif(-2.0f * (float)m / (float)NB, &s, &c);
    tw[i] = make_float2(c, s);
}

// Tap spectrum: the forward transform of h (zero-padded to 16384) in pass
// D's lane order, times 1/16384 (exact).  One workgroup.
__global__ __launch_bounds__(WGB, 1) void fft16k_spectrum_kernel(const float *h, int32_t M, const float2 *tw,
                                                                 float2 *hs) {
    __shared__ float lds[2 * NB];
    const int t = threadIdx.x;
    float zr[16], zi[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int n = 1024 * q + t;
        zr[q] = n < M ? h[n] : 0.f;
        zi[q] = 0.f;
    }
    fft16k_forward(zr, zi, lds, imag_plane(lds), tw, t);
    const float sc = 1.0f / (float)NB;
#pragma unroll
    for (int j = 0; j < 16; ++j) hs[16 * t + j] = make_float2(zr[j] * sc, zi[j] * sc);
}

}  // namespace

size_t fft16k_table_bytes() { return (size_t)(TWC_OFF + 64) * sizeof(float2) + (size_t)NB * sizeof(float2); }

hipError_t launch_fft16k_prepare(const float *h, int32_t M, void *tab, hipStream_t st) {
    float2 *tw = static_cast<float2 *>(tab);
    float2 *hs = tw + (TWC_OFF + 64);
    hipLaunchKernelGGL(fft16k_twiddle_kernel, dim3((TWC_OFF + 64 + 255) / 256), dim3(256), 0, st, tw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fft16k_spectrum_kernel, dim3(1), dim3(WGB), 0, st, h, M, static_cast<const float2 *>(tw), hs);
    return hipGetLastError();
}

hipError_t launch_fft16k(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy, int32_t M,
                         const void *tab, bool correlate, const float *hist, hipStream_t st) {
    if (N == 0) return hipSuccess;
    F16Args a{};
    a.x = x;
    a.y = y;
    a.C = C;
    a.N = N;
    a.ldx = ldx;
    a.ldy = ldy;
    a.ntiles = (N + HOPB - 1) / HOPB;
    a.nblocks = (C + 1) / 2 * a.ntiles;
    a.tw = static_cast<const float2 *>(tab);
    a.hs = a.tw + (TWC_OFF + 64);
    a.hist = (!correlate && M > 1) ? hist : nullptr;
    a.hlen = M > 1 ? M - 1 : 0;
    a.correlate = correlate ? 1 : 0;
    hipLaunchKernelGGL(fir16k_kernel, dim3((unsigned)a.nblocks), dim3(WGB), 0, st, a);
    return hipGetLastError();
}

}  // namespace tfx
