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
//   pass A  (over a, lane L = 64 b + 4 d + e):  16-point DFT, then * W^(L k1)
//   pass B  (over b, lane (k1, c = 4 d + e)):   16-point DFT, then * W^(16 c k2)
//   pass C  (over d, lane (k1, k2, e)):         16-point DFT, then * W^(256 e k3)
//   pass D  (over e, lane (k1, k2, q)):         four 4-point DFTs (k3 = 4 q + r)
// The 1024 lanes L are virtual: thread t of a 512-thread workgroup runs lanes
// t and t + 512, each with 16 values, so a block needs 64 data registers a
// thread and two blocks share a CU (one overlapping the other's loads,
// barriers and LDS traffic).  The three exchanges go through one LDS plane of
// 16384 floats (64 KB), the real parts first, then the imaginary parts.
// Exchanges B->C and C->D rotate the 4-element groups of a 64-element row by
// the row index k2, which makes every access pattern free of bank conflicts
// (checked on the CPU for 64 banks per wave and 32 per half-wave, and for the
// 16-byte reads of pass D; the lanes of a wave are 64 consecutive virtual
// lanes either way).  The inverse runs the passes backwards with conjugate
// twiddles and ends in pass A's layout.  The spectrum product is done in
// registers in pass D's lane order, in which the tap spectrum is stored: it is
// computed by this same forward transform from the zero-padded taps (fp32)
// and scaled by 1/16384.
#include <hip/hip_runtime.h>

#include "tfx_device.h"
#include "tfx_internal.h"

namespace tfx {

namespace {

constexpr int NB = FFT16_POINTS;  // 16384
constexpr int HOPB = FFT16_HOP;   // 8192 outputs per block
#ifndef TFX_FFT16_NV
#define TFX_FFT16_NV 2
#endif
constexpr int NV = TFX_FFT16_NV;  // virtual lanes per thread: t + VS v
constexpr int WGB = 1024 / NV;    // threads per workgroup
constexpr int VS = WGB;           // virtual-lane stride

// Twiddle tables (float2, rows of 16 entries padded to TWS = 18 so that the
// 16-byte reads of 16 lanes from 16 different rows hit 64 different banks):
//   TWB[c][k] = W^(16 c k) (c < 64), TWC[e][k] = W^(256 e k) (e < 4),
//   TLO[c][k] = W^(c k) (c < 16).
// Pass A's W^(L k) is formed as TWB[L >> 4][k] TLO[L & 15][k].  The whole set
// (12 KB) is copied into LDS by each workgroup: read from global memory at
// every pass, the twiddle loads' latency took some 40 % of the kernel's time.
constexpr int TWS = 18;
constexpr int TWB_ROW = 0, TWC_ROW = 64, TLO_ROW = 68, TW_ROWS = 84;
constexpr int TW_FLOAT2 = TW_ROWS * TWS;  // 1512

// Multiplies the lane's 16 values by a row of the twiddle table (or its
// conjugate), the row's 16-byte pieces read from LDS as they are used.
template <bool CONJ>
__device__ __forceinline__ void twiddle_lds(float (&zr)[16], float (&zi)[16], const float2 *row) {
    const float4 *r4 = reinterpret_cast<const float4 *>(row);
#pragma unroll
    for (int g = 0; g < 8; ++g) {
        const float4 w = r4[g];
        if (g > 0) cmul_tw<CONJ>(zr[2 * g], zi[2 * g], make_float2(w.x, w.y));
        cmul_tw<CONJ>(zr[2 * g + 1], zi[2 * g + 1], make_float2(w.z, w.w));
    }
}

// Pass A's row W^(L k) = TWB[L >> 4][k] TLO[L & 15][k], applied as its two
// factors one after the other.
template <bool CONJ>
__device__ __forceinline__ void twiddle_lds_a(float (&zr)[16], float (&zi)[16], const float2 *tw, int L) {
    twiddle_lds<CONJ>(zr, zi, tw + (TWB_ROW + (L >> 4)) * TWS);
    twiddle_lds<CONJ>(zr, zi, tw + (TLO_ROW + (L & 15)) * TWS);
}

// Copies the twiddle tables into the workgroup's LDS copy (every load issued
// before the first store; the caller passes a barrier before the first use).
__device__ __forceinline__ void tw_stage(float2 *twl, const float2 *tw, int t) {
    constexpr int N4 = TW_FLOAT2 / 2, R = (N4 + WGB - 1) / WGB;
    const float4 *src = reinterpret_cast<const float4 *>(tw);
    float4 *dst = reinterpret_cast<float4 *>(twl);
    float4 w[R];
#pragma unroll
    for (int r = 0; r < R; ++r) w[r] = src[min(t + r * WGB, N4 - 1)];
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (t + r * WGB < N4) dst[t + r * WGB] = w[r];
}

// Lane coordinates of virtual lane L = t + 512 v.
struct Lane {
    int L, k1, c, d, e, k2, q;
    __device__ __forceinline__ explicit Lane(int l)
        : L(l), k1(l >> 6), c(l & 63), d((l & 63) >> 2), e(l & 3), k2((l >> 2) & 15), q(l & 3) {}
};

// Address maps of the exchanges (element j of the lane):
//   A->B  write 1024 j + L                      read 1024 k1 + 64 j + c
//   B->C  write rot64(1024 k1 + 4 d + e, j, d)   read rot64(rc, j, k2) (k2 = j)
//   C->D  write rot64(rc, j, k2) (k3 = j)        read 16-byte groups in pass D
// with rot64(base, j, r) = base + 68 j - 64 [j >= 16 - r] (row j of 64
// elements, the group rotated by r) and rc = 1024 k1 + 68 k2 + e.
// A Map holds the two row bases (base and base - 64) as byte offsets the
// compiler cannot see through, so an access costs one select and its step
// is the LDS instruction's immediate offset.
struct Map {
    int o0, o1, r, step;
    __device__ __forceinline__ Map(int base, int step_, int r_) : r(r_), step(step_) {
        o0 = 4 * base;
        o1 = 4 * (base - 64);
        asm volatile("" : "+v"(o0), "+v"(o1));
    }
    __device__ __forceinline__ float *at(float *P, int j) const {
        return reinterpret_cast<float *>(reinterpret_cast<char *>(P) + (j >= 16 - r ? o1 : o0) + 4 * step * j);
    }
};
__device__ __forceinline__ Map map_a(const Lane &l) { return Map(l.L, 1024, 0); }
__device__ __forceinline__ Map map_b(const Lane &l) { return Map(1024 * l.k1 + l.c, 64, 0); }
__device__ __forceinline__ Map rot_w(const Lane &l) { return Map(1024 * l.k1 + 4 * l.d + l.e, 68, l.d); }
__device__ __forceinline__ Map rot_c(const Lane &l) { return Map(1024 * l.k1 + 68 * l.k2 + l.e, 4, l.k2); }

// A copy of the thread index the compiler cannot see through: addresses
// derived from it are recomputed where they are used instead of being kept
// in registers from one phase of an exchange to the next.
__device__ __forceinline__ int opaque(int t) {
    asm volatile("" : "+v"(t));
    return t;
}

// One LDS exchange of both virtual lanes' 16 values through the plane P:
// value j of lane v goes to P[W(lane, j)] and comes back from P[R(lane, j)],
// the real parts first.  The caller has passed a barrier since the last read
// of P; the exchange ends after its own last read (no barrier).
template <class WA, class RA>
__device__ __forceinline__ void exchange(float (&zr)[NV][16], float (&zi)[NV][16], float *P, int t, WA wad,
                                         RA rad) {
    {
        const int u = opaque(t);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const Map m = wad(Lane(u + VS * v));
#pragma unroll
            for (int j = 0; j < 16; ++j) *m.at(P, j) = zr[v][j];
        }
    }
    __syncthreads();
    {
        const int u = opaque(t);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const Map m = rad(Lane(u + VS * v));
#pragma unroll
            for (int j = 0; j < 16; ++j) zr[v][j] = *m.at(P, j);
        }
    }
    __syncthreads();
    {
        const int u = opaque(t);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const Map m = wad(Lane(u + VS * v));
#pragma unroll
            for (int j = 0; j < 16; ++j) *m.at(P, j) = zi[v][j];
        }
    }
    __syncthreads();
    {
        const int u = opaque(t);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const Map m = rad(Lane(u + VS * v));
#pragma unroll
            for (int j = 0; j < 16; ++j) zi[v][j] = *m.at(P, j);
        }
    }
}

// Pass D's side of the exchange C <-> D: lane (k1, k2, q) owns the 16-byte
// groups k3 = 4 q + r (r = 0..3) of row 1024 k1 + 64 k2, rotated by k2 like
// pass C's accesses; one plane (z = real or imaginary parts) at a time.
__device__ __forceinline__ int group_addr(const Lane &l, int r) {
    return 1024 * l.k1 + 64 * l.k2 + 4 * ((4 * l.q + r + l.k2) & 15);
}
__device__ __forceinline__ void load_groups(float (&z)[NV][16], const float *P, int t) {
    const int u = opaque(t);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const Lane l(u + VS * v);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float4 w = *reinterpret_cast<const float4 *>(P + group_addr(l, r));
            z[v][4 * r] = w.x;
            z[v][4 * r + 1] = w.y;
            z[v][4 * r + 2] = w.z;
            z[v][4 * r + 3] = w.w;
        }
    }
}
__device__ __forceinline__ void store_groups(const float (&z)[NV][16], float *P, int t) {
    const int u = opaque(t);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const Lane l(u + VS * v);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            *reinterpret_cast<float4 *>(P + group_addr(l, r)) =
                make_float4(z[v][4 * r], z[v][4 * r + 1], z[v][4 * r + 2], z[v][4 * r + 3]);
    }
}
// Pass C's side: element j of lane (k1, k2, e) at rot_c.
__device__ __forceinline__ void store_rot_c(const float (&z)[NV][16], float *P, int t) {
    const int u = opaque(t);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const Map m = rot_c(Lane(u + VS * v));
#pragma unroll
        for (int j = 0; j < 16; ++j) *m.at(P, j) = z[v][j];
    }
}
__device__ __forceinline__ void load_rot_c(float (&z)[NV][16], float *P, int t) {
    const int u = opaque(t);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const Map m = rot_c(Lane(u + VS * v));
#pragma unroll
        for (int j = 0; j < 16; ++j) z[v][j] = *m.at(P, j);
    }
}

// Forward transform.  In: virtual lane L holds z[1024 a + L] in zr/zi[v][a].
// Out: virtual lane L = 64 k1 + 4 k2 + q holds
// Z[k1 + 16 k2 + 256 (4 q + r) + 4096 k4] in zr/zi[v][4 r + k4].  The caller
// has passed a barrier since the last read of P; ends after the last read.
// (Each pass derives its lane coordinates afresh from the thread index.)
__device__ __forceinline__ void fft16k_forward(float (&zr)[NV][16], float (&zi)[NV][16], float *P, const float2 *tw,
                                               int t) {
    {  // pass A
        const int u = opaque(t);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            dft16<-1>(zr[v], zi[v]);
            twiddle_lds_a<false>(zr[v], zi[v], tw, u + VS * v);
        }
    }
    exchange(zr, zi, P, t, map_a, map_b);
    {  // pass B
        const int u = opaque(t);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            dft16<-1>(zr[v], zi[v]);
            twiddle_lds<false>(zr[v], zi[v], tw + (TWB_ROW + ((u + VS * v) & 63)) * TWS);
        }
    }
    __syncthreads();
    exchange(zr, zi, P, t, rot_w, rot_c);
    {  // pass C
        const int u = opaque(t);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            dft16<-1>(zr[v], zi[v]);
            twiddle_lds<false>(zr[v], zi[v], tw + (TWC_ROW + (u & 3)) * TWS);
        }
    }
    // exchange C -> D, pass D reading (k3 = 4 q + r, e = 0..3) as 16-byte groups
    __syncthreads();
    store_rot_c(zr, P, t);
    __syncthreads();
    load_groups(zr, P, t);
    __syncthreads();
    store_rot_c(zi, P, t);
    __syncthreads();
    load_groups(zi, P, t);
    // pass D
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            dft4<-1>(zr[v][4 * r], zi[v][4 * r], zr[v][4 * r + 1], zi[v][4 * r + 1], zr[v][4 * r + 2],
                     zi[v][4 * r + 2], zr[v][4 * r + 3], zi[v][4 * r + 3]);
}

// Inverse of fft16k_forward without the 1/16384 factor: from its output
// layout back to its input layout, lane v's 16 values passed to out(zr, zi, v)
// once final.  Begins with a barrier before its first
// LDS write; ends after its last read.
template <class OUT>
__device__ __forceinline__ void fft16k_inverse(float (&zr)[NV][16], float (&zi)[NV][16], float *P, const float2 *tw,
                                               int t, OUT out) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            dft4<1>(zr[v][4 * r], zi[v][4 * r], zr[v][4 * r + 1], zi[v][4 * r + 1], zr[v][4 * r + 2],
                    zi[v][4 * r + 2], zr[v][4 * r + 3], zi[v][4 * r + 3]);
    // exchange D -> C: 16-byte group writes, reads in pass C's order
    __syncthreads();
    store_groups(zr, P, t);
    __syncthreads();
    load_rot_c(zr, P, t);
    __syncthreads();
    store_groups(zi, P, t);
    __syncthreads();
    load_rot_c(zi, P, t);
    {  // pass C inverse: lane (k1, k2, e) over k3
        const int u = opaque(t);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            twiddle_lds<true>(zr[v], zi[v], tw + (TWC_ROW + (u & 3)) * TWS);
            dft16<1>(zr[v], zi[v]);
        }
    }
    __syncthreads();
    exchange(zr, zi, P, t, rot_c, rot_w);
    {  // pass B inverse: lane (k1, c) over k2
        const int u = opaque(t);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            twiddle_lds<true>(zr[v], zi[v], tw + (TWB_ROW + ((u + VS * v) & 63)) * TWS);
            dft16<1>(zr[v], zi[v]);
        }
    }
    __syncthreads();
    exchange(zr, zi, P, t, map_b, map_a);
    {  // pass A inverse: lane L over k1; each lane's values handed to out
       // as soon as they are final (their registers free for the next lane)
        const int u = opaque(t);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            twiddle_lds_a<true>(zr[v], zi[v], tw, u + VS * v);
            dft16<1>(zr[v], zi[v]);
            out(zr[v], zi[v], v);
        }
    }
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

// Stores rows Q0 .. Q0 + 7 of virtual lane L's values (samples n0 + 1024 q +
// L) to ya and, when yb is set, yb, up to N.
template <int Q0>
__device__ __forceinline__ void store_rows(const float (&zr)[16], const float (&zi)[16], float *ya, float *yb,
                                           int64_t n0, int64_t N, int L) {
    if (n0 + HOPB <= N) {
#pragma unroll
        for (int q = 0; q < 8; ++q) ya[n0 + 1024 * q + L] = zr[Q0 + q];
        if (yb) {
#pragma unroll
            for (int q = 0; q < 8; ++q) yb[n0 + 1024 * q + L] = zi[Q0 + q];
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t n = n0 + 1024 * q + L;
        if (n < N) {
            ya[n] = zr[Q0 + q];
            if (yb) yb[n] = zi[Q0 + q];
        }
    }
}

__global__ __launch_bounds__(WGB, 8 / NV) void fir16k_kernel(F16Args a) {
    __shared__ __align__(16) float P[NB];
    __shared__ __align__(16) float2 twl[TW_FLOAT2];
    const int t = threadIdx.x;
    tw_stage(twl, a.tw, t);
    const int64_t lb = xcd_block(blockIdx.x, a.nblocks);
    const int64_t pair = lb / a.ntiles, tile = lb - pair * a.ntiles;
    const int64_t ca = 2 * pair, cb = ca + 1;
    const bool has_b = cb < a.C;
    const float *xa = a.x + ca * a.ldx, *xb = has_b ? a.x + cb * a.ldx : nullptr;
    const int64_t n0 = tile * HOPB;
    const int64_t base = a.correlate ? n0 : n0 - HOPB;
    // virtual lane L = t + 512 v holds z[1024 q + L] in [v][q]
    float zr[NV][16], zi[NV][16];
    if (base >= 0 && base + NB <= a.N) {
        const float *pa = xa + base + t;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int q = 0; q < 16; ++q) zr[v][q] = pa[1024 * q + VS * v];
        if (has_b) {
            const float *pb = xb + base + t;
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int q = 0; q < 16; ++q) zi[v][q] = pb[1024 * q + VS * v];
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int q = 0; q < 16; ++q) zi[v][q] = 0.f;
        }
    } else {
        const float *ha = a.hist ? a.hist + ca * a.hlen : nullptr;
        const float *hb = (a.hist && has_b) ? a.hist + cb * a.hlen : nullptr;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int64_t n = base + 1024 * q + VS * v + t;
                const bool in = n >= 0 && n < a.N;
                const bool inh = n < 0 && n >= -a.hlen;
                zr[v][q] = in ? xa[n] : ((inh && ha) ? ha[a.hlen + n] : 0.f);
                zi[v][q] = (in && has_b) ? xb[n] : ((inh && hb) ? hb[a.hlen + n] : 0.f);
            }
    }
    __syncthreads();  // the twiddle tables
    fft16k_forward(zr, zi, P, twl, t);
    __builtin_amdgcn_sched_barrier(0);
    {
        const float sg = a.correlate ? -1.f : 1.f;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            // eight bins at a time: their 4 loads issued together, the next
            // ones held back by a scheduling fence (registers)
#pragma unroll
            for (int hf = 0; hf < 2; ++hf) {
                // (the lane index laundered per group, and the products pinned
                // below: otherwise all 16 loads are issued first and hold 64
                // registers)
                const float4 *h4 = reinterpret_cast<const float4 *>(a.hs + 16 * (opaque(t) + VS * v));
                float4 hq[4];
#pragma unroll
                for (int g = 0; g < 4; ++g) hq[g] = h4[4 * hf + g];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int b = 8 * hf + 2 * g;
                    cmul_tw<false>(zr[v][b], zi[v][b], make_float2(hq[g].x, sg * hq[g].y));
                    cmul_tw<false>(zr[v][b + 1], zi[v][b + 1], make_float2(hq[g].z, sg * hq[g].w));
                    // the products made here, before the next group's loads
                    asm volatile("" : "+v"(zr[v][b]), "+v"(zi[v][b]), "+v"(zr[v][b + 1]), "+v"(zi[v][b + 1]));
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    // rows 8..15 of the block (convolution) or 0..7 (correlation) are the tile
    // (two paths with constant row indices: a run-time index into the data
    // arrays would move them to scratch memory)
    float *ya = a.y + ca * a.ldy, *yb = has_b ? a.y + cb * a.ldy : nullptr;
    fft16k_inverse(zr, zi, P, twl, t, [&](const float (&r)[16], const float (&i)[16], int v) {
        if (a.correlate)
            store_rows<0>(r, i, ya, yb, n0, a.N, t + VS * v);
        else
            store_rows<8>(r, i, ya, yb, n0, a.N, t + VS * v);
    });
}

// Twiddle tables in fp32 from sincospi of exact arguments (2 m / 16384), in
// the padded row layout above (pad entries zero).
__global__ void fft16k_twiddle_kernel(float2 *tw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= TW_FLOAT2) return;
    const int row = i / TWS, k = i % TWS;
    if (k >= 16) {
        tw[i] = make_float2(0.f, 0.f);
        return;
    }
    int m;
    if (row < TWC_ROW) m = (16 * (row - TWB_ROW) * k) & (NB - 1);
    else if (row < TLO_ROW) m = (256 * (row - TWC_ROW) * k) & (NB - 1);
    else m = ((row - TLO_ROW) * k) & (NB - 1);
    float s, c;
    sincospif(-2.0f * (float)m / (float)NB, &s, &c);
    tw[i] = make_float2(c, s);
}

// Tap spectrum: the forward transform of h (zero-padded to 16384) in pass
// D's lane order, times 1/16384 (exact).  One workgroup.
__global__ __launch_bounds__(WGB, 1) void fft16k_spectrum_kernel(const float *h, int32_t M, const float2 *tw,
                                                                 float2 *hs) {
    __shared__ __align__(16) float P[NB];
    __shared__ __align__(16) float2 twl[TW_FLOAT2];
    const int t = threadIdx.x;
    tw_stage(twl, tw, t);
    float zr[NV][16], zi[NV][16];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int n = 1024 * q + VS * v + t;
            zr[v][q] = n < M ? h[n] : 0.f;
            zi[v][q] = 0.f;
        }
    __syncthreads();  // the twiddle tables
    fft16k_forward(zr, zi, P, twl, t);
    const float sc = 1.0f / (float)NB;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int j = 0; j < 16; ++j) hs[16 * (t + VS * v) + j] = make_float2(zr[v][j] * sc, zi[v][j] * sc);
}

}  // namespace

size_t fft16k_table_bytes() { return (size_t)TW_FLOAT2 * sizeof(float2) + (size_t)NB * sizeof(float2); }

hipError_t launch_fft16k_prepare(const float *h, int32_t M, void *tab, hipStream_t st) {
    float2 *tw = static_cast<float2 *>(tab);
    float2 *hs = tw + TW_FLOAT2;
    hipLaunchKernelGGL(fft16k_twiddle_kernel, dim3((TW_FLOAT2 + 255) / 256), dim3(256), 0, st, tw);
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
    a.hs = a.tw + TW_FLOAT2;
    a.hist = (!correlate && M > 1) ? hist : nullptr;
    a.hlen = M > 1 ? M - 1 : 0;
    a.correlate = correlate ? 1 : 0;
    hipLaunchKernelGGL(fir16k_kernel, dim3((unsigned)a.nblocks), dim3(WGB), 0, st, a);
    return hipGetLastError();
}

}  // namespace tfx
