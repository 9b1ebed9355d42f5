// tfx_device.h -- device building blocks shared by the forward (tfx_chain.hip)
// and adjoint (tfx_backward.hip) kernels: look-back records, DPP moves, the
// 4096-point FFT, and the chunk-carry engine of the linear-recurrence scan.
#pragma once
#include <hip/hip_runtime.h>

#include "tfx_internal.h"

namespace tfx {

// ------------------------------------------------------------------ records
// Look-back records.  Every (channel, tile, section) owns 4 64-bit words: the
// tile aggregate (2 floats) and the inclusive prefix (2 floats), each word
// (epoch << 32) | float bits, written and read with relaxed agent-scope
// atomics: every word validates itself, so no acquire/release fence is
// needed.  (Each XCD of the chip has its own L2, and an agent-scope fence
// writes back or invalidates the whole L2; fences in a spin loop would thrash
// it for every tile on the XCD.)  The cross-tile values are fp32 even for
// sections carried in fp64 inside the tile: across tiles the state is damped
// by PhiT = A^3072, so rounding there accumulates over a few tiles only.  The
// epoch advances once per run (block 0 of the filter-kernel variant that does
// not match the workspace's high-Q word advances it, stream-ordered against
// the variant that does the work), so a run never clears the words the
// previous run left and needs no memset.
constexpr uint32_t EPOCH_MASK = 0x3FFFFFFFu;
constexpr int64_t SPIN_MAX = int64_t(1) << 22;

__device__ __forceinline__ uint64_t ld_word(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_word(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_epoch(const uint32_t *hdr, int word) {
    return __hip_atomic_load(hdr + word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Run by the filter-kernel variant that does not match the high-Q word
// before it exits: its block 0 advances the look-back epoch for the next run.
__device__ __forceinline__ void advance_epoch(uint32_t *hdr) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t ne = (hdr[HDR_EPOCH] + 1u) & EPOCH_MASK;
        hdr[HDR_EPOCH] = ne == 0u ? 1u : ne;
    }
}

// Logical block id of block b for L2 reuse across the chip's 8 XCDs, which
// take block ids round robin (block b runs on XCD b % 8) and each have their
// own L2.  Within every window of 8 K block ids (K = 2^ks), XCD x takes the
// K consecutive logical ids x K .. x K + K - 1, so neighbouring tiles of a
// channel pair, whose input blocks overlap, read through one L2; ks = 0 and
// the last, partial window keep b.  The look-back stays free of deadlock
// while an XCD can hold K blocks at once: if every resident block waited,
// the lowest unfinished logical tile would not be resident, so its XCD
// would be full of unfinished blocks dispatched before it, all from its own
// window (earlier windows' blocks have lower logical ids) -- at most K - 1.
// (readfirstlane keeps the result in scalar registers.)
__device__ __forceinline__ uint32_t xcd_order(uint32_t b, uint32_t nblocks, uint32_t ks) {
    const uint32_t W = 8u << ks, w0 = b & ~(W - 1u), r = b & (W - 1u);
    return __builtin_amdgcn_readfirstlane(w0 + W > nblocks ? b : w0 + ((r & 7u) << ks) + (r >> 3));
}

// Lanes 0, 1 of a wave store the tagged pair (f0, f1) (wave-uniform) into
// slot 0 (aggregate) or 1 (inclusive prefix) of record r.
__device__ __forceinline__ void publish(uint64_t *recs, int64_t r, int slot, uint32_t epoch, float f0, float f1,
                                       int lane) {
    if (lane < 2)
        st_word(&recs[r * REC_WORDS + slot * 2 + lane],
                ((uint64_t)epoch << 32) | (uint32_t)__float_as_uint(lane == 0 ? f0 : f1));
}

// Decodes the 4 words w of a record.  Returns 2 when the inclusive prefix is
// out (f0, f1 = prefix), 1 when only the aggregate is (f0, f1 = aggregate),
// else 0.
__device__ __forceinline__ int decode_record(const uint64_t (&w)[4], uint32_t epoch, float &f0, float &f1) {
    const uint64_t e = epoch;
    const bool inc = (w[2] >> 32) == e && (w[3] >> 32) == e;
    const bool agg = (w[0] >> 32) == e && (w[1] >> 32) == e;
    f0 = __uint_as_float((uint32_t)(inc ? w[2] : w[0]));
    f1 = __uint_as_float((uint32_t)(inc ? w[3] : w[1]));
    return inc ? 2 : (agg ? 1 : 0);
}

// ---------------------------------------------------------------- lane moves
// DPP lane move of a float / double (dpp_ctrl CTRL, rows ROWS written, lanes
// reading outside their row get 0).
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xFFFFFFFF), CTRL, ROWS, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int DPP_ROW_SHR = 0x110;    // + n: lane - n within a row of 16
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane - 1 across the wave
constexpr int DPP_ROW_BCAST15 = 0x142;
constexpr int DPP_ROW_BCAST31 = 0x143;

// Element (i, j) of a 2x2 row-major matrix, or of its transpose (TR).
template <bool TR, typename CT>
__device__ __forceinline__ CT m2(const CT *P, int i, int j) {
    return TR ? P[2 * j + i] : P[2 * i + j];
}
// w += P t (P or its transpose)
template <bool TR, typename CT>
__device__ __forceinline__ void madd2(CT &w0, CT &w1, const CT *P, CT t0, CT t1) {
    const CT n0 = m2<TR>(P, 0, 0) * t0 + m2<TR>(P, 0, 1) * t1 + w0;
    const CT n1 = m2<TR>(P, 1, 0) * t0 + m2<TR>(P, 1, 1) * t1 + w1;
    w0 = n0;
    w1 = n1;
}

// Table access by carry precision; the fp32 tables may sit in a SecTab
// (global memory) or in its LDS copy (SecLds).
template <typename CT> struct Tab;
template <> struct Tab<float> {
    template <class TB> static __device__ __forceinline__ const float *fold(const TB &t, int k) { return t.fold[k]; }
    template <class TB> static __device__ __forceinline__ const float *psi(const TB &t, int w) { return t.psi[w]; }
    template <class TB> static __device__ __forceinline__ const float *lb(const TB &t, int j) { return t.lb[j]; }
};
template <> struct Tab<double> {
    static __device__ __forceinline__ const double *fold(const SecTab &t, int k) { return t.fold_d[k]; }
    static __device__ __forceinline__ const double *psi(const SecTab &t, int w) { return t.psi_d[w]; }
    static __device__ __forceinline__ const double *lb(const SecTab &t, int j) { return t.lb_d[j]; }
};

// Copies the fp32 tables (the leading sizeof(SL) bytes of each SecTab) of
// sections [s0, s0 + n) into LDS (whole workgroup; the caller synchronises
// before and after).
template <class SL>
__device__ __forceinline__ void stage_tables(SL *dst, const SecTab *src, int s0, int n, int tid, int nthreads) {
    constexpr int V = sizeof(SL) / 16;
    for (int e = tid; e < n * V; e += nthreads) {
        const int s = e / V, i = e % V;
        reinterpret_cast<float4 *>(&dst[s])[i] = reinterpret_cast<const float4 *>(&src[s0 + s])[i];
    }
}

// ------------------------------------------------------------ matrix cores
// Operand types of the 32 x 32 x 16 matrix-core products of the Toeplitz FIR
// (frames of TP = 32 samples; a staged frame row holds 32 operands and 8 of
// padding, 2-byte units).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int TP = 32;        // frame length = output columns
constexpr int TROW = TP + 8;  // staged frame row (2-byte units)

// Compute modes of the matrix-core FIR (tfx_compute values).
enum { TZ_BF16 = 1, TZ_F16 = 2, TZ_BF16X3 = 3 };

template <int MODE> struct Op;
template <> struct Op<TZ_BF16> {
    typedef __bf16 T;
    typedef bf16x8 V;
    static __device__ __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Op<TZ_F16> {
    typedef _Float16 T;
    typedef f16x8 V;
    static __device__ __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct Op<TZ_BF16X3> : Op<TZ_BF16> {};

// ------------------------------------------------------------------ staging
// LDS layout of lane chunks of LC samples: LC samples then 4 floats of
// padding, so a lane's chunk starts 16 LC + 16 bytes after its neighbour's
// and 16-byte reads of 16 lanes hit distinct banks (LC = 16, 24, 32).  The
// defaults are the chain kernel's chunk length L.
template <int LC = L> struct Chunk {
    static constexpr int T = GL * LC;       // samples per group tile
    static constexpr int STRIDE = LC + 4;   // floats per staged chunk
    static constexpr int STG = GL * STRIDE;  // floats per staged tile
    static __device__ __forceinline__ int phys(int i) { return (i / LC) * STRIDE + (i % LC); }
};
constexpr int CSTRIDE = Chunk<>::STRIDE;
constexpr int STG_FLOATS = Chunk<>::STG;
__device__ __forceinline__ int cphys(int i) { return Chunk<>::phys(i); }

template <int LC = L>
__device__ __forceinline__ void load_chunk(const float *stg, int gl, float (&v)[LC]) {
#pragma unroll
    for (int q = 0; q < LC / 4; ++q) {
        const float4 t4 = *reinterpret_cast<const float4 *>(&stg[gl * Chunk<LC>::STRIDE + 4 * q]);
        v[4 * q + 0] = t4.x;
        v[4 * q + 1] = t4.y;
        v[4 * q + 2] = t4.z;
        v[4 * q + 3] = t4.w;
    }
}
template <int LC = L>
__device__ __forceinline__ void store_chunk(float *stg, int gl, const float (&v)[LC]) {
#pragma unroll
    for (int q = 0; q < LC / 4; ++q)
        *reinterpret_cast<float4 *>(&stg[gl * Chunk<LC>::STRIDE + 4 * q]) =
            make_float4(v[4 * q + 0], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}

// One group (GL lanes) stages the tile's samples src[0..rem) (zeros past rem)
// into stg in the chunk layout.  vec: src is 16-byte aligned.
template <int LC = L>
__device__ __forceinline__ void stage_tile(float *stg, const float *src, int64_t rem, bool valid, bool vec, int gl) {
    typedef Chunk<LC> K;
    if (vec && rem >= K::T) {
        float4 t4[K::T / (4 * GL)];
#pragma unroll
        for (int k = 0; k < K::T / (4 * GL); ++k)
            t4[k] = valid ? reinterpret_cast<const float4 *>(src)[gl + GL * k] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int k = 0; k < K::T / (4 * GL); ++k)
            *reinterpret_cast<float4 *>(&stg[K::phys(4 * (gl + GL * k))]) = t4[k];
    } else {  // ragged last tile or unaligned rows
#pragma unroll 4
        for (int k = 0; k < K::T / GL; ++k) {
            const int i = gl + GL * k;
            stg[K::phys(i)] = (valid && i < rem) ? src[i] : 0.f;
        }
    }
}

// One group writes its staged tile (chunk layout) to dst[0..rem).
template <int LC = L>
__device__ __forceinline__ void store_tile(float *dst, const float *stg, int64_t rem, bool vec, int gl) {
    typedef Chunk<LC> K;
    if (vec && rem >= K::T) {
#pragma unroll
        for (int k = 0; k < K::T / (4 * GL); ++k) {
            const int f = gl + GL * k;
            reinterpret_cast<float4 *>(dst)[f] = *reinterpret_cast<const float4 *>(&stg[K::phys(4 * f)]);
        }
    } else {
#pragma unroll 4
        for (int k = 0; k < K::T / GL; ++k) {
            const int i = gl + GL * k;
            if (i < rem) dst[i] = stg[K::phys(i)];
        }
    }
}

// --------------------------------------------------------------------- FFT
// 16-point DFT constants: cos / sin of 2 pi m / 16, m = 0..9.
constexpr float c16[10] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508978f, 0.0f,
                           -0.38268343236508978f, -0.70710678118654752f, -0.92387953251128674f, -1.0f,
                           -0.92387953251128674f};
constexpr float s16[10] = {0.0f, 0.38268343236508978f, 0.70710678118654752f, 0.92387953251128674f, 1.0f,
                           0.92387953251128674f, 0.70710678118654752f, 0.38268343236508978f, 0.0f,
                           -0.38268343236508978f};

// X_k = sum_n a_n w^{nk}, w = SIGN * i
template <int SIGN>
__device__ __forceinline__ void dft4(float &r0, float &i0, float &r1, float &i1, float &r2, float &i2, float &r3,
                                     float &i3) {
    const float sr02 = r0 + r2, si02 = i0 + i2, dr02 = r0 - r2, di02 = i0 - i2;
    const float sr13 = r1 + r3, si13 = i1 + i3, dr13 = r1 - r3, di13 = i1 - i3;
    const float wr = SIGN < 0 ? di13 : -di13;
    const float wi = SIGN < 0 ? -dr13 : dr13;
    r0 = sr02 + sr13;
    i0 = si02 + si13;
    r1 = dr02 + wr;
    i1 = di02 + wi;
    r2 = sr02 - sr13;
    i2 = si02 - si13;
    r3 = dr02 - wr;
    i3 = di02 - wi;
}

// In-register 16-point DFT, X_k = sum_n v_n e^{SIGN 2 pi i n k / 16}, as a
// 4 x 4 decomposition (n = 4 n1 + n2, k = k1 + 4 k2).
template <int SIGN>
__device__ __forceinline__ void dft16(float (&zr)[16], float (&zi)[16]) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2)
        dft4<SIGN>(zr[n2], zi[n2], zr[4 + n2], zi[4 + n2], zr[8 + n2], zi[8 + n2], zr[12 + n2], zi[12 + n2]);
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
        for (int n2 = 1; n2 < 4; ++n2) {
            const int m = n2 * k1;
            const float c = c16[m], s = SIGN < 0 ? -s16[m] : s16[m];
            const float r = zr[4 * k1 + n2], i = zi[4 * k1 + n2];
            zr[4 * k1 + n2] = r * c - i * s;
            zi[4 * k1 + n2] = r * s + i * c;
        }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
        dft4<SIGN>(zr[4 * k1], zi[4 * k1], zr[4 * k1 + 1], zi[4 * k1 + 1], zr[4 * k1 + 2], zi[4 * k1 + 2],
                   zr[4 * k1 + 3], zi[4 * k1 + 3]);
    float tr[16], ti[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            tr[k1 + 4 * k2] = zr[4 * k1 + k2];
            ti[k1 + 4 * k2] = zi[4 * k1 + k2];
        }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        zr[k] = tr[k];
        zi[k] = ti[k];
    }
}

// (r, i) *= w, or *= conj(w) (CONJ)
template <bool CONJ>
__device__ __forceinline__ void cmul_tw(float &r, float &i, float2 w) {
    const float ws = CONJ ? -w.y : w.y;
    const float nr = r * w.x - i * ws;
    const float ni = r * ws + i * w.x;
    r = nr;
    i = ni;
}

// The two LDS exchanges of the FFT store element (k1, b, c) at
// 256 k1 + 16 ((b + k1) & 15) + c and element (k1, k2, c) at
// 256 k1 + 16 ((k2 + k1) & 15) + ((c + k1) & 15): bijections onto [0, 4096),
// bank-conflict-free for every lane order used below (checked on the CPU for
// 32 banks per half-wave and 64 per wave).  In each loop a lane's addresses
// are one lane constant plus the loop's immediate step, minus 256 (or 16)
// once the rotation wraps, so an access costs a compare and a select.
//
// Twiddles (w = e^{-2 pi i / 4096}; the inverse uses the conjugates) come
// from the 32 rows of TWL, copied into LDS by the workgroup (twl_stage):
// global twiddle loads left the transforms waiting on L2 at every pass.  Pass
// twiddles that are not a row entry are the product of two:
// w^(t k) = w^(16 (t >> 4) k) w^((t & 15) k) and
// w^((16 b + c) k1) = w^(16 k1 b) w^(c k1).  Row r is read 16 bytes at a
// time; its entry 0 is 1 and is skipped.
template <bool CONJ>
__device__ __forceinline__ void twiddle_lds(float (&zr)[16], float (&zi)[16], const float2 *twl, int r) {
    const float4 *r4 = reinterpret_cast<const float4 *>(twl + r * TWL_S);
#pragma unroll
    for (int g = 0; g < 8; ++g) {
        const float4 w = r4[g];
        if (g > 0) cmul_tw<CONJ>(zr[2 * g], zi[2 * g], make_float2(w.x, w.y));  // entry 0 is 1
        cmul_tw<CONJ>(zr[2 * g + 1], zi[2 * g + 1], make_float2(w.z, w.w));
    }
}
// Copies TWL (the workspace's twiddle region) into the workgroup's LDS copy;
// the caller passes a barrier before the first transform.
__device__ __forceinline__ void twl_stage(float2 *twl, const float2 *twid, int tid, int nthreads) {
    const float4 *src = reinterpret_cast<const float4 *>(twid);
    float4 *dst = reinterpret_cast<float4 *>(twl);
    for (int e = tid; e < TWL_ENTRIES / 2; e += nthreads) dst[e] = src[e];
}

// Forward 4096-point DFT (e^{-2 pi i n k / 4096}) of the values held by the
// 256 lanes of a workgroup.  In: lane t holds z[256 a + t], a = 0..15.  Out:
// lane t holds Z[t + 256 k3], k3 = 0..15.  Three radix-16 passes with two LDS
// exchanges through lds[0 .. 8192) floats.  Ends with the data in registers
// and every lane past its last LDS read (callers may reuse lds after a
// barrier).
// twl: the workgroup's LDS copy of TWL.
__device__ __forceinline__ void fft4096_forward(float (&zr)[16], float (&zi)[16], float *lds, const float2 *twl,
                                                int tid) {
    float *Lr = lds, *Li = lds + NFFT;
    dft16<-1>(zr, zi);
    twiddle_lds<false>(zr, zi, twl, tid >> 4);
    twiddle_lds<false>(zr, zi, twl, 16 + (tid & 15));
    {
        const int b = tid >> 4, c = tid & 15, w0 = 16 * b + c;
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) {
            const int ad = (k1 >= 16 - b ? w0 - 256 : w0) + 272 * k1;
            Lr[ad] = zr[k1];
            Li[ad] = zi[k1];
        }
    }
    __syncthreads();
    {
        const int k1 = tid >> 4, c = tid & 15, r0 = 272 * k1 + c;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const int ad = (b >= 16 - k1 ? r0 - 256 : r0) + 16 * b;
            zr[b] = Lr[ad];
            zi[b] = Li[ad];
        }
        dft16<-1>(zr, zi);
        twiddle_lds<false>(zr, zi, twl, c);
        __syncthreads();
        const int w1 = 272 * k1 + ((c + k1) & 15);
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) {
            const int ad = (k2 >= 16 - k1 ? w1 - 256 : w1) + 16 * k2;
            Lr[ad] = zr[k2];
            Li[ad] = zi[k2];
        }
    }
    __syncthreads();
    {
        const int k1 = tid & 15, k2 = tid >> 4, r1 = 256 * k1 + 16 * ((k2 + k1) & 15) + k1;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int ad = (c >= 16 - k1 ? r1 - 16 : r1) + c;
            zr[c] = Lr[ad];
            zi[c] = Li[ad];
        }
        dft16<-1>(zr, zi);
    }
}

// Inverse of fft4096_forward without the 1/4096 factor (e^{+2 pi i n k /
// 4096}): in the forward's output layout, out in its input layout.  Begins
// with a barrier before its first LDS write.
__device__ __forceinline__ void fft4096_inverse(float (&zr)[16], float (&zi)[16], float *lds, const float2 *twl,
                                                int tid) {
    float *Lr = lds, *Li = lds + NFFT;
    {
        const int k1 = tid & 15, k2 = tid >> 4, r1 = 256 * k1 + 16 * ((k2 + k1) & 15) + k1;
        dft16<1>(zr, zi);
        twiddle_lds<true>(zr, zi, twl, k2);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int ad = (c >= 16 - k1 ? r1 - 16 : r1) + c;
            Lr[ad] = zr[c];
            Li[ad] = zi[c];
        }
    }
    __syncthreads();
    {
        const int k1 = tid >> 4, c = tid & 15, w1 = 272 * k1 + ((c + k1) & 15);
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) {
            const int ad = (k2 >= 16 - k1 ? w1 - 256 : w1) + 16 * k2;
            zr[k2] = Lr[ad];
            zi[k2] = Li[ad];
        }
        dft16<1>(zr, zi);
        twiddle_lds<true>(zr, zi, twl, k1);  // w^(16 k1 b)
        const float2 wc = twl[(16 + c) * TWL_S + k1];  // w^(c k1), the lane's constant
#pragma unroll
        for (int b = 0; b < 16; ++b) cmul_tw<true>(zr[b], zi[b], wc);
        __syncthreads();
        const int r0 = 272 * k1 + c;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            const int ad = (b >= 16 - k1 ? r0 - 256 : r0) + 16 * b;
            Lr[ad] = zr[b];
            Li[ad] = zi[b];
        }
    }
    __syncthreads();
    {
        const int b = tid >> 4, c = tid & 15, w0 = 16 * b + c;
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) {
            const int ad = (k1 >= 16 - b ? w0 - 256 : w0) + 272 * k1;
            zr[k1] = Lr[ad];
            zi[k1] = Li[ad];
        }
        dft16<1>(zr, zi);
    }
}

// Z *= H (or conj(H)) bin by bin, H = the tap spectrum in the per-lane layout
// hspec[t][k3] = H[t + 256 k3].  The loads go in groups of four bins with a
// compiler barrier between groups, so at most four bins' spectra sit in
// registers beside the data.
__device__ __forceinline__ void spectrum_product(float (&zr)[16], float (&zi)[16], const float2 *hspec, int tid,
                                                 bool conj) {
    const float sg = conj ? -1.f : 1.f;
    const float4 *h4 = reinterpret_cast<const float4 *>(hspec + 16 * tid);
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4) {
        const float4 p = h4[2 * g4], q = h4[2 * g4 + 1];
        const float2 w[4] = {make_float2(p.x, sg * p.y), make_float2(p.z, sg * p.w), make_float2(q.x, sg * q.y),
                             make_float2(q.z, sg * q.w)};
#pragma unroll
        for (int u = 0; u < 4; ++u) cmul_tw<false>(zr[4 * g4 + u], zi[4 * g4 + u], w[u]);
        asm volatile("" ::: "memory");
    }
}

// Loads the complex block z[m] = xa[base + m] + i xb[base + m], m = 256 q + tid
// (zeros outside [0, N) and past limit; xb may be null) into the forward FFT
// input layout.  With a history (streaming: the hlen samples before the
// block, ha / hb, hb may be null) the samples at n in [-hlen, 0) come from
// ha[hlen + n].  A block wholly inside takes no per-element checks.
__device__ __forceinline__ void load_pair_block(float (&zr)[16], float (&zi)[16], const float *xa, const float *xb,
                                                int64_t base, int64_t N, int64_t limit, int tid,
                                                const float *ha = nullptr, const float *hb = nullptr,
                                                int64_t hlen = 0) {
    const int64_t hi = N < limit ? N : limit;
    if (base >= 0 && base + NFFT <= hi) {
        const float *pa = xa + base + tid;
#pragma unroll
        for (int q = 0; q < 16; ++q) zr[q] = pa[256 * q];
        if (xb) {
            const float *pb = xb + base + tid;
#pragma unroll
            for (int q = 0; q < 16; ++q) zi[q] = pb[256 * q];
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) zi[q] = 0.f;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t n = base + 256 * q + tid;
        const bool in = n >= 0 && n < hi;
        const bool inh = n < 0 && n >= -hlen;
        zr[q] = in ? xa[n] : (inh ? ha[hlen + n] : 0.f);
        zi[q] = (in && xb) ? xb[n] : ((inh && hb) ? hb[hlen + n] : 0.f);
    }
}

// Stores the 3072 outputs of a tile held as zr/zi[q0 .. q0 + 12) (lane tid
// holds sample 256 (q - q0) + tid) to ya[n0 + .] and, when yb is set,
// yb[n0 + .], up to N.  A tile wholly inside takes no per-element checks.
template <int Q0>
__device__ __forceinline__ void store_pair_tile(const float (&zr)[16], const float (&zi)[16], float *ya, float *yb,
                                                int64_t n0, int64_t N, int tid) {
    if (n0 + 12 * 256 <= N) {
        float *pa = ya + n0 + tid;
#pragma unroll
        for (int q = 0; q < 12; ++q) pa[256 * q] = zr[Q0 + q];
        if (yb) {
            float *pb = yb + n0 + tid;
#pragma unroll
            for (int q = 0; q < 12; ++q) pb[256 * q] = zi[Q0 + q];
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        const int64_t n = n0 + 256 * q + tid;
        if (n < N) {
            ya[n] = zr[Q0 + q];
            if (yb) yb[n] = zi[Q0 + q];
        }
    }
}

// ------------------------------------------------------------ chunk carry
// The recurrence  s_{k+1} = Phi s_k + z_k  over the chunks of a tile (Phi =
// A^24 of one section, or its transpose for the adjoint), carried across
// tiles by a decoupled look-back or started from a known tile prefix.

struct CarryCtx {
    int lane, gw, grp;
    bool lookback;        // prefix by look-back (else `known`)
    int64_t pos;          // tile position in processing order
    uint64_t *recs;       // records of this channel/section: rec(q) = rec0 + q * rstride
    int64_t rec0, rstride;
    uint32_t epoch;
    uint32_t *hdr;
    double known0, known1;  // prefix when !lookback, or at pos == 0
    float *prefix_out;      // optional: receives the tile prefix (2 floats)
};

// Decoupled look-back of one tile by one full wave.  Publishes the tile
// aggregate (agg), then returns the state entering the tile.  Lane l watches
// predecessor pos-1-l (a window of 64 tiles per step); a lane stops
// re-reading its record once the aggregate or the prefix is out, so the spin
// costs one 32-byte read per still-missing predecessor.
template <typename CT, bool TR, class TB>
__device__ void lookback(const TB &tb, const CarryCtx &cc, CT agg0, CT agg1, CT &P0, CT &P1) {
    const int lane = cc.lane;
    publish(cc.recs, cc.rec0 + cc.pos * cc.rstride, 0, cc.epoch, (float)agg0, (float)agg1, lane);
    CT acc0 = 0, acc1 = 0;
    CT M00 = 1, M01 = 0, M10 = 0, M11 = 1;  // (PhiT)^(64 * windows consumed)
    int64_t base = cc.pos - 1;
    while (true) {
        const int64_t q = base - lane;
        // 0 missing, 1 aggregate, 2 prefix, 3 before the first tile; a tile
        // beyond the look-back depth counts as a prefix of zero
        int st = q < 0 ? 3 : ((tb.depth > 0 && q < cc.pos - tb.depth) ? 2 : 0);
        float r0 = 0.f, r1 = 0.f;
        int64_t spins = 0;
        while (true) {
            if (st == 0) {
                const uint64_t *p = cc.recs + (cc.rec0 + q * cc.rstride) * REC_WORDS;
                uint64_t w[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) w[i] = ld_word(p + i);
                st = decode_record(w, cc.epoch, r0, r1);
            }
            const unsigned long long fm = __ballot(st == 2);
            const int first = fm ? (__ffsll(fm) - 1) : 63;
            if (!__ballot(st == 0 && lane <= first)) break;
            if (++spins > SPIN_MAX) {  // never expected: report and finish
                atomicOr(&cc.hdr[HDR_ERROR], 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
        const unsigned long long fm = __ballot(st == 2);
        const int first = fm ? (__ffsll(fm) - 1) : 64;
        CT v0 = 0, v1 = 0;
        if (lane <= first && (st == 1 || st == 2)) {
            v0 = (CT)r0;
            v1 = (CT)r1;
        }
        CT R0, R1;
        if (first == 0) {
            R0 = __shfl(v0, 0);
            R1 = __shfl(v1, 0);
        } else {
            // lane 0 <- sum_l PhiT^l v_l
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const int d = 1 << k;
                const CT t0 = __shfl_down(v0, d), t1 = __shfl_down(v1, d);
                if (lane + d < 64) madd2<TR>(v0, v1, Tab<CT>::lb(tb, k), t0, t1);
            }
            R0 = __shfl(v0, 0);
            R1 = __shfl(v1, 0);
        }
        acc0 += M00 * R0 + M01 * R1;
        acc1 += M10 * R0 + M11 * R1;
        if (fm) break;
        const CT *B = Tab<CT>::lb(tb, 6);  // PhiT^64
        const CT n00 = M00 * m2<TR>(B, 0, 0) + M01 * m2<TR>(B, 1, 0);
        const CT n01 = M00 * m2<TR>(B, 0, 1) + M01 * m2<TR>(B, 1, 1);
        const CT n10 = M10 * m2<TR>(B, 0, 0) + M11 * m2<TR>(B, 1, 0);
        const CT n11 = M10 * m2<TR>(B, 0, 1) + M11 * m2<TR>(B, 1, 1);
        M00 = n00;
        M01 = n01;
        M10 = n10;
        M11 = n11;
        base -= 64;
    }
    P0 = acc0;
    P1 = acc1;
}

// Given the lane's chunk state z (the chunk's final state from a zero
// entering state), returns the state entering the lane's chunk.  Inclusive
// scan over the wave's 64 chunks (DPP row shifts within rows of 16 lanes,
// then row broadcasts weighted by the lane's own power of Phi), the group's
// wave aggregates combined through LDS with Psi = Phi^64, the tile prefix by
// look-back (publishing the inclusive prefix) or from `known`, then folded
// into every chunk with the table of Phi^k.  Contains two workgroup
// barriers; s_agg / s_pre slot `buf` must not be in use by a neighbouring
// call (callers alternate two slots).
template <typename CT, bool TR, class TB>
__device__ void carry(const TB &tb, const CarryCtx &cc, float z0, float z1, float &e0, float &e1,
                      double (*s_agg)[GWAVES][2], double (*s_pre)[2], int buf) {
    const int lane = cc.lane;
    CT w0 = (CT)z0, w1 = (CT)z1;
    {
        CT t0 = dpp<DPP_ROW_SHR + 1>(w0), t1 = dpp<DPP_ROW_SHR + 1>(w1);
        madd2<TR>(w0, w1, Tab<CT>::fold(tb, 1), t0, t1);
        t0 = dpp<DPP_ROW_SHR + 2>(w0);
        t1 = dpp<DPP_ROW_SHR + 2>(w1);
        madd2<TR>(w0, w1, Tab<CT>::fold(tb, 2), t0, t1);
        t0 = dpp<DPP_ROW_SHR + 4>(w0);
        t1 = dpp<DPP_ROW_SHR + 4>(w1);
        madd2<TR>(w0, w1, Tab<CT>::fold(tb, 4), t0, t1);
        t0 = dpp<DPP_ROW_SHR + 8>(w0);
        t1 = dpp<DPP_ROW_SHR + 8>(w1);
        madd2<TR>(w0, w1, Tab<CT>::fold(tb, 8), t0, t1);
        t0 = dpp<DPP_ROW_BCAST15, 0xA>(w0);  // rows 1, 3 take lane 15 of rows 0, 2
        t1 = dpp<DPP_ROW_BCAST15, 0xA>(w1);
        madd2<TR>(w0, w1, Tab<CT>::fold(tb, (lane & 15) + 1), t0, t1);
        t0 = dpp<DPP_ROW_BCAST31, 0xC>(w0);  // rows 2, 3 take lane 31
        t1 = dpp<DPP_ROW_BCAST31, 0xC>(w1);
        madd2<TR>(w0, w1, Tab<CT>::fold(tb, (lane & 31) + 1), t0, t1);
    }
    if (lane == 63) {
        s_agg[buf][cc.gw][0] = (double)w0;
        s_agg[buf][cc.gw][1] = (double)w1;
    }
    __syncthreads();
    // wave-entering states for a zero tile-entering state; E ends as the
    // tile aggregate
    const CT *Psi = Tab<CT>::psi(tb, 1);
    CT E0 = 0, E1 = 0, ew0 = 0, ew1 = 0;
#pragma unroll
    for (int w = 0; w < GWAVES; ++w) {
        if (w == cc.gw) {
            ew0 = E0;
            ew1 = E1;
        }
        CT g0 = (CT)s_agg[buf][w][0], g1 = (CT)s_agg[buf][w][1];
        madd2<TR>(g0, g1, Psi, E0, E1);
        E0 = g0;
        E1 = g1;
    }
    if (cc.gw == 0) {
        CT P0 = (CT)cc.known0, P1 = (CT)cc.known1;
        if (cc.lookback) {
            if (cc.pos > 0) lookback<CT, TR, TB>(tb, cc, E0, E1, P0, P1);
            CT i0 = E0, i1 = E1;
            madd2<TR>(i0, i1, Tab<CT>::lb(tb, 0), P0, P1);  // PhiT P + E
            publish(cc.recs, cc.rec0 + cc.pos * cc.rstride, 1, cc.epoch, (float)i0, (float)i1, lane);
        }
        if (lane == 0) {
            s_pre[buf][0] = (double)P0;
            s_pre[buf][1] = (double)P1;
            if (cc.prefix_out) {
                cc.prefix_out[0] = (float)P0;
                cc.prefix_out[1] = (float)P1;
            }
        }
    }
    __syncthreads();
    CT x0 = ew0, x1 = ew1;  // wave-entering state
    madd2<TR>(x0, x1, Tab<CT>::psi(tb, cc.gw), (CT)s_pre[buf][0], (CT)s_pre[buf][1]);
    CT s0 = dpp<DPP_WAVE_SHR1>(w0), s1 = dpp<DPP_WAVE_SHR1>(w1);  // lane 0 reads 0
    madd2<TR>(s0, s1, Tab<CT>::fold(tb, lane), x0, x1);
    e0 = (float)s0;
    e1 = (float)s1;
}

// ------------------------------------------------ cascade-level carry
// The same chunk scan as `carry`, with the tile-entering state P known (no
// look-back) and a single workgroup barrier.  Returns the chunk-entering
// state e of the lane's chunk and the group's tile aggregate E (the state at
// the tile's end from a zero tile-entering state).  s_agg slot `buf` must
// not be in use by a neighbouring call (callers alternate two slots).
template <typename CT, class TB>
__device__ void carry_local(const TB &tb, int lane, int gw, float z0, float z1, CT P0, CT P1, float &e0, float &e1,
                            CT &E0, CT &E1, double (*s_agg)[GWAVES][2], int buf) {
    CT w0 = (CT)z0, w1 = (CT)z1;
    {
        CT t0 = dpp<DPP_ROW_SHR + 1>(w0), t1 = dpp<DPP_ROW_SHR + 1>(w1);
        madd2<false>(w0, w1, Tab<CT>::fold(tb, 1), t0, t1);
        t0 = dpp<DPP_ROW_SHR + 2>(w0);
        t1 = dpp<DPP_ROW_SHR + 2>(w1);
        madd2<false>(w0, w1, Tab<CT>::fold(tb, 2), t0, t1);
        t0 = dpp<DPP_ROW_SHR + 4>(w0);
        t1 = dpp<DPP_ROW_SHR + 4>(w1);
        madd2<false>(w0, w1, Tab<CT>::fold(tb, 4), t0, t1);
        t0 = dpp<DPP_ROW_SHR + 8>(w0);
        t1 = dpp<DPP_ROW_SHR + 8>(w1);
        madd2<false>(w0, w1, Tab<CT>::fold(tb, 8), t0, t1);
        t0 = dpp<DPP_ROW_BCAST15, 0xA>(w0);
        t1 = dpp<DPP_ROW_BCAST15, 0xA>(w1);
        madd2<false>(w0, w1, Tab<CT>::fold(tb, (lane & 15) + 1), t0, t1);
        t0 = dpp<DPP_ROW_BCAST31, 0xC>(w0);
        t1 = dpp<DPP_ROW_BCAST31, 0xC>(w1);
        madd2<false>(w0, w1, Tab<CT>::fold(tb, (lane & 31) + 1), t0, t1);
    }
    if (lane == 63) {
        s_agg[buf][gw][0] = (double)w0;
        s_agg[buf][gw][1] = (double)w1;
    }
    __syncthreads();
    const CT *Psi = Tab<CT>::psi(tb, 1);
    CT A0 = 0, A1 = 0, ew0 = 0, ew1 = 0;
#pragma unroll
    for (int w = 0; w < GWAVES; ++w) {
        if (w == gw) {
            ew0 = A0;
            ew1 = A1;
        }
        CT g0 = (CT)s_agg[buf][w][0], g1 = (CT)s_agg[buf][w][1];
        madd2<false>(g0, g1, Psi, A0, A1);
        A0 = g0;
        A1 = g1;
    }
    E0 = A0;
    E1 = A1;
    CT x0 = ew0, x1 = ew1;  // wave-entering state
    madd2<false>(x0, x1, Tab<CT>::psi(tb, gw), P0, P1);
    CT s0 = dpp<DPP_WAVE_SHR1>(w0), s1 = dpp<DPP_WAVE_SHR1>(w1);
    madd2<false>(s0, s1, Tab<CT>::fold(tb, lane), x0, x1);
    e0 = (float)s0;
    e1 = (float)s1;
}

// ---------------------------------------------- cascade-level section form
// TDF-II over the chunk from (s1, s2), in place; with CAP the state after
// sample r_cap (if 0 <= r_cap < LC) is returned in (c1, c2).
template <int LC, bool CAP = false>
__device__ __forceinline__ void section_from(const float *co, float (&v)[LC], float s1, float s2, int r_cap,
                                             float &c1, float &c2) {
    const float b0 = co[0], b1 = co[1], b2 = co[2], a1 = co[3], a2 = co[4];
#pragma unroll
    for (int r = 0; r < LC; ++r) {
        const float xv = v[r];
        const float yv = fmaf(b0, xv, s1);
        s1 = fmaf(b1, xv, fmaf(-a1, yv, s2));
        s2 = fmaf(b2, xv, -a2 * yv);
        v[r] = yv;
        if (CAP && r == r_cap) {
            c1 = s1;
            c2 = s2;
        }
    }
}

// e += Phi^lane Psi^gw P: how a tile-entering state P moves a lane's
// chunk-entering state (carry_local is linear in its prefix).
template <class TB>
__device__ __forceinline__ void fold_prefix(const TB &tb, int lane, int gw, float P0, float P1, float &e0, float &e1) {
    float x0 = 0.f, x1 = 0.f;
    madd2<false>(x0, x1, Tab<float>::psi(tb, gw), P0, P1);
    madd2<false>(e0, e1, Tab<float>::fold(tb, lane), x0, x1);
}

// Phase-A form of a section (zero tile-entering state): zero-state response
// over the chunk, the in-tile carry to the chunk-entering state e, and the
// zero-input response of e added in place.  !RUN: only the state is needed
// (the last section), so the zero-state pass keeps no output and no
// correction follows.
template <int LC, bool RUN>
__device__ __forceinline__ void casc_section_a(const SecLdsC &tb, float (&v)[LC], int lane, int gw,
                                               double (*s_agg)[GWAVES][2], int buf, float &e0, float &e1, float &E0,
                                               float &E1) {
    const float b0 = tb.coef[0], b1 = tb.coef[1], b2 = tb.coef[2], a1 = tb.coef[3], a2 = tb.coef[4];
    float s1 = 0.f, s2 = 0.f;
    if (RUN) {
#pragma unroll
        for (int r = 0; r < LC; ++r) {
            const float xv = v[r];
            const float yv = fmaf(b0, xv, s1);
            s1 = fmaf(b1, xv, fmaf(-a1, yv, s2));
            s2 = fmaf(b2, xv, -a2 * yv);
            v[r] = yv;
        }
    } else {  // s' = A s + B x: 4 operations a sample
        const float B0 = fmaf(-a1, b0, b1), B1 = fmaf(-a2, b0, b2);
#pragma unroll
        for (int r = 0; r < LC; ++r) {
            const float xv = v[r];
            const float n1 = fmaf(B0, xv, fmaf(-a1, s1, s2));
            s2 = fmaf(B1, xv, -a2 * s1);
            s1 = n1;
        }
    }
    carry_local<float, SecLdsC>(tb, lane, gw, s1, s2, 0.f, 0.f, e0, e1, E0, E1, s_agg, buf);
    if (RUN) {
        float z1 = e0, z2 = e1;
#pragma unroll
        for (int r = 0; r < LC; ++r) {
            v[r] += z1;
            const float n1 = fmaf(-a1, z1, z2);
            z2 = -a2 * z1;
            z1 = n1;
        }
    }
}

// Phase-C form (known tile-entering state P): zero-state response, carry,
// then the zero-input response of the chunk-entering state added in place;
// with CAP the state after sample r_cap is returned in (c1, c2).
template <int LC, bool CAP>
__device__ __forceinline__ void casc_section_c(const SecLdsC &tb, float (&v)[LC], int lane, int gw, float P0,
                                               float P1, double (*s_agg)[GWAVES][2], int buf, int r_cap, float &c1,
                                               float &c2) {
    const float b0 = tb.coef[0], b1 = tb.coef[1], b2 = tb.coef[2], a1 = tb.coef[3], a2 = tb.coef[4];
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int r = 0; r < LC; ++r) {
        const float xv = v[r];
        const float yv = fmaf(b0, xv, s1);
        s1 = fmaf(b1, xv, fmaf(-a1, yv, s2));
        s2 = fmaf(b2, xv, -a2 * yv);
        v[r] = yv;
        if (CAP && r == r_cap) {
            c1 = s1;
            c2 = s2;
        }
    }
    float z1, z2, E0, E1;
    carry_local<float, SecLdsC>(tb, lane, gw, s1, s2, P0, P1, z1, z2, E0, E1, s_agg, buf);
#pragma unroll
    for (int r = 0; r < LC; ++r) {
        v[r] += z1;
        const float n1 = fmaf(-a1, z1, z2);
        z2 = -a2 * z1;
        z1 = n1;
        if (CAP && r == r_cap) {  // state after the sample = zero-state + zero-input states
            c1 += z1;
            c2 += z2;
        }
    }
}

// Decoupled look-back over the whole cascade state (D = 2S <= 16 components,
// section s at components 2s, 2s+1), by one wave.  Lanes form 4 rows of 16:
// row r watches predecessor pos-1-r, lane c of a row component c.  Every
// record holds the tile aggregate (D tagged words) then the inclusive prefix
// (D words).  T (LDS) holds the cascade's tile transition Phi_T, its square
// and its fourth power, D x D row-major each.  Publishes the aggregate E
// (LDS, D floats), writes the tile-entering state to P (LDS) and publishes
// the inclusive prefix Phi_T P + E.  `known`: the state entering tile 0
// (null = zero).  Mw: a D x D LDS matrix of this wave (the pending window
// weight).
struct CascCtx {
    int lane, D;
    int depth;         // look-back depth (0 = unbounded)
    uint64_t *rec;     // record of tile 0 of this channel; tile q at rec + q * 2D
    int64_t pos;       // tile position
    uint32_t epoch;
    uint32_t *hdr;
    const float *known;
};

// sum_d Tm[c][d] v(src_row, d) for lanes c < D of every row (0 elsewhere);
// Tm is D x D row-major.
__device__ __forceinline__ float row_matvec(const float *Tm, int D, int c, float v, int src_row) {
    float acc = 0.f;
    const float *tr = Tm + (c < D ? c : 0) * D;
    for (int d = 0; d < D; ++d) acc = fmaf(tr[d], __shfl(v, src_row * 16 + d), acc);
    return c < D ? acc : 0.f;
}

__device__ void casc_lookback(const CascCtx &cc, const float *T, const float *E, float *P, float *Mw) {
    const int lane = cc.lane, row = lane >> 4, c = lane & 15, D = cc.D;
    const bool active = c < D;
    const int W = 2 * D;
    const uint64_t tag = (uint64_t)cc.epoch << 32;
    const float Ec = active ? E[c] : 0.f;
    if (row == 0 && active) st_word(cc.rec + cc.pos * W + c, tag | __float_as_uint(Ec));
    float acc = 0.f;
    if (cc.pos == 0) {
        acc = (active && cc.known) ? cc.known[c] : 0.f;
    } else {
        // pending window weight (Phi_T^4)^windows, in LDS: lane l holds
        // entries 4 l .. 4 l + 3 of the D x D row-major matrix
        const int DD = D * D;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = 4 * lane + u;
            if (e < DD) Mw[e] = (e / D == e % D) ? 1.f : 0.f;
        }
        const unsigned long long rmask0 = (D >= 16 ? 0xFFFFull : ((1ull << D) - 1ull));
        int64_t base = cc.pos - 1;
        while (true) {
            const int64_t q = base - row;
            float va = 0.f, vi = 0.f;
            bool ha = false, hi = false;
            if (cc.depth > 0 && q < cc.pos - cc.depth) {  // beyond the look-back depth: a zero prefix
                hi = ha = true;
            } else if (q < 0) {  // before tile 0: the prefix entering tile 0
                hi = ha = true;
                vi = (q == -1 && cc.known && active) ? cc.known[c] : 0.f;
            }
            int st[4];
            int first = 4;
            int64_t spins = 0;
            bool poll = true;  // this lane's row still misses a record
            while (true) {
                if (poll && active && q >= 0) {
                    const uint64_t *p = cc.rec + q * W;
                    const uint64_t wa = ld_word(p + c), wi = ld_word(p + D + c);
                    if ((wa >> 32) == cc.epoch) {
                        ha = true;
                        va = __uint_as_float((uint32_t)wa);
                    }
                    if ((wi >> 32) == cc.epoch) {
                        hi = true;
                        vi = __uint_as_float((uint32_t)wi);
                    }
                }
                // a row is complete when every component's word is out (the
                // words of one record may become visible in any order)
                const unsigned long long bi = __ballot(!active || hi), ba = __ballot(!active || ha);
                first = 4;
                bool need = false;
#pragma unroll
                for (int r = 3; r >= 0; --r) {
                    const unsigned long long rm = rmask0 << (16 * r);
                    st[r] = ((bi & rm) == rm) ? 2 : (((ba & rm) == rm) ? 1 : 0);
                    if (st[r] == 2) first = r;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r <= first && st[r] == 0) need = true;
                if (!need) break;
                if (++spins > SPIN_MAX) {  // never expected: report and finish
                    if (lane == 0) atomicOr(&cc.hdr[HDR_ERROR], 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
                poll = st[row] == 0;
            }
            // row r contributes Phi_T^r times its aggregate (rows before the
            // first complete prefix) or its prefix (that row); later rows 0
            float v = (row < first) ? va : (row == first ? vi : 0.f);
            if (!active) v = 0.f;
            float t1 = row_matvec(T, D, c, v, (row + 1) & 3);  // rows 0, 2 += Phi_T * rows 1, 3
            if (row == 0 || row == 2) v += t1;
            float t2 = row_matvec(T + DD, D, c, v, 2);  // row 0 += Phi_T^2 * row 2
            if (row == 0) v += t2;
            // acc += (window weight) * R, R = row 0's vector
            acc += row_matvec(Mw, D, c, v, 0);
            if (first < 4) break;
            // next window: M <- M Phi_T^4 in place.  Every lane reads before
            // any lane writes: the wave's LDS accesses are issued in program
            // order.
            float nm[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = 4 * lane + u;
                if (e < DD) {
                    const int i = e / D, j = e % D;
                    for (int d = 0; d < D; ++d) nm[u] = fmaf(Mw[i * D + d], T[2 * DD + d * D + j], nm[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = 4 * lane + u;
                if (e < DD) Mw[e] = nm[u];
            }
            base -= 4;
        }
    }
    // tile-entering state, and the inclusive prefix Phi_T P + E
    if (row == 0 && active) P[c] = acc;
    const float inc = Ec + row_matvec(T, D, c, acc, 0);
    if (row == 0 && active) st_word(cc.rec + cc.pos * W + D + c, tag | __float_as_uint(inc));
}

}  // namespace tfx
