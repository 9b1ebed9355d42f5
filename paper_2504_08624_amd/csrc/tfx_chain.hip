// tfx_chain.hip -- fused multichannel FIR + IIR-SOS chain for gfx950.
//
// One kernel template covers every forward form of the library:
//   FIR part   none | direct LDS-tiled convolution | overlap-save FFT
//   IIR part   none | per-section chunked linear-recurrence scan
// The FIR output of a tile never leaves the chip: it lands in the registers
// of the lanes that run the recursion on it.
//
// The filtering is the textbook definition (causal FIR convolution and the
// transposed-direct-form-II section recursion; the paper, Sec. 3, names these
// filters and the coefficient-driven lfilter).  The parallel decomposition is
// this library's own:
//
// Tiles.  A workgroup of 256 lanes holds two channel groups of 128 lanes, one
// for each channel of an even/odd pair.  A group owns a tile of T = 3072
// consecutive samples of its channel; lane i owns the 24-sample chunk
// [24i, 24i+24) in registers.  Workgroup ids are tile-major (all pairs of tile
// t before tile t+1), and workgroups are dispatched in id order, so a tile's
// predecessors in time are always resident or finished when it waits on them
// (no global atomic counter: on this chip one contended device-scope atomic
// per workgroup serialises across the eight XCDs).
//
// FFT FIR.  The pair is packed as one complex signal (real = even channel,
// imaginary = odd channel); as the taps are real, one complex FFT filters both
// channels exactly.  Per tile: 4096-point FFT of the block starting 1024
// samples before the tile, product with the precomputed tap spectrum,
// inverse FFT, the first 1024 outputs dropped.  Each FFT is three radix-16
// passes (one 16-point DFT per lane in registers) with XOR-swizzled,
// bank-conflict-free LDS exchanges between passes.
//
// IIR scan, one section at a time (the cascade stays in registers):
//   1. zero-state response of the lane's chunk (TDF-II, fp32): y0[t] and the
//      final state z;
//   2. inclusive scan of z over the 64 lanes of a wave with the powers
//      Phi^(2^j) of the 2x2 chunk transition Phi = A^24;
//   3. the group's wave aggregates combined through LDS with Psi = Phi^64;
//   4. decoupled look-back across tiles of the channel: publish the tile
//      aggregate, reduce predecessors' aggregates (weighted by powers of
//      PhiT = A^T) up to the first published inclusive prefix, 64 tiles per
//      step;
//   5. each lane folds the prefix into its chunk-entering state with a table
//      of Phi^k and adds the zero-input response of that state, generated
//      by the same recursion with x = 0 (3 operations per sample).
// The carry (steps 2-5) runs in fp32, or in fp64 for sections whose pole
// radius exceeds 0.999; the per-sample recursion is fp32.
#include <hip/hip_runtime.h>

#include "tfx_internal.h"

namespace tfx {

// Look-back records.  Every (channel, tile, section) owns 4 64-bit words:
// the tile aggregate (2 floats) and the inclusive prefix (2 floats), each
// word (epoch << 32) | float bits, written and read with relaxed agent-scope
// atomics: every word validates itself, so no acquire/release fence is
// needed.  (On this chip each XCD has its own L2, and an agent-scope fence
// writes back or invalidates the whole L2; fences in a spin loop would thrash
// it for every tile on the XCD.)  The cross-tile values are fp32 even for
// sections carried in fp64 inside the tile: across tiles the state is damped
// by PhiT = A^3072, so rounding there accumulates over a few tiles only.
// The epoch advances once per launch (a one-thread kernel behind every run),
// so a run never has to clear the words the previous run left and repeated
// runs need no memset.
constexpr uint32_t EPOCH_MASK = 0x3FFFFFFFu;
constexpr int64_t SPIN_MAX = int64_t(1) << 22;
constexpr int REC_WORDS = 4;
enum { HDR_ERROR = 1, HDR_EPOCH = 2 };

// LDS layout of lane chunks: 24 samples then 4 floats of padding, so a lane's
// chunk starts 112 bytes after its neighbour's and 16-byte reads of 16 lanes
// hit distinct banks.
constexpr int CSTRIDE = L + 4;
constexpr int STG_FLOATS = GL * CSTRIDE;
__device__ __forceinline__ int cphys(int i) { return (i / L) * CSTRIDE + (i % L); }
constexpr int DIRECT_GROUP_FLOATS = ((T + KBLK_MAX + L - 1) / L + 1) * CSTRIDE;

template <int FIRM>
constexpr int lds_floats() {
    return FIRM == FIR_DIRECT ? GROUPS * DIRECT_GROUP_FLOATS
                              : (FIRM == FIR_FFT ? 2 * NFFT : GROUPS * STG_FLOATS);
}
static_assert(GROUPS * STG_FLOATS <= 2 * NFFT, "staging must fit in the FFT buffers");

__device__ __forceinline__ uint64_t ld_word(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_word(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// w += P t for a 2x2 row-major P
template <typename CT>
__device__ __forceinline__ void madd2(CT &w0, CT &w1, const CT *P, CT t0, CT t1) {
    const CT n0 = P[0] * t0 + P[1] * t1 + w0;
    const CT n1 = P[2] * t0 + P[3] * t1 + w1;
    w0 = n0;
    w1 = n1;
}

// --------------------------------------------------------------- main kernel

struct KArgs {
    const float *x;
    float *y;
    int64_t C, N, ldx, ldy;
    const float *h;
    int32_t M, KBL;
    const SecTab *tab;
    int32_t S;
    const float *state_in;
    float *state_out;
    float *ckpt;
    uint64_t *recs;
    uint32_t *hdr;
    int64_t ntiles, cpad;
    int32_t vec;          // x and y rows 16-byte aligned: float4 tile I/O
    const float2 *twid;   // e^{-2 pi i j / 4096}
    const float2 *hspec;  // tap spectrum / 4096
};

// ------------------------------------------------------------------ FFT part

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

// z[j] *= w (CONJ: *= conj(w)) with w = twid[idx(j)]
template <bool CONJ>
__device__ __forceinline__ void cmul_tw(float &r, float &i, float2 w) {
    const float ws = CONJ ? -w.y : w.y;
    const float nr = r * w.x - i * ws;
    const float ni = r * ws + i * w.x;
    r = nr;
    i = ni;
}

// Swizzled LDS addresses of the two exchanges (see the file comment); both are
// bijections onto [0, 4096) and conflict-free for the lane orders used.
__device__ __forceinline__ int ex1(int k1, int b, int c) { return 256 * k1 + 16 * ((b + k1) & 15) + c; }
__device__ __forceinline__ int ex2(int k1, int k2, int c) { return 256 * k1 + 16 * ((k2 + k1) & 15) + (c ^ k1); }

// Overlap-save block of the pair: on return lane t holds the circular
// convolution outputs c[256 a + t], a = 0..15 (real: even channel, imaginary:
// odd channel).  The block input is x[n0 - 1024 + m], m < 4096.
__device__ void fft_block(const KArgs &a, float *lds, int64_t pair, int64_t n0, int tid, float (&zr)[16],
                          float (&zi)[16]) {
    float *Lr = lds, *Li = lds + NFFT;
    const int64_t chA = 2 * pair, chB = 2 * pair + 1;
    const float *xA = a.x + chA * a.ldx;
    const float *xB = chB < a.C ? a.x + chB * a.ldx : nullptr;
    const int64_t base = n0 - FFT_DISCARD;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t n = base + 256 * q + tid;
        const bool in = n >= 0 && n < a.N;
        zr[q] = in ? xA[n] : 0.f;
        zi[q] = (in && xB) ? xB[n] : 0.f;
    }
    // ---- forward: pass over a (lane = 16 b + c)
    dft16<-1>(zr, zi);
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) cmul_tw<false>(zr[k1], zi[k1], a.twid[(tid * k1) & (NFFT - 1)]);
    {
        const int b = tid >> 4, c = tid & 15;
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) {
            Lr[ex1(k1, b, c)] = zr[k1];
            Li[ex1(k1, b, c)] = zi[k1];
        }
    }
    __syncthreads();
    {  // pass over b (lane = 16 k1 + c)
        const int k1 = tid >> 4, c = tid & 15;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            zr[b] = Lr[ex1(k1, b, c)];
            zi[b] = Li[ex1(k1, b, c)];
        }
        dft16<-1>(zr, zi);
#pragma unroll
        for (int k2 = 1; k2 < 16; ++k2) cmul_tw<false>(zr[k2], zi[k2], a.twid[(16 * c * k2) & (NFFT - 1)]);
        __syncthreads();
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) {
            Lr[ex2(k1, k2, c)] = zr[k2];
            Li[ex2(k1, k2, c)] = zi[k2];
        }
    }
    __syncthreads();
    {  // pass over c (lane = 16 k2 + k1); X[k1 + 16 k2 + 256 k3] = X[tid + 256 k3]
        const int k1 = tid & 15, k2 = tid >> 4;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            zr[c] = Lr[ex2(k1, k2, c)];
            zi[c] = Li[ex2(k1, k2, c)];
        }
        dft16<-1>(zr, zi);
        // ---- spectrum product (the 1/4096 of the inverse is folded into H)
#pragma unroll
        for (int k3 = 0; k3 < 16; ++k3) cmul_tw<false>(zr[k3], zi[k3], a.hspec[tid + 256 * k3]);
        // ---- inverse: pass over k3
        dft16<1>(zr, zi);
#pragma unroll
        for (int c = 1; c < 16; ++c) cmul_tw<true>(zr[c], zi[c], a.twid[(16 * c * k2) & (NFFT - 1)]);
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            Lr[ex2(k1, k2, c)] = zr[c];
            Li[ex2(k1, k2, c)] = zi[c];
        }
    }
    __syncthreads();
    {  // pass over k2 (lane = 16 k1 + c)
        const int k1 = tid >> 4, c = tid & 15;
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) {
            zr[k2] = Lr[ex2(k1, k2, c)];
            zi[k2] = Li[ex2(k1, k2, c)];
        }
        dft16<1>(zr, zi);
#pragma unroll
        for (int b = 0; b < 16; ++b) cmul_tw<true>(zr[b], zi[b], a.twid[((16 * b + c) * k1) & (NFFT - 1)]);
        __syncthreads();
#pragma unroll
        for (int b = 0; b < 16; ++b) {
            Lr[ex1(k1, b, c)] = zr[b];
            Li[ex1(k1, b, c)] = zi[b];
        }
    }
    __syncthreads();
    {  // pass over k1 (lane = 16 b + c): outputs c[256 a + tid]
        const int b = tid >> 4, c = tid & 15;
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) {
            zr[k1] = Lr[ex1(k1, b, c)];
            zi[k1] = Li[ex1(k1, b, c)];
        }
        dft16<1>(zr, zi);
    }
}

// ------------------------------------------------------------------ IIR part

template <typename CT> struct Tab;
template <> struct Tab<float> {
    static __device__ __forceinline__ const float *fold(const SecTab &t, int k) { return t.fold[k]; }
    static __device__ __forceinline__ const float *psi(const SecTab &t, int w) { return t.psi[w]; }
    static __device__ __forceinline__ const float *lb(const SecTab &t, int j) { return t.lb[j]; }
};
template <> struct Tab<double> {
    static __device__ __forceinline__ const double *fold(const SecTab &t, int k) { return t.fold_d[k]; }
    static __device__ __forceinline__ const double *psi(const SecTab &t, int w) { return t.psi_d[w]; }
    static __device__ __forceinline__ const double *lb(const SecTab &t, int j) { return t.lb_d[j]; }
};

// Decoupled look-back of one (channel, tile, section) by one full wave.
// Publishes the tile aggregate, then returns the state entering the tile.
// Lane l watches predecessor base - l (a window of 64 tiles per step); a lane
// stops re-reading its record once the aggregate or the prefix is out, so the
// spin costs one 32-byte read per still-missing predecessor.
template <typename CT>
__device__ void lookback(const KArgs &a, const SecTab &tb, int64_t ch, int64_t tile, int s, int lane,
                         uint32_t epoch, CT agg0, CT agg1, CT &P0, CT &P1) {
    const int64_t S = a.S;
    const int64_t rec0 = ch * a.ntiles * S + s;  // record of tile q: rec0 + q * S
    publish(a.recs, rec0 + tile * S, 0, epoch, (float)agg0, (float)agg1, lane);
    CT acc0 = 0, acc1 = 0;
    CT M0 = 1, M1 = 0, M2 = 0, M3 = 1;  // PhiT^(64 * windows consumed)
    int64_t base = tile - 1;
    while (true) {
        const int64_t q = base - lane;
        int st = q < 0 ? 3 : 0;  // 0 missing, 1 aggregate, 2 prefix, 3 before tile 0
        float r0 = 0.f, r1 = 0.f;
        int64_t spins = 0;
        while (true) {
            if (st == 0) {
                const uint64_t *p = a.recs + (rec0 + q * S) * REC_WORDS;
                uint64_t w[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) w[i] = ld_word(p + i);
                st = decode_record(w, epoch, r0, r1);
            }
            const unsigned long long fm = __ballot(st == 2);
            const int first = fm ? (__ffsll(fm) - 1) : 63;
            if (!__ballot(st == 0 && lane <= first)) break;
            if (++spins > SPIN_MAX) {  // never expected: report and finish
                atomicOr(&a.hdr[HDR_ERROR], 1u);
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
                if (lane + d < 64) madd2(v0, v1, Tab<CT>::lb(tb, k), t0, t1);
            }
            R0 = __shfl(v0, 0);
            R1 = __shfl(v1, 0);
        }
        acc0 += M0 * R0 + M1 * R1;
        acc1 += M2 * R0 + M3 * R1;
        if (fm) break;
        const CT *B = Tab<CT>::lb(tb, 6);
        const CT n0 = M0 * B[0] + M1 * B[2], n1 = M0 * B[1] + M1 * B[3];
        const CT n2 = M2 * B[0] + M3 * B[2], n3 = M2 * B[1] + M3 * B[3];
        M0 = n0; M1 = n1; M2 = n2; M3 = n3;
        base -= 64;
    }
    P0 = acc0;
    P1 = acc1;
}

struct TileCtx {
    int64_t tile, ch;
    uint32_t epoch;
    int tid, lane, grp, gl, gw;
    bool valid, is_last;
    int r_last, owner;
};

// One section over the group's tile: zero-state response, carry, correction.
// s_agg / s_pre are double-buffered by section parity, so no barrier is
// needed at the end of a section.
template <typename CT>
__device__ void run_section(const KArgs &a, const SecTab &tb, int s, float (&v)[L], const TileCtx &c,
                            double (*s_agg)[GWAVES][2], double (*s_pre)[2]) {
    const float b0 = tb.coef[0], b1 = tb.coef[1], b2 = tb.coef[2];
    const float a1 = tb.coef[3], a2 = tb.coef[4];
    const int buf = (s & 1) * GROUPS + c.grp;
    float s1 = 0.f, s2 = 0.f, c1 = 0.f, c2 = 0.f;
    if (c.is_last) {
#pragma unroll
        for (int r = 0; r < L; ++r) {
            const float xv = v[r];
            const float yv = fmaf(b0, xv, s1);
            s1 = fmaf(b1, xv, fmaf(-a1, yv, s2));
            s2 = fmaf(b2, xv, -a2 * yv);
            v[r] = yv;
            if (r == c.r_last) {
                c1 = s1;
                c2 = s2;
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < L; ++r) {
            const float xv = v[r];
            const float yv = fmaf(b0, xv, s1);
            s1 = fmaf(b1, xv, fmaf(-a1, yv, s2));
            s2 = fmaf(b2, xv, -a2 * yv);
            v[r] = yv;
        }
    }
    // 2. inclusive scan over the wave's 64 chunks: within rows of 16 lanes by
    //    DPP row shifts (out-of-row sources read 0), then the row totals by
    //    row broadcasts, weighted by the lane's own power of Phi
    CT w0 = (CT)s1, w1 = (CT)s2;
    {
        CT t0 = dpp<DPP_ROW_SHR + 1>(w0), t1 = dpp<DPP_ROW_SHR + 1>(w1);
        madd2(w0, w1, Tab<CT>::fold(tb, 1), t0, t1);
        t0 = dpp<DPP_ROW_SHR + 2>(w0);
        t1 = dpp<DPP_ROW_SHR + 2>(w1);
        madd2(w0, w1, Tab<CT>::fold(tb, 2), t0, t1);
        t0 = dpp<DPP_ROW_SHR + 4>(w0);
        t1 = dpp<DPP_ROW_SHR + 4>(w1);
        madd2(w0, w1, Tab<CT>::fold(tb, 4), t0, t1);
        t0 = dpp<DPP_ROW_SHR + 8>(w0);
        t1 = dpp<DPP_ROW_SHR + 8>(w1);
        madd2(w0, w1, Tab<CT>::fold(tb, 8), t0, t1);
        t0 = dpp<DPP_ROW_BCAST15, 0xA>(w0);  // rows 1, 3 take lane 15 of rows 0, 2
        t1 = dpp<DPP_ROW_BCAST15, 0xA>(w1);
        madd2(w0, w1, Tab<CT>::fold(tb, (c.lane & 15) + 1), t0, t1);
        t0 = dpp<DPP_ROW_BCAST31, 0xC>(w0);  // rows 2, 3 take lane 31
        t1 = dpp<DPP_ROW_BCAST31, 0xC>(w1);
        madd2(w0, w1, Tab<CT>::fold(tb, (c.lane & 31) + 1), t0, t1);
    }
    if (c.lane == 63) {
        s_agg[buf][c.gw][0] = (double)w0;
        s_agg[buf][c.gw][1] = (double)w1;
    }
    __syncthreads();
    // 3. wave-entering states for a zero tile-entering state; E ends as the
    //    tile aggregate
    const CT *Psi = Tab<CT>::psi(tb, 1);
    CT E0 = 0, E1 = 0, ew0 = 0, ew1 = 0;
#pragma unroll
    for (int w = 0; w < GWAVES; ++w) {
        if (w == c.gw) {
            ew0 = E0;
            ew1 = E1;
        }
        const CT g0 = (CT)s_agg[buf][w][0], g1 = (CT)s_agg[buf][w][1];
        const CT n0 = Psi[0] * E0 + Psi[1] * E1 + g0;
        const CT n1 = Psi[2] * E0 + Psi[3] * E1 + g1;
        E0 = n0;
        E1 = n1;
    }
    // 4. tile prefix, by the group's first wave
    if (c.gw == 0) {
        CT P0 = 0, P1 = 0;
        if (c.tile == 0) {
            if (a.state_in && c.valid) {
                P0 = (CT)a.state_in[(c.ch * a.S + s) * 2 + 0];
                P1 = (CT)a.state_in[(c.ch * a.S + s) * 2 + 1];
            }
        } else {
            lookback<CT>(a, tb, c.ch, c.tile, s, c.lane, c.epoch, E0, E1, P0, P1);
        }
        {
            const CT *PT = Tab<CT>::lb(tb, 0);
            const int64_t r = (c.ch * a.ntiles + c.tile) * a.S + s;
            publish(a.recs, r, 1, c.epoch, (float)(PT[0] * P0 + PT[1] * P1 + E0),
                    (float)(PT[2] * P0 + PT[3] * P1 + E1), c.lane);
        }
        if (c.lane == 0) {
            s_pre[buf][0] = (double)P0;
            s_pre[buf][1] = (double)P1;
            if (a.ckpt && c.valid) {
                a.ckpt[((c.ch * a.ntiles + c.tile) * a.S + s) * 2 + 0] = (float)P0;
                a.ckpt[((c.ch * a.ntiles + c.tile) * a.S + s) * 2 + 1] = (float)P1;
            }
        }
    }
    __syncthreads();
    // 5. chunk-entering state, then its zero-input response added in place
    const CT P0 = (CT)s_pre[buf][0], P1 = (CT)s_pre[buf][1];
    const CT *Pw = Tab<CT>::psi(tb, c.gw);
    const CT e0 = ew0 + Pw[0] * P0 + Pw[1] * P1;
    const CT e1 = ew1 + Pw[2] * P0 + Pw[3] * P1;
    const CT pv0 = dpp<DPP_WAVE_SHR1>(w0), pv1 = dpp<DPP_WAVE_SHR1>(w1);  // lane 0 reads 0
    const CT *F = Tab<CT>::fold(tb, c.lane);
    float z1 = (float)(pv0 + F[0] * e0 + F[1] * e1);
    float z2 = (float)(pv1 + F[2] * e0 + F[3] * e1);
    if (c.is_last) {
#pragma unroll
        for (int r = 0; r < L; ++r) {
            v[r] += z1;
            const float n1 = fmaf(-a1, z1, z2);
            z2 = -a2 * z1;
            z1 = n1;
            if (r == c.r_last) {  // state after the last sample = ZSR + ZIR states
                c1 += z1;
                c2 += z2;
            }
        }
        if (c.valid && c.gl == c.owner && a.state_out) {
            a.state_out[(c.ch * a.S + s) * 2 + 0] = c1;
            a.state_out[(c.ch * a.S + s) * 2 + 1] = c2;
        }
    } else {
#pragma unroll
        for (int r = 0; r < L; ++r) {
            v[r] += z1;
            const float n1 = fmaf(-a1, z1, z2);
            z2 = -a2 * z1;
            z1 = n1;
        }
    }
}

__device__ __forceinline__ void load_chunk(const float *stg, int gl, float (&v)[L]) {
#pragma unroll
    for (int q = 0; q < L / 4; ++q) {
        const float4 t4 = *reinterpret_cast<const float4 *>(&stg[gl * CSTRIDE + 4 * q]);
        v[4 * q + 0] = t4.x;
        v[4 * q + 1] = t4.y;
        v[4 * q + 2] = t4.z;
        v[4 * q + 3] = t4.w;
    }
}

template <int FIRM, bool HAS_SOS>
__global__ __launch_bounds__(WG) void chain_kernel(KArgs a) {
    __shared__ __align__(16) float lds[lds_floats<FIRM>()];
    __shared__ double s_agg[2 * GROUPS][GWAVES][2];
    __shared__ double s_pre[2 * GROUPS][2];
    __shared__ uint32_t s_epoch;

    TileCtx c;
    c.tid = threadIdx.x;
    c.lane = c.tid & 63;
    c.grp = c.tid / GL;
    c.gl = c.tid % GL;
    c.gw = c.gl >> 6;
    const uint64_t id = blockIdx.x;
    c.epoch = 0;
    if (HAS_SOS) {
        if (c.tid == 0) s_epoch = __hip_atomic_load(&a.hdr[HDR_EPOCH], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        c.epoch = s_epoch;
    }
    const uint64_t npairs = (uint64_t)(a.cpad / 2);
    c.tile = (int64_t)(id / npairs);
    const int64_t pair = (int64_t)(id % npairs);
    c.ch = 2 * pair + c.grp;
    c.valid = c.ch < a.C;
    const int64_t n0 = c.tile * T;
    float v[L];
    float *stg = lds + c.grp * (FIRM == FIR_DIRECT ? DIRECT_GROUP_FLOATS : STG_FLOATS);

    if (FIRM == FIR_NONE) {
        const float *xc = a.x + c.ch * a.ldx + n0;
        const int64_t rem = a.N - n0;  // samples of this tile inside the signal
        if (a.vec && rem >= T) {
            float4 t4[T / (4 * GL)];
#pragma unroll
            for (int k = 0; k < T / (4 * GL); ++k)
                t4[k] = c.valid ? reinterpret_cast<const float4 *>(xc)[c.gl + GL * k] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int k = 0; k < T / (4 * GL); ++k)
                *reinterpret_cast<float4 *>(&stg[cphys(4 * (c.gl + GL * k))]) = t4[k];
        } else {  // ragged last tile or unaligned rows
#pragma unroll 4
            for (int k = 0; k < T / GL; ++k) {
                const int i = c.gl + GL * k;
                stg[cphys(i)] = (c.valid && i < rem) ? xc[i] : 0.f;
            }
        }
        __syncthreads();
        load_chunk(stg, c.gl, v);
    } else if (FIRM == FIR_DIRECT) {
        const float *xc = a.x + c.ch * a.ldx;
        const int p0 = c.gl * L;
        float acc[L];
#pragma unroll
        for (int r = 0; r < L; ++r) acc[r] = 0.f;
        for (int k0 = 0; k0 < a.M; k0 += a.KBL) {
            __syncthreads();
            const int64_t src0 = n0 - (k0 + a.KBL - 1);
            for (int i0 = 0; i0 < T + a.KBL; i0 += 8 * GL) {
                float t8[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = i0 + c.gl + GL * u;
                    const int64_t n = src0 + i;
                    t8[u] = (c.valid && i < T + a.KBL && n >= 0 && n < a.N) ? xc[n] : 0.f;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = i0 + c.gl + GL * u;
                    if (i < T + a.KBL) stg[cphys(i)] = t8[u];
                }
            }
            __syncthreads();
            const int kend = min(a.KBL, a.M - k0);
            for (int kb = 0; kb < kend; kb += KB) {
                // window W[i] = x[n0 + p0 - kbase - (KB-1) + i], i < L + KB
                const int base0 = p0 + a.KBL - KB - kb;
                float W[L + KB];
#pragma unroll
                for (int q = 0; q < (L + KB) / 4; ++q) {
                    const float4 t4 = *reinterpret_cast<const float4 *>(&stg[cphys(base0 + 4 * q)]);
                    W[4 * q + 0] = t4.x;
                    W[4 * q + 1] = t4.y;
                    W[4 * q + 2] = t4.z;
                    W[4 * q + 3] = t4.w;
                }
                const int kbase = k0 + kb;
#pragma unroll
                for (int j = 0; j < KB; ++j) {
                    const float hj = (kbase + j < a.M) ? a.h[kbase + j] : 0.f;
#pragma unroll
                    for (int r = 0; r < L; ++r) acc[r] = fmaf(hj, W[r - j + KB - 1], acc[r]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < L; ++r) v[r] = acc[r];
    } else {  // FIR_FFT
        float zr[16], zi[16];
        fft_block(a, lds, pair, n0, c.tid, zr, zi);
        if (!HAS_SOS) {
            const int64_t chA = 2 * pair, chB = chA + 1;
            float *yA = a.y + chA * a.ldy;
            float *yB = a.y + chB * a.ldy;
#pragma unroll
            for (int q = 4; q < 16; ++q) {
                const int64_t n = n0 + 256 * (q - 4) + c.tid;
                if (n < a.N) {
                    yA[n] = zr[q];
                    if (chB < a.C) yB[n] = zi[q];
                }
            }
            return;
        }
        __syncthreads();  // FFT buffers become the two staging areas
        float *stA = lds, *stB = lds + STG_FLOATS;
#pragma unroll
        for (int q = 4; q < 16; ++q) {
            const int j = 256 * (q - 4) + c.tid;
            stA[cphys(j)] = zr[q];
            stB[cphys(j)] = zi[q];
        }
        __syncthreads();
        load_chunk(stg, c.gl, v);
    }

    if (HAS_SOS) {
        c.is_last = (c.tile == a.ntiles - 1);
        const int64_t plast = a.N - 1 - n0;
        c.r_last = c.is_last ? (int)(plast % L) : 0;
        c.owner = c.is_last ? (int)(plast / L) : -1;
        for (int s = 0; s < a.S; ++s) {
            const SecTab &tb = a.tab[s];
            if (tb.hiq)
                run_section<double>(a, tb, s, v, c, s_agg, s_pre);
            else
                run_section<float>(a, tb, s, v, c, s_agg, s_pre);
        }
    }

    __syncthreads();
#pragma unroll
    for (int q = 0; q < L / 4; ++q)
        *reinterpret_cast<float4 *>(&stg[c.gl * CSTRIDE + 4 * q]) =
            make_float4(v[4 * q + 0], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    __syncthreads();
    if (c.valid) {
        float *yc = a.y + c.ch * a.ldy + n0;
        const int64_t rem = a.N - n0;
        if (a.vec && rem >= T) {
#pragma unroll
            for (int k = 0; k < T / (4 * GL); ++k) {
                const int f = c.gl + GL * k;
                reinterpret_cast<float4 *>(yc)[f] = *reinterpret_cast<const float4 *>(&stg[cphys(4 * f)]);
            }
        } else {
#pragma unroll 4
            for (int k = 0; k < T / GL; ++k) {
                const int i = c.gl + GL * k;
                if (i < rem) yc[i] = stg[cphys(i)];
            }
        }
    }
}

// Advances the look-back epoch after a run (stream-ordered behind it).
__global__ void bump_epoch_kernel(uint32_t *hdr) {
    uint32_t ne = (hdr[HDR_EPOCH] + 1u) & EPOCH_MASK;
    hdr[HDR_EPOCH] = ne == 0u ? 1u : ne;
}

// ------------------------------------------------------------------- host

static size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

WsLayout ws_layout(int64_t C, int64_t N, int32_t S, int32_t M_merged, int32_t n_fir, int32_t fir_mode) {
    WsLayout w{};
    w.ntiles = (N + T - 1) / T;
    w.cpad = C + (C & 1);
    size_t off = 0;
    w.hdr = off;
    off += 256;
    w.tab = off;
    off += al256(sizeof(SecTab) * (size_t)S);
    const size_t nrec = (size_t)w.cpad * (size_t)w.ntiles * (size_t)S;
    w.recs = off;
    off += al256(nrec * REC_WORDS * sizeof(uint64_t));
    w.taps = w.merge = off;
    if (n_fir > 1) {
        off += al256((size_t)M_merged * sizeof(float));
        w.merge = off;
        off += al256((size_t)M_merged * 2 * sizeof(double));
    }
    w.twid = w.hspec = w.tw64 = off;
    if (fir_mode == FIR_FFT) {
        off += al256(NFFT * sizeof(float2));
        w.hspec = off;
        off += al256(NFFT * sizeof(float2));
        w.tw64 = off;
        off += al256(NFFT * sizeof(double2));
    }
    w.total = (S > 0 || n_fir > 1 || fir_mode == FIR_FFT) ? off : 0;
    return w;
}

// kernels of the prepare step (tfx_tables.hip)
hipError_t launch_tables(const ChainPlan &p, const WsLayout &lay, const float *h, int32_t M);
hipError_t launch_state_passthrough(const float *in, float *out, int64_t n, hipStream_t st);

template <int F, bool S>
static hipError_t launch_main(const KArgs &k, int64_t nblocks, hipStream_t st) {
    hipLaunchKernelGGL((chain_kernel<F, S>), dim3((unsigned)nblocks), dim3(WG), 0, st, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !S) return e;
    hipLaunchKernelGGL(bump_epoch_kernel, dim3(1), dim3(1), 0, st, k.hdr);
    return hipGetLastError();
}

static int32_t merged_taps(const StageList &f) {
    int32_t Mtot = 0;
    for (int i = 0; i < f.n; ++i) Mtot += (i == 0) ? f.len[i] : f.len[i] - 1;
    return Mtot;
}

static const float *taps_ptr(const ChainPlan &p, const WsLayout &lay) {
    if (p.firs.n == 1) return p.firs.ptr[0];
    if (p.firs.n > 1) return reinterpret_cast<const float *>(static_cast<const char *>(p.ws) + lay.taps);
    return nullptr;
}

hipError_t launch_prepare(const ChainPlan &p) {
    const int32_t Mtot = merged_taps(p.firs);
    const WsLayout lay = ws_layout(p.C, p.N, p.S, Mtot, p.firs.n, p.fir_mode);
    return launch_tables(p, lay, taps_ptr(p, lay), Mtot);
}

hipError_t launch_run(const ChainPlan &p) {
    const int32_t Mtot = merged_taps(p.firs);
    const WsLayout lay = ws_layout(p.C, p.N, p.S, Mtot, p.firs.n, p.fir_mode);
    char *ws = static_cast<char *>(p.ws);
    if (p.N == 0) {
        if (p.state_out && p.S > 0) return launch_state_passthrough(p.state_in, p.state_out, p.C * p.S * 2, p.stream);
        return hipSuccess;
    }
    KArgs k{};
    k.x = p.x;
    k.y = p.y;
    k.C = p.C;
    k.N = p.N;
    k.ldx = p.ldx;
    k.ldy = p.ldy;
    k.M = Mtot;
    k.h = taps_ptr(p, lay);
    k.KBL = 0;
    if (Mtot > 0) {
        const int32_t m16 = (Mtot + KB - 1) / KB * KB;
        k.KBL = m16 < KBLK_MAX ? m16 : KBLK_MAX;
    }
    k.S = p.S;
    k.state_in = p.state_in;
    k.state_out = p.state_out;
    k.ckpt = p.ckpt;
    k.ntiles = lay.ntiles;
    k.cpad = lay.cpad;
    k.hdr = reinterpret_cast<uint32_t *>(ws + lay.hdr);
    k.tab = reinterpret_cast<const SecTab *>(ws + lay.tab);
    k.recs = reinterpret_cast<uint64_t *>(ws + lay.recs);
    k.vec = ((reinterpret_cast<uintptr_t>(p.x) | reinterpret_cast<uintptr_t>(p.y)) % 16 == 0 && p.ldx % 4 == 0 &&
             p.ldy % 4 == 0) ? 1 : 0;
    k.twid = reinterpret_cast<const float2 *>(ws + lay.twid);
    k.hspec = reinterpret_cast<const float2 *>(ws + lay.hspec);
    const int64_t nblocks = (lay.cpad / 2) * lay.ntiles;
    const bool s = p.S > 0;
    switch (Mtot > 0 ? p.fir_mode : FIR_NONE) {
        case FIR_DIRECT: return s ? launch_main<FIR_DIRECT, true>(k, nblocks, p.stream)
                                  : launch_main<FIR_DIRECT, false>(k, nblocks, p.stream);
        case FIR_FFT: return s ? launch_main<FIR_FFT, true>(k, nblocks, p.stream)
                               : launch_main<FIR_FFT, false>(k, nblocks, p.stream);
        default: return s ? launch_main<FIR_NONE, true>(k, nblocks, p.stream)
                          : launch_main<FIR_NONE, false>(k, nblocks, p.stream);
    }
}

}  // namespace tfx
