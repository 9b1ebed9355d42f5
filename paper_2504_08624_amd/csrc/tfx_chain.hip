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
// radius exceeds 0.999; the per-sample recursion is fp32.  The shared pieces
// (records, DPP moves, FFT passes, carry engine) live in tfx_device.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <type_traits>

#include "tfx_device.h"
#include "tfx_mc.h"

namespace tfx {

constexpr int DIRECT_GROUP_FLOATS = ((T + KBLK_MAX + L - 1) / L + 1) * CSTRIDE;
// kernel variant of FIR_FFT for filters of more than one tap partition
constexpr int FIR_FFT_PARTS = 4;
// Kernel-internal FIR mode: the matrix-core (block-Toeplitz) FIR fused into the
// chain kernel, bf16 or fp16 operands.
constexpr int FIR_TZ_BF16 = 5, FIR_TZ_F16 = 6;
template <int FIRM>
constexpr bool is_tz() { return FIRM == FIR_TZ_BF16 || FIRM == FIR_TZ_F16; }

template <int FIRM>
constexpr bool is_fft() { return FIRM == FIR_FFT || FIRM == FIR_FFT_PARTS; }

// LDS of the cascade-level look-back (floats): Phi_T, Phi_T^2, Phi_T^4 and a
// window weight per group (D x D each), tile aggregate and prefix per group.
// After the FFT the tail of its buffers beyond the two staging areas is free.
constexpr int FFT_TAIL_FLOATS = 2 * NFFT - GROUPS * STG_FLOATS;
__host__ __device__ constexpr bool casc_in_tail(int FIRM, int S) {
    return (FIRM == FIR_FFT || FIRM == 4) && casc_floats(2 * S) <= FFT_TAIL_FLOATS;
}

template <int FIRM>
constexpr int lds_floats() {
    // the partitioned FFT keeps its spectrum accumulator in LDS after the
    // FFT buffers
    return FIRM == FIR_DIRECT ? GROUPS * DIRECT_GROUP_FLOATS
                              : (FIRM == FIR_FFT_PARTS ? 4 * NFFT : (FIRM == FIR_FFT ? 2 * NFFT : GROUPS * STG_FLOATS));
}
static_assert(GROUPS * STG_FLOATS <= 2 * NFFT, "staging must fit in the FFT buffers");

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
    int32_t correlate;    // FIR part: y[n] = sum_k h[k] x[n+k] (adjoint) instead of convolution
    const float2 *twid;   // e^{-2 pi i j / 4096}
    const float2 *hspec;  // [nparts][4096] spectra of the tap partitions / 4096
    int32_t nparts;
    const CascTab *casc;  // cascade tile-transition powers (cascade-level look-back)
    const CascZir *zir;   // zero-input response tables of the cascade
    const McTab *mc;      // matrix-core cascade tables
    const void *tzb;      // fused Toeplitz FIR: B operand table [2 Q][64][8]
    int32_t tzQ;          // its frame lags Q
    const float *hist;    // streaming: the M - 1 FIR inputs before the block, [C][M - 1] (null = zeros)
    int64_t ldh;          // M - 1
    uint32_t xcd_ks;      // block order: xcd_order's log2 K (0 = block ids in order)
};

// FIR input x[ch][n] of the block, n < N, with the streaming history for
// n in [-(M - 1), 0) and zeros before it.
__device__ __forceinline__ float fir_input(const KArgs &a, const float *xc, int64_t ch, int64_t n) {
    if (n >= 0) return n < a.N ? xc[n] : 0.f;
    return (a.hist && n >= -a.ldh) ? a.hist[ch * a.ldh + a.ldh + n] : 0.f;
}

// Fused matrix-core FIR of a tile (both channels of the pair), written into
// the two staging areas.  With frames of TP = 32 samples,
//     y[32 b + i] = sum_{q, m} x[32 (b - q) + m] h[32 q + i - m],
// a (frames x 32 Q) by (32 Q x 32) product per channel whose tap operand B is
// the prepared table of the stand-alone Toeplitz kernel.  The tile is 96
// frames per channel, three 32-frame accumulator tiles, six for the pair;
// wave w takes tiles w and w + 4.  The signal operand A (frames converted to
// bf16 / fp16) is staged in the staging areas TZ_QC lags at a time: frames
// F0 - (q1 - 1) .. F0 + 95 of each channel, where tile u's row for lag q and
// frame F0 + 32 t + r is 32 t + r + q1 - 1 - q.
constexpr int TZ_QC = 64;
constexpr int TZ_PF = 4;  // tap-fragment loads in flight
constexpr int TZ_SU = 2;  // operand staging loads in flight per thread
constexpr int TZ_ROWS = T / TP + TZ_QC - 1;
static_assert(GROUPS * TZ_ROWS * TROW * 2 <= GROUPS * STG_FLOATS * 4, "Toeplitz operands must fit in the staging");
// MCL: the output goes to the matrix-core cascade's chunk layout (chunk k
// of channel g at g * 96 * 36 + 36 k) instead of the staging areas.
template <int MODE, bool MCL = false>
__device__ void tz_tile(const KArgs &a, float *lds, int64_t pair, int64_t n0, int tid) {
    typedef Op<MODE> O;
    typedef typename O::T Tt;
    typedef typename O::V V;
    typedef Tt T4 __attribute__((ext_vector_type(4)));
    Tt *ast = reinterpret_cast<Tt *>(lds);  // [GROUPS][TZ_ROWS][TROW]
    const int lane = tid & 63, w = tid >> 6, r32 = lane & 31, kh = lane >> 5;
    const int ntl = w < 2 ? 2 : 1;  // tiles of this wave: w, w + 4
    const int64_t F0 = n0 / TP;
    const V *bt = static_cast<const V *>(a.tzb);
    f32x16 acc[2];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[k][r] = 0.f;
    for (int q0 = 0; q0 < a.tzQ; q0 += TZ_QC) {
        const int q1 = min(a.tzQ, q0 + TZ_QC);
        const int nrows = T / TP + (q1 - q0) - 1;
        const int64_t fbase = F0 - (q1 - 1);
        __syncthreads();  // the previous pass's operand reads
#pragma unroll
        for (int g = 0; g < GROUPS; ++g) {
            const int64_t ch = 2 * pair + g;
            const float *xc = a.x + ch * a.ldx;
            Tt *ag = ast + g * TZ_ROWS * TROW;
            const int total = nrows * (TP / 4);
            const int64_t nlo = fbase * TP, nhi = (fbase + nrows) * TP;
            if (ch < a.C && a.vec && nlo >= 0 && nhi <= a.N) {
                // inside the signal: TZ_SU four-sample loads in flight per thread
                for (int e0 = tid; e0 < total; e0 += TZ_SU * WG) {
                    float4 t[TZ_SU];
#pragma unroll
                    for (int k = 0; k < TZ_SU; ++k) {
                        // clamped, not skipped: loads inside a branch are each waited for
                        const int e = min(e0 + k * WG, total - 1);
                        t[k] = *reinterpret_cast<const float4 *>(xc + nlo + 4 * e);
                    }
#pragma unroll
                    for (int k = 0; k < TZ_SU; ++k) {
                        const int e = e0 + k * WG;
                        if (e < total) {
                            T4 t4;
                            t4[0] = (Tt)t[k].x;
                            t4[1] = (Tt)t[k].y;
                            t4[2] = (Tt)t[k].z;
                            t4[3] = (Tt)t[k].w;
                            *reinterpret_cast<T4 *>(&ag[(e >> 3) * TROW + 4 * (e & 7)]) = t4;
                        }
                    }
                }
                continue;
            }
            for (int e = tid; e < total; e += WG) {
                const int row = e >> 3, c4 = e & 7;  // TP / 4 = 8 four-sample pieces a row
                const int64_t n = (fbase + row) * TP + 4 * c4;
                float v4[4];
                if (ch < a.C && a.vec && n >= 0 && n + 3 < a.N) {
                    const float4 t = *reinterpret_cast<const float4 *>(xc + n);
                    v4[0] = t.x;
                    v4[1] = t.y;
                    v4[2] = t.z;
                    v4[3] = t.w;
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) v4[u] = ch < a.C ? fir_input(a, xc, ch, n + u) : 0.f;
                }
                T4 t4;
#pragma unroll
                for (int u = 0; u < 4; ++u) t4[u] = (Tt)v4[u];
                *reinterpret_cast<T4 *>(&ag[row * TROW + 4 * c4]) = t4;
            }
        }
        __syncthreads();
        // steps st = 2 q + hh; tap fragments are loaded TZ_PF steps ahead
        // through a ring, every load index clamped to the last step (no
        // branch around a load), and each step reads the next step's signal
        // fragments before it issues its own products
        const int s0 = 2 * q0, s1 = 2 * q1;
        V bq[TZ_PF];
#pragma unroll
        for (int i = 0; i < TZ_PF; ++i) bq[i] = bt[(int64_t)min(s0 + i, s1 - 1) * 64 + lane];
        auto afrag = [&](int st, int k) -> V {
            const int q = st >> 1, hh = st & 1, u = w + 4 * k, g = u / 3, t = u % 3;
            const int row = 32 * t + r32 + (q1 - 1 - q);
            return *reinterpret_cast<const V *>(&ast[(g * TZ_ROWS + row) * TROW + 16 * hh + 8 * kh]);
        };
        // NT accumulator tiles (1 or 2, wave-uniform) over the steps
        auto steps = [&](auto nt_c) {
            constexpr int NT = decltype(nt_c)::value;
            V acur[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k) acur[k] = afrag(s0, k);
            int sb = s0;
            for (; sb + TZ_PF <= s1; sb += TZ_PF) {
#pragma unroll
                for (int i = 0; i < TZ_PF; ++i) {
                    const int st = sb + i, sn = min(st + 1, s1 - 1);
                    V anext[NT];
#pragma unroll
                    for (int k = 0; k < NT; ++k) anext[k] = afrag(sn, k);
#pragma unroll
                    for (int k = 0; k < NT; ++k) acc[k] = O::mma(acur[k], bq[i], acc[k]);
                    bq[i] = bt[(int64_t)min(st + TZ_PF, s1 - 1) * 64 + lane];
#pragma unroll
                    for (int k = 0; k < NT; ++k) acur[k] = anext[k];
                    __builtin_amdgcn_sched_group_barrier(0x100, NT, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, NT, 0);
                    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                }
            }
#pragma unroll
            for (int i = 0; i < TZ_PF; ++i) {  // the remaining steps
                const int st = sb + i;
                if (st < s1) {
#pragma unroll
                    for (int k = 0; k < NT; ++k) acc[k] = O::mma(afrag(st, k), bq[i], acc[k]);
                }
            }
        };
        if (ntl == 2)
            steps(std::integral_constant<int, 2>());
        else
            steps(std::integral_constant<int, 1>());
    }
    __syncthreads();  // every operand read done: the staging areas take the output
    // accumulator (row i, column c): lane c + 32 (i / 4 % 2), register
    // 4 (i / 8) + i % 4; output sample 32 (32 t + i) + c of the channel's tile
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (k < ntl) {
            const int u = w + 4 * k, g = u / 3, t = u % 3;
            if constexpr (MCL) {
                float *st = lds + g * (T / TP) * 36;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int i = 8 * (r >> 2) + 4 * kh + (r & 3);
                    st[36 * (32 * t + i) + r32] = acc[k][r];
                }
            } else {
                float *st = lds + g * STG_FLOATS;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int i = 8 * (r >> 2) + 4 * kh + (r & 3);
                    st[cphys(32 * (32 * t + i) + r32)] = acc[k][r];
                }
            }
        }
    }
    __syncthreads();
}

// Overlap-save block of the pair.  Convolution: the block starts 1024 samples
// before the tile and outputs c[256 a + t], a = 4..15, are the tile.
// Correlation (the FIR adjoint, spectrum conjugated): the block starts at the
// tile and outputs a = 0..11 are the tile.  Filters longer than 1025 taps
// (PARTS) are uniformly partitioned: partition p = taps [1025 p, 1025 p +
// 1025) filters its own input block, shifted by 1025 p samples (earlier for
// the convolution, later for the correlation); the products with the
// partition spectra are summed in the frequency domain and inverted once.
// tw: the workgroup's LDS copy of the twiddle table, staged by the caller.
template <bool PARTS>
__device__ void fft_block(const KArgs &a, float *lds, int64_t pair, int64_t n0, int tid, float (&zr)[16],
                          float (&zi)[16], const float2 *tw) {
    const int64_t chA = 2 * pair, chB = 2 * pair + 1;
    const float *xA = a.x + chA * a.ldx;
    const float *xB = chB < a.C ? a.x + chB * a.ldx : nullptr;
    const float *hA = a.hist ? a.hist + chA * a.ldh : nullptr;
    const float *hB = (a.hist && chB < a.C) ? a.hist + chB * a.ldh : nullptr;
    const int64_t hlen = a.hist ? a.ldh : 0;
    const int64_t base = a.correlate ? n0 : n0 - FFT_DISCARD;
    if (!PARTS) {
        load_pair_block(zr, zi, xA, xB, base, a.N, a.N, tid, hA, hB, hlen);
        fft4096_forward(zr, zi, lds, tw, tid);
        spectrum_product(zr, zi, a.hspec, tid, a.correlate != 0);
    } else {
        // spectrum accumulator: lane t owns bins t + 256 k3 (no sharing, no
        // barrier), after the two FFT buffers
        float2 *acc = reinterpret_cast<float2 *>(lds + 2 * NFFT);
#pragma unroll 1
        for (int p = 0; p < a.nparts; ++p) {
            const int64_t shift = (int64_t)FFT_PART * p;
            __syncthreads();  // the previous pass's last LDS reads
            load_pair_block(zr, zi, xA, xB, a.correlate ? base + shift : base - shift, a.N, a.N, tid, hA, hB, hlen);
            fft4096_forward(zr, zi, lds, tw, tid);
            const float2 *hs = a.hspec + (int64_t)p * NFFT;
            const float sg = a.correlate ? -1.f : 1.f;
#pragma unroll 4
            for (int k3 = 0; k3 < 16; ++k3) {
                const float2 w = hs[16 * tid + k3];
                const float wi = sg * w.y;
                float2 s = p ? acc[tid + 256 * k3] : make_float2(0.f, 0.f);
                s.x = fmaf(zr[k3], w.x, fmaf(-zi[k3], wi, s.x));
                s.y = fmaf(zr[k3], wi, fmaf(zi[k3], w.x, s.y));
                acc[tid + 256 * k3] = s;
            }
        }
#pragma unroll
        for (int k3 = 0; k3 < 16; ++k3) {
            const float2 s = acc[tid + 256 * k3];
            zr[k3] = s.x;
            zi[k3] = s.y;
        }
    }
    fft4096_inverse(zr, zi, lds, tw, tid);
    if (a.correlate) {  // move the tile to a = 4..15 like the convolution case
#pragma unroll
        for (int q = 15; q >= 4; --q) {
            zr[q] = zr[q - 4];
            zi[q] = zi[q - 4];
        }
    }
}

// Direct FIR of a group's tile: lane gl gets the outputs gl * L .. gl * L +
// L - 1 of the tile starting at n0 (convolution, or the adjoint correlation)
// in v.  stg: the group's DIRECT_GROUP_FLOATS of LDS.  Contains workgroup
// barriers (every lane of the workgroup calls it).
__device__ void direct_tile(const KArgs &a, float *stg, int64_t ch, bool valid, int gl, int64_t n0, float (&v)[L]) {
    const float *xc = a.x + ch * a.ldx;
    const int p0 = gl * L;
    float acc[L];
#pragma unroll
    for (int r = 0; r < L; ++r) acc[r] = 0.f;
    for (int k0 = 0; k0 < a.M; k0 += a.KBL) {
        __syncthreads();
        // stage x[src0 + i], i < T + KBL: convolution needs x[n - k],
        // correlation x[n + k]
        const int64_t src0 = a.correlate ? n0 + k0 : n0 - (k0 + a.KBL - 1);
        for (int i0 = 0; i0 < T + a.KBL; i0 += 8 * GL) {
            float t8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + gl + GL * u;
                const int64_t n = src0 + i;
                t8[u] = (valid && i < T + a.KBL) ? fir_input(a, xc, ch, n) : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + gl + GL * u;
                if (i < T + a.KBL) stg[cphys(i)] = t8[u];
            }
        }
        __syncthreads();
        const int kend = min(a.KBL, a.M - k0);
        for (int kb = 0; kb < kend; kb += KB) {
            // convolution: W[i] = x[n0 + p0 - kbase - (KB-1) + i];
            // correlation: W[i] = x[n0 + p0 + kbase + i]
            const int base0 = a.correlate ? p0 + kb : p0 + a.KBL - KB - kb;
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
            if (a.correlate) {
#pragma unroll
                for (int j = 0; j < KB; ++j) {
                    const float hj = (kbase + j < a.M) ? a.h[kbase + j] : 0.f;
#pragma unroll
                    for (int r = 0; r < L; ++r) acc[r] = fmaf(hj, W[r + j], acc[r]);
                }
            } else {
#pragma unroll
                for (int j = 0; j < KB; ++j) {
                    const float hj = (kbase + j < a.M) ? a.h[kbase + j] : 0.f;
#pragma unroll
                    for (int r = 0; r < L; ++r) acc[r] = fmaf(hj, W[r - j + KB - 1], acc[r]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < L; ++r) v[r] = acc[r];
}

struct TileCtx {
    int64_t tile, ch;
    uint32_t epoch;
    int tid, lane, grp, gl, gw;
    bool valid, is_last;
    int r_last, owner;
};

// One section over the group's tile: zero-state response, carry, then the
// zero-input response of each chunk-entering state added in place.  s_agg /
// s_pre are double-buffered by section parity (no barrier needed at the end).
// KNOWN: the section's tile-entering state `known` has been produced by the
// cascade-level look-back (no look-back here; the checkpoint is written by
// the caller).
template <typename CT, class TB, bool STOUT, bool KNOWN = false>
__device__ void run_section(const KArgs &a, const TB &tb, int s, float (&v)[L], const TileCtx &c,
                            double (*s_agg)[GWAVES][2], double (*s_pre)[2], const float *known = nullptr) {
    const float b0 = tb.coef[0], b1 = tb.coef[1], b2 = tb.coef[2];
    const float a1 = tb.coef[3], a2 = tb.coef[4];
    float s1 = 0.f, s2 = 0.f, c1 = 0.f, c2 = 0.f;
    if (STOUT && c.is_last) {
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
    CarryCtx cc;
    cc.lane = c.lane;
    cc.gw = c.gw;
    cc.grp = c.grp;
    cc.lookback = true;
    cc.pos = c.tile;
    cc.recs = a.recs;
    cc.rec0 = c.ch * a.ntiles * a.S + s;
    cc.rstride = a.S;
    cc.epoch = c.epoch;
    cc.hdr = a.hdr;
    cc.known0 = cc.known1 = 0.0;
    if (c.tile == 0 && a.state_in && c.valid) {
        cc.known0 = a.state_in[(c.ch * a.S + s) * 2 + 0];
        cc.known1 = a.state_in[(c.ch * a.S + s) * 2 + 1];
    }
    cc.prefix_out = (a.ckpt && c.valid) ? a.ckpt + ((c.ch * a.ntiles + c.tile) * a.S + s) * 2 : nullptr;
    float z1, z2;
    if constexpr (KNOWN) {
        CT E0, E1;
        carry_local<CT, TB>(tb, c.lane, c.gw, s1, s2, (CT)known[0], (CT)known[1], z1, z2, E0, E1, s_agg,
                            (s & 1) * GROUPS + c.grp);
    } else {
        carry<CT, false, TB>(tb, cc, s1, s2, z1, z2, s_agg, s_pre, (s & 1) * GROUPS + c.grp);
    }
    if (STOUT && c.is_last) {
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

// HIQ: the variant with the FP64 carry.  Both variants are launched; the one
// that does not match the workspace's high-Q word exits at once, so the
// common case is compiled without the FP64 path's registers.
// CASC: the cascade (at most CASC_MAX sections, none needing FP64) is run in
// three phases per tile: (A) every section over the tile from a zero
// tile-entering state, giving the cascade's tile aggregate; (B) one
// decoupled look-back of the whole 2S-component cascade state; (C) every
// section again from its now known tile-entering state, with no look-back.
// This trades a second in-tile pass for S - 1 fewer cross-tile round trips,
// which dominate the per-section form.
// Completes a tile of a cascade-level cascade: v holds the response to a zero
// tile-entering state (phase A), P (D = 2S floats, LDS) the state entering
// the tile.  By linearity the output at sample r of chunk k gains
// G[r] . (F^(L k) P): the entering state carried k chunks into the tile,
// then through the cascade to its output, with no further pass per section.
// With k = 16 a + b (a = the lane's 16-lane row), F^(L k) P = F^(L b) R_a,
// R_a = F^(16 L a) P: lane (a, i) forms component i of R_a, each lane takes
// the row's components by lane shuffles.  F is block lower triangular, and
// so are its powers.  The powers are read from LDS (zt_stage): mb[(i D + j)
// 16 + b] = (F^(L b))[i][j] and ma[(a D + j) 16 + i] = (F^(16 L a))[i][j];
// G, read at lane-uniform indices, from global memory.
template <int D>
__device__ __forceinline__ void casc_zir_add(float (&v)[L], const CascZir *zt, const float *mb, const float *P, int k) {
    const int a = k >> 4, b = k & 15, ri = k & 15;
    const float *ma = mb + D * D * 16;
    float ra = 0.f;  // component ri of R_a
    if (ri < D) {
#pragma unroll
        for (int j = 0; j < D; ++j) ra = fmaf(ma[(a * D + j) * 16 + ri], P[j], ra);
    }
    const int row0 = (__lane_id() & ~15);
    float r[D];
#pragma unroll
    for (int j = 0; j < D; ++j) r[j] = __shfl(ra, row0 + j);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float zi = 0.f;  // component i of F^(L b) R_a
#pragma unroll
        for (int j = 0; j < (i | 1) + 1; ++j) zi = fmaf(mb[(i * D + j) * 16 + b], r[j], zi);
#pragma unroll
        for (int q = 0; q < L; ++q) v[q] = fmaf(zt->G[q][i], zi, v[q]);
    }
}

// Copies the rows j < D of Mb and MaT (16 floats each) into LDS at dst, in
// 16-byte pieces, every load issued before the first store.
__device__ __forceinline__ void zt_stage(float *dst, const CascZir *zt, int D, int tid) {
    constexpr int PER = 4;  // pieces per thread per round
    const int nmb = D * D * 4, n = nmb + ZIR_A * D * 4;
    for (int e0 = tid; e0 < n; e0 += PER * WG) {
        float4 t[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = min(e0 + u * WG, n - 1), row = e >> 2, c4 = e & 3;
            const float *src = e < nmb ? &zt->Mb[row / D][row % D][4 * c4]
                                       : &zt->MaT[(row - D * D) / D][(row - D * D) % D][4 * c4];
            t[u] = *reinterpret_cast<const float4 *>(src);
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = e0 + u * WG;
            if (e < n) reinterpret_cast<float4 *>(dst)[e] = t[u];
        }
    }
}

// Cascades up to ZIR_MAX sections (larger ones would cost the kernel
// registers, hence occupancy) use the zero-input response tables.
__device__ __forceinline__ void casc_zir(float (&v)[L], const CascZir *zt, const float *mb, const float *P, int k,
                                         int S) {
    switch (S) {
    case 1: casc_zir_add<2>(v, zt, mb, P, k); break;
    case 2: casc_zir_add<4>(v, zt, mb, P, k); break;
    case 3: casc_zir_add<6>(v, zt, mb, P, k); break;
    case 4: casc_zir_add<8>(v, zt, mb, P, k); break;
    case 5: casc_zir_add<10>(v, zt, mb, P, k); break;
    default: casc_zir_add<12>(v, zt, mb, P, k); break;
    }
}

// Workgroups per CU the variants with the table form are held to (four
// waves per SIMD: at most 128 registers).
template <int FIRM, bool HAS_SOS, bool HIQ, bool CASC, bool STOUT>
constexpr int chain_min_blocks() {
    return (HAS_SOS && CASC && !HIQ && !STOUT && (FIRM == FIR_NONE || FIRM == FIR_FFT)) ? 4 : 1;
}

template <int FIRM, bool HAS_SOS, bool HIQ, bool CASC, bool STOUT>
__global__ __launch_bounds__(WG, (chain_min_blocks<FIRM, HAS_SOS, HIQ, CASC, STOUT>())) void chain_kernel(KArgs a) {
    __shared__ __align__(16) float lds[lds_floats<FIRM>()];
    __shared__ double s_agg[2 * GROUPS][GWAVES][2];
    __shared__ double s_pre[2 * GROUPS][2];
    __shared__ uint32_t s_epoch;
    constexpr bool FFT = FIRM == FIR_FFT || FIRM == FIR_FFT_PARTS;
    // dynamic: the fp32 tables (LDS_SECTIONS sections at a time, or all of a
    // cascade-level cascade without their look-back powers), then the
    // cascade look-back area unless it sits in the FFT buffers' tail
    extern __shared__ __align__(16) unsigned char s_dyn[];
    SecLds *s_tab = reinterpret_cast<SecLds *>(s_dyn);
    SecLdsC *s_tabc = reinterpret_cast<SecLdsC *>(s_dyn);
    // with the FFT FIR the same area first holds the transforms' twiddles
    // (the tables go there once the FIR is done; the launch sizes the area
    // for both)
    float2 *s_twl = reinterpret_cast<float2 *>(s_dyn);

    if (HAS_SOS && (a.hdr[HDR_HIQ] != 0u) != HIQ) {  // the other variant runs
        advance_epoch(a.hdr);
        return;
    }
    TileCtx c;
    c.tid = threadIdx.x;
    c.lane = c.tid & 63;
    c.grp = c.tid / GL;
    c.gl = c.tid % GL;
    c.gw = c.gl >> 6;
    c.epoch = 0;
    if (FFT) {
        // the section tables are staged once the FIR is done: its twiddles
        // hold their LDS area until then
        twl_stage(s_twl, a.twid, c.tid, WG);
        if (HAS_SOS && c.tid == 0) s_epoch = load_epoch(a.hdr, HDR_EPOCH);
        __syncthreads();
        if (HAS_SOS) c.epoch = s_epoch;
    } else if (HAS_SOS) {
        if (c.tid == 0) s_epoch = load_epoch(a.hdr, HDR_EPOCH);
        // the tables' loads overlap the FIR part of the tile
        if (CASC)
            stage_tables(s_tabc, a.tab, 0, a.S, c.tid, WG);
        else
            stage_tables(s_tab, a.tab, 0, min(a.S, LDS_SECTIONS), c.tid, WG);
        __syncthreads();
        c.epoch = s_epoch;
    }
    const uint64_t npairs = (uint64_t)(a.cpad / 2);
    const uint64_t id = xcd_order(blockIdx.x, gridDim.x, a.xcd_ks);
    c.tile = (int64_t)(id / npairs);
    const int64_t pair = (int64_t)(id % npairs);
    c.ch = 2 * pair + c.grp;
    c.valid = c.ch < a.C;
    const int64_t n0 = c.tile * T;
    float v[L];
    float *stg = lds + c.grp * (FIRM == FIR_DIRECT ? DIRECT_GROUP_FLOATS : STG_FLOATS);

    if (FIRM == FIR_NONE) {
        stage_tile(stg, a.x + c.ch * a.ldx + n0, a.N - n0, c.valid, a.vec != 0, c.gl);
        __syncthreads();
        load_chunk(stg, c.gl, v);
    } else if constexpr (is_tz<FIRM>()) {
        tz_tile<FIRM == FIR_TZ_BF16 ? TZ_BF16 : TZ_F16>(a, lds, pair, n0, c.tid);
        load_chunk(stg, c.gl, v);
    } else if (FIRM == FIR_DIRECT) {
        direct_tile(a, stg, c.ch, c.valid, c.gl, n0, v);
    } else {  // FIR_FFT
        float zr[16], zi[16];
        fft_block<FIRM == FIR_FFT_PARTS>(a, lds, pair, n0, c.tid, zr, zi, s_twl);
        if (!HAS_SOS) {
            const int64_t chA = 2 * pair, chB = chA + 1;
            store_pair_tile<4>(zr, zi, a.y + chA * a.ldy, chB < a.C ? a.y + chB * a.ldy : nullptr, n0, a.N, c.tid);
            return;
        }
        __syncthreads();  // FFT buffers become the two staging areas, the twiddles' area the tables
        if (CASC)
            stage_tables(s_tabc, a.tab, 0, a.S, c.tid, WG);
        else
            stage_tables(s_tab, a.tab, 0, min(a.S, LDS_SECTIONS), c.tid, WG);
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

    if (HAS_SOS && CASC) {
        c.is_last = STOUT && (c.tile == a.ntiles - 1);
        const int64_t plast = a.N - 1 - n0;
        c.r_last = c.is_last ? (int)(plast % L) : 0;
        c.owner = c.is_last ? (int)(plast / L) : -1;
        if (FIRM == FIR_DIRECT) store_chunk(stg, c.gl, v);  // keep the cascade input chunk
        // cascade look-back area: T (3 D x D), window weights, E and P
        const int D = 2 * a.S, DD = D * D;
        float *cr = casc_in_tail(FIRM, a.S) ? lds + GROUPS * STG_FLOATS
                                            : reinterpret_cast<float *>(s_dyn + a.S * sizeof(SecLdsC));
        float *cT = cr, *cM = cr + 3 * DD + c.grp * DD, *cE = cr + (3 + GROUPS) * DD + 32 * c.grp, *cP = cE + 16;
        for (int e = c.tid; e < 3 * DD; e += WG) {  // read in phase B, after phase A's barriers
            const int k = e / DD, i = (e % DD) / D, j = e % D;
            cT[e] = a.casc->T[k][i][j];
        }
        // (A) zero tile-entering state: the cascade's tile aggregate and its
        //     response to the tile's input
        float eA0 = 0.f, eA1 = 0.f;
        for (int s = 0; s < a.S; ++s) {
            float e0, e1, E0, E1;
            const int buf = (s & 1) * GROUPS + c.grp;
            casc_section_a<L, true>(s_tabc[s], v, c.lane, c.gw, s_agg, buf, e0, e1, E0, E1);
            if (s == 0) {
                eA0 = e0;
                eA1 = e1;
            }
            if (c.gl == 0) {
                cE[2 * s] = E0;
                cE[2 * s + 1] = E1;
            }
        }
        // (the table form costs registers: kept to the variants where it
        // does not lower occupancy)
        constexpr bool ZIR = !STOUT && (FIRM == FIR_NONE || FIRM == FIR_FFT || FIRM == FIR_FFT_PARTS);
        // its powers go to the staging areas, unused from phase A's first
        // barrier until the output is staged (ordered by phase B's barrier)
        if (ZIR && a.S <= ZIR_MAX) zt_stage(lds, a.zir, 2 * a.S, c.tid);
        // (B) one look-back of the cascade state (first wave of each group)
        if (c.gw == 0) {
            CascCtx cc;
            cc.lane = c.lane;
            cc.D = 2 * a.S;
            cc.depth = a.casc->depth;
            cc.rec = a.recs + c.ch * a.ntiles * (int64_t)(4 * a.S);
            cc.pos = c.tile;
            cc.epoch = c.epoch;
            cc.hdr = a.hdr;
            cc.known = (a.state_in && c.valid) ? a.state_in + c.ch * a.S * 2 : nullptr;
            casc_lookback(cc, cT, cE, cP, cM);
            if (a.ckpt && c.valid && c.lane < D) a.ckpt[(c.ch * a.ntiles + c.tile) * a.S * 2 + c.lane] = cP[c.lane];
        }
        __syncthreads();
        if (ZIR && a.S <= ZIR_MAX) {
            // (C) the entering state's zero-input response added to phase A's output
            casc_zir(v, a.zir, lds, cP, c.gl, a.S);
        } else {
        // (C') otherwise: every section from its known tile-entering state;
        //     section 0 reuses phase A's carry (its input is unchanged)
        load_chunk(stg, c.gl, v);
        const int r_cap = c.gl == c.owner ? c.r_last : -1;
        for (int s = 0; s < a.S; ++s) {
            const SecLdsC &tb = s_tabc[s];
            float c1 = 0.f, c2 = 0.f;
            if (s == 0) {
                float e0 = eA0, e1 = eA1;
                fold_prefix(tb, c.lane, c.gw, cP[0], cP[1], e0, e1);
                if (STOUT && c.is_last) section_from<L, true>(tb.coef, v, e0, e1, r_cap, c1, c2);
                else section_from<L>(tb.coef, v, e0, e1, -1, c1, c2);
            } else {
                const int buf = (s & 1) * GROUPS + c.grp;
                if (STOUT && c.is_last)
                    casc_section_c<L, true>(tb, v, c.lane, c.gw, cP[2 * s], cP[2 * s + 1], s_agg, buf, r_cap, c1, c2);
                else
                    casc_section_c<L, false>(tb, v, c.lane, c.gw, cP[2 * s], cP[2 * s + 1], s_agg, buf, -1, c1, c2);
            }
            if (STOUT && r_cap >= 0 && c.valid && a.state_out) {
                a.state_out[(c.ch * a.S + s) * 2 + 0] = c1;
                a.state_out[(c.ch * a.S + s) * 2 + 1] = c2;
            }
        }
        }
    } else if (HAS_SOS) {
        c.is_last = STOUT && (c.tile == a.ntiles - 1);
        const int64_t plast = a.N - 1 - n0;
        c.r_last = c.is_last ? (int)(plast % L) : 0;
        c.owner = c.is_last ? (int)(plast / L) : -1;
        for (int s = 0; s < a.S; ++s) {
            if (s > 0 && s % LDS_SECTIONS == 0) {  // next block of tables
                __syncthreads();
                stage_tables(s_tab, a.tab, s, min(a.S - s, LDS_SECTIONS), c.tid, WG);
                __syncthreads();
            }
            const SecLds &tl = s_tab[s % LDS_SECTIONS];
            if (HIQ && tl.hiq)
                run_section<double, SecTab, STOUT>(a, a.tab[s], s, v, c, s_agg, s_pre);
            else
                run_section<float, SecLds, STOUT>(a, tl, s, v, c, s_agg, s_pre);
        }
    }

    __syncthreads();
    store_chunk(stg, c.gl, v);
    __syncthreads();
    if (c.valid) store_tile(a.y + c.ch * a.ldy + n0, stg, a.N - n0, a.vec != 0, c.gl);
}

template <int FIRM>
constexpr int mc_lds_floats() {
    return FIRM == FIR_FFT ? 2 * NFFT
         : is_tz<FIRM>() ? (GROUPS * STG_FLOATS > MC_X_FLOATS ? GROUPS * STG_FLOATS : MC_X_FLOATS)
                           : (FIRM == FIR_DIRECT ? (GROUPS * DIRECT_GROUP_FLOATS > MC_X_FLOATS
                                                        ? GROUPS * DIRECT_GROUP_FLOATS
                                                        : MC_X_FLOATS)
                                                 : MC_X_FLOATS);
}
static_assert(2 * NFFT >= MC_X_FLOATS, "chunks must fit in the FFT buffers");

template <int FIRM>
__global__ __launch_bounds__(WG, 4) void chain_mc_kernel(KArgs a) {
    __shared__ __align__(16) float lds[mc_lds_floats<FIRM>()];
    __shared__ uint32_t s_epoch;
    __shared__ __align__(16) float2 s_twl[FIRM == FIR_FFT ? TWL_ENTRIES : 2];  // the transforms' twiddles
    if (a.hdr[HDR_HIQ] != 0u) {  // the FP64-carry variant runs
        advance_epoch(a.hdr);
        return;
    }
    const int tid = threadIdx.x;
    if (tid == 0) s_epoch = load_epoch(a.hdr, HDR_EPOCH);
    const uint64_t npairs = (uint64_t)(a.cpad / 2);
    const uint64_t id = xcd_order(blockIdx.x, gridDim.x, a.xcd_ks);
    const int64_t tile = (int64_t)(id / npairs);
    const int64_t pair = (int64_t)(id % npairs);
    const int64_t n0 = tile * T;
    const int64_t rem = a.N - n0;  // samples of the tile inside the signal (> 0)
    float *X = lds;                // [192][MC_XS]: sample j of channel g at g * 96 * 36 + 36 (j / 32) + j % 32

    // ---- FIR (or the input) into X
    if constexpr (FIRM == FIR_FFT) {
        float zr[16], zi[16];
        twl_stage(s_twl, a.twid, tid, WG);
        __syncthreads();
        fft_block<false>(a, lds, pair, n0, tid, zr, zi, s_twl);
        __syncthreads();  // the FFT buffers become X
#pragma unroll
        for (int q = 4; q < 16; ++q) {
            const int j = 256 * (q - 4) + tid;
            X[MC_XS * (j >> 5) + (j & 31)] = zr[q];
            X[MC_NCH * MC_XS + MC_XS * (j >> 5) + (j & 31)] = zi[q];
        }
    } else if constexpr (is_tz<FIRM>()) {
        static_assert(MC_LC == TP && MC_XS == 36, "the matrix-core FIR's frames are the cascade's chunks");
        tz_tile<FIRM == FIR_TZ_BF16 ? TZ_BF16 : TZ_F16, true>(a, lds, pair, n0, tid);
    } else if constexpr (FIRM == FIR_DIRECT) {
        const int grp = tid / GL, gl = tid % GL;
        const int64_t ch = 2 * pair + grp;
        float v[L];
        direct_tile(a, lds + grp * DIRECT_GROUP_FLOATS, ch, ch < a.C, gl, n0, v);
        __syncthreads();  // the direct FIR's staging becomes X
#pragma unroll
        for (int r = 0; r < L; ++r) {
            const int j = gl * L + r;
            X[grp * MC_NCH * MC_XS + MC_XS * (j >> 5) + (j & 31)] = v[r];
        }
    } else {
        const float *src[GROUPS];
#pragma unroll
        for (int g = 0; g < GROUPS; ++g) src[g] = 2 * pair + g < a.C ? a.x + (2 * pair + g) * a.ldx + n0 : nullptr;
        mc_stage_pair(X, src, rem, a.vec != 0, tid);
    }
    McCtx m;
    m.mt = a.mc;
    m.ct = a.casc;
    m.S = a.S;
    m.pos = tile;
    m.hdr = a.hdr;
#pragma unroll
    for (int g = 0; g < GROUPS; ++g) {
        const int64_t ch = 2 * pair + g;
        const bool valid = ch < a.C;
        m.rec[g] = a.recs + ch * a.ntiles * (int64_t)(4 * a.S);
        m.known[g] = (a.state_in && valid) ? a.state_in + ch * a.S * 2 : nullptr;
        m.ckpt[g] = (a.ckpt && valid) ? a.ckpt + (ch * a.ntiles + tile) * a.S * 2 : nullptr;
    }
    __syncthreads();  // s_epoch
    m.epoch = s_epoch;
    mc_cascade_tile(lds, m, tid);

    // ---- store both channels
    float *dst[GROUPS];
#pragma unroll
    for (int g = 0; g < GROUPS; ++g) dst[g] = 2 * pair + g < a.C ? a.y + (2 * pair + g) * a.ldy + n0 : nullptr;
    mc_store_pair(X, dst, rem, a.vec != 0, tid);
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
    w.casc = off;
    if (S > 0 && S <= CASC_MAX) off += al256(sizeof(CascTab));
    w.zir = off;
    if (S > 0 && S <= CASC_MAX) off += al256(sizeof(CascZir));
    w.mc = off;
    if (S > 0 && S <= CASC_MAX) off += al256(sizeof(McTab));
    w.taps = w.merge = off;
    if (n_fir > 1) {
        off += al256((size_t)M_merged * sizeof(float));
        w.merge = off;
        off += al256((size_t)M_merged * 2 * sizeof(double));
    }
    w.twid = w.hspec = w.tw64 = off;
    if (fir_mode == FIR_FFT) {
        off += al256(TWID_ENTRIES * sizeof(float2));
        w.hspec = off;
        off += al256((size_t)fft_parts(M_merged) * NFFT * sizeof(float2));
        w.tw64 = off;
        off += al256(NFFT * sizeof(double2));
    }
    w.ttab = off;
    if (fir_mode == FIR_TOEPLITZ) off += al256(toeplitz_table_bytes(M_merged, 3));  // largest (split) table
    w.f16 = off;
    if (fir_mode == FIR_FFT16) off += al256(fft16k_table_bytes());
    w.total = (S > 0 || n_fir > 1 || fir_mode == FIR_FFT || fir_mode == FIR_TOEPLITZ || fir_mode == FIR_FFT16) ? off : 0;
    return w;
}

// kernel of the prepare step (tfx_tables.hip)
hipError_t launch_state_passthrough(const float *in, float *out, int64_t n, hipStream_t st);

template <int F, bool S, bool STOUT>
static hipError_t launch_variants(const KArgs &k, int64_t nblocks, hipStream_t st) {
    // (with the FFT FIR the dynamic area first holds the twiddles)
    constexpr size_t twl = (F == FIR_FFT || F == FIR_FFT_PARTS) ? sizeof(float2) * TWL_ENTRIES : 0;
    const size_t dyn = std::max(twl, S ? sizeof(SecLds) * (size_t)(k.S < LDS_SECTIONS ? k.S : LDS_SECTIONS) : 0);
    if constexpr (S) {
        const size_t dync = std::max(twl, sizeof(SecLdsC) * (size_t)k.S +
                                              (casc_in_tail(F, k.S) ? 0 : sizeof(float) * (size_t)casc_floats(2 * k.S)));
        constexpr bool mc = !STOUT && (F == FIR_NONE || F == FIR_FFT || F == FIR_DIRECT || is_tz<F>());
        if (mc && k.S >= MC_MIN_SECTIONS && k.S <= CASC_MAX) {
            if constexpr (mc)
                hipLaunchKernelGGL((chain_mc_kernel<F>), dim3((unsigned)nblocks), dim3(WG), 0, st, k);
        } else if (k.S <= CASC_MAX)
            hipLaunchKernelGGL((chain_kernel<F, S, false, true, STOUT>), dim3((unsigned)nblocks), dim3(WG), dync, st, k);
        else
            hipLaunchKernelGGL((chain_kernel<F, S, false, false, STOUT>), dim3((unsigned)nblocks), dim3(WG), dyn, st, k);
    } else {
        hipLaunchKernelGGL((chain_kernel<F, S, false, false, false>), dim3((unsigned)nblocks), dim3(WG), dyn, st, k);
    }
    hipError_t e = hipGetLastError();
    if constexpr (S) {
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((chain_kernel<F, S, true, false, STOUT>), dim3((unsigned)nblocks), dim3(WG), dyn, st, k);
        e = hipGetLastError();
    }
    return e;
}

// STOUT: the variants that record the final state of every section (only
// when the caller asks for it, so the common variants carry no such code).
template <int F, bool S>
static hipError_t launch_main(const KArgs &k, int64_t nblocks, hipStream_t st) {
    if (S && k.state_out) return launch_variants<F, S, true>(k, nblocks, st);
    return launch_variants<F, S, false>(k, nblocks, st);
}

// xcd_order's log2 K for the current device and a grid of npairs channel
// pairs per tile: 32 block ids per XCD on the whole 256-CU chip (32 CUs per
// XCD, each holding at least one block).  Block ids stay in order on anything
// smaller (a partitioned device), and when npairs is a multiple of 8: then
// every tile of pair p already runs on XCD p % 8.
uint32_t xcd_window(int64_t npairs) {
    if (npairs % 8 == 0) return 0;
    static std::atomic<int> cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int n = cus[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = -1;
        cus[dev].store(n, std::memory_order_relaxed);
    }
    return n >= 256 ? 5u : 0u;
}

int32_t merged_taps(const StageList &f) {
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
    hipError_t e = launch_tables(p, lay, taps_ptr(p, lay), Mtot);
    if (e != hipSuccess) return e;
    if (Mtot > 0 && p.fir_mode == FIR_FFT16)
        return launch_fft16k_prepare(taps_ptr(p, lay), Mtot, static_cast<char *>(p.ws) + lay.f16, p.stream);
    if (p.fir_mode != FIR_TOEPLITZ) return e;
    return launch_toeplitz_prepare(taps_ptr(p, lay), Mtot, p.cmp, static_cast<char *>(p.ws) + lay.ttab, p.stream);
}

// Streaming: hist_out[c][j] = the input M - 1 - j samples before the
// block's end (from the block, then from hist_in, then zeros).
__global__ void hist_update_kernel(const float *x, int64_t ldx, const float *hin, float *hout, int64_t C, int64_t N,
                                   int64_t H) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= C * H) return;
    const int64_t c = e / H, j = e % H;
    const int64_t n = N - H + j;
    hout[e] = n >= 0 ? x[c * ldx + n] : (hin ? hin[c * H + H + n] : 0.f);
}

hipError_t launch_run(const ChainPlan &p) {
    int32_t Mtot = merged_taps(p.firs);
    const WsLayout lay = ws_layout(p.C, p.n_layout ? p.n_layout : p.N, p.S, Mtot, p.firs.n, p.fir_mode);
    if (p.hist_out && Mtot > 1) {  // stream-ordered before the filter, which reads hist_in only
        const int64_t n = p.C * (int64_t)(Mtot - 1);
        hipLaunchKernelGGL(hist_update_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, p.stream, p.x, p.ldx,
                           p.hist_in, p.hist_out, p.C, p.N, (int64_t)(Mtot - 1));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
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
    // matrix-core FIR with a cascade behind it, bf16 or fp16 operands: fused
    // into the chain kernel (the split-bf16 form and a FIR alone run the
    // stand-alone Toeplitz kernel)
    const bool tz_fused = Mtot > 0 && p.fir_mode == FIR_TOEPLITZ && p.S > 0 && (p.cmp == TZ_BF16 || p.cmp == TZ_F16);
    if (Mtot > 0 && p.fir_mode == FIR_FFT16) {
        // 16384-point FFT FIR into y, then the cascade in place over y (each
        // tile of the cascade kernel reads only the samples it writes)
        hipError_t e = launch_fft16k(p.x, p.y, p.C, p.N, p.ldx, p.ldy, Mtot, ws + lay.f16, false, p.hist_in, p.stream);
        if (e != hipSuccess || p.S == 0) return e;
        k.x = p.y;
        k.ldx = p.ldy;
        Mtot = 0;
    }
    if (Mtot > 0 && p.fir_mode == FIR_TOEPLITZ && !tz_fused) {
        // matrix-core FIR into y, then the cascade in place over y (each
        // tile reads only the samples it writes)
        hipError_t e = launch_toeplitz(p.x, p.y, p.C, p.N, p.ldx, p.ldy, Mtot, p.cmp, ws + lay.ttab, p.stream,
                                       p.hist_in);
        if (e != hipSuccess || p.S == 0) return e;
        k.x = p.y;
        k.ldx = p.ldy;
        Mtot = 0;
    }
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
    k.ntiles = (p.N + T - 1) / T;  // the block's tiles (streaming: the layout may be for a longer block)
    k.cpad = lay.cpad;
    k.hdr = reinterpret_cast<uint32_t *>(ws + lay.hdr);
    k.tab = reinterpret_cast<const SecTab *>(ws + lay.tab);
    k.recs = reinterpret_cast<uint64_t *>(ws + lay.recs);
    k.vec = ((reinterpret_cast<uintptr_t>(p.x) | reinterpret_cast<uintptr_t>(p.y)) % 16 == 0 && p.ldx % 4 == 0 &&
             p.ldy % 4 == 0) ? 1 : 0;
    k.twid = reinterpret_cast<const float2 *>(ws + lay.twid);
    k.hspec = reinterpret_cast<const float2 *>(ws + lay.hspec);
    k.nparts = fft_parts(Mtot);
    k.casc = reinterpret_cast<const CascTab *>(ws + lay.casc);
    k.zir = reinterpret_cast<const CascZir *>(ws + lay.zir);
    k.mc = reinterpret_cast<const McTab *>(ws + lay.mc);
    k.hist = Mtot > 1 ? p.hist_in : nullptr;
    k.ldh = Mtot > 1 ? Mtot - 1 : 0;
    k.xcd_ks = xcd_window(lay.cpad / 2);
    const int64_t nblocks = (lay.cpad / 2) * k.ntiles;
    const bool s = p.S > 0;
    if (tz_fused) {
        k.tzb = ws + lay.ttab;
        k.tzQ = toeplitz_lags(Mtot);
        return p.cmp == TZ_BF16 ? launch_main<FIR_TZ_BF16, true>(k, nblocks, p.stream)
                                : launch_main<FIR_TZ_F16, true>(k, nblocks, p.stream);
    }
    switch (Mtot > 0 ? p.fir_mode : FIR_NONE) {
        case FIR_DIRECT: return s ? launch_main<FIR_DIRECT, true>(k, nblocks, p.stream)
                                  : launch_main<FIR_DIRECT, false>(k, nblocks, p.stream);
        case FIR_FFT:
            if (k.nparts > 1)
                return s ? launch_main<FIR_FFT_PARTS, true>(k, nblocks, p.stream)
                         : launch_main<FIR_FFT_PARTS, false>(k, nblocks, p.stream);
            return s ? launch_main<FIR_FFT, true>(k, nblocks, p.stream)
                     : launch_main<FIR_FFT, false>(k, nblocks, p.stream);
        default: return s ? launch_main<FIR_NONE, true>(k, nblocks, p.stream)
                          : launch_main<FIR_NONE, false>(k, nblocks, p.stream);
    }
}

hipError_t launch_fir_pass(const ChainPlan &p, const WsLayout &lay, const float *in, int64_t ldin, float *out,
                           int64_t ldout, bool correlate) {
    const int32_t Mtot = merged_taps(p.firs);
    if (p.N == 0 || Mtot == 0) return hipSuccess;
    char *ws = static_cast<char *>(p.ws);
    if (p.fir_mode == FIR_FFT16)
        return launch_fft16k(in, out, p.C, p.N, ldin, ldout, Mtot, ws + lay.f16, correlate, nullptr, p.stream);
    KArgs k{};
    k.x = in;
    k.y = out;
    k.C = p.C;
    k.N = p.N;
    k.ldx = ldin;
    k.ldy = ldout;
    k.M = Mtot;
    k.h = taps_ptr(p, lay);
    const int32_t m16 = (Mtot + KB - 1) / KB * KB;
    k.KBL = m16 < KBLK_MAX ? m16 : KBLK_MAX;
    k.S = 0;
    k.ntiles = lay.ntiles;
    k.cpad = lay.cpad;
    k.vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) % 16 == 0 && ldin % 4 == 0 &&
             ldout % 4 == 0) ? 1 : 0;
    k.correlate = correlate ? 1 : 0;
    k.twid = reinterpret_cast<const float2 *>(ws + lay.twid);
    k.hspec = reinterpret_cast<const float2 *>(ws + lay.hspec);
    k.nparts = fft_parts(Mtot);
    k.xcd_ks = xcd_window(lay.cpad / 2);
    const int64_t nblocks = (lay.cpad / 2) * lay.ntiles;
    if (p.fir_mode == FIR_FFT && k.nparts > 1) return launch_main<FIR_FFT_PARTS, false>(k, nblocks, p.stream);
    return p.fir_mode == FIR_FFT ? launch_main<FIR_FFT, false>(k, nblocks, p.stream)
                                 : launch_main<FIR_DIRECT, false>(k, nblocks, p.stream);
}

}  // namespace tfx
