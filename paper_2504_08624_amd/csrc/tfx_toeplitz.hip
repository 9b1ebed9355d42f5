// tfx_toeplitz.hip -- FIR convolution as a block-Toeplitz matrix product on
// the gfx950 matrix cores (bf16 or fp16 operands, fp32 accumulation, and a
// split-bf16 mode with three products for close-to-fp32 accuracy).
//
// The signal of a channel is cut into frames of P = 32 samples, Y[b][i] =
// y[32 b + i].  With q the frame lag and m the sample within a frame,
//     y[32 b + i] = sum_{q, m} x[32 (b - q) + m] h[32 q + i - m]
// (h = 0 outside [0, M)); for each i the pairs (q, m), q < Q = ceil((M-1)/32)
// + 1, m < 32, meet every tap exactly once.  So Y = A B with
//     A[b][(q, m)] = x[32 (b - q) + m]     (Toeplitz in frames: depends on b - q)
//     B[(q, m)][i] = h[32 q + i - m]       (Toeplitz taps, the same for every channel)
// a (frames x 32Q) by (32Q x 32) product: 2 M flops per output sample plus
// under 1 % for the triangle of zero taps.  One v_mfma_f32_32x32x16 step
// covers 32 frames x 32 outputs x 16 values of (q, m): a fixed q and
// m in [16 hh, 16 hh + 16).
//
// Operand flow.  B is the same for every tile: the prepare step writes it
// once, already in the matrix core's per-lane operand layout (16 bytes per
// lane per step), and every wave streams it from L2.  A is a sliding window
// over frames: a workgroup stages the frames it needs, converted to the
// operand precision, into LDS once per block of lags, and each wave reads
// its fragments from there.  A wave holds FB = 4 accumulator tiles (32 frames
// each) and reuses each B fragment for all four.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tfx_device.h"

namespace tfx {

constexpr int TFB = 4;                      // accumulator tiles per wave
constexpr int TWAVES = 4;                   // waves per workgroup
constexpr int TFRAMES = TFB * 32 * TWAVES;  // frames per workgroup tile (512)
constexpr int TQC = 192;                    // lags per LDS stage
constexpr int TZ_SU = 8;                    // staging loads in flight per thread
// Filters with more than TZ_Q3 lags stage too many rows for three
// workgroups per CU, and take the deeper tap-fragment prefetch.
constexpr int TZ_Q3 = 171;

// B operand table: step s = 2 q + hh, lane l, element v holds
// h[32 q + (l % 32) - 16 hh - 8 (l / 32) - v]  (0 outside [0, M)),
// as hi (and, split mode, lo = h - hi) parts.  Layout [nsteps][64][8].
template <int MODE>
__global__ void toeplitz_btab_kernel(const float *h, int32_t M, int32_t nsteps, typename Op<MODE>::T *hi,
                                     typename Op<MODE>::T *lo) {
    typedef typename Op<MODE>::T T;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nsteps * 64 * 8) return;
    const int v = (int)(e & 7), l = (int)((e >> 3) & 63);
    const int s = (int)(e >> 9);
    const int q = s >> 1, hh = s & 1;
    const int k = 32 * q + (l & 31) - 16 * hh - 8 * (l >> 5) - v;
    const float t = (k >= 0 && k < M) ? h[k] : 0.f;
    const T th = (T)t;
    hi[e] = th;
    if (MODE == TZ_BF16X3) lo[e] = (T)(t - (float)th);
}

struct TzArgs {
    const float *x;
    float *y;
    int64_t C, N, ldx, ldy;
    int32_t Q;            // frame lags
    int64_t nft;          // frame tiles per channel
    const void *bhi, *blo;
    int32_t vec;          // x rows 16-byte aligned
    const float *hist;    // streaming: the M - 1 inputs before the block, [C][M - 1] (null = zeros)
    int64_t ldh;          // M - 1
};

// One workgroup: 512 consecutive frames (16384 outputs) of one channel.
// PF: tap-fragment steps loaded ahead (more hides more L2 latency but costs
// registers: 8 leaves two waves per SIMD, 4 three).
template <int MODE, int PF>
__global__ __launch_bounds__(64 * TWAVES) void toeplitz_kernel(TzArgs a) {
    typedef Op<MODE> O;
    typedef typename O::T T;
    typedef typename O::V V;
    typedef T T4 __attribute__((ext_vector_type(4)));
    constexpr int NA = MODE == TZ_BF16X3 ? 2 : 1;  // staged A parts (hi, lo)
    // [NA][rows][TROW]: one operand part in dynamic LDS with rows = TFRAMES +
    // min(Q, TQC) - 1 (short filters stage fewer rows, so more workgroups fit
    // a CU; at most 56 KB); the split mode's two parts statically, for TQC lags
    constexpr int NSTAT = MODE == TZ_BF16X3 ? NA * (TFRAMES + TQC - 1) * TROW : 8;
    __shared__ __align__(16) T lds_stat[NSTAT];
    extern __shared__ __align__(16) unsigned char tz_dyn[];
    T *lds_base = MODE == TZ_BF16X3 ? lds_stat : reinterpret_cast<T *>(tz_dyn);
    const int rows_max = MODE == TZ_BF16X3 ? TFRAMES + TQC - 1 : TFRAMES + min(a.Q, TQC) - 1;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t ch = blockIdx.x / a.nft;
    const int64_t b0 = (blockIdx.x % a.nft) * TFRAMES;  // first frame of the tile
    const float *xc = a.x + ch * a.ldx;
    const V *bhi = static_cast<const V *>(a.bhi);
    const V *blo = static_cast<const V *>(a.blo);

    f32x16 acc[TFB];
#pragma unroll
    for (int j = 0; j < TFB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;

    const int r32 = lane & 31, kh = lane >> 5;
    for (int q0 = 0; q0 < a.Q; q0 += TQC) {
        const int q1 = min(a.Q, q0 + TQC);
        // stage frames fbase .. fbase + TFRAMES + (q1 - q0) - 2
        const int64_t fbase = b0 - (q1 - 1);
        const int nrows = TFRAMES + (q1 - q0) - 1;
        __syncthreads();
        const int total = nrows * (TP / 4);
        const int64_t nlo = fbase * TP, nhi = (fbase + nrows) * TP;
        if (a.vec && nlo >= 0 && nhi <= a.N) {
            // inside the signal: TZ_SU four-sample loads in flight per thread
            for (int e0 = tid; e0 < total; e0 += TZ_SU * 64 * TWAVES) {
                float4 t[TZ_SU];
#pragma unroll
                for (int k = 0; k < TZ_SU; ++k) {
                    // clamped, not skipped: loads inside a branch are each waited for
                    const int e = min(e0 + k * 64 * TWAVES, total - 1);
                    t[k] = *reinterpret_cast<const float4 *>(xc + nlo + 4 * e);
                }
#pragma unroll
                for (int k = 0; k < TZ_SU; ++k) {
                    const int e = e0 + k * 64 * TWAVES;
                    if (e < total) {
                        const int row = e / (TP / 4), c4 = e % (TP / 4);
                        const float v4[4] = {t[k].x, t[k].y, t[k].z, t[k].w};
                        T4 hi4, lo4;
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            hi4[u] = (T)v4[u];
                            lo4[u] = (T)(v4[u] - (float)hi4[u]);
                        }
                        *reinterpret_cast<T4 *>(&lds_base[row * TROW + 4 * c4]) = hi4;
                        if (MODE == TZ_BF16X3) *reinterpret_cast<T4 *>(&lds_base[(NA - 1) * rows_max * TROW + row * TROW + 4 * c4]) = lo4;
                    }
                }
            }
        } else {
        for (int e = tid; e < total; e += 64 * TWAVES) {
            const int row = e / (TP / 4), c4 = e % (TP / 4);
            const int64_t n = (fbase + row) * TP + 4 * c4;
            float v4[4];
            if (a.vec && n >= 0 && n + 3 < a.N) {
                const float4 t = *reinterpret_cast<const float4 *>(xc + n);
                v4[0] = t.x;
                v4[1] = t.y;
                v4[2] = t.z;
                v4[3] = t.w;
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int64_t m = n + u;
                    v4[u] = m >= 0 ? (m < a.N ? xc[m] : 0.f)
                                   : ((a.hist && m >= -a.ldh) ? a.hist[ch * a.ldh + a.ldh + m] : 0.f);
                }
            }
            T4 hi4, lo4;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                hi4[u] = (T)v4[u];
                lo4[u] = (T)(v4[u] - (float)hi4[u]);
            }
            *reinterpret_cast<T4 *>(&lds_base[row * TROW + 4 * c4]) = hi4;
            if (MODE == TZ_BF16X3) *reinterpret_cast<T4 *>(&lds_base[(NA - 1) * rows_max * TROW + row * TROW + 4 * c4]) = lo4;
        }
        }
        __syncthreads();
        // steps s = 2 q + hh; the tap fragments are loaded PF steps ahead
        // (a ring of PF fragments: slot i holds step sb + i).  Every load index
        // is clamped to the last step instead of skipped, so the main loop has
        // no branch (loads inside a branch are each waited for at its end).
        const int s0 = 2 * q0, s1 = 2 * q1;
        // signal fragment of step st for accumulator tile j (part 0: hi, 1: lo)
        auto afrag = [&](int st, int j, int part) -> V {
            const int q = st >> 1, hh = st & 1;
            // frame b = b0 + 32 (w * TFB + j) + r32; staged row b - q - fbase
            const int row = 32 * (w * TFB + j) + r32 + (q1 - 1 - q);
            return *reinterpret_cast<const V *>(&lds_base[part * rows_max * TROW + row * TROW + 16 * hh + 8 * kh]);
        };
        V bq[PF], bl[PF];
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int64_t si = min(s0 + i, s1 - 1);
            bq[i] = bhi[si * 64 + lane];
            if (MODE == TZ_BF16X3) bl[i] = blo[si * 64 + lane];
        }
        int sb = s0;
        if (MODE != TZ_BF16X3) {
            // full groups of PF steps; each step loads the next step's signal
            // fragments before it issues its own products
            V acur[TFB];
#pragma unroll
            for (int j = 0; j < TFB; ++j) acur[j] = afrag(s0, j, 0);
            for (; sb + PF <= s1; sb += PF) {
#pragma unroll
                for (int i = 0; i < PF; ++i) {
                    const int st = sb + i, sn = min(st + 1, s1 - 1);
                    V anext[TFB];
#pragma unroll
                    for (int j = 0; j < TFB; ++j) anext[j] = afrag(sn, j, 0);
#pragma unroll
                    for (int j = 0; j < TFB; ++j) acc[j] = O::mma(acur[j], bq[i], acc[j]);
                    bq[i] = bhi[(int64_t)min(st + PF, s1 - 1) * 64 + lane];
#pragma unroll
                    for (int j = 0; j < TFB; ++j) acur[j] = anext[j];
                    // keep that order in the schedule: the next step's LDS
                    // reads, this step's products, then the tap refill
                    __builtin_amdgcn_sched_group_barrier(0x100, TFB, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, TFB, 0);
                    __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
                }
            }
        }
        // the remaining steps (all of them in split mode)
        for (; sb < s1; sb += PF) {
#pragma unroll
            for (int i = 0; i < PF; ++i) {
                const int st = sb + i;
                if (st < s1) {
#pragma unroll
                    for (int j = 0; j < TFB; ++j) {
                        const V ah = afrag(st, j, 0);
                        acc[j] = O::mma(ah, bq[i], acc[j]);
                        if (MODE == TZ_BF16X3) {
                            const V al = afrag(st, j, NA - 1);
                            acc[j] = O::mma(ah, bl[i], acc[j]);
                            acc[j] = O::mma(al, bq[i], acc[j]);
                        }
                    }
                    // the fragment's last use is issued: refill its slot in place
                    const int64_t sf = min(st + PF, s1 - 1);
                    bq[i] = bhi[sf * 64 + lane];
                    if (MODE == TZ_BF16X3) bl[i] = blo[sf * 64 + lane];
                }
            }
        }
    }
    // accumulator (row i, column c): lane c + 32 (i / 4 % 2), register
    // 4 (i / 8) + i % 4; output sample 32 (frame) + column
    float *yc = a.y + ch * a.ldy;
#pragma unroll
    for (int j = 0; j < TFB; ++j) {
        const int64_t fb = b0 + 32 * (w * TFB + j);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 8 * (r >> 2) + 4 * kh + (r & 3);
            const int64_t n = (fb + i) * TP + r32;
            if (n < a.N) yc[n] = acc[j][r];
        }
    }
}

// ------------------------------------------------------------------- host

int32_t toeplitz_lags(int32_t M) { return (M - 1 + TP - 1) / TP + 1; }

size_t toeplitz_table_bytes(int32_t M, int32_t cmp) {
    const size_t steps = 2 * (size_t)toeplitz_lags(M);
    return steps * 64 * 8 * 2 * (cmp == TZ_BF16X3 ? 2 : 1);
}

hipError_t launch_toeplitz_prepare(const float *h, int32_t M, int32_t cmp, void *tab, hipStream_t st) {
    const int32_t nsteps = 2 * toeplitz_lags(M);
    const int64_t n = (int64_t)nsteps * 64 * 8;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    char *t = static_cast<char *>(tab);
    switch (cmp) {
        case TZ_BF16:
            hipLaunchKernelGGL(toeplitz_btab_kernel<TZ_BF16>, grid, block, 0, st, h, M, nsteps,
                               reinterpret_cast<__bf16 *>(t), nullptr);
            break;
        case TZ_F16:
            hipLaunchKernelGGL(toeplitz_btab_kernel<TZ_F16>, grid, block, 0, st, h, M, nsteps,
                               reinterpret_cast<_Float16 *>(t), nullptr);
            break;
        default:
            hipLaunchKernelGGL(toeplitz_btab_kernel<TZ_BF16X3>, grid, block, 0, st, h, M, nsteps,
                               reinterpret_cast<__bf16 *>(t), reinterpret_cast<__bf16 *>(t + n * 2));
            break;
    }
    return hipGetLastError();
}

hipError_t launch_toeplitz(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy, int32_t M,
                           int32_t cmp, const void *tab, hipStream_t st, const float *hist) {
    if (N == 0) return hipSuccess;
    TzArgs a{};
    a.x = x;
    a.y = y;
    a.C = C;
    a.N = N;
    a.ldx = ldx;
    a.ldy = ldy;
    a.Q = toeplitz_lags(M);
    const int64_t frames = (N + TP - 1) / TP;
    a.nft = (frames + TFRAMES - 1) / TFRAMES;
    const int64_t n = 2 * (int64_t)a.Q * 64 * 8;
    a.bhi = tab;
    a.blo = static_cast<const char *>(tab) + n * 2;
    a.vec = (reinterpret_cast<uintptr_t>(x) % 16 == 0 && ldx % 4 == 0) ? 1 : 0;
    a.hist = M > 1 ? hist : nullptr;
    a.ldh = M - 1;
    const dim3 grid((unsigned)(C * a.nft)), block(64 * TWAVES);
    const size_t dyn = cmp == TZ_BF16X3 ? 0 : (TFRAMES + (size_t)std::min(a.Q, TQC) - 1) * TROW * 2;  // 2-byte operands
    const bool deep = a.Q > TZ_Q3;
    switch (cmp) {
        case TZ_BF16:
            if (deep) hipLaunchKernelGGL((toeplitz_kernel<TZ_BF16, 8>), grid, block, dyn, st, a);
            else hipLaunchKernelGGL((toeplitz_kernel<TZ_BF16, 4>), grid, block, dyn, st, a);
            break;
        case TZ_F16:
            if (deep) hipLaunchKernelGGL((toeplitz_kernel<TZ_F16, 8>), grid, block, dyn, st, a);
            else hipLaunchKernelGGL((toeplitz_kernel<TZ_F16, 4>), grid, block, dyn, st, a);
            break;
        default: hipLaunchKernelGGL((toeplitz_kernel<TZ_BF16X3, 4>), grid, block, dyn, st, a); break;
    }
    return hipGetLastError();
}

}  // namespace tfx
