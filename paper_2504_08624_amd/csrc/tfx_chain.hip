// tfx_chain.hip -- fused multichannel FIR + IIR-SOS chain for gfx950.
//
// One kernel covers the three forward forms of the library:
//   * FIR only       (direct LDS-tiled convolution),
//   * SOS only       (chunked parallel linear-recurrence scan),
//   * FIR -> SOS     (the FIR tile output stays in registers and feeds the scan).
//
// The filtering itself is the textbook definition (FIR convolution and the
// transposed-direct-form-II section recursion; the paper, Sec. 3, names
// these filters and the coefficient-driven lfilter).  How it is parallelised
// is this library's own design:
//
// Tile / chunk layout.  A workgroup of WG=256 lanes owns a tile of T=8192
// consecutive samples of one channel; lane i owns chunk [32i, 32i+32) of the
// tile in 32 registers.  Tiles are handed out by an atomic counter so that a
// tile's predecessors in time have always started (forward progress of the
// look-back below).
//
// IIR scan, one section at a time (the cascade stays in registers):
//   1. zero-state response of the lane's chunk, TDF-II, fp32: y0[t] and the
//      final state z (2 floats);
//   2. inclusive scan of z over the 64 lanes of a wave with the powers
//      Phi^(2^j) of the 2x2 chunk transition Phi = A^32 (Kogge-Stone);
//   3. wave aggregates combined through LDS with Psi = Phi^64;
//   4. decoupled look-back across tiles: a tile publishes its aggregate,
//      then reduces predecessors' aggregates (weighted by PhiT^k, PhiT = A^T)
//      up to the first published inclusive prefix, 64 predecessors per step;
//   5. every lane folds the tile prefix into its chunk-entering state with a
//      table of Phi^k and corrects y[t] = y0[t] + (row 0 of A^t) . s_in.
// The carry (steps 2-5) runs in fp32, or in fp64 for sections whose pole
// radius exceeds 0.999; the per-sample recursion is always fp32.
#include <hip/hip_runtime.h>

#include "tfx_internal.h"

namespace tfx {

// Look-back flag word: (epoch << 2) | status.  The epoch advances once per
// launch (the last workgroup to finish bumps it), so a run never has to clear
// the flags left by the previous one and repeated runs need no memset.
enum : uint32_t { FLAG_NONE = 0, FLAG_AGG = 1, FLAG_INC = 2 };
constexpr uint32_t EPOCH_MASK = 0x3FFFFFFFu;
constexpr int64_t SPIN_MAX = int64_t(1) << 24;
// Workspace header words.
enum { HDR_TILE = 0, HDR_ERROR = 1, HDR_EPOCH = 2, HDR_DONE = 3 };

// LDS index with 4 floats of padding every 32: a lane's 32-sample chunk then
// starts 144 bytes after its neighbour's, so 16-byte reads are conflict-free.
__device__ __forceinline__ int phys(int i) { return i + ((i >> 5) << 2); }

__device__ __forceinline__ uint32_t load_acquire(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_release(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ tables

__device__ void mat2_mul(const double *A, const double *B, double *C) {
    const double c0 = A[0] * B[0] + A[1] * B[2];
    const double c1 = A[0] * B[1] + A[1] * B[3];
    const double c2 = A[2] * B[0] + A[3] * B[2];
    const double c3 = A[2] * B[1] + A[3] * B[3];
    C[0] = c0; C[1] = c1; C[2] = c2; C[3] = c3;
}

__device__ void put4(float *f, double *d, const double *m) {
    for (int i = 0; i < 4; ++i) {
        f[i] = (float)m[i];
        if (d) d[i] = m[i];
    }
}

// All powers are formed in FP64 from the fp32 coefficients and rounded once.
__device__ void build_section(SecTab *tb, const float *co) {
    const double b0 = co[0], b1 = co[1], b2 = co[2], a1 = co[3], a2 = co[4];
    for (int i = 0; i < 5; ++i) tb->coef[i] = co[i];
    tb->pad[0] = tb->pad[1] = 0;
    const double A[4] = {-a1, 1.0, -a2, 0.0};
    double g0 = 1.0, g1 = 0.0;  // row 0 of A^t
    for (int t = 0; t < L; ++t) {
        tb->g[t][0] = (float)g0;
        tb->g[t][1] = (float)g1;
        const double n0 = -a1 * g0 - a2 * g1, n1 = g0;
        g0 = n0; g1 = n1;
    }
    double P[4] = {A[0], A[1], A[2], A[3]};
    for (int t = 0; t < L; ++t) {
        put4(tb->apow[t], nullptr, P);
        if (t + 1 < L) mat2_mul(P, A, P);
    }
    const double Phi[4] = {P[0], P[1], P[2], P[3]};
    double F[4] = {1.0, 0.0, 0.0, 1.0};
    for (int k = 0; k < 64; ++k) {
        put4(tb->fold[k], tb->fold_d[k], F);
        mat2_mul(F, Phi, F);
    }
    const double Psi[4] = {F[0], F[1], F[2], F[3]};
    double W[4] = {1.0, 0.0, 0.0, 1.0};
    for (int w = 0; w < WAVES; ++w) {
        put4(tb->psi[w], tb->psi_d[w], W);
        mat2_mul(W, Psi, W);
    }
    double B[4] = {W[0], W[1], W[2], W[3]};  // PhiT = A^T
    for (int j = 0; j < 7; ++j) {
        put4(tb->lb[j], tb->lb_d[j], B);
        mat2_mul(B, B, B);
    }
    const double disc = a1 * a1 - 4.0 * a2;
    double r;
    if (disc < 0.0) {
        r = sqrt(a2);
    } else {
        const double sq = sqrt(disc);
        r = fmax(fabs(0.5 * (-a1 + sq)), fabs(0.5 * (-a1 - sq)));
    }
    tb->hiq = r > 0.999 ? 1 : 0;
}

struct PrepArgs {
    SecTab *tab;
    int32_t S;
    StageList sos;
    uint32_t *flags;
    int64_t nflags;
    uint32_t *hdr;
};

// Builds every section's tables and initialises the look-back flags and the
// workspace header.  Needed once per (workspace, coefficients).
__global__ void prep_kernel(PrepArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gid; i < a.nflags; i += stride) a.flags[i] = 0u;
    if (gid == 0) {
        a.hdr[HDR_TILE] = 0u;
        a.hdr[HDR_ERROR] = 0u;
        a.hdr[HDR_EPOCH] = 1u;
        a.hdr[HDR_DONE] = 0u;
    }
    if (gid < a.S) {
        int s = (int)gid, st = 0;
        while (s >= a.sos.len[st]) {
            s -= a.sos.len[st];
            ++st;
        }
        build_section(&a.tab[gid], a.sos.ptr[st] + 5 * s);
    }
}

struct MergeArgs {
    StageList firs;
    double *buf0, *buf1;
    float *out;
};

// Convolves the tap vectors of several FIR stages into one (FP64, one block).
__global__ void merge_taps_kernel(MergeArgs a) {
    int Mcur = a.firs.len[0];
    for (int k = threadIdx.x; k < Mcur; k += blockDim.x) a.buf0[k] = a.firs.ptr[0][k];
    __syncthreads();
    double *cur = a.buf0, *nxt = a.buf1;
    for (int st = 1; st < a.firs.n; ++st) {
        const int Mi = a.firs.len[st];
        const float *hi = a.firs.ptr[st];
        const int Mn = Mcur + Mi - 1;
        for (int k = threadIdx.x; k < Mn; k += blockDim.x) {
            const int jlo = k - Mi + 1 > 0 ? k - Mi + 1 : 0;
            const int jhi = k < Mcur - 1 ? k : Mcur - 1;
            double acc = 0.0;
            for (int j = jlo; j <= jhi; ++j) acc += cur[j] * (double)hi[k - j];
            nxt[k] = acc;
        }
        __syncthreads();
        double *t = cur; cur = nxt; nxt = t;
        Mcur = Mn;
    }
    for (int k = threadIdx.x; k < Mcur; k += blockDim.x) a.out[k] = (float)cur[k];
}

__global__ void state_passthrough_kernel(const float *in, float *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in ? in[i] : 0.f;
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
    uint32_t *flags;
    double *recs;
    uint32_t *hdr;
    int64_t ntiles;
};

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

// Decoupled look-back of one (tile, section) by a full wave.  Publishes the
// tile aggregate, then returns the state entering the tile.
template <typename CT>
__device__ void lookback(const KArgs &a, const SecTab &tb, int64_t ch, int64_t tile, int s,
                         int lane, uint32_t epoch, CT agg0, CT agg1, CT &P0, CT &P1) {
    const int64_t S = a.S;
    const int64_t rself = (ch * a.ntiles + tile) * S + s;
    if (lane == 0) {
        a.recs[rself * 4 + 0] = (double)agg0;
        a.recs[rself * 4 + 1] = (double)agg1;
        store_release(&a.flags[rself], (epoch << 2) | FLAG_AGG);
    }
    CT acc0 = 0, acc1 = 0;
    CT M0 = 1, M1 = 0, M2 = 0, M3 = 1;  // PhiT^(64 * windows consumed)
    int64_t base = tile - 1;
    while (true) {
        const int64_t q = base - lane;
        uint32_t f = FLAG_NONE;
        if (q >= 0) {
            const int64_t r = (ch * a.ntiles + q) * S + s;
            int64_t spins = 0;
            while (true) {
                const uint32_t w = load_acquire(&a.flags[r]);
                if ((w >> 2) == epoch && (w & 3u) != FLAG_NONE) {
                    f = w & 3u;
                    break;
                }
                if (++spins > SPIN_MAX) {  // never expected: report and finish
                    atomicOr(&a.hdr[HDR_ERROR], 1u);
                    f = FLAG_INC;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        const unsigned long long incmask = __ballot(q >= 0 && f == FLAG_INC);
        const int istar = incmask ? (__ffsll(incmask) - 1) : 64;
        CT v0 = 0, v1 = 0;
        if (q >= 0 && lane <= istar) {
            const int64_t r = (ch * a.ntiles + q) * S + s;
            const int off = (lane == istar) ? 2 : 0;
            v0 = (CT)a.recs[r * 4 + off];
            v1 = (CT)a.recs[r * 4 + off + 1];
        }
        // lane 0 <- sum_i PhiT^i v_i
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const int d = 1 << j;
            const CT t0 = __shfl_down(v0, d), t1 = __shfl_down(v1, d);
            if (lane + d < 64) {
                const CT *B = Tab<CT>::lb(tb, j);
                const CT n0 = B[0] * t0 + B[1] * t1 + v0;
                const CT n1 = B[2] * t0 + B[3] * t1 + v1;
                v0 = n0;
                v1 = n1;
            }
        }
        const CT R0 = __shfl(v0, 0), R1 = __shfl(v1, 0);
        acc0 += M0 * R0 + M1 * R1;
        acc1 += M2 * R0 + M3 * R1;
        if (incmask) break;
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
    int tid, lane, wave;
    bool is_last;
    int r_last, owner;
};

// One section over the tile: zero-state response, carry, correction.
template <typename CT>
__device__ void run_section(const KArgs &a, const SecTab &tb, int s, float (&v)[L],
                            const TileCtx &c, double (*s_agg)[2], double *s_pre) {
    const float b0 = tb.coef[0], b1 = tb.coef[1], b2 = tb.coef[2];
    const float a1 = tb.coef[3], a2 = tb.coef[4];
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
    // 2. inclusive scan over the wave's 64 chunks
    CT w0 = (CT)s1, w1 = (CT)s2;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const int d = 1 << j;
        const CT t0 = __shfl_up(w0, d), t1 = __shfl_up(w1, d);
        if (c.lane >= d) {
            const CT *P = Tab<CT>::fold(tb, d);
            const CT n0 = P[0] * t0 + P[1] * t1 + w0;
            const CT n1 = P[2] * t0 + P[3] * t1 + w1;
            w0 = n0;
            w1 = n1;
        }
    }
    if (c.lane == 63) {
        s_agg[c.wave][0] = (double)w0;
        s_agg[c.wave][1] = (double)w1;
    }
    __syncthreads();
    // 3. wave-entering states for a zero tile-entering state; E ends as the
    //    tile aggregate
    const CT *Psi = Tab<CT>::psi(tb, 1);
    CT E0 = 0, E1 = 0, ew0 = 0, ew1 = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        if (w == c.wave) {
            ew0 = E0;
            ew1 = E1;
        }
        const CT g0 = (CT)s_agg[w][0], g1 = (CT)s_agg[w][1];
        const CT n0 = Psi[0] * E0 + Psi[1] * E1 + g0;
        const CT n1 = Psi[2] * E0 + Psi[3] * E1 + g1;
        E0 = n0;
        E1 = n1;
    }
    // 4. tile prefix
    if (c.wave == 0) {
        CT P0 = 0, P1 = 0;
        if (c.tile == 0) {
            if (a.state_in) {
                P0 = (CT)a.state_in[(c.ch * a.S + s) * 2 + 0];
                P1 = (CT)a.state_in[(c.ch * a.S + s) * 2 + 1];
            }
        } else {
            lookback<CT>(a, tb, c.ch, c.tile, s, c.lane, c.epoch, E0, E1, P0, P1);
        }
        if (c.lane == 0) {
            const CT *PT = Tab<CT>::lb(tb, 0);
            const int64_t r = (c.ch * a.ntiles + c.tile) * a.S + s;
            a.recs[r * 4 + 2] = (double)(PT[0] * P0 + PT[1] * P1 + E0);
            a.recs[r * 4 + 3] = (double)(PT[2] * P0 + PT[3] * P1 + E1);
            store_release(&a.flags[r], (c.epoch << 2) | FLAG_INC);
            s_pre[0] = (double)P0;
            s_pre[1] = (double)P1;
            if (a.ckpt) {
                a.ckpt[((c.ch * a.ntiles + c.tile) * a.S + s) * 2 + 0] = (float)P0;
                a.ckpt[((c.ch * a.ntiles + c.tile) * a.S + s) * 2 + 1] = (float)P1;
            }
        }
    }
    __syncthreads();
    // 5. chunk-entering state and correction
    const CT P0 = (CT)s_pre[0], P1 = (CT)s_pre[1];
    const CT *Pw = Tab<CT>::psi(tb, c.wave);
    const CT e0 = ew0 + Pw[0] * P0 + Pw[1] * P1;
    const CT e1 = ew1 + Pw[2] * P0 + Pw[3] * P1;
    CT pv0 = __shfl_up(w0, 1), pv1 = __shfl_up(w1, 1);
    if (c.lane == 0) {
        pv0 = 0;
        pv1 = 0;
    }
    const CT *F = Tab<CT>::fold(tb, c.lane);
    const CT si0 = pv0 + F[0] * e0 + F[1] * e1;
    const CT si1 = pv1 + F[2] * e0 + F[3] * e1;
    const float sf0 = (float)si0, sf1 = (float)si1;
#pragma unroll
    for (int r = 0; r < L; ++r) v[r] = fmaf(tb.g[r][0], sf0, fmaf(tb.g[r][1], sf1, v[r]));
    if (c.is_last && c.tid == c.owner && a.state_out) {
        const float *Ap = tb.apow[c.r_last];
        a.state_out[(c.ch * a.S + s) * 2 + 0] = fmaf(Ap[0], sf0, fmaf(Ap[1], sf1, c1));
        a.state_out[(c.ch * a.S + s) * 2 + 1] = fmaf(Ap[2], sf0, fmaf(Ap[3], sf1, c2));
    }
    __syncthreads();  // s_agg / s_pre are reused by the next section
}

template <bool HAS_FIR>
constexpr int xs_len() {
    return HAS_FIR ? ((T + KBLK_MAX + 32) / 32) * 36 : (T / 32) * 36;
}

template <bool HAS_FIR, bool HAS_SOS>
__global__ __launch_bounds__(WG) void chain_kernel(KArgs a) {
    __shared__ __align__(16) float xs[xs_len<HAS_FIR>()];
    __shared__ double s_agg[WAVES][2];
    __shared__ double s_pre[2];
    __shared__ uint32_t s_id, s_epoch;

    TileCtx c;
    c.tid = threadIdx.x;
    c.lane = c.tid & 63;
    c.wave = c.tid >> 6;
    uint64_t id;
    c.epoch = 0;
    if (HAS_SOS) {
        if (c.tid == 0) {
            s_id = atomicAdd(&a.hdr[HDR_TILE], 1u);
            s_epoch = __hip_atomic_load(&a.hdr[HDR_EPOCH], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        id = s_id;
        c.epoch = s_epoch;
    } else {
        id = blockIdx.x;
    }
    c.tile = (int64_t)(id / (uint64_t)a.C);
    c.ch = (int64_t)(id % (uint64_t)a.C);
    const int64_t n0 = c.tile * T;
    const float *xc = a.x + c.ch * a.ldx;
    const int p0 = c.tid * L;
    float v[L];

    if (HAS_FIR) {
        float acc[L];
#pragma unroll
        for (int r = 0; r < L; ++r) acc[r] = 0.f;
        for (int k0 = 0; k0 < a.M; k0 += a.KBL) {
            __syncthreads();
            const int64_t src0 = n0 - (k0 + a.KBL - 1);
            for (int i = c.tid; i < T + a.KBL; i += WG) {
                const int64_t n = src0 + i;
                xs[phys(i)] = (n >= 0 && n < a.N) ? xc[n] : 0.f;
            }
            __syncthreads();
            const int kend = min(a.KBL, a.M - k0);
            for (int kb = 0; kb < kend; kb += KB) {
                const int base0 = p0 + a.KBL - KB - kb;
                float W[L + KB];
#pragma unroll
                for (int q = 0; q < (L + KB) / 4; ++q) {
                    const float4 t4 = *reinterpret_cast<const float4 *>(&xs[phys(base0 + 4 * q)]);
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
    } else {
        for (int i = c.tid; i < T; i += WG) {
            const int64_t n = n0 + i;
            xs[phys(i)] = (n < a.N) ? xc[n] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < L / 4; ++q) {
            const float4 t4 = *reinterpret_cast<const float4 *>(&xs[phys(p0 + 4 * q)]);
            v[4 * q + 0] = t4.x;
            v[4 * q + 1] = t4.y;
            v[4 * q + 2] = t4.z;
            v[4 * q + 3] = t4.w;
        }
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
        *reinterpret_cast<float4 *>(&xs[phys(p0 + 4 * q)]) =
            make_float4(v[4 * q + 0], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    __syncthreads();
    float *yc = a.y + c.ch * a.ldy;
    for (int i = c.tid; i < T; i += WG) {
        const int64_t n = n0 + i;
        if (n < a.N) yc[n] = xs[phys(i)];
    }
    if (HAS_SOS && c.tid == 0) {
        // every workgroup has taken its tile id and read the epoch once all
        // have arrived here: the last one re-arms the header for the next run
        const uint32_t done = atomicAdd(&a.hdr[HDR_DONE], 1u);
        if (done == gridDim.x - 1) {
            uint32_t ne = (c.epoch + 1u) & EPOCH_MASK;
            if (ne == 0u) ne = 1u;
            __hip_atomic_store(&a.hdr[HDR_TILE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.hdr[HDR_DONE], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.hdr[HDR_EPOCH], ne, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------------- host

static size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

WsLayout ws_layout(int64_t C, int64_t N, int32_t S, int32_t M_merged, int32_t n_fir) {
    WsLayout w{};
    w.ntiles = (N + T - 1) / T;
    size_t off = 0;
    w.hdr = off;
    off += 256;
    w.tab = off;
    off += al256(sizeof(SecTab) * (size_t)S);
    const size_t nrec = (size_t)C * (size_t)w.ntiles * (size_t)S;
    w.flags = off;
    off += al256(nrec * sizeof(uint32_t));
    w.recs = off;
    off += al256(nrec * 4 * sizeof(double));
    w.taps = off;
    w.merge = off;
    if (n_fir > 1) {
        off += al256((size_t)M_merged * sizeof(float));
        w.merge = off;
        off += al256((size_t)M_merged * 2 * sizeof(double));
    }
    w.total = (S > 0 || n_fir > 1) ? off : 0;
    return w;
}

template <bool F, bool S>
static hipError_t launch_main(const KArgs &k, int64_t nblocks, hipStream_t st) {
    hipLaunchKernelGGL((chain_kernel<F, S>), dim3((unsigned)nblocks), dim3(WG), 0, st, k);
    return hipGetLastError();
}

static int32_t merged_taps(const StageList &f) {
    int32_t Mtot = 0;
    for (int i = 0; i < f.n; ++i) Mtot += (i == 0) ? f.len[i] : f.len[i] - 1;
    return Mtot;
}

hipError_t launch_prepare(const ChainPlan &p) {
    const int32_t Mtot = merged_taps(p.firs);
    const WsLayout lay = ws_layout(p.C, p.N, p.S, Mtot, p.firs.n);
    char *ws = static_cast<char *>(p.ws);
    hipError_t e;
    if (p.firs.n > 1) {
        MergeArgs m;
        m.firs = p.firs;
        m.buf0 = reinterpret_cast<double *>(ws + lay.merge);
        m.buf1 = m.buf0 + Mtot;
        m.out = reinterpret_cast<float *>(ws + lay.taps);
        hipLaunchKernelGGL(merge_taps_kernel, dim3(1), dim3(256), 0, p.stream, m);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (p.S > 0) {
        PrepArgs pa;
        pa.tab = reinterpret_cast<SecTab *>(ws + lay.tab);
        pa.S = p.S;
        pa.sos = p.sos;
        pa.flags = reinterpret_cast<uint32_t *>(ws + lay.flags);
        pa.nflags = p.C * lay.ntiles * p.S;
        pa.hdr = reinterpret_cast<uint32_t *>(ws + lay.hdr);
        const int64_t work = pa.nflags > p.S ? pa.nflags : p.S;
        int64_t nb = (work + 255) / 256;
        if (nb > 1024) nb = 1024;
        if (nb < 1) nb = 1;
        hipLaunchKernelGGL(prep_kernel, dim3((unsigned)nb), dim3(256), 0, p.stream, pa);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_run(const ChainPlan &p) {
    const int32_t Mtot = merged_taps(p.firs);
    const WsLayout lay = ws_layout(p.C, p.N, p.S, Mtot, p.firs.n);
    char *ws = static_cast<char *>(p.ws);
    if (p.N == 0) {
        if (p.state_out && p.S > 0) {
            const int64_t n = p.C * p.S * 2;
            hipLaunchKernelGGL(state_passthrough_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                               p.stream, p.state_in, p.state_out, n);
            return hipGetLastError();
        }
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
    k.h = p.firs.n == 1 ? p.firs.ptr[0] : (p.firs.n > 1 ? reinterpret_cast<const float *>(ws + lay.taps) : nullptr);
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
    k.hdr = reinterpret_cast<uint32_t *>(ws + lay.hdr);
    k.tab = reinterpret_cast<const SecTab *>(ws + lay.tab);
    k.flags = reinterpret_cast<uint32_t *>(ws + lay.flags);
    k.recs = reinterpret_cast<double *>(ws + lay.recs);
    const int64_t nblocks = p.C * lay.ntiles;
    const bool f = Mtot > 0, s = p.S > 0;
    if (f && s) return launch_main<true, true>(k, nblocks, p.stream);
    if (f) return launch_main<true, false>(k, nblocks, p.stream);
    if (s) return launch_main<false, true>(k, nblocks, p.stream);
    return launch_main<false, false>(k, nblocks, p.stream);
}

}  // namespace tfx
