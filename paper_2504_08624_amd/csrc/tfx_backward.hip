// tfx_backward.hip -- adjoint of the FIR / IIR-SOS chain (gradients with
// respect to the chain input, the FIR taps and the section coefficients).
//
// SOS section, forward s_{n+1} = A s_n + B x_n, y_n = C s_n + D x_n with
// A = [[-a1, 1], [-a2, 0]], B = (b1 - a1 b0, b2 - a2 b0), C = (1, 0), D = b0
// (transposed direct form II).  For upstream gradient g = dL/dy the adjoint
// state lambda_n = dL/ds_n obeys, backwards in time,
//     lambda_n = A^T lambda_{n+1} + C^T g_n,      lambda_N = 0,
//     dL/dx_n  = D g_n + B^T lambda_{n+1},
// and the coefficient gradients are sums over samples (and channels):
//     dL/dA = sum lambda_{n+1} s_n^T,  dL/dB = sum lambda_{n+1} x_n,
//     dL/dD = sum g_n x_n,
// mapped to (b0, b1, b2, a1, a2) through the definitions of A, B, D.  Since
// A^T has the same form as A, the adjoint recursion is the same 2x2 linear
// recurrence run in reverse time, and this kernel reuses the forward's
// chunked scan: lane l of a channel group owns chunk 127 - l of the tile (so
// lane order is reverse time), tiles are dispatched last first, and the scan
// tables are used transposed.  Section signals are recomputed per tile from
// the forward's checkpointed tile-entering states (no per-sample storage):
// one forward pass over the tile records every chunk-entering state of every
// section, and the input of section s is then rebuilt in each lane's
// registers from those states.
//
// FIR, y = h * x: dL/dx[n] = sum_k h[k] g[n + k] (the forward kernel's
// correlation mode) and dL/dh[k] = sum_{c,n} g[c,n] x[c,n-k], computed per
// tile as a circular cross-correlation with 4096-point FFTs (a channel pair
// packed as one complex signal: the real part of conj(FFT(g)) FFT(x) sums both
// channels' correlations).  Coefficient gradients are per-tile partial sums
// reduced in a fixed order in FP64, so results are bit-identical run to run.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tfx_device.h"

namespace tfx {

struct BArgs {
    const float *f;   // cascade input (the chain input, or its FIR output)
    const float *x;   // FFT_FIR: the chain input; the FIR output is recomputed per tile
    int64_t ldx;
    const float2 *twid, *hspec;
    const float *g;   // gradient of the cascade output
    float *gf;        // gradient of the cascade input
    int64_t C, N, ldf, ldg, ldo;
    const SecTab *tab;
    int32_t S;
    const float *ckpt;  // [C][ntiles][S][2] forward tile-entering states
    double *part;       // [S][5][cpad * ntiles] per group-tile partial sums
    uint64_t *recs;     // adjoint look-back records [cpad][ntiles][S]
    uint32_t *hdr;
    int64_t ntiles, cpad;
    int32_t vecf, vecg, veco;
    uint32_t xcd_ks;  // block order (xcd_order)
};

// TDF-II section over a lane's chunk from state (s1, s2), in place.
__device__ __forceinline__ void tdf2_chunk(float (&v)[L], const float *co, float s1, float s2) {
    const float b0 = co[0], b1 = co[1], b2 = co[2], a1 = co[3], a2 = co[4];
#pragma unroll
    for (int r = 0; r < L; ++r) {
        const float xv = v[r];
        const float yv = fmaf(b0, xv, s1);
        s1 = fmaf(b1, xv, fmaf(-a1, yv, s2));
        s2 = fmaf(b2, xv, -a2 * yv);
        v[r] = yv;
    }
}

// HIQ: the variant with the FP64 carry; both are launched and the one that
// does not match the workspace's high-Q word exits at once.  FFT_FIR: the
// cascade input is the overlap-save FFT FIR output of the chain input,
// recomputed for the tile here instead of read from memory.
template <bool HIQ, bool FFT_FIR>
__global__ __launch_bounds__(WG, 3) void sos_bwd_kernel(BArgs a) {
    // staging of both groups' tiles, or the FFT buffers
    __shared__ __align__(16) float stg_all[FFT_FIR ? 2 * NFFT : GROUPS * STG_FLOATS];
    // dynamic: fp32 tables of the S sections, then the chunk-entering forward
    // states sig[grp][s][chunk]
    extern __shared__ __align__(16) SecLds s_tab[];
    __shared__ double s_agg[2 * GROUPS][GWAVES][2];
    __shared__ double s_pre[2 * GROUPS][2];
    __shared__ double s_red[2][GROUPS][GWAVES][5];
    __shared__ uint32_t s_epoch;

    if ((a.hdr[HDR_HIQ] != 0u) != HIQ) return;
    const int tid = threadIdx.x, lane = tid & 63, grp = tid / GL, gl = tid % GL, gw = gl >> 6;
    if (tid == 0) s_epoch = load_epoch(a.hdr, HDR_EPOCH);
    const uint64_t npairs = (uint64_t)(a.cpad / 2);
    const uint64_t id = xcd_order(blockIdx.x, gridDim.x, a.xcd_ks);
    const int64_t pos = (int64_t)(id / npairs);  // reverse-time processing position
    const int64_t tile = a.ntiles - 1 - pos;
    const int64_t pair = (int64_t)(id % npairs);
    const int64_t ch = 2 * pair + grp;
    const bool valid = ch < a.C;
    const int64_t n0 = tile * T;
    const int S = a.S;
    float *stg = stg_all + grp * STG_FLOATS;
    const int mc = GL - 1 - gl;  // the chunk this lane owns in reverse time
    float2 *sig = reinterpret_cast<float2 *>(s_tab + S) + grp * S * GL;
    // the FFT FIR's twiddles sit in the chunk-state area until step 2 (the
    // launch sizes the area for both)
    float2 *s_twl = reinterpret_cast<float2 *>(s_tab + S);
    stage_tables(s_tab, a.tab, 0, S, tid, WG);

    // 1. stage f; lanes take their forward chunk (gl) and their reverse-time
    //    chunk (mc)
    if (FFT_FIR) {
        float zr[16], zi[16];
        const float *xA = a.x + 2 * pair * a.ldx;
        const float *xB = 2 * pair + 1 < a.C ? xA + a.ldx : nullptr;
        twl_stage(s_twl, a.twid, tid, WG);
        load_pair_block(zr, zi, xA, xB, n0 - FFT_DISCARD, a.N, a.N, tid);
        __syncthreads();  // the twiddles
        fft4096_forward(zr, zi, stg_all, s_twl, tid);
        spectrum_product(zr, zi, a.hspec, tid, false);
        fft4096_inverse(zr, zi, stg_all, s_twl, tid);
        __syncthreads();  // the FFT buffers become the two staging areas
#pragma unroll
        for (int q = 4; q < 16; ++q) {
            const int j = 256 * (q - 4) + tid;
            const bool in = n0 + j < a.N;  // zero past the signal, as staged input is
            stg_all[cphys(j)] = in ? zr[q] : 0.f;
            stg_all[STG_FLOATS + cphys(j)] = in ? zi[q] : 0.f;
        }
    } else {
        stage_tile(stg, a.f + ch * a.ldf + n0, a.N - n0, valid, a.vecf != 0, gl);
    }
    __syncthreads();
    const uint32_t epoch = s_epoch;
    float v[L], fr[L];
    load_chunk(stg, gl, v);
    load_chunk(stg, mc, fr);

    // 2. forward recompute from the checkpointed tile-entering states,
    //    recording every section's chunk-entering state
    for (int s = 0; s < S; ++s) {
        const SecLds &tb = s_tab[s];
        const float b0 = tb.coef[0], b1 = tb.coef[1], b2 = tb.coef[2], a1 = tb.coef[3], a2 = tb.coef[4];
        float s1 = 0.f, s2 = 0.f;
#pragma unroll
        for (int r = 0; r < L; ++r) {
            const float xv = v[r];
            const float yv = fmaf(b0, xv, s1);
            s1 = fmaf(b1, xv, fmaf(-a1, yv, s2));
            s2 = fmaf(b2, xv, -a2 * yv);
            v[r] = yv;
        }
        CarryCtx cc;
        cc.lane = lane;
        cc.gw = gw;
        cc.grp = grp;
        cc.lookback = false;
        cc.pos = tile;
        cc.recs = nullptr;
        cc.rec0 = 0;
        cc.rstride = 0;
        cc.epoch = 0;
        cc.hdr = a.hdr;
        cc.known0 = valid ? a.ckpt[((ch * a.ntiles + tile) * S + s) * 2 + 0] : 0.0;
        cc.known1 = valid ? a.ckpt[((ch * a.ntiles + tile) * S + s) * 2 + 1] : 0.0;
        cc.prefix_out = nullptr;
        float z1, z2;
        if (HIQ && tb.hiq)
            carry<double, false>(a.tab[s], cc, s1, s2, z1, z2, s_agg, s_pre, (s & 1) * GROUPS + grp);
        else
            carry<float, false>(tb, cc, s1, s2, z1, z2, s_agg, s_pre, (s & 1) * GROUPS + grp);
        sig[s * GL + gl] = make_float2(z1, z2);
        if (s + 1 < S) {
#pragma unroll
            for (int r = 0; r < L; ++r) {
                v[r] += z1;
                const float n1 = fmaf(-a1, z1, z2);
                z2 = -a2 * z1;
                z1 = n1;
            }
        }
    }
    // 3. stage g (over f); lanes take their reverse-time chunk
    __syncthreads();
    stage_tile(stg, a.g + ch * a.ldg + n0, a.N - n0, valid, a.vecg != 0, gl);
    __syncthreads();
    float gr[L];
    load_chunk(stg, mc, gr);

    // 4. sections in reverse order.  xo holds the output of section s over
    //    chunk mc: the input rebuilt for section s + 1 in the previous
    //    iteration (for the last section it is computed once), so the state
    //    s1 before sample r is xo[r] - b0 xs[r] (y = b0 x + s1) without a
    //    further pass.
    float xo[L];
    for (int s = S - 1; s >= 0; --s) {
        const SecLds &tb = s_tab[s];
        const float b0 = tb.coef[0], b1 = tb.coef[1], b2 = tb.coef[2], a1 = tb.coef[3], a2 = tb.coef[4];
        const float B0 = fmaf(-a1, b0, b1), B1 = fmaf(-a2, b0, b2);
        // (a) input of section s over chunk mc
        float xs[L];
#pragma unroll
        for (int r = 0; r < L; ++r) xs[r] = fr[r];
        for (int j = 0; j < s; ++j) {
            const float2 st = sig[j * GL + mc];
            tdf2_chunk(xs, s_tab[j].coef, st.x, st.y);
        }
        if (s == S - 1) {
#pragma unroll
            for (int r = 0; r < L; ++r) xo[r] = xs[r];
            const float2 st = sig[s * GL + mc];
            tdf2_chunk(xo, tb.coef, st.x, st.y);
        }
        // (b) adjoint zero-state response of the chunk, last sample first
        float m0 = 0.f, m1 = 0.f;
#pragma unroll
        for (int r = L - 1; r >= 0; --r) {
            const float n0v = fmaf(-a1, m0, fmaf(-a2, m1, gr[r]));
            m1 = m0;
            m0 = n0v;
        }
        // (c) carry in reverse time: the adjoint state entering the chunk from
        //     its end
        CarryCtx cc;
        cc.lane = lane;
        cc.gw = gw;
        cc.grp = grp;
        cc.lookback = true;
        cc.pos = pos;
        cc.recs = a.recs;
        cc.rec0 = ch * a.ntiles * S + s;
        cc.rstride = S;
        cc.epoch = epoch;
        cc.hdr = a.hdr;
        cc.known0 = cc.known1 = 0.0;  // lambda_N = 0
        cc.prefix_out = nullptr;
        float e0, e1;
        const int buf = ((S - 1 - s) & 1) * GROUPS + grp;
        if (HIQ && tb.hiq)
            carry<double, true>(a.tab[s], cc, m0, m1, e0, e1, s_agg, s_pre, buf);
        else
            carry<float, true>(tb, cc, m0, m1, e0, e1, s_agg, s_pre, buf);
        // (d) the adjoint recursion from the true state: input gradient and
        //     coefficient-gradient sums (24 terms per chunk by fp32 fused
        //     multiply-adds, then FP64 across chunks and tiles)
        float dA00 = 0.f, dA10 = 0.f, dB0 = 0.f, dB1 = 0.f, dD = 0.f;
        m0 = e0;
        m1 = e1;  // lambda_{n+1}
#pragma unroll
        for (int r = L - 1; r >= 0; --r) {
            const float gv = gr[r];
            const float gx = fmaf(b0, gv, fmaf(B0, m0, B1 * m1));
            const float sf = fmaf(-b0, xs[r], xo[r]);  // s1 before sample r
            dA00 = fmaf(m0, sf, dA00);
            dA10 = fmaf(m1, sf, dA10);
            dB0 = fmaf(m0, xs[r], dB0);
            dB1 = fmaf(m1, xs[r], dB1);
            dD = fmaf(gv, xs[r], dD);
            const float n0v = fmaf(-a1, m0, fmaf(-a2, m1, gv));
            m1 = m0;
            m0 = n0v;
            gr[r] = gx;
        }
#pragma unroll
        for (int r = 0; r < L; ++r) xo[r] = xs[r];  // output of section s - 1
        // (e) group sums, in a fixed order
        // within rows of 16 lanes in fp32 (16 chunk sums), across rows in FP64
        float rf[5] = {dA00, dA10, dB0, dB1, dD};
#pragma unroll
        for (int k = 0; k < 5; ++k) {
#pragma unroll
            for (int d = 1; d <= 8; d <<= 1) rf[k] += __shfl_xor(rf[k], d);
        }
        double red[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            red[k] = (double)rf[k];
            red[k] += __shfl_xor(red[k], 16);
            red[k] += __shfl_xor(red[k], 32);
        }
        const int rb = (S - 1 - s) & 1;
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) s_red[rb][grp][gw][k] = red[k];
        }
        __syncthreads();
        if (gl == 0 && valid) {
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < GWAVES; ++w) t += s_red[rb][grp][w][k];
                a.part[((int64_t)s * 5 + k) * (a.cpad * a.ntiles) + ch * a.ntiles + tile] = t;
            }
        }
    }
    // 5. gradient of the cascade input
    __syncthreads();
    store_chunk(stg, mc, gr);
    __syncthreads();
    if (valid) store_tile(a.gf + ch * a.ldo + n0, stg, a.N - n0, a.veco != 0, gl);
}

// Section-coefficient gradients from the per-tile partial sums.  One block
// per (section, sum): lane-strided FP64 partial sums in a fixed order, then
// a fixed tree; a second kernel maps each section's five sums to the
// gradients [b0 b1 b2 a1 a2] of its stage row.
struct SosGradArgs {
    const double *part;
    const SecTab *tab;
    int32_t S;
    int64_t C, ntiles, cpad;
    double *sums;  // [S][5]
    GradList out;
};

constexpr int RED_THREADS = 256;

// sum_{j >= 0, t + j s < n} p[t + j s] in index order, eight loads in flight.
template <typename T>
__device__ __forceinline__ double strided_sum(const T *p, int64_t n, int64_t t, int64_t s) {
    double acc = 0.0;
    int64_t i = t;
    for (; i + 7 * s < n; i += 8 * s) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[i + u * s];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += (double)v[u];
    }
    for (; i < n; i += s) acc += (double)p[i];
    return acc;
}

__device__ double block_sum_fixed(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = RED_THREADS / 2; w >= 1; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(RED_THREADS) void sos_grad_reduce_kernel(SosGradArgs a) {
    __shared__ double sh[RED_THREADS];
    const int64_t stride = a.cpad * a.ntiles;
    const int64_t n = a.C * a.ntiles;  // entries ch * ntiles + tile, ch < C
    const double *p = a.part + (int64_t)blockIdx.x * stride;  // block = 5 s + k
    const double t = block_sum_fixed(strided_sum(p, n, threadIdx.x, RED_THREADS), sh);
    if (threadIdx.x == 0) a.sums[blockIdx.x] = t;
}

__global__ void sos_grad_map_kernel(SosGradArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.S) return;
    double d[5];
    for (int k = 0; k < 5; ++k) d[k] = a.sums[5 * s + k];
    const double b0 = a.tab[s].coef[0], a1 = a.tab[s].coef[3], a2 = a.tab[s].coef[4];
    const double dA00 = d[0], dA10 = d[1], dB0 = d[2], dB1 = d[3], dD = d[4];
    int st = 0, j = s;
    while (j >= a.out.len[st]) {
        j -= a.out.len[st];
        ++st;
    }
    float *o = a.out.ptr[st];
    if (!o) return;
    o[5 * j + 0] = (float)(dD - a1 * dB0 - a2 * dB1);  // b0 enters D and both entries of B
    o[5 * j + 1] = (float)dB0;
    o[5 * j + 2] = (float)dB1;
    o[5 * j + 3] = (float)(-dA00 - b0 * dB0);  // a1 enters A[0][0] and B[0]
    o[5 * j + 4] = (float)(-dA10 - b0 * dB1);  // a2 enters A[1][0] and B[1]
}

// Tap-gradient partials.  Block (pair-tile, lag block kb): for the lags k in
// [1025 kb, 1025 kb + 1025),
//   part[kb][blk][k - 1025 kb] = sum over the pair's two channels and the
//                                tile's samples n of g[n] x[n - k],
// one 4096-point circular cross-correlation: with z the x block starting
// 1024 + 1025 kb samples before the tile and w the tile's g (zero past it),
// Re IFFT(conj(W) Z)[d] at d = 1024 - (k - 1025 kb) is that sum (no
// wrap-around, as d + 3071 < 4096), both channels at once.
struct GhArgs {
    const float *x, *g;
    int64_t C, N, ldx, ldg;
    int32_t M;
    int64_t cpad;
    const float2 *twid;
    float *part;  // [lag block][pair-tile block][1025]
};

__global__ __launch_bounds__(WG) void fir_gh_part_kernel(GhArgs a) {
    // FFT buffers, then the g block's spectrum (lane t keeps bins t + 256 k)
    __shared__ __align__(16) float lds[2 * NFFT];
    __shared__ __align__(16) float2 wspec[NFFT];
    __shared__ __align__(16) float2 s_twl[TWL_ENTRIES];
    const int tid = threadIdx.x;
    twl_stage(s_twl, a.twid, tid, WG);
    const int64_t npairs = a.cpad / 2;
    const int64_t tile = blockIdx.x / npairs, pair = blockIdx.x % npairs;
    const int64_t k0 = (int64_t)blockIdx.y * FFT_PART;
    const int64_t chA = 2 * pair, chB = chA + 1;
    const int64_t n0 = tile * T;
    float zr[16], zi[16];
    // g tile [n0, n0 + 3072), zero past it
    load_pair_block(zr, zi, a.g + chA * a.ldg, chB < a.C ? a.g + chB * a.ldg : nullptr, n0, a.N, n0 + T, tid);
    __syncthreads();  // the twiddle table
    fft4096_forward(zr, zi, lds, s_twl, tid);
#pragma unroll
    for (int k = 0; k < 16; ++k) wspec[tid + 256 * k] = make_float2(zr[k], zi[k]);
    // x block [n0 - 1024 - k0, n0 + 3072 - k0)
    load_pair_block(zr, zi, a.x + chA * a.ldx, chB < a.C ? a.x + chB * a.ldx : nullptr, n0 - FFT_DISCARD - k0,
                    a.N, a.N, tid);
    __syncthreads();  // the first FFT's last LDS reads
    fft4096_forward(zr, zi, lds, s_twl, tid);
#pragma unroll
    for (int k = 0; k < 16; ++k) {  // conj(W) Z
        const float2 w = wspec[tid + 256 * k];
        const float r = w.x * zr[k] + w.y * zi[k];
        const float i = w.x * zi[k] - w.y * zr[k];
        zr[k] = r;
        zi[k] = i;
    }
    fft4096_inverse(zr, zi, lds, s_twl, tid);
    // lane tid holds d = 256 q + tid; lag k = k0 + 1024 - d
    float *out = a.part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * FFT_PART;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int d = 256 * q + tid;
        if (d <= FFT_DISCARD) out[FFT_DISCARD - d] = zr[q] * (1.0f / NFFT);
    }
}

// FIR gradients of a single-partition FFT FIR (M <= 1025) in one pass over
// the tiles.  For tile t of a channel pair, with B the upstream-gradient
// block [n0, n0 + 4096) (zero past the signal) and X the input tile
// [n0, n0 + 3072) zero-padded to 4096 points:
//   dL/dx[n0 + d] = IFFT(conj(H) FFT(B))[d], d < 3072, since
//                   dL/dx[n] = sum_k h[k] g[n + k] and k + d < 4096;
//   sum_{m in tile} x[m] g[m + k] = Re IFFT(conj(FFT(X)) FFT(B))[k], k <= 1024,
// for both channels of the pair at once (the two packed channels' cross
// terms are purely imaginary, so the real part is the sum of the two
// correlations).  One FFT of B serves both.  A workgroup walks the (tile,
// pair) items xcd_order maps blockIdx.x, + gridDim.x, ... to (neighbouring
// tiles on one XCD) and sums conj(FFT(X)) FFT(B) over them in
// fp32 registers (lane t keeps bins t + 256 k3); its sum is written once, and
// FP64 reductions in a fixed order plus one inverse DFT per lag give dL/dh.
struct FirBwdArgs {
    const float *x, *g;
    float *gx;
    int64_t C, N, ldx, ldg, ldgx;
    int64_t cpad, ntiles;
    const float2 *twid, *hspec;
    float2 *spart;  // [workgroup][16][256] summed spectra, bin 256 k3 + t at [k3][t]
    int32_t want_gh;
    uint32_t xcd_ks;  // item order (xcd_order over the item index)
};

__global__ __launch_bounds__(WG) void fir_bwd_kernel(FirBwdArgs a) {
    __shared__ __align__(16) float lds[2 * NFFT];
    __shared__ __align__(16) float2 s_twl[TWL_ENTRIES];
    const int tid = threadIdx.x;
    twl_stage(s_twl, a.twid, tid, WG);  // visible after the first tile's barrier
    const int64_t npairs = a.cpad / 2, nitems = npairs * a.ntiles;
    float ar[16], ai[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) ar[k] = ai[k] = 0.f;
    for (int64_t ip = blockIdx.x; ip < nitems; ip += gridDim.x) {
        const int64_t it = xcd_order((uint32_t)ip, (uint32_t)nitems, a.xcd_ks);
        const int64_t tile = it / npairs, pair = it % npairs;
        const int64_t chA = 2 * pair, chB = chA + 1;
        const int64_t n0 = tile * T;
        const bool hasB = chB < a.C;
        float zr[16], zi[16];
        // keeps the twiddle and spectrum loads inside the loop: hoisted out of
        // it they would hold some 150 registers for the whole kernel
        asm volatile("" ::: "memory");
        __syncthreads();  // the previous tile's last LDS reads
        load_pair_block(zr, zi, a.g + chA * a.ldg, hasB ? a.g + chB * a.ldg : nullptr, n0, a.N, a.N, tid);
        fft4096_forward(zr, zi, lds, s_twl, tid);
        if (a.want_gh) {
            float br[16], bi[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                br[k] = zr[k];
                bi[k] = zi[k];
            }
            load_pair_block(zr, zi, a.x + chA * a.ldx, hasB ? a.x + chB * a.ldx : nullptr, n0, a.N, n0 + T, tid);
            __syncthreads();  // the B transform's last LDS reads
            fft4096_forward(zr, zi, lds, s_twl, tid);
#pragma unroll
            for (int k = 0; k < 16; ++k) {  // += conj(X) B
                ar[k] = fmaf(zr[k], br[k], fmaf(zi[k], bi[k], ar[k]));
                ai[k] = fmaf(zr[k], bi[k], fmaf(-zi[k], br[k], ai[k]));
                zr[k] = br[k];
                zi[k] = bi[k];
            }
        }
        spectrum_product(zr, zi, a.hspec, tid, true);
        fft4096_inverse(zr, zi, lds, s_twl, tid);
        store_pair_tile<0>(zr, zi, a.gx + chA * a.ldgx, hasB ? a.gx + chB * a.ldgx : nullptr, n0, a.N, tid);
    }
    if (a.want_gh) {
        float2 *o = a.spart + (int64_t)blockIdx.x * NFFT;
#pragma unroll
        for (int k = 0; k < 16; ++k) o[256 * k + tid] = make_float2(ar[k], ai[k]);
    }
}

// sum1[split][f] = sum of the workgroup spectra w in [split * SPEC_SPLIT,
// (split + 1) * SPEC_SPLIT) at bin f, in FP64 and in workgroup order.
constexpr int SPEC_SPLIT = 64;
constexpr int FIR_BWD_WGS = 512;  // two per CU fit (about 230 VGPRs)

__global__ void fir_spec_reduce1_kernel(const float2 *spart, int64_t nwg, double2 *sum1) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w0 = (int64_t)blockIdx.y * SPEC_SPLIT;
    const int64_t w1 = min(nwg, w0 + SPEC_SPLIT);
    double sr = 0.0, si = 0.0;
#pragma unroll 8
    for (int64_t w = w0; w < w1; ++w) {
        const float2 v = spart[w * NFFT + f];
        sr += (double)v.x;
        si += (double)v.y;
    }
    sum1[(int64_t)blockIdx.y * NFFT + f] = make_double2(sr, si);
}

__global__ void fir_spec_reduce2_kernel(const double2 *sum1, int32_t nsplit, double2 *spec) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < nsplit; ++k) {
        const double2 v = sum1[(int64_t)k * NFFT + f];
        sr += v.x;
        si += v.y;
    }
    spec[f] = make_double2(sr, si);
}

// dL/dh[k] = Re(sum_f P[f] e^{+2 pi i f k / 4096}) / 4096 for the lags
// k = 4 blockIdx.x + u, u < 4: thread t takes bins f = t + 256 j for all four
// lags, then a fixed-order block sum per lag.
constexpr int GH_DFT_LAGS = 4;
__global__ void fir_gh_dft_kernel(const double2 *spec, const double2 *tw64, int32_t M, float *gh) {
    __shared__ double wsum[GH_DFT_LAGS][WG / 64];
    const int k0 = blockIdx.x * GH_DFT_LAGS, t = threadIdx.x;
    double acc[GH_DFT_LAGS] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
        const int f = t + 256 * j;
        const double2 p = spec[f];
#pragma unroll
        for (int u = 0; u < GH_DFT_LAGS; ++u) {
            // e^{-i theta}: Re(p e^{+i theta}) = p.x w.x + p.y w.y
            const double2 w = tw64[(f * (k0 + u)) & (NFFT - 1)];
            acc[u] = fma(p.x, w.x, fma(p.y, w.y, acc[u]));
        }
    }
#pragma unroll
    for (int u = 0; u < GH_DFT_LAGS; ++u) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) acc[u] += __shfl_xor(acc[u], d);
        if ((t & 63) == 0) wsum[u][t >> 6] = acc[u];
    }
    __syncthreads();
    if (t < GH_DFT_LAGS && k0 + t < M)
        gh[k0 + t] = (float)(((wsum[t][0] + wsum[t][1]) + (wsum[t][2] + wsum[t][3])) / NFFT);
}

// Two-level FP64 reduction of the tap-gradient partials, in a fixed order:
// level 1 sums the partials of 128 consecutive blocks per lag
// (sum1[split][k]), level 2 the splits in order.
constexpr int GH_SPLIT = 128;

__global__ void fir_gh_reduce1_kernel(const float *part, int32_t M, int64_t nparts, double *sum1) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const int64_t i0 = (int64_t)blockIdx.y * GH_SPLIT;
    const int64_t i1 = min(nparts, i0 + GH_SPLIT);
    const int kb = k / FFT_PART, kk = k % FFT_PART;
    const float *p = part + ((int64_t)kb * nparts + i0) * FFT_PART + kk;
    sum1[(int64_t)blockIdx.y * M + k] = strided_sum(p, (i1 - i0) * FFT_PART, 0, FFT_PART);
}

__global__ void fir_gh_reduce2_kernel(const double *sum1, int32_t M, int32_t nsplit, float *dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    dst[k] = (float)strided_sum(sum1 + k, (int64_t)nsplit * M, 0, M);
}

// out = a (*) b, FP64 (a == null stands for the unit impulse).
__global__ void conv_f64_kernel(const double *a, int32_t na, const float *b, int32_t nb, double *out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (a == nullptr) {
        if (k < nb) out[k] = b[k];
        return;
    }
    if (k >= na + nb - 1) return;
    const int jlo = k - nb + 1 > 0 ? k - nb + 1 : 0;
    const int jhi = k < na - 1 ? k : na - 1;
    double acc = 0.0;
    for (int j = jlo; j <= jhi; ++j) acc += a[j] * (double)b[k - j];
    out[k] = acc;
}

// Gradient of one of several merged FIR stages: with H = h_i (*) O (O the
// convolution of the other stages' taps), dL/dh_i[k] = sum_j O[j] gH[j + k].
__global__ void stage_tap_grad_kernel(const double *O, int32_t nO, const float *gH, int32_t Mi, float *out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Mi) return;
    double acc = 0.0;
    for (int j = 0; j < nO; ++j) acc += O[j] * (double)gH[j + k];
    out[k] = (float)acc;
}

// ------------------------------------------------------------------- host

// kernels of the prepare step (tfx_tables.hip)
hipError_t launch_twiddles(float2 *twid, double2 *tw64, hipStream_t st);
hipError_t launch_state_passthrough(const float *in, float *out, int64_t n, hipStream_t st);

static size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

BwdLayout bwd_layout(int64_t C, int64_t N, int32_t S, int32_t M_merged, int32_t n_fir, int32_t fir_mode) {
    BwdLayout b{};
    b.fwd = ws_layout(C, N, S, M_merged, n_fir, fir_mode);
    const int64_t ntiles = b.fwd.ntiles, cpad = b.fwd.cpad, npairs = cpad / 2;
    // the forward layout ends with a 256-aligned total (or 0 when it needs nothing)
    size_t off = b.fwd.total ? b.fwd.total : 256;
    if (b.fwd.total == 0) b.fwd.hdr = 0;
    b.part_sos = off;
    off += al256((size_t)S * 5 * cpad * ntiles * sizeof(double));
    b.sos_sum = off;
    off += al256((size_t)S * 5 * sizeof(double));
    const bool both = n_fir > 0 && S > 0;
    const bool fused = both && fir_mode == FIR_FFT && fft_parts(M_merged) == 1;  // FIR recomputed in the adjoint
    b.fbuf = off;
    if (both && !fused) off += al256((size_t)C * N * sizeof(float));
    b.gfbuf = off;
    if (both) off += al256((size_t)C * N * sizeof(float));
    b.nlag = 0;
    b.spec_path = n_fir > 0 && fir_mode == FIR_FFT && fft_parts(M_merged) == 1;
    b.spec_wg = b.spec_nsplit = 0;
    b.part_gh = b.gh1 = b.gH = b.obuf = b.twid = b.tw64 = b.spec = off;
    if (n_fir > 0 && ntiles > 0) {
        if (b.spec_path) {
            const int64_t nitems = npairs * ntiles;
            b.spec_wg = nitems < FIR_BWD_WGS ? nitems : FIR_BWD_WGS;
            b.spec_nsplit = (b.spec_wg + SPEC_SPLIT - 1) / SPEC_SPLIT;
            off += al256((size_t)b.spec_wg * NFFT * sizeof(float2));
            b.gh1 = off;
            off += al256((size_t)b.spec_nsplit * NFFT * sizeof(double2));
            b.spec = off;
            off += al256(NFFT * sizeof(double2));
        } else {
            b.nlag = (M_merged + FFT_PART - 1) / FFT_PART;
            off += al256((size_t)b.nlag * npairs * ntiles * FFT_PART * sizeof(float));
            b.gh1 = off;
            off += al256((size_t)((npairs * ntiles + GH_SPLIT - 1) / GH_SPLIT) * M_merged * sizeof(double));
        }
        b.gH = off;
        off += al256((size_t)M_merged * sizeof(float));
        b.obuf = off;
        if (n_fir > 1) off += al256((size_t)M_merged * 2 * sizeof(double));
        b.twid = b.tw64 = off;
        if (fir_mode != FIR_FFT) {
            off += al256(TWID_ENTRIES * sizeof(float2));
            b.tw64 = off;
            off += al256(NFFT * sizeof(double2));
        }
    }
    b.total = off;
    return b;
}

hipError_t launch_backward(const BwdPlan &bp) {
    const ChainPlan &p = bp.fwd;
    const int32_t M = merged_taps(p.firs);
    const BwdLayout lay = bwd_layout(p.C, p.N, p.S, M, p.firs.n, p.fir_mode);
    char *ws = static_cast<char *>(p.ws);
    hipStream_t st = p.stream;
    hipError_t e;
    if (p.N == 0) {  // every gradient sum is empty
        if ((e = launch_header_init(p.ws, p.ws_bytes, st)) != hipSuccess) return e;
        for (int i = 0; i < bp.gsos.n; ++i)
            if (bp.gsos.ptr[i] && (e = launch_state_passthrough(nullptr, bp.gsos.ptr[i], 5 * (int64_t)bp.gsos.len[i], st)))
                return e;
        for (int i = 0; i < bp.gfir.n; ++i)
            if (bp.gfir.ptr[i] && (e = launch_state_passthrough(nullptr, bp.gfir.ptr[i], bp.gfir.len[i], st)))
                return e;
        return hipSuccess;
    }
    const bool has_fir = p.firs.n > 0, has_sos = p.S > 0;
    const float *h = has_fir ? (p.firs.n == 1 ? p.firs.ptr[0] : reinterpret_cast<const float *>(ws + lay.fwd.taps))
                             : nullptr;
    // tables, merged taps, spectrum; clears the look-back records
    if ((e = launch_tables(p, lay.fwd, h, M)) != hipSuccess) return e;
    if (has_fir && p.fir_mode == FIR_FFT16 &&
        (e = launch_fft16k_prepare(h, M, ws + lay.fwd.f16, st)) != hipSuccess)
        return e;
    // the cascade input f and the gradient of the cascade input gf
    const float *f = p.x;
    int64_t ldf = p.ldx;
    float *gf = bp.gx;
    int64_t ldgf = bp.ldgx;
    // a single-partition FFT FIR is recomputed inside the adjoint kernel;
    // other FIR forms are run into a buffer first
    const bool fuse = has_fir && has_sos && p.fir_mode == FIR_FFT && fft_parts(M) == 1;
    if (has_fir && has_sos) {
        if (!fuse) {
            float *fb = reinterpret_cast<float *>(ws + lay.fbuf);
            if ((e = launch_fir_pass(p, lay.fwd, p.x, p.ldx, fb, p.N, false)) != hipSuccess) return e;
            f = fb;
            ldf = p.N;
        }
        gf = reinterpret_cast<float *>(ws + lay.gfbuf);
        ldgf = p.N;
    }
    const int64_t ntiles = lay.fwd.ntiles, cpad = lay.fwd.cpad, npairs = cpad / 2;
    if (has_sos) {
        BArgs b{};
        b.f = f;
        b.g = bp.gy;
        b.gf = has_fir ? gf : bp.gx;
        b.C = p.C;
        b.N = p.N;
        b.ldf = ldf;
        b.ldg = bp.ldg;
        b.ldo = has_fir ? ldgf : bp.ldgx;
        b.tab = reinterpret_cast<const SecTab *>(ws + lay.fwd.tab);
        b.S = p.S;
        b.ckpt = p.ckpt;
        b.part = reinterpret_cast<double *>(ws + lay.part_sos);
        b.recs = reinterpret_cast<uint64_t *>(ws + lay.fwd.recs);
        b.hdr = reinterpret_cast<uint32_t *>(ws + lay.fwd.hdr);
        b.ntiles = ntiles;
        b.cpad = cpad;
        b.vecf = (reinterpret_cast<uintptr_t>(b.f) % 16 == 0 && b.ldf % 4 == 0) ? 1 : 0;
        b.vecg = (reinterpret_cast<uintptr_t>(b.g) % 16 == 0 && b.ldg % 4 == 0) ? 1 : 0;
        b.veco = (reinterpret_cast<uintptr_t>(b.gf) % 16 == 0 && b.ldo % 4 == 0) ? 1 : 0;
        b.xcd_ks = xcd_window(npairs);
        const size_t dyn = (size_t)p.S * sizeof(SecLds) +
                           std::max((size_t)p.S * GROUPS * GL * sizeof(float2),
                                    fuse ? sizeof(float2) * TWL_ENTRIES : (size_t)0);
        const dim3 grid((unsigned)(npairs * ntiles)), block(WG);
        if (fuse) {
            b.x = p.x;
            b.ldx = p.ldx;
            b.twid = reinterpret_cast<const float2 *>(ws + lay.fwd.twid);
            b.hspec = reinterpret_cast<const float2 *>(ws + lay.fwd.hspec);
            hipLaunchKernelGGL((sos_bwd_kernel<false, true>), grid, block, dyn, st, b);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL((sos_bwd_kernel<true, true>), grid, block, dyn, st, b);
        } else {
            hipLaunchKernelGGL((sos_bwd_kernel<false, false>), grid, block, dyn, st, b);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL((sos_bwd_kernel<true, false>), grid, block, dyn, st, b);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        SosGradArgs r{};
        r.part = b.part;
        r.tab = b.tab;
        r.S = p.S;
        r.C = p.C;
        r.ntiles = ntiles;
        r.cpad = cpad;
        r.out = bp.gsos;
        r.sums = reinterpret_cast<double *>(ws + lay.sos_sum);
        hipLaunchKernelGGL(sos_grad_reduce_kernel, dim3((unsigned)(5 * p.S)), dim3(RED_THREADS), 0, st, r);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(sos_grad_map_kernel, dim3((unsigned)((p.S + 63) / 64)), dim3(64), 0, st, r);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!has_fir) return hipSuccess;
    const float *gfc = has_sos ? gf : bp.gy;
    const int64_t ldgfc = has_sos ? ldgf : bp.ldg;
    bool any = false;
    for (int i = 0; i < bp.gfir.n; ++i) any = any || bp.gfir.ptr[i] != nullptr;
    float *gH = p.firs.n == 1 ? bp.gfir.ptr[0] : reinterpret_cast<float *>(ws + lay.gH);
    if (lay.spec_path) {
        // input gradient and tap-gradient spectra in one pass, then the
        // fixed-order reductions and the inverse DFT per lag
        FirBwdArgs fb{};
        fb.x = p.x;
        fb.g = gfc;
        fb.gx = bp.gx;
        fb.C = p.C;
        fb.N = p.N;
        fb.ldx = p.ldx;
        fb.ldg = ldgfc;
        fb.ldgx = bp.ldgx;
        fb.cpad = cpad;
        fb.ntiles = ntiles;
        fb.twid = reinterpret_cast<const float2 *>(ws + lay.fwd.twid);
        fb.hspec = reinterpret_cast<const float2 *>(ws + lay.fwd.hspec);
        fb.spart = reinterpret_cast<float2 *>(ws + lay.part_gh);
        fb.want_gh = any ? 1 : 0;
        fb.xcd_ks = lay.spec_wg % 8 == 0 ? xcd_window(npairs) : 0;  // item ip runs on XCD ip % 8
        hipLaunchKernelGGL(fir_bwd_kernel, dim3((unsigned)lay.spec_wg), dim3(WG), 0, st, fb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (!any) return hipSuccess;
        double2 *sum1 = reinterpret_cast<double2 *>(ws + lay.gh1);
        double2 *spec = reinterpret_cast<double2 *>(ws + lay.spec);
        hipLaunchKernelGGL(fir_spec_reduce1_kernel, dim3(NFFT / 256, (unsigned)lay.spec_nsplit), dim3(256), 0, st,
                           static_cast<const float2 *>(fb.spart), lay.spec_wg, sum1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(fir_spec_reduce2_kernel, dim3(NFFT / 256), dim3(256), 0, st,
                           static_cast<const double2 *>(sum1), (int32_t)lay.spec_nsplit, spec);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(fir_gh_dft_kernel, dim3((unsigned)((M + GH_DFT_LAGS - 1) / GH_DFT_LAGS)), dim3(WG), 0, st,
                           static_cast<const double2 *>(spec), reinterpret_cast<const double2 *>(ws + lay.fwd.tw64),
                           M, gH);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
        // input gradient: correlation of the cascade-input gradient with the taps
        if ((e = launch_fir_pass(p, lay.fwd, gfc, ldgfc, bp.gx, bp.ldgx, true)) != hipSuccess) return e;
        if (!any) return hipSuccess;
        GhArgs g{};
        g.x = p.x;
        g.g = gfc;
        g.C = p.C;
        g.N = p.N;
        g.ldx = p.ldx;
        g.ldg = ldgfc;
        g.M = M;
        g.cpad = cpad;
        g.twid = reinterpret_cast<const float2 *>(ws + lay.fwd.twid);
        g.part = reinterpret_cast<float *>(ws + lay.part_gh);
        if (p.fir_mode != FIR_FFT) {  // the direct path's prepare leaves no twiddles
            g.twid = reinterpret_cast<const float2 *>(ws + lay.twid);
            if ((e = launch_twiddles(reinterpret_cast<float2 *>(ws + lay.twid),
                                     reinterpret_cast<double2 *>(ws + lay.tw64), st)) != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(fir_gh_part_kernel, dim3((unsigned)(npairs * ntiles), (unsigned)lay.nlag), dim3(WG), 0,
                           st, g);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t nbx = npairs * ntiles;
        const int32_t nsplit = (int32_t)((nbx + GH_SPLIT - 1) / GH_SPLIT);
        double *sum1 = reinterpret_cast<double *>(ws + lay.gh1);
        hipLaunchKernelGGL(fir_gh_reduce1_kernel, dim3((unsigned)((M + 255) / 256), (unsigned)nsplit), dim3(256), 0,
                           st, static_cast<const float *>(g.part), M, nbx, sum1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(fir_gh_reduce2_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st,
                           static_cast<const double *>(sum1), M, nsplit, gH);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (p.firs.n == 1) return hipSuccess;
    // several FIR stages: chain rule through the tap convolution
    double *o0 = reinterpret_cast<double *>(ws + lay.obuf), *o1 = o0 + M;
    for (int i = 0; i < p.firs.n; ++i) {
        if (!bp.gfir.ptr[i]) continue;
        const double *cur = nullptr;
        int32_t nc = 0;
        for (int j = 0; j < p.firs.n; ++j) {
            if (j == i) continue;
            double *dst = (cur == o0) ? o1 : o0;
            const int32_t nn = cur ? nc + p.firs.len[j] - 1 : p.firs.len[j];
            hipLaunchKernelGGL(conv_f64_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, cur, nc,
                               p.firs.ptr[j], p.firs.len[j], dst);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            cur = dst;
            nc = nn;
        }
        const int32_t Mi = p.firs.len[i];
        hipLaunchKernelGGL(stage_tap_grad_kernel, dim3((unsigned)((Mi + 255) / 256)), dim3(256), 0, st, cur, nc,
                           static_cast<const float *>(gH), Mi, bp.gfir.ptr[i]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tfx
