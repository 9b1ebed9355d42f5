// tfx_tables.hip -- the prepare step: per-section scan tables, FFT twiddles and
// tap spectrum, merged taps, workspace initialisation.  Everything is formed
// in FP64 from the fp32 coefficients the filter kernel will see, and rounded
// once.  These kernels run once per (workspace, coefficients); the filter
// kernel (tfx_chain.hip) only reads what they leave in the workspace.
#include <hip/hip_runtime.h>

#include "tfx_internal.h"

namespace tfx {

__device__ void mat2_mul(const double *A, const double *B, double *C) {
    const double c0 = A[0] * B[0] + A[1] * B[2];
    const double c1 = A[0] * B[1] + A[1] * B[3];
    const double c2 = A[2] * B[0] + A[3] * B[2];
    const double c3 = A[2] * B[1] + A[3] * B[3];
    C[0] = c0;
    C[1] = c1;
    C[2] = c2;
    C[3] = c3;
}

__device__ void put4(float *f, double *d, const double *m) {
    for (int i = 0; i < 4; ++i) {
        f[i] = (float)m[i];
        if (d) d[i] = m[i];
    }
}

// R = A^e (FP64 2 x 2) by binary powering; R may alias nothing.
__device__ void mat2_pow(const double *A, int e, double *R) {
    double P[4] = {A[0], A[1], A[2], A[3]};
    R[0] = 1.0;
    R[1] = 0.0;
    R[2] = 0.0;
    R[3] = 1.0;
    while (e > 0) {
        if (e & 1) mat2_mul(R, P, R);
        e >>= 1;
        if (e > 0) mat2_mul(P, P, P);
    }
}

__device__ double mat2_maxabs(const double *M) {
    return fmax(fmax(fabs(M[0]), fabs(M[1])), fmax(fabs(M[2]), fabs(M[3])));
}

// Transition powers of one TDF-II section, built by one block of 256
// threads.  With state s = (s1, s2) the section is s' = A s + B x,
// y = s1 + b0 x, A = [[-a1, 1], [-a2, 0]], so a state s entering a chunk
// becomes Phi s = A^Lc s after Lc samples.  Thread k < 64 writes the fold
// power Phi^k, thread j < 9 the look-back power W^(2^j) of the tile
// transition W = Phi^128, and threads k < 64 test W^(k+1) for the look-back
// depth (the first d <= 64 with max |W^d| <= 2^-60, 0 if none).  Every power
// is formed by binary powering in FP64 and rounded once.
__device__ void build_section_block(SecTab *tb, const float *co, int Lc, int tid) {
    __shared__ int s_dep;
    const double a1 = co[3], a2 = co[4];
    const double A[4] = {-a1, 1.0, -a2, 0.0};
    double Phi[4], Psi[4], W[4], R[4];
    mat2_pow(A, Lc, Phi);
    mat2_pow(Phi, 64, Psi);
    mat2_pow(Psi, GWAVES, W);
    if (tid == 0) s_dep = 65;
    __syncthreads();
    if (tid < 64) {
        mat2_pow(Phi, tid, R);
        put4(tb->fold[tid], tb->fold_d[tid], R);
        mat2_pow(W, tid + 1, R);
        if (mat2_maxabs(R) <= DEPTH_EPS) atomicMin(&s_dep, tid + 1);
    }
    if (tid < GWAVES) {
        mat2_pow(Psi, tid, R);
        put4(tb->psi[tid], tb->psi_d[tid], R);
    }
    if (tid < 9) {
        mat2_pow(W, 1 << tid, R);
        put4(tb->lb[tid], tb->lb_d[tid], R);
    }
    __syncthreads();
    if (tid == 0) {
        for (int i = 0; i < 5; ++i) tb->coef[i] = co[i];
        tb->pad = 0;
        tb->depth = s_dep > 64 ? 0 : s_dep;
        tb->hiq = section_hiq(a1, a2) ? 1 : 0;
    }
}

// Element (i, j) of the cascade's one-sample transition F under zero input
// (D = 2S state components, section s at 2s, 2s + 1): block (s, s) is the
// section's A; block (s, t), t < s, is B_s (prod_{t<l<s} b0_l) C, since
// section s's input is section s-1's output.
__device__ double cascade_f(const double (*co)[5], int D, int i, int j) {
    if (i >= D || j >= D) return 0.0;
    const int si = i >> 1, ri = i & 1, sj = j >> 1, cj = j & 1;
    const double b0 = co[si][0], b1 = co[si][1], b2 = co[si][2], a1 = co[si][3], a2 = co[si][4];
    if (si == sj) return ri == 0 ? (cj == 0 ? -a1 : 1.0) : (cj == 0 ? -a2 : 0.0);
    if (sj < si && cj == 0) {
        double pr = ri == 0 ? b1 - a1 * b0 : b2 - a2 * b0;
        for (int l = sj + 1; l < si; ++l) pr *= co[l][0];
        return pr;
    }
    return 0.0;
}

// Tile-transition powers of the whole cascade for the cascade-level
// look-back, in FP64, by one block of 256 threads (one matrix element
// each).  The cascade's one-sample transition F (zero input): block (i, i) =
// A_i; block (i, j), j < i = B_i (prod_{j<l<i} D_l) C, since section i's
// input is section i-1's output; Phi_T = F^(128 Lc) = (F^Lc)^128.
__device__ void mm16(const double (*A)[16], const double (*B)[16], double (*R)[16], int i, int j) {
    double acc = 0.0;
    for (int k = 0; k < 16; ++k) acc += A[i][k] * B[k][j];
    __syncthreads();  // every read of A and B done (R may alias either)
    R[i][j] = acc;
    __syncthreads();
}

// max |M| over the block (every thread gets it)
__device__ double block_maxabs(const double (*M)[16], int i, int j, int tid) {
    __shared__ double wmax[4];
    double v = fabs(M[i][j]);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d));
    if ((tid & 63) == 0) wmax[tid >> 6] = v;
    __syncthreads();
    v = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    __syncthreads();
    return v;
}

// co(s, k): coefficient k of section s; Lc: the chunk length (tile 128 Lc).
template <class Co>
__device__ void casc_table_block(Co co_at, int32_t S, int Lc, CascTab *out, int tid) {
    __shared__ double co[CASC_MAX][5];
    __shared__ double M0[16][16], M1[16][16], Pw[7][16][16];
    const int i = tid >> 4, j = tid & 15;
    if (tid < S * 5) co[tid / 5][tid % 5] = co_at(tid / 5, tid % 5);
    __syncthreads();
    M1[i][j] = cascade_f(co, 2 * S, i, j);
    Pw[0][i][j] = i == j ? 1.0 : 0.0;
    __syncthreads();
    for (int e = Lc; e > 0; e >>= 1) {  // Pw[0] = F^Lc by binary powering
        if (e & 1) mm16(Pw[0], M1, Pw[0], i, j);
        if (e > 1) mm16(M1, M1, M1, i, j);
    }
    for (int t = 0; t < 7; ++t) mm16(Pw[0], Pw[0], Pw[0], i, j);  // F^(128 Lc), the tile transition
    for (int t = 1; t < 7; ++t) mm16(Pw[t - 1], Pw[t - 1], Pw[t], i, j);  // Phi_T^(2^t)
    out->T[0][i][j] = (float)Pw[0][i][j];
    out->T[1][i][j] = (float)Pw[1][i][j];
    out->T[2][i][j] = (float)Pw[2][i][j];
    // look-back depth: a d <= 64 with max |Phi_T^d| <= 2^-60 (0 if none),
    // found by doubling, then bisection between the last failing power of
    // two and the first passing one; every accepted d is checked directly
    int first = -1;
    for (int t = 0; t < 7 && first < 0; ++t)
        if (block_maxabs(Pw[t], i, j, tid) <= DEPTH_EPS) first = t;
    int dep = 0;
    if (first == 0) {
        dep = 1;
    } else if (first > 0) {
        int lo = 1 << (first - 1), hi = 1 << first;
        M0[i][j] = Pw[first - 1][i][j];  // Phi_T^lo
        __syncthreads();
        for (int t = first - 2; t >= 0; --t) {
            mm16(M0, Pw[t], M1, i, j);  // Phi_T^(lo + 2^t)
            if (block_maxabs(M1, i, j, tid) <= DEPTH_EPS) {
                hi = lo + (1 << t);
            } else {
                lo += 1 << t;
                M0[i][j] = M1[i][j];
                __syncthreads();
            }
        }
        dep = hi;
    }
    if (tid == 0) out->depth = dep;
}

// Zero-input response tables of the cascade (CascZir), in FP64 then
// rounded, one block of 256 threads (one matrix element each) per entry:
// k < ZIR_B gives F^(Lc k), ZIR_B <= k < ZIR_B + ZIR_A gives F^(16 Lc a),
// a = k - ZIR_B, by binary powering; k == ZIR_B + ZIR_A gives the output rows
// G[r] = c F^r, r < Lc, where c[2s] = prod_{t>s} b0_t (the s1 register of
// section s reaches the output through the b0 of every later section) and
// c[2s+1] = 0.
template <class Co>
__device__ void zir_block(Co co_at, int32_t S, int Lc, int k, CascZir *out, int tid) {
    __shared__ double co[CASC_MAX][5];
    __shared__ double Fm[16][16], P[16][16];
    __shared__ double g[16];
    const int i = tid >> 4, j = tid & 15;
    if (tid < S * 5) co[tid / 5][tid % 5] = co_at(tid / 5, tid % 5);
    __syncthreads();
    const int D = 2 * S;
    Fm[i][j] = cascade_f(co, D, i, j);
    P[i][j] = i == j ? 1.0 : 0.0;
    __syncthreads();
    if (k < ZIR_B + ZIR_A) {
        const int e0 = k < ZIR_B ? Lc * k : ZIR_B * Lc * (k - ZIR_B);
        for (int e = e0; e > 0; e >>= 1) {
            if (e & 1) mm16(P, Fm, P, i, j);
            if (e > 1) mm16(Fm, Fm, Fm, i, j);
        }
        if (k < ZIR_B) out->Mb[i][j][k] = (float)P[i][j];
        else out->MaT[k - ZIR_B][j][i] = (float)P[i][j];
        return;
    }
    if (tid < 16) {
        double c = 0.0;
        if (tid < D && (tid & 1) == 0) {
            c = 1.0;
            for (int t = (tid >> 1) + 1; t < S; ++t) c *= co[t][0];
        }
        g[tid] = c;
    }
    __syncthreads();
    for (int r = 0; r < Lc; ++r) {  // G[r] = g, then g <- g F
        double acc = 0.0;
        if (tid < 16) {
            out->G[r][tid] = (float)g[tid];
            for (int q = 0; q < 16; ++q) acc += g[q] * Fm[q][tid];
        }
        __syncthreads();
        if (tid < 16) g[tid] = acc;
        __syncthreads();
    }
}

// Matrix-core cascade tables (McTab), in FP64 then rounded, one block of
// 256 threads: the chunk's impulse response h, the input columns F^m b, the
// output rows c F^r, the chunk transition Fc = F^32 and the segment
// transition Fc^12, each laid out as the kernel's operands.
template <class Co>
__device__ void mc_block(Co co_at, int32_t S, McTab *out, int tid) {
    __shared__ double co[CASC_MAX][5];
    __shared__ double Pw[16][16], Q[16][16];
    __shared__ double V[MC_LC][16];   // F^m b
    __shared__ double Gm[MC_LC][16];  // c F^r
    __shared__ double hh[MC_LC];
    const int i = tid >> 4, j = tid & 15;
    if (tid < S * 5) co[tid / 5][tid % 5] = co_at(tid / 5, tid % 5);
    __syncthreads();
    const int D = 2 * S;
    Pw[i][j] = cascade_f(co, D, i, j);
    if (tid < 16) {
        // b: section s sees the input through the b0 of every earlier
        // section; c: the s1 register of section s reaches the output
        // through the b0 of every later one
        double bb = 0.0, cc = 0.0;
        if (tid < D) {
            const int sc = tid >> 1;
            double g = 1.0;
            for (int l = 0; l < sc; ++l) g *= co[l][0];
            bb = ((tid & 1) ? co[sc][2] - co[sc][4] * co[sc][0] : co[sc][1] - co[sc][3] * co[sc][0]) * g;
            if ((tid & 1) == 0) {
                cc = 1.0;
                for (int t = sc + 1; t < S; ++t) cc *= co[t][0];
            }
        }
        V[0][tid] = bb;
        Gm[0][tid] = cc;
    }
    __syncthreads();
    // doubling: with Pw = F^(2^l), V[2^l + v] = Pw V[v] and
    // Gm[2^l + v] = Gm[v] Pw for v < 2^l (thread (i, j): component i of
    // vector j), then Pw <- Pw^2; five levels give 32 vectors and Pw = F^32
    for (int l = 0; l < 5; ++l) {
        const int n = 1 << l;
        double vv = 0.0, gg = 0.0;
        if (j < n) {
            for (int k = 0; k < 16; ++k) {
                vv += Pw[i][k] * V[j][k];
                gg += Gm[j][k] * Pw[k][i];
            }
        }
        __syncthreads();
        if (j < n) {
            V[n + j][i] = vv;
            Gm[n + j][i] = gg;
        }
        mm16(Pw, Pw, Pw, i, j);
    }
    if (tid < MC_LC) {  // h[0] = d, h[n] = c F^(n-1) b
        double hv = 0.0;
        if (tid == 0) {
            hv = S > 0 ? 1.0 : 0.0;
            for (int l = 0; l < S; ++l) hv *= co[l][0];
        } else {
            for (int k = 0; k < 16; ++k) hv += Gm[tid - 1][k] * V[0][k];
        }
        hh[tid] = hv;
    }
    __syncthreads();
    for (int e = tid; e < 64 * 24; e += 256) {
        const int l = e / 24, q = e % 24, rb = q / 8, t = q % 8;
        const int row = 16 * rb + (l & 15), m = 8 * (l >> 4) + t;
        double v;
        if (row < MC_LC) v = row >= m ? hh[row - m] : 0.0;
        else v = V[MC_LC - 1 - m][row - MC_LC];  // H[:, m] = F^(31 - m) b
        out->W[l][q] = (float)v;
    }
    for (int e = tid; e < 64 * 8; e += 256) {
        const int l = e / 8, q = e % 8, rb = q / 4, k = q % 4;
        out->Gt[l][q] = (float)Gm[16 * rb + (l & 15)][4 * (l >> 4) + k];
    }
    out->Fr[i][j] = (float)Pw[i][mc_src(i, j)];  // Fc = F^32
    mm16(Pw, Pw, Q, i, j);  // Fc^2
    mm16(Q, Q, Q, i, j);    // Fc^4
    mm16(Q, Q, Pw, i, j);   // Fc^8
    mm16(Pw, Q, Q, i, j);   // Fc^12
    out->Fsr[i][j] = (float)Q[i][mc_src(i, j)];
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
        double *t = cur;
        cur = nxt;
        nxt = t;
        Mcur = Mn;
    }
    for (int k = threadIdx.x; k < Mcur; k += blockDim.x) a.out[k] = (float)cur[k];
}

// Entry i of the twiddle tables (i < 4096), each e^{-2 pi i e / 4096} for an
// exact integer e mod 4096, in FP64 and rounded once: tw64[i] (e = i) and,
// for i < TWL_ENTRIES, the padded fp32 table TWL of the FFT kernels.
__device__ void write_twiddle(float2 *twid, double2 *tw64, int i) {
    double sn, cs;
    sincospi(-2.0 * (double)i / NFFT, &sn, &cs);
    tw64[i] = make_double2(cs, sn);
    if (i < TWL_ENTRIES) {  // TWL[r][k]: e = 16 r k (r < 16), (r - 16) k; pads zero
        const int r = i / TWL_S, k = i % TWL_S;
        const int eL = ((r < 16 ? 16 * r : r - 16) * k) & (NFFT - 1);
        sincospi(-2.0 * (double)eL / NFFT, &sn, &cs);
        twid[i] = k < 16 ? make_float2((float)cs, (float)sn) : make_float2(0.f, 0.f);
    }
}

__global__ void fft_twiddle_kernel(float2 *twid, double2 *tw64) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < NFFT) write_twiddle(twid, tw64, k);
}

// hspec[p][k] = (sum_j h[1025 p + j] e^{-2 pi i j k / 4096}) / 4096, the DFT
// of tap partition p (j < 1025, zero-padded), in FP64, stored in the FFT
// kernels' per-lane order (bin t + 256 k3 at [t][k3]).  One block of 256
// lanes covers 16 bins: lane (kk, jj) sums taps j = jj (mod 16) of bin
// k = 16 blk + kk, stepping its twiddle by e^{-2 pi i 16 k / 4096} (at most
// 65 steps from an exact start, so the FP64 twiddle error stays near
// 1e-14, far below the fp32 rounding of the result); the 16 partial sums
// are added by a fixed shuffle tree.
__device__ void spectrum_block(const float *h_all, int32_t M_all, int part, int blk, float2 *hspec_all, int tid) {
    __shared__ float hs[FFT_PART + 15];
    const int kk = tid >> 4, jj = tid & 15;
    const int k = blk * 16 + kk;
    const float *h = h_all + (int64_t)part * FFT_PART;
    const int rest = M_all - part * FFT_PART;
    const int M = rest < FFT_PART ? rest : FFT_PART;
    for (int j = tid; j < FFT_PART + 15; j += 256) hs[j] = j < M ? h[j] : 0.f;  // zero-padded to 16 | length
    __syncthreads();
    double wr, wi, sr, si;
    sincospi(-2.0 * (double)((jj * k) & (NFFT - 1)) / NFFT, &wi, &wr);
    sincospi(-2.0 * (double)((16 * k) & (NFFT - 1)) / NFFT, &si, &sr);
    double hr = 0.0, hi = 0.0;
#pragma unroll 5
    for (int m = 0; m < (FFT_PART + 15) / 16; ++m) {
        const double hv = (double)hs[jj + 16 * m];
        hr = fma(hv, wr, hr);
        hi = fma(hv, wi, hi);
        const double nr = wr * sr - wi * si;
        wi = fma(wr, si, wi * sr);
        wr = nr;
    }
#pragma unroll
    for (int d = 8; d >= 1; d >>= 1) {
        hr += __shfl_xor(hr, d);
        hi += __shfl_xor(hi, d);
    }
    if (jj == 0)  // per-lane layout: bin t + 256 k3 at [t][k3]
        hspec_all[(int64_t)part * NFFT + 16 * (k & 255) + (k >> 8)] = make_float2((float)(hr / NFFT), (float)(hi / NFFT));
}

// The prepare step of a chain in one launch.  Blocks take roles by index:
// tap-spectrum blocks (which also write the twiddle tables), one block per
// section (scan tables), one block for the cascade's tile transition; every
// block also clears a share of the look-back records (tag 0 never matches
// an epoch), and block 0 arms the header (epoch 1, error 0, high-Q word).
struct PrepareArgs {
    const float *h;
    int32_t M, nspec;  // nspec = 256 * partitions, or 0 without an FFT FIR
    float2 *twid, *hspec;
    double2 *tw64;
    SecTab *tab;
    int32_t S, casc;
    StageList sos;
    CascTab *ctab;
    McTab *mc;     // matrix-core cascade tables (null: not wanted)
    CascZir *zir;  // zero-input response tables (null: not wanted)
    uint64_t *recs;
    int64_t nwords;
    uint32_t *hdr;
};

__global__ __launch_bounds__(256) void prepare_kernel(PrepareArgs a) {
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    for (int64_t i = (int64_t)b * 256 + tid; i < a.nwords; i += (int64_t)gridDim.x * 256) a.recs[i] = 0ull;
    if (b == 0) {  // header words; the cascade's high-Q word: one section per thread, loads in parallel
        __shared__ uint32_t s_any;
        if (tid == 0) s_any = 0u;
        __syncthreads();
        for (int q = tid; q < a.S; q += 256) {
            int sec = q, st = 0;
            while (sec >= a.sos.len[st]) {
                sec -= a.sos.len[st];
                ++st;
            }
            if (section_hiq(a.sos.ptr[st][5 * sec + 3], a.sos.ptr[st][5 * sec + 4])) atomicOr(&s_any, 1u);
        }
        __syncthreads();
        if (tid == 0) {
            a.hdr[HDR_ERROR] = 0u;
            a.hdr[HDR_EPOCH] = 1u;
            a.hdr[HDR_HIQ] = s_any;
        }
    }
    if (b < a.nspec) {
        const int blk = b % (NFFT / 16), part = b / (NFFT / 16);
        spectrum_block(a.h, a.M, part, blk, a.hspec, tid);
        if (part == 0 && tid < 16) write_twiddle(a.twid, a.tw64, blk * 16 + tid);
    } else if (b < a.nspec + a.S) {
        int s = b - a.nspec, st = 0;
        while (s >= a.sos.len[st]) {
            s -= a.sos.len[st];
            ++st;
        }
        build_section_block(&a.tab[b - a.nspec], a.sos.ptr[st] + 5 * s, L, tid);
    } else if (a.casc && b == a.nspec + a.S) {
        const StageList &sl = a.sos;
        casc_table_block(
            [&](int s, int k) {
                int st = 0;
                while (s >= sl.len[st]) {
                    s -= sl.len[st];
                    ++st;
                }
                return (double)sl.ptr[st][5 * s + k];
            },
            a.S, L, a.ctab, tid);
    } else if (a.casc && a.mc && b == a.nspec + a.S + 1) {
        const StageList &sl = a.sos;
        mc_block(
            [&](int s, int k) {
                int st = 0;
                while (s >= sl.len[st]) {
                    s -= sl.len[st];
                    ++st;
                }
                return (double)sl.ptr[st][5 * s + k];
            },
            a.S, a.mc, tid);
    } else if (a.casc && a.zir && b > a.nspec + a.S + 1 && b <= a.nspec + a.S + 2 + ZIR_B + ZIR_A) {
        const StageList &sl = a.sos;
        zir_block(
            [&](int s, int k) {
                int st = 0;
                while (s >= sl.len[st]) {
                    s -= sl.len[st];
                    ++st;
                }
                return (double)sl.ptr[st][5 * s + k];
            },
            a.S, L, b - (a.nspec + a.S + 2), a.zir, tid);
    }
}

__global__ void state_passthrough_kernel(const float *in, float *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in ? in[i] : 0.f;
}

// Batched clips: section tables of every clip (chunk length lc), the block
// map, cleared look-back records, epoch 1.  Thread g < nsec builds section g, found by a
// binary search over the clips' first table index.
struct BatchPrepArgs {
    const ClipDesc *desc;
    int32_t nclips;
    SecTab *tab;
    int64_t nsec;
    uint64_t *recs;
    int64_t nwords;
    uint32_t *hdr;
    int32_t lc;
    CascTab *ctab;  // per clip, or null
    McTab *mtab;    // per clip, or null
    int32_t *map;   // block id -> clip, nblocks entries
    int64_t nblocks;
};

// Blocks g < nsec build section g; blocks nsec + c build clip c's cascade
// tables (when ctab is set); every block clears a share of the records.
__global__ __launch_bounds__(256) void batch_prep_kernel(BatchPrepArgs a) {
    const int tid = threadIdx.x;
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < a.nwords; i += (int64_t)gridDim.x * 256) a.recs[i] = 0ull;
    // block map: the last clip whose first block is <= b (first blocks never
    // decrease; a clip without blocks shares its first block with the next)
    for (int64_t b = (int64_t)blockIdx.x * 256 + tid; b < a.nblocks; b += (int64_t)gridDim.x * 256) {
        int lo = 0, hi = a.nclips - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (a.desc[mid].blk0 <= b) lo = mid;
            else hi = mid - 1;
        }
        a.map[b] = lo;
    }
    if (blockIdx.x == 0 && tid == 0) {
        a.hdr[HDR_ERROR] = 0u;
        a.hdr[HDR_EPOCH] = 1u;
        uint32_t any = 0u;
        for (int c = 0; c < a.nclips; ++c)
            for (int s = 0; s < a.desc[c].S; ++s)
                any |= section_hiq(a.desc[c].sos[5 * s + 3], a.desc[c].sos[5 * s + 4]) ? 1u : 0u;
        a.hdr[HDR_HIQ] = any;
    }
    const int64_t nroles = a.nsec + (a.ctab ? a.nclips : 0) + (a.mtab ? a.nclips : 0);
    for (int64_t g = blockIdx.x; g < nroles; g += gridDim.x) {
        if (g < a.nsec) {
            // the last clip with tab0 <= g: tab0 grows with the clip index by
            // S, so that clip has S > 0 and holds section g
            int lo = 0, hi = a.nclips - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (a.desc[mid].tab0 <= g) lo = mid;
                else hi = mid - 1;
            }
            build_section_block(&a.tab[g], a.desc[lo].sos + 5 * (g - a.desc[lo].tab0), a.lc, tid);
        } else if (g < a.nsec + a.nclips) {
            const ClipDesc &d = a.desc[g - a.nsec];
            if (d.S > 0) {
                const float *co = d.sos;
                casc_table_block([&](int s, int k) { return (double)co[5 * s + k]; }, d.S, a.lc,
                                 &a.ctab[g - a.nsec], tid);
            }
        } else {
            const int c = (int)(g - a.nsec - a.nclips);
            const ClipDesc &d = a.desc[c];
            if (d.S > 0) {
                const float *co = d.sos;
                mc_block([&](int s, int k) { return (double)co[5 * s + k]; }, d.S, &a.mtab[c], tid);
            }
        }
        __syncthreads();  // the role's shared memory is reused by the next one
    }
}

hipError_t launch_batch_prepare(const BatchLayout &lay, int lc, int32_t nclips, void *ws, hipStream_t st) {
    char *w = static_cast<char *>(ws);
    BatchPrepArgs a;
    a.desc = reinterpret_cast<const ClipDesc *>(w + lay.desc);
    a.nclips = nclips;
    a.tab = reinterpret_cast<SecTab *>(w + lay.tab);
    a.nsec = lay.nsec;
    a.recs = reinterpret_cast<uint64_t *>(w + lay.recs);
    a.nwords = lay.nrec * 4;
    a.hdr = reinterpret_cast<uint32_t *>(w + lay.hdr);
    a.lc = lc;
    a.ctab = lay.casc_on ? reinterpret_cast<CascTab *>(w + lay.casc) : nullptr;
    a.mtab = lay.mc_on ? reinterpret_cast<McTab *>(w + lay.mc) : nullptr;
    a.map = reinterpret_cast<int32_t *>(w + lay.map);
    a.nblocks = lay.nblocks;
    const int64_t nroles = a.nsec + (a.ctab ? nclips : 0) + (a.mtab ? nclips : 0);
    int64_t nb = (a.nwords + 255) / 256;
    if (nb > 2048) nb = 2048;
    if (nb < nroles) nb = nroles < 2048 ? nroles : 2048;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(batch_prep_kernel, dim3((unsigned)nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_tables(const ChainPlan &p, const WsLayout &lay, const float *h, int32_t M) {
    char *ws = static_cast<char *>(p.ws);
    hipError_t e;
    if (p.firs.n > 1) {
        MergeArgs m;
        m.firs = p.firs;
        m.buf0 = reinterpret_cast<double *>(ws + lay.merge);
        m.buf1 = m.buf0 + M;
        m.out = reinterpret_cast<float *>(ws + lay.taps);
        hipLaunchKernelGGL(merge_taps_kernel, dim3(1), dim3(256), 0, p.stream, m);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    PrepareArgs a{};
    const bool fft = p.firs.n > 0 && p.fir_mode == FIR_FFT;
    a.h = h;
    a.M = M;
    a.nspec = fft ? (NFFT / 16) * fft_parts(M) : 0;
    a.twid = reinterpret_cast<float2 *>(ws + lay.twid);
    a.hspec = reinterpret_cast<float2 *>(ws + lay.hspec);
    a.tw64 = reinterpret_cast<double2 *>(ws + lay.tw64);
    a.tab = reinterpret_cast<SecTab *>(ws + lay.tab);
    a.S = p.S;
    a.casc = (p.S > 0 && p.S <= CASC_MAX) ? 1 : 0;
    a.sos = p.sos;
    a.ctab = reinterpret_cast<CascTab *>(ws + lay.casc);
    // cascades of up to ZIR_MAX sections take the zero-input response
    // tables, longer ones (up to CASC_MAX) the matrix-core form
    a.mc = (a.casc && p.S >= MC_MIN_SECTIONS) ? reinterpret_cast<McTab *>(ws + lay.mc) : nullptr;
    a.zir = (a.casc && p.S <= ZIR_MAX) ? reinterpret_cast<CascZir *>(ws + lay.zir) : nullptr;
    a.recs = reinterpret_cast<uint64_t *>(ws + lay.recs);
    a.nwords = p.S > 0 ? lay.cpad * lay.ntiles * p.S * REC_WORDS : 0;
    a.hdr = reinterpret_cast<uint32_t *>(ws + lay.hdr);
    int64_t nb = a.nspec + a.S + (a.casc ? 2 : 0) + (a.zir ? ZIR_B + ZIR_A + 1 : 0);
    int64_t nclear = (a.nwords + 255) / 256;
    if (nclear > 1024) nclear = 1024;
    if (nb < nclear) nb = nclear;
    // a workspace with room for the header gets its header words written
    // even when there is nothing else to build
    if (nb == 0 && p.ws && p.ws_bytes >= 256) nb = 1;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(prepare_kernel, dim3((unsigned)nb), dim3(256), 0, p.stream, a);
    return hipGetLastError();
}

// Header words of a workspace that a call uses without building anything
// (empty signals, identity cascades): error 0, epoch 1, no high-Q section.
__global__ void header_init_kernel(uint32_t *hdr) {
    hdr[HDR_ERROR] = 0u;
    hdr[HDR_EPOCH] = 1u;
    hdr[HDR_HIQ] = 0u;
}

hipError_t launch_header_init(void *ws, size_t ws_bytes, hipStream_t st) {
    if (!ws || ws_bytes < 256) return hipSuccess;
    hipLaunchKernelGGL(header_init_kernel, dim3(1), dim3(1), 0, st, static_cast<uint32_t *>(ws));
    return hipGetLastError();
}

// Status word of a workspace: OR it into *flags (written only when a bit is
// set), then optionally clear it.  One thread; stream-ordered after the
// calls that used the workspace.
__global__ void ws_status_kernel(uint32_t *hdr, uint32_t *flags, int32_t clear) {
    const uint32_t v = __hip_atomic_load(hdr + HDR_ERROR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v) *flags |= v;
    if (clear) __hip_atomic_store(hdr + HDR_ERROR, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t launch_ws_status(void *ws, uint32_t *flags, int32_t clear, hipStream_t st) {
    hipLaunchKernelGGL(ws_status_kernel, dim3(1), dim3(1), 0, st, static_cast<uint32_t *>(ws), flags, clear);
    return hipGetLastError();
}

hipError_t launch_twiddles(float2 *twid, double2 *tw64, hipStream_t st) {
    hipLaunchKernelGGL(fft_twiddle_kernel, dim3(NFFT / 256), dim3(256), 0, st, twid, tw64);
    return hipGetLastError();
}

hipError_t launch_state_passthrough(const float *in, float *out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(state_passthrough_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

}  // namespace tfx
