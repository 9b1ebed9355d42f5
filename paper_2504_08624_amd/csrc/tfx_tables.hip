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

// Transition powers of one TDF-II section.  With state s = (s1, s2) the
// section is s' = A s + B x, y = s1 + b0 x, A = [[-a1, 1], [-a2, 0]], so a
// state s entering a chunk becomes A^Lc s after Lc samples.
__device__ void build_section(SecTab *tb, const float *co, int Lc) {
    const double a1 = co[3], a2 = co[4];
    for (int i = 0; i < 5; ++i) tb->coef[i] = co[i];
    tb->pad = 0;
    const double A[4] = {-a1, 1.0, -a2, 0.0};
    double P[4] = {A[0], A[1], A[2], A[3]};
    for (int t = 1; t < Lc; ++t) mat2_mul(P, A, P);
    const double Phi[4] = {P[0], P[1], P[2], P[3]};
    double F[4] = {1.0, 0.0, 0.0, 1.0};
    for (int k = 0; k < 64; ++k) {
        put4(tb->fold[k], tb->fold_d[k], F);
        mat2_mul(F, Phi, F);
    }
    const double Psi[4] = {F[0], F[1], F[2], F[3]};
    double W[4] = {1.0, 0.0, 0.0, 1.0};
    for (int w = 0; w < GWAVES; ++w) {
        put4(tb->psi[w], tb->psi_d[w], W);
        mat2_mul(W, Psi, W);
    }
    double B[4] = {W[0], W[1], W[2], W[3]};  // PhiT = A^T
    {  // look-back depth
        double Q[4] = {W[0], W[1], W[2], W[3]};
        tb->depth = 0;
        for (int k = 1; k <= 64; ++k) {
            if (fmax(fmax(fabs(Q[0]), fabs(Q[1])), fmax(fabs(Q[2]), fabs(Q[3]))) <= DEPTH_EPS) {
                tb->depth = k;
                break;
            }
            mat2_mul(Q, W, Q);
        }
    }
    for (int j = 0; j < 9; ++j) {
        put4(tb->lb[j], tb->lb_d[j], B);
        mat2_mul(B, B, B);
    }
    tb->hiq = section_hiq(a1, a2) ? 1 : 0;
}

struct PrepArgs {
    SecTab *tab;
    int32_t S;
    StageList sos;
    uint64_t *recs;
    int64_t nwords;
    uint32_t *hdr;
};

// Section tables; clears the look-back records (tag 0 never matches an
// epoch); arms the header (epoch 1).
__global__ void prep_kernel(PrepArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gid; i < a.nwords; i += stride) a.recs[i] = 0ull;
    if (gid == 0) {
        a.hdr[HDR_ERROR] = 0u;
        a.hdr[HDR_EPOCH] = 1u;
        uint32_t any = 0u;
        for (int s = 0, st = 0, j = 0; s < a.S; ++s, ++j) {
            while (j >= a.sos.len[st]) {
                j -= a.sos.len[st];
                ++st;
            }
            const float *co = a.sos.ptr[st] + 5 * j;
            any |= section_hiq(co[3], co[4]) ? 1u : 0u;
        }
        a.hdr[HDR_HIQ] = any;
    }
    if (gid < a.S) {
        int s = (int)gid, st = 0;
        while (s >= a.sos.len[st]) {
            s -= a.sos.len[st];
            ++st;
        }
        build_section(&a.tab[gid], a.sos.ptr[st] + 5 * s, L);
    }
}

// Tile-transition powers of the whole cascade for the cascade-level
// look-back, in FP64.  The cascade's one-sample transition F (zero input):
// block (i, i) = A_i; block (i, j), j < i = B_i (prod_{j<l<i} D_l) C, since
// section i's input is section i-1's output; Phi_T = F^3072 = (F^8 F^16)^128.
// One block of 256 threads, one matrix element each.
__device__ void mm16(const double (*A)[16], const double (*B)[16], double (*R)[16], int i, int j) {
    double acc = 0.0;
    for (int k = 0; k < 16; ++k) acc += A[i][k] * B[k][j];
    __syncthreads();  // every read of A and B done (R may alias neither, but callers reuse buffers)
    R[i][j] = acc;
    __syncthreads();
}

__global__ void casc_table_kernel(StageList sos, int32_t S, CascTab *out) {
    __shared__ double co[CASC_MAX][5];
    __shared__ double M0[16][16], M1[16][16], M2[16][16], M3[16][16];
    const int tid = threadIdx.x, i = tid >> 4, j = tid & 15;
    if (tid < S * 5) {
        int s = tid / 5, st = 0;
        const int k = tid % 5;
        while (s >= sos.len[st]) {
            s -= sos.len[st];
            ++st;
        }
        co[tid / 5][k] = sos.ptr[st][5 * s + k];
    }
    __syncthreads();
    const int D = 2 * S;
    double f = 0.0;
    if (i < D && j < D) {
        const int si = i >> 1, ri = i & 1, sj = j >> 1, cj = j & 1;
        const double b0 = co[si][0], b1 = co[si][1], b2 = co[si][2], a1 = co[si][3], a2 = co[si][4];
        if (si == sj) {
            f = ri == 0 ? (cj == 0 ? -a1 : 1.0) : (cj == 0 ? -a2 : 0.0);
        } else if (sj < si && cj == 0) {
            double pr = ri == 0 ? b1 - a1 * b0 : b2 - a2 * b0;
            for (int l = sj + 1; l < si; ++l) pr *= co[l][0];
            f = pr;
        }
    }
    M0[i][j] = f;
    __syncthreads();
    mm16(M0, M0, M1, i, j);  // F^2
    mm16(M1, M1, M0, i, j);  // F^4
    mm16(M0, M0, M2, i, j);  // F^8
    mm16(M2, M2, M1, i, j);  // F^16
    mm16(M1, M2, M3, i, j);  // F^24
    for (int t = 0; t < 7; ++t) {  // F^(24 * 128) = F^3072
        mm16(M3, M3, M0, i, j);
        M3[i][j] = M0[i][j];
        __syncthreads();
    }
    out->T[0][i][j] = (float)M3[i][j];
    {  // look-back depth: the first d with max |Phi_T^d| <= 2^-60
        __shared__ double amax[256];
        __shared__ int dep;
        if (tid == 0) dep = 0;
        M0[i][j] = M3[i][j];
        __syncthreads();
        for (int k = 1; k <= 64; ++k) {
            amax[tid] = fabs(M0[i][j]);
            __syncthreads();
            for (int w = 128; w >= 1; w >>= 1) {
                if (tid < w) amax[tid] = fmax(amax[tid], amax[tid + w]);
                __syncthreads();
            }
            const bool hit = amax[0] <= DEPTH_EPS;
            __syncthreads();
            if (hit) {
                if (tid == 0) dep = k;
                break;
            }
            mm16(M0, M3, M1, i, j);
            M0[i][j] = M1[i][j];
            __syncthreads();
        }
        __syncthreads();
        if (tid == 0) out->depth = dep;
    }
    mm16(M3, M3, M1, i, j);
    out->T[1][i][j] = (float)M1[i][j];
    mm16(M1, M1, M2, i, j);
    out->T[2][i][j] = (float)M2[i][j];
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

// twid[k] = e^{-2 pi i k / 4096} in fp32 (filter kernel) and fp64 (spectrum)
__global__ void fft_twiddle_kernel(float2 *twid, double2 *tw64) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NFFT) return;
    double s, c;
    sincospi(-2.0 * (double)k / NFFT, &s, &c);
    twid[k] = make_float2((float)c, (float)s);
    tw64[k] = make_double2(c, s);
}

// hspec[p][k] = (sum_j h[1025 p + j] e^{-2 pi i j k / 4096}) / 4096, the
// direct DFT of tap partition p (j < 1025, zero-padded) in FP64 (exact
// twiddle indices j k mod 4096).  Block (blk, p) of 256 lanes covers 16 bins:
// lane (kk, jj) sums taps j = jj (mod 16) of bin 16 blk + kk, then the 16
// partial sums are added in a fixed order.
__global__ void fft_spectrum_kernel(const float *h_all, int32_t M_all, const double2 *tw64, float2 *hspec_all) {
    __shared__ double pr[16][17], pi[16][17];
    const int kk = threadIdx.x >> 4, jj = threadIdx.x & 15;
    const int k = blockIdx.x * 16 + kk;
    const float *h = h_all + (int64_t)blockIdx.y * FFT_PART;
    const int rest = M_all - (int)blockIdx.y * FFT_PART;
    const int M = rest < FFT_PART ? rest : FFT_PART;
    float2 *hspec = hspec_all + (int64_t)blockIdx.y * NFFT;
    double hr = 0.0, hi = 0.0;
    for (int j = jj; j < M; j += 16) {
        const double2 w = tw64[(j * k) & (NFFT - 1)];
        hr += (double)h[j] * w.x;
        hi += (double)h[j] * w.y;
    }
    pr[kk][jj] = hr;
    pi[kk][jj] = hi;
    __syncthreads();
    if (jj == 0) {
        double sr = 0.0, si = 0.0;
        for (int u = 0; u < 16; ++u) {
            sr += pr[kk][u];
            si += pi[kk][u];
        }
        hspec[k] = make_float2((float)(sr / NFFT), (float)(si / NFFT));
    }
}

__global__ void state_passthrough_kernel(const float *in, float *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in ? in[i] : 0.f;
}

// Batched clips: section tables of every clip (chunk length lc), cleared
// look-back records, epoch 1.  Thread g < nsec builds section g, found by a
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
};

__global__ void batch_prep_kernel(BatchPrepArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gid; i < a.nwords; i += stride) a.recs[i] = 0ull;
    if (gid == 0) {
        a.hdr[HDR_ERROR] = 0u;
        a.hdr[HDR_EPOCH] = 1u;
        uint32_t any = 0u;
        for (int c = 0; c < a.nclips; ++c)
            for (int s = 0; s < a.desc[c].S; ++s)
                any |= section_hiq(a.desc[c].sos[5 * s + 3], a.desc[c].sos[5 * s + 4]) ? 1u : 0u;
        a.hdr[HDR_HIQ] = any;
    }
    for (int64_t g = gid; g < a.nsec; g += stride) {
        // the last clip with tab0 <= g: tab0 grows with the clip index by S,
        // so that clip has S > 0 and holds section g
        int lo = 0, hi = a.nclips - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (a.desc[mid].tab0 <= g) lo = mid;
            else hi = mid - 1;
        }
        build_section(&a.tab[g], a.desc[lo].sos + 5 * (g - a.desc[lo].tab0), a.lc);
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
    const int64_t work = a.nwords > a.nsec ? a.nwords : a.nsec;
    int64_t nb = (work + 255) / 256;
    if (nb > 2048) nb = 2048;
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
    if (p.firs.n > 0 && p.fir_mode == FIR_FFT) {
        double2 *tw64 = reinterpret_cast<double2 *>(ws + lay.tw64);
        hipLaunchKernelGGL(fft_twiddle_kernel, dim3(NFFT / 256), dim3(256), 0, p.stream,
                           reinterpret_cast<float2 *>(ws + lay.twid), tw64);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(fft_spectrum_kernel, dim3(NFFT / 16, fft_parts(M)), dim3(256), 0, p.stream, h, M, tw64,
                           reinterpret_cast<float2 *>(ws + lay.hspec));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (p.S > 0) {
        PrepArgs pa;
        pa.tab = reinterpret_cast<SecTab *>(ws + lay.tab);
        pa.S = p.S;
        pa.sos = p.sos;
        pa.recs = reinterpret_cast<uint64_t *>(ws + lay.recs);
        pa.nwords = lay.cpad * lay.ntiles * p.S * 4;
        pa.hdr = reinterpret_cast<uint32_t *>(ws + lay.hdr);
        const int64_t work = pa.nwords > p.S ? pa.nwords : p.S;
        int64_t nb = (work + 255) / 256;
        if (nb > 1024) nb = 1024;
        if (nb < 1) nb = 1;
        hipLaunchKernelGGL(prep_kernel, dim3((unsigned)nb), dim3(256), 0, p.stream, pa);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (p.S <= CASC_MAX) {
            hipLaunchKernelGGL(casc_table_kernel, dim3(1), dim3(256), 0, p.stream, p.sos, p.S,
                               reinterpret_cast<CascTab *>(ws + lay.casc));
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    return hipSuccess;
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
