// tfx_mc.h -- the matrix-core form of a short SOS cascade, shared by the
// chain kernel and the batched kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "tfx_device.h"

namespace tfx {

// --------------------------------------------------- matrix-core cascade
// Cascades of up to CASC_MAX sections (no FP64-carry section), no final-state
// output: the cascade runs on the matrix cores instead of section by section.
// A workgroup holds the tile of a channel pair as 192 chunks of MC_LC = 32
// samples (chunk K = 96 ch + k).  With the tables of McTab:
//   (1) [Tc; H] X on the matrix cores (16 x 16 x 4 fp32 steps): the chunks'
//       zero-state outputs Y0 = Tc X and the state each chunk leaves from a
//       zero entering state, U = H X;
//   (2) the chunk states s_(k+1) = Fc s_k + u_k in 16 segments of 12 chunks,
//       one 16-lane row per segment and one lane per state component (the
//       12 x 12 product by DPP row rotations), from zero: each segment's
//       aggregate;
//   (3) per channel, the tile aggregate from the segment aggregates (powers
//       Fs = Fc^12), one decoupled look-back of the whole cascade state (as in
//       the per-section form, the tile transition F^3072), then every
//       segment's entering state;
//   (4) the recurrence of (2) again from those states: every chunk's
//       entering state S;
//   (5) Y = Y0 + G S on the matrix cores, staged through LDS and stored.
// The per-sample work is on the matrix cores; the vector units do the
// 12-step recurrences (about 20 instructions per chunk step) and the FFT.
typedef float mcf4 __attribute__((ext_vector_type(4)));
constexpr int MC_XS = 36;                       // LDS floats per staged chunk (32 + 4 padding)
constexpr int MC_US = 20;                       // LDS floats per chunk state (16 + 4 padding)
constexpr int MC_CHUNKS = GROUPS * MC_NCH;      // 192
constexpr int MC_X_FLOATS = MC_CHUNKS * MC_XS;  // 6912
constexpr int MC_G_OFF = MC_CHUNKS * MC_US;     // segment aggregates [16][16]
constexpr int MC_E_OFF = MC_G_OFF + 256;        // segment-entering states [16][16]
constexpr int MC_LB_OFF = MC_E_OFF + 256;       // cascade look-back area
static_assert(MC_LB_OFF + casc_floats(16) <= MC_X_FLOATS, "look-back area must fit beside the chunk states");
static_assert(MC_NCH == 8 * MC_SEG && WG == 256, "16 segments of 12 chunks over four waves");

// value of lane mc_src(i, D_) of the lane's 16-lane row
template <int D_>
__device__ __forceinline__ float mc_rot(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x120 + D_, 0xF, 0xF, true));
}

// u + M s for the 16-component state s held one component per lane of a
// 16-lane row; f[d] = M[i][mc_src(i, d)] on lane i.  Four partial sums in a
// fixed order.
__device__ __forceinline__ float mc_step(float s, const float (&f)[16], float u) {
    float a0 = fmaf(f[0], s, u);
    float a1 = f[1] * mc_rot<1>(s);
    float a2 = f[2] * mc_rot<2>(s);
    float a3 = f[3] * mc_rot<3>(s);
    a0 = fmaf(f[4], mc_rot<4>(s), a0);
    a1 = fmaf(f[5], mc_rot<5>(s), a1);
    a2 = fmaf(f[6], mc_rot<6>(s), a2);
    a3 = fmaf(f[7], mc_rot<7>(s), a3);
    a0 = fmaf(f[8], mc_rot<8>(s), a0);
    a1 = fmaf(f[9], mc_rot<9>(s), a1);
    a2 = fmaf(f[10], mc_rot<10>(s), a2);
    a3 = fmaf(f[11], mc_rot<11>(s), a3);
    a0 = fmaf(f[12], mc_rot<12>(s), a0);
    a1 = fmaf(f[13], mc_rot<13>(s), a1);
    a2 = fmaf(f[14], mc_rot<14>(s), a2);
    a3 = fmaf(f[15], mc_rot<15>(s), a3);
    return (a0 + a1) + (a2 + a3);
}

__device__ __forceinline__ void mc_load16(float (&f)[16], const float *src) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 t = reinterpret_cast<const float4 *>(src)[q];
        f[4 * q] = t.x;
        f[4 * q + 1] = t.y;
        f[4 * q + 2] = t.z;
        f[4 * q + 3] = t.w;
    }
}

// The cascade part of a tile (phases (1) to (5)) on a channel pair whose
// input chunks are in X (LDS, [192][MC_XS]); leaves the output chunks in X.
// Every lane of the workgroup calls it.
static_assert(GROUPS == 2, "McCtx users select between the two groups");
struct McCtx {
    const McTab *mt;
    const CascTab *ct;
    int32_t S;
    uint64_t *rec[GROUPS];      // look-back records of tile 0 of each channel
    int64_t pos;                // tile position
    uint32_t epoch;
    uint32_t *hdr;
    const float *known[GROUPS]; // state entering tile 0 ([S][2]) or null
    float *ckpt[GROUPS];        // where this tile's entering state goes ([S][2]) or null
};

static __device__ void mc_cascade_tile(float *lds, const McCtx &m, int tid) {
    const int lane = tid & 63, w = tid >> 6;
    float *X = lds;
    const McTab *mt = m.mt;
    float aw[24];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const float4 t = reinterpret_cast<const float4 *>(mt->W[lane])[q];
        aw[4 * q] = t.x;
        aw[4 * q + 1] = t.y;
        aw[4 * q + 2] = t.z;
        aw[4 * q + 3] = t.w;
    }
    __syncthreads();

    // ---- (1) Y0 and U: wave w takes chunks 48 w .. 48 w + 47, three column
    //      blocks of 16; lane l feeds samples 8 (l >> 4) + t of chunk l & 15
    const int lq = lane >> 4, lc = lane & 15;
    mcf4 acc[3][3];
#pragma unroll
    for (int rb = 0; rb < 3; ++rb)
#pragma unroll
        for (int cb = 0; cb < 3; ++cb) acc[rb][cb] = mcf4{0.f, 0.f, 0.f, 0.f};
    {
        float bx[3][8];
#pragma unroll
        for (int cb = 0; cb < 3; ++cb) {
            const int K = 48 * w + 16 * cb + lc;
            const float4 *p = reinterpret_cast<const float4 *>(X + MC_XS * K + 8 * lq);
            const float4 b0 = p[0], b1 = p[1];
            bx[cb][0] = b0.x; bx[cb][1] = b0.y; bx[cb][2] = b0.z; bx[cb][3] = b0.w;
            bx[cb][4] = b1.x; bx[cb][5] = b1.y; bx[cb][6] = b1.z; bx[cb][7] = b1.w;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t)
#pragma unroll
            for (int rb = 0; rb < 3; ++rb)
#pragma unroll
                for (int cb = 0; cb < 3; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[8 * rb + t], bx[cb][t], acc[rb][cb], 0, 0, 0);
    }
    const int D = 2 * m.S, DD = D * D;
    float *U = lds;  // [192][MC_US] chunk states, over X
    float *Gs = lds + MC_G_OFF, *Es = lds + MC_E_OFF;
    float *cT = lds + MC_LB_OFF;
    __syncthreads();  // every wave's reads of X are done
#pragma unroll
    for (int cb = 0; cb < 3; ++cb) {
        const int K = 48 * w + 16 * cb + lc;
        *reinterpret_cast<mcf4 *>(U + MC_US * K + 4 * lq) = acc[2][cb];
    }
    for (int e = tid; e < 3 * DD; e += WG) {  // tile-transition powers for the look-back
        const int k = e / DD, i = (e % DD) / D, j = e % D;
        cT[e] = m.ct->T[k][i][j];
    }
    const int ri = lane & 15, sg = 4 * w + lq, K0 = MC_SEG * sg;  // segment sg: chunks K0 .. K0 + 11
    float fr[16];
    mc_load16(fr, mt->Fr[ri]);
    __syncthreads();

    // ---- (2) segment aggregates from a zero entering state
    {
        float sv = 0.f;
#pragma unroll
        for (int m = 0; m < MC_SEG; ++m) sv = mc_step(sv, fr, U[MC_US * (K0 + m) + ri]);
        Gs[16 * sg + ri] = sv;
    }
    __syncthreads();

    // ---- (3) per channel (waves 0 and 2): tile aggregate, look-back,
    //      segment-entering states
    if ((w & 1) == 0) {
        const int grp = w >> 1;
        float fs[16];
        mc_load16(fs, mt->Fsr[ri]);
        float *cM = cT + 3 * DD + grp * DD, *cE = cT + (3 + GROUPS) * DD + 32 * grp, *cP = cE + 16;
        float ev = 0.f;
#pragma unroll
        for (int j = 0; j < 8; ++j) ev = mc_step(ev, fs, Gs[16 * (8 * grp + j) + ri]);
        if (lane < 16) cE[ri] = ev;
        CascCtx cc;
        cc.lane = lane;
        cc.D = D;
        cc.depth = m.ct->depth;
        // (the per-group pointers selected, not indexed: a run-time index
        // into the context's arrays would move them to scratch memory)
        cc.rec = grp == 0 ? m.rec[0] : m.rec[1];
        cc.pos = m.pos;
        cc.epoch = m.epoch;
        cc.hdr = m.hdr;
        cc.known = grp == 0 ? m.known[0] : m.known[1];
        casc_lookback(cc, cT, cE, cP, cM);
        float *ck = grp == 0 ? m.ckpt[0] : m.ckpt[1];
        if (ck && lane < D) ck[lane] = cP[lane];
        ev = ri < D ? cP[ri] : 0.f;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (lane < 16) Es[16 * (8 * grp + j) + ri] = ev;
            ev = mc_step(ev, fs, Gs[16 * (8 * grp + j) + ri]);
        }
    }
    __syncthreads();

    // ---- (4) every chunk's entering state, in place of U
    {
        float sv = Es[16 * sg + ri];
#pragma unroll
        for (int m = 0; m < MC_SEG; ++m) {
            const int idx = MC_US * (K0 + m) + ri;
            const float u = U[idx];
            U[idx] = sv;
            sv = mc_step(sv, fr, u);
        }
    }
    __syncthreads();

    // ---- (5) Y = Y0 + G S (state component 4 (l >> 4) + k at step k)
    {
        float gt[8];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const float4 t = reinterpret_cast<const float4 *>(mt->Gt[lane])[q];
            gt[4 * q] = t.x;
            gt[4 * q + 1] = t.y;
            gt[4 * q + 2] = t.z;
            gt[4 * q + 3] = t.w;
        }
        mcf4 sv[3];
#pragma unroll
        for (int cb = 0; cb < 3; ++cb) sv[cb] = *reinterpret_cast<const mcf4 *>(U + MC_US * (48 * w + 16 * cb + lc) + 4 * lq);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < 3; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(gt[4 * rb + k], sv[cb][k], acc[rb][cb], 0, 0, 0);
    }
    __syncthreads();  // every wave's reads of S are done
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 3; ++cb) {
            const int K = 48 * w + 16 * cb + lc;
            *reinterpret_cast<mcf4 *>(X + MC_XS * K + 16 * rb + 4 * lq) = acc[rb][cb];
        }
    __syncthreads();

}

// Stages the tile of a channel pair into X: src[g] (null: the channel does
// not exist) holds rem samples from the tile's start (zeros past rem);
// vec: rows 16-byte aligned.
__device__ __forceinline__ void mc_stage_pair(float *X, const float *const (&src)[GROUPS], int64_t rem, bool vec,
                                              int tid) {
#pragma unroll
    for (int g = 0; g < GROUPS; ++g) {
        float *dst = X + g * MC_NCH * MC_XS;
        if (src[g] && vec && rem >= T) {
            float4 t4[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) t4[k] = reinterpret_cast<const float4 *>(src[g])[tid + WG * k];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int j = 4 * (tid + WG * k);
                *reinterpret_cast<float4 *>(dst + MC_XS * (j >> 5) + (j & 31)) = t4[k];
            }
        } else {
            for (int j = tid; j < T; j += WG) dst[MC_XS * (j >> 5) + (j & 31)] = (src[g] && j < rem) ? src[g][j] : 0.f;
        }
    }
}

// Writes the pair's output chunks from X: dst[g] (null: skip) receives rem
// samples (at most one tile).
__device__ __forceinline__ void mc_store_pair(const float *X, float *const (&dst)[GROUPS], int64_t rem, bool vec,
                                              int tid) {
#pragma unroll
    for (int g = 0; g < GROUPS; ++g) {
        if (!dst[g]) continue;
        const float *src = X + g * MC_NCH * MC_XS;
        if (vec && rem >= T) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int j = 4 * (tid + WG * k);
                reinterpret_cast<float4 *>(dst[g])[tid + WG * k] =
                    *reinterpret_cast<const float4 *>(src + MC_XS * (j >> 5) + (j & 31));
            }
        } else {
            for (int j = tid; j < T; j += WG)
                if (j < rem) dst[g][j] = src[MC_XS * (j >> 5) + (j & 31)];
        }
    }
}

}  // namespace tfx
