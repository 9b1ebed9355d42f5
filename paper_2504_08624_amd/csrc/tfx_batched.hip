// tfx_batched.hip -- a ragged batch of clips (each with its own channel
// count, length and SOS cascade) filtered by one kernel launch.
//
// The launch covers every (clip, tile, channel pair) of the batch: blocks are
// numbered clip by clip in a chosen clip order, tile-major within a clip, so a
// tile's predecessors in time always have lower block ids and the decoupled
// look-back of the chain kernel carries over unchanged.  A block finds its
// clip in the block map the prepare step leaves in the workspace (one read;
// a 64-way search over the descriptor table took two dependent rounds); every clip has its own
// section tables and look-back records.  The chunk length LC (and with it
// the tile length 128 LC) is a template parameter, chosen per batch by the
// autotuner among 16, 24 and 32.
#include <hip/hip_runtime.h>

#include "tfx_device.h"
#include "tfx_mc.h"

namespace tfx {

template <int LC, typename CT, class TB>
__device__ void batch_section(const TB &tb, float (&v)[LC], const CarryCtx &cc, double (*s_agg)[GWAVES][2],
                              double (*s_pre)[2], int buf) {
    const float b0 = tb.coef[0], b1 = tb.coef[1], b2 = tb.coef[2];
    const float a1 = tb.coef[3], a2 = tb.coef[4];
    float s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int r = 0; r < LC; ++r) {
        const float xv = v[r];
        const float yv = fmaf(b0, xv, s1);
        s1 = fmaf(b1, xv, fmaf(-a1, yv, s2));
        s2 = fmaf(b2, xv, -a2 * yv);
        v[r] = yv;
    }
    float z1, z2;
    carry<CT, false, TB>(tb, cc, s1, s2, z1, z2, s_agg, s_pre, buf);
#pragma unroll
    for (int r = 0; r < LC; ++r) {
        v[r] += z1;
        const float n1 = fmaf(-a1, z1, z2);
        z2 = -a2 * z1;
        z1 = n1;
    }
}

struct BatchArgs {
    const ClipDesc *desc;
    const int32_t *map;  // block id -> clip (written by the prepare step)
    int32_t nclips;
    const SecTab *tab;
    const CascTab *ctab;  // per clip (cascade-level variant)
    const McTab *mtab;    // per clip (matrix-core variant)
    uint64_t *recs;
    uint32_t *hdr;
};

// The block's clip (from the prepare step's block map) and the look-back
// epoch, written to LDS by thread 0 (the caller synchronises).
__device__ __forceinline__ void find_clip(const BatchArgs &a, int64_t id, int tid, int *s_clip, uint32_t *s_epoch) {
    if (tid == 0) {
        *s_clip = a.map[id];
        *s_epoch = load_epoch(a.hdr, HDR_EPOCH);
    }
}

// HIQ: the variant with the FP64 carry; both run, the one that does not match
// the batch's high-Q word advances the look-back epoch and exits.
// CASC: every clip's cascade (at most CASC_MAX sections, none needing FP64)
// in the three phases of the chain kernel's cascade-level form: the cascade
// over the tile from a zero state (tile aggregate), one look-back of the
// whole 2S-component state, the cascade again from the known state.
template <int LC, bool HIQ, bool CASC>
__global__ __launch_bounds__(WG) void batch_kernel(BatchArgs a) {
    typedef Chunk<LC> K;
    __shared__ __align__(16) float lds[GROUPS * K::STG];
    __shared__ double s_agg[2 * GROUPS][GWAVES][2];
    __shared__ double s_pre[2 * GROUPS][2];
    __shared__ uint32_t s_epoch;
    __shared__ int s_clip;
    // dynamic: fp32 tables (LDS_SECTIONS at a time; CASC: all of them without
    // their look-back powers, then the cascade look-back area)
    extern __shared__ __align__(16) unsigned char s_dyn[];
    SecLds *s_tab = reinterpret_cast<SecLds *>(s_dyn);
    SecLdsC *s_tabc = reinterpret_cast<SecLdsC *>(s_dyn);

    if ((a.hdr[HDR_HIQ] != 0u) != HIQ) {  // the other variant runs
        advance_epoch(a.hdr);
        return;
    }
    const int tid = threadIdx.x, lane = tid & 63, grp = tid / GL, gl = tid % GL, gw = gl >> 6;
    const int64_t id = blockIdx.x;
    find_clip(a, id, tid, &s_clip, &s_epoch);
    __syncthreads();
    const ClipDesc &d = a.desc[s_clip];
    const uint32_t epoch = s_epoch;
    const int64_t npairs = d.cpad / 2, local = id - d.blk0;
    const int64_t tile = local / npairs, pair = local % npairs;
    const int64_t ch = 2 * pair + grp;
    const bool valid = ch < d.C;
    const int64_t n0 = tile * K::T;
    float *stg = lds + grp * K::STG;
    float v[LC];
    if constexpr (CASC) {
        const int S = d.S, D = 2 * S, DD = D * D;
        // tables, then the cascade look-back area
        float *cr = reinterpret_cast<float *>(s_dyn + S * sizeof(SecLdsC));
        float *cT = cr, *cM = cr + 3 * DD + grp * DD, *cE = cr + (3 + GROUPS) * DD + 32 * grp, *cP = cE + 16;
        const CascTab &ct = a.ctab[s_clip];
        stage_tables(s_tabc, a.tab, (int)d.tab0, S, tid, WG);
        for (int e = tid; e < 3 * DD; e += WG) {
            const int k = e / DD, i = (e % DD) / D, j = e % D;
            cT[e] = ct.T[k][i][j];
        }
        stage_tile<LC>(stg, d.x + ch * d.ldx + n0, d.N - n0, valid, d.vec != 0, gl);
        __syncthreads();
        load_chunk<LC>(stg, gl, v);
        if (S > 0) {  // (no state otherwise: y = x; block-uniform)
            // (A) zero tile-entering state: the cascade's tile aggregate; the
            //     last section only needs its state
            float eA0 = 0.f, eA1 = 0.f;
            for (int s = 0; s < S; ++s) {
                float e0, e1, E0, E1;
                const int buf = (s & 1) * GROUPS + grp;
                if (s + 1 < S)
                    casc_section_a<LC, true>(s_tabc[s], v, lane, gw, s_agg, buf, e0, e1, E0, E1);
                else
                    casc_section_a<LC, false>(s_tabc[s], v, lane, gw, s_agg, buf, e0, e1, E0, E1);
                if (s == 0) {
                    eA0 = e0;
                    eA1 = e1;
                }
                if (gl == 0) {
                    cE[2 * s] = E0;
                    cE[2 * s + 1] = E1;
                }
            }
            // (B) one look-back of the cascade state (first wave of each group)
            if (gw == 0) {
                CascCtx cc;
                cc.lane = lane;
                cc.D = D;
                cc.depth = ct.depth;
                cc.rec = a.recs + (d.rec0 + ch * d.ntiles * S) * REC_WORDS;
                cc.pos = tile;
                cc.epoch = epoch;
                cc.hdr = a.hdr;
                cc.known = nullptr;
                casc_lookback(cc, cT, cE, cP, cM);
            }
            __syncthreads();
            // (C) every section from its known tile-entering state; section 0
            //     reuses phase A's carry (its input is unchanged)
            load_chunk<LC>(stg, gl, v);
            for (int s = 0; s < S; ++s) {
                const SecLdsC &tb = s_tabc[s];
                float c1, c2;
                if (s == 0) {
                    float e0 = eA0, e1 = eA1;
                    fold_prefix(tb, lane, gw, cP[0], cP[1], e0, e1);
                    section_from<LC>(tb.coef, v, e0, e1, -1, c1, c2);
                } else {
                    casc_section_c<LC, false>(tb, v, lane, gw, cP[2 * s], cP[2 * s + 1], s_agg,
                                              (s & 1) * GROUPS + grp, -1, c1, c2);
                }
            }
        }
    } else {
        stage_tables(s_tab, a.tab, (int)d.tab0, min(d.S, LDS_SECTIONS), tid, WG);
        stage_tile<LC>(stg, d.x + ch * d.ldx + n0, d.N - n0, valid, d.vec != 0, gl);
        __syncthreads();
        load_chunk<LC>(stg, gl, v);
        for (int s = 0; s < d.S; ++s) {
            if (s > 0 && s % LDS_SECTIONS == 0) {  // next block of tables
                __syncthreads();
                stage_tables(s_tab, a.tab, (int)d.tab0 + s, min(d.S - s, LDS_SECTIONS), tid, WG);
                __syncthreads();
            }
            const SecLds &tb = s_tab[s % LDS_SECTIONS];
            CarryCtx cc;
            cc.lane = lane;
            cc.gw = gw;
            cc.grp = grp;
            cc.lookback = true;
            cc.pos = tile;
            cc.recs = a.recs;
            cc.rec0 = d.rec0 + ch * d.ntiles * d.S + s;
            cc.rstride = d.S;
            cc.epoch = epoch;
            cc.hdr = a.hdr;
            cc.known0 = cc.known1 = 0.0;
            cc.prefix_out = nullptr;
            const int buf = (s & 1) * GROUPS + grp;
            if (HIQ && tb.hiq)
                batch_section<LC, double>(a.tab[d.tab0 + s], v, cc, s_agg, s_pre, buf);
            else
                batch_section<LC, float>(tb, v, cc, s_agg, s_pre, buf);
        }
    }
    __syncthreads();
    store_chunk<LC>(stg, gl, v);
    __syncthreads();
    if (valid) store_tile<LC>(d.y + ch * d.ldy + n0, stg, d.N - n0, d.vec != 0, gl);
}

// Matrix-core form (chunk length 24, i.e. 3072-sample tiles, every cascade
// of at most CASC_MAX sections without FP64-carry sections): each block
// stages its tile of a channel pair and runs the cascade of its clip on the
// matrix cores (mc_cascade_tile, with the clip's own tables); the look-back
// records are the clip's, as in the cascade-level form.
__global__ __launch_bounds__(WG, 4) void batch_mc_kernel(BatchArgs a) {
    __shared__ __align__(16) float lds[MC_X_FLOATS];
    __shared__ uint32_t s_epoch;
    __shared__ int s_clip;
    if (a.hdr[HDR_HIQ] != 0u) {  // the FP64-carry variant runs
        advance_epoch(a.hdr);
        return;
    }
    const int tid = threadIdx.x;
    const int64_t id = blockIdx.x;
    find_clip(a, id, tid, &s_clip, &s_epoch);
    __syncthreads();
    const ClipDesc &d = a.desc[s_clip];
    const int64_t npairs = d.cpad / 2, local = id - d.blk0;
    const int64_t tile = local / npairs, pair = local % npairs;
    const int64_t n0 = tile * T, rem = d.N - n0;
    const float *src[GROUPS];
#pragma unroll
    for (int g = 0; g < GROUPS; ++g) src[g] = 2 * pair + g < d.C ? d.x + (2 * pair + g) * d.ldx + n0 : nullptr;
    mc_stage_pair(lds, src, rem, d.vec != 0, tid);
    if (d.S > 0) {  // block-uniform
        McCtx m;
        m.mt = &a.mtab[s_clip];
        m.ct = &a.ctab[s_clip];
        m.S = d.S;
        m.pos = tile;
        m.epoch = s_epoch;
        m.hdr = a.hdr;
#pragma unroll
        for (int g = 0; g < GROUPS; ++g) {
            m.rec[g] = a.recs + (d.rec0 + (2 * pair + g) * d.ntiles * d.S) * REC_WORDS;
            m.known[g] = nullptr;
            m.ckpt[g] = nullptr;
        }
        mc_cascade_tile(lds, m, tid);
    } else {
        __syncthreads();
    }
    // (the output pointers formed here, not held across the cascade)
    float *dst[GROUPS];
#pragma unroll
    for (int g = 0; g < GROUPS; ++g) dst[g] = 2 * pair + g < d.C ? d.y + (2 * pair + g) * d.ldy + n0 : nullptr;
    mc_store_pair(lds, dst, rem, d.vec != 0, tid);
}

// The descriptor table reaches the device through kernel arguments, 32
// clips per launch: no host buffer has to outlive the call.
constexpr int DESC_CHUNK = 32;
struct DescChunk {
    ClipDesc d[DESC_CHUNK];
    int32_t first, n;
};
__global__ void desc_write_kernel(ClipDesc *dst, DescChunk c) {
    const int i = threadIdx.x;
    if (i < c.n) dst[c.first + i] = c.d[i];
}

hipError_t upload_descriptors(const ClipDesc *desc, int32_t n, const BatchLayout &lay, void *ws, hipStream_t st) {
    ClipDesc *dst = reinterpret_cast<ClipDesc *>(static_cast<char *>(ws) + lay.desc);
    for (int32_t f = 0; f < n; f += DESC_CHUNK) {
        DescChunk c{};
        c.first = f;
        c.n = n - f < DESC_CHUNK ? n - f : DESC_CHUNK;
        for (int i = 0; i < c.n; ++i) c.d[i] = desc[f + i];
        hipLaunchKernelGGL(desc_write_kernel, dim3(1), dim3(DESC_CHUNK), 0, st, dst, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------------- host

static size_t al256b(size_t b) { return (b + 255) & ~size_t(255); }

BatchLayout batch_plan(const ClipIn *clips, int32_t n, int lc, int order, ClipDesc *desc) {
    BatchLayout lay{};
    const int64_t T_ = (int64_t)GL * lc;
    // processing order: as given, or by tile count, longest first (stable)
    int32_t *ord = new int32_t[n > 0 ? n : 1];
    for (int i = 0; i < n; ++i) ord[i] = i;
    if (order == 1) {
        for (int i = 1; i < n; ++i) {  // insertion sort, stable
            const int32_t k = ord[i];
            const int64_t tk = (clips[k].N + T_ - 1) / T_;
            int j = i - 1;
            while (j >= 0 && (clips[ord[j]].N + T_ - 1) / T_ < tk) {
                ord[j + 1] = ord[j];
                --j;
            }
            ord[j + 1] = k;
        }
    }
    int64_t blk = 0, tab = 0, rec = 0;
    for (int j = 0; j < n; ++j) {
        const ClipIn &c = clips[ord[j]];
        ClipDesc d{};
        d.x = c.x;
        d.y = c.y;
        d.sos = c.sos;
        d.C = c.C;
        d.N = c.N;
        d.ldx = c.ldx;
        d.ldy = c.ldy;
        d.S = c.S;
        d.ntiles = (c.N + T_ - 1) / T_;
        d.cpad = c.C + (c.C & 1);
        d.blk0 = blk;
        d.tab0 = tab;
        d.rec0 = rec;
        d.vec = ((reinterpret_cast<uintptr_t>(c.x) | reinterpret_cast<uintptr_t>(c.y)) % 16 == 0 && c.ldx % 4 == 0 &&
                 c.ldy % 4 == 0) ? 1 : 0;
        blk += d.cpad / 2 * d.ntiles;
        tab += c.S;
        if (c.S > lay.smax) lay.smax = c.S;
        rec += d.cpad * d.ntiles * c.S;
        if (desc) desc[j] = d;
    }
    delete[] ord;
    lay.nblocks = blk;
    lay.nsec = tab;
    lay.nrec = rec;
    size_t off = 0;
    lay.hdr = off;
    off += 256;
    lay.desc = off;
    off += al256b(sizeof(ClipDesc) * (size_t)(n > 0 ? n : 1));
    lay.map = off;
    off += al256b(sizeof(int32_t) * (size_t)(blk > 0 ? blk : 1));
    lay.tab = off;
    off += al256b(sizeof(SecTab) * (size_t)tab);
    lay.recs = off;
    off += al256b((size_t)rec * REC_WORDS * sizeof(uint64_t));
    lay.casc = off;
    lay.casc_on = lay.smax > 0 && lay.smax <= CASC_MAX;
    if (lay.casc_on) off += al256b(sizeof(CascTab) * (size_t)n);
    lay.mc = off;
    // 3072-sample tiles and a longest cascade of MC_MIN_SECTIONS or more: the
    // matrix-core form (whose cost hardly depends on the section count)
    lay.mc_on = lay.casc_on && lc == L && lay.smax >= MC_MIN_SECTIONS;
    if (lay.mc_on) off += al256b(sizeof(McTab) * (size_t)n);
    lay.total = off;
    return lay;
}

hipError_t launch_batch_run(const BatchLayout &lay, int lc, int32_t nclips, void *ws, hipStream_t st) {
    if (lay.nblocks == 0) return hipSuccess;
    char *w = static_cast<char *>(ws);
    BatchArgs a;
    a.desc = reinterpret_cast<const ClipDesc *>(w + lay.desc);
    a.map = reinterpret_cast<const int32_t *>(w + lay.map);
    a.nclips = nclips;
    a.tab = reinterpret_cast<const SecTab *>(w + lay.tab);
    a.recs = reinterpret_cast<uint64_t *>(w + lay.recs);
    a.hdr = reinterpret_cast<uint32_t *>(w + lay.hdr);
    a.ctab = reinterpret_cast<const CascTab *>(w + lay.casc);
    a.mtab = reinterpret_cast<const McTab *>(w + lay.mc);
    const dim3 grid((unsigned)lay.nblocks), block(WG);
    const size_t dyn = sizeof(SecLds) * (size_t)(lay.smax < LDS_SECTIONS ? lay.smax : LDS_SECTIONS);
    const size_t dync = sizeof(SecLdsC) * (size_t)lay.smax + sizeof(float) * (size_t)casc_floats(2 * lay.smax);
    const bool cs = lay.casc_on;
    hipError_t e = hipSuccess;
    switch (lc) {
        case 16:
            if (cs) hipLaunchKernelGGL((batch_kernel<16, false, true>), grid, block, dync, st, a);
            else hipLaunchKernelGGL((batch_kernel<16, false, false>), grid, block, dyn, st, a);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL((batch_kernel<16, true, false>), grid, block, dyn, st, a);
            break;
        case 32:
            if (cs) hipLaunchKernelGGL((batch_kernel<32, false, true>), grid, block, dync, st, a);
            else hipLaunchKernelGGL((batch_kernel<32, false, false>), grid, block, dyn, st, a);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL((batch_kernel<32, true, false>), grid, block, dyn, st, a);
            break;
        default:
            if (lay.mc_on) hipLaunchKernelGGL(batch_mc_kernel, grid, block, 0, st, a);
            else if (cs) hipLaunchKernelGGL((batch_kernel<24, false, true>), grid, block, dync, st, a);
            else hipLaunchKernelGGL((batch_kernel<24, false, false>), grid, block, dyn, st, a);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL((batch_kernel<24, true, false>), grid, block, dyn, st, a);
            break;
    }
    e = hipGetLastError();
    return e;
}

}  // namespace tfx
