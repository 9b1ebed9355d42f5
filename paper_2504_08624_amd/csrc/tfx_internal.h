// Internal declarations shared by the kernel translation units and the C ABI.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>
#include <math.h>

#include "tfx.h"

namespace tfx {

// ---- tiling ------------------------------------------------------------------
// A channel group of GL = 128 lanes owns one tile of T = GL * L consecutive
// samples of one channel; lane i of the group owns chunk [i*L, (i+1)*L) and keeps
// it in registers from the FIR output through every section to the store.  A
// workgroup holds GROUPS = 2 channel groups (an even/odd channel pair), which is
// also the pair the two-channel complex FFT filters together.
constexpr int L = 24;
constexpr int GL = 128;
constexpr int GWAVES = GL / 64;
constexpr int GROUPS = 2;
constexpr int WG = GL * GROUPS;
constexpr int T = GL * L;  // 3072

// ---- direct FIR ----------------------------------------------------------------
constexpr int KB = 16;          // taps per register block
constexpr int KBLK_MAX = 1024;  // taps staged per LDS pass

// ---- overlap-save FFT FIR --------------------------------------------------------
constexpr int NFFT = 4096;              // complex points, 16 x 16 x 16
constexpr int FFT_DISCARD = NFFT - T;   // 1024 leading outputs dropped per block
constexpr int FFT_PART = FFT_DISCARD + 1;  // taps per partition of a long filter
// The twiddles the FFT kernels keep in LDS: rows r < 16 hold W^(16 r k),
// rows 16 + c hold W^(c k) (W = e^{-2 pi i / 4096}, k < 16), each padded to
// TWL_S entries so that 16 lanes reading 16 different rows hit 64 banks.
constexpr int TWL_S = 18, TWL_ROWS = 32, TWL_ENTRIES = TWL_ROWS * TWL_S;
// The fp32 twiddle region of the workspace holds TWL alone (float2 entries).
constexpr int TWID_ENTRIES = TWL_ENTRIES;
__host__ __device__ constexpr int fft_parts(int M) { return (M + FFT_PART - 1) / FFT_PART; }
// One 16384-point FFT per block of 8192 outputs (tfx_fft16k.hip): filters of
// up to 8193 taps.
constexpr int FFT16_POINTS = 16384;
constexpr int FFT16_HOP = 8192;
constexpr int FFT16_MAX_TAPS = FFT16_HOP + 1;

constexpr int MAX_STAGES = 64;
constexpr int MAX_SECTIONS = 256;
constexpr int MAX_TAPS = 65536;
constexpr int BWD_MAX_SECTIONS = 16;  // adjoint: chunk states of every section stay in LDS

enum FirMode { FIR_NONE = 0, FIR_DIRECT = 1, FIR_FFT = 2, FIR_TOEPLITZ = 3, FIR_FFT16 = 4 };

// Per-section tables built on the device from the fp32 coefficients (in FP64,
// then rounded).  2x2 matrices are row-major {m00, m01, m10, m11}.
//   A    = [[-a1, 1], [-a2, 0]]     one-sample state transition (TDF-II)
//   Phi  = A^L                       chunk transition
//   Psi  = Phi^64                    wave transition
//   PhiT = Psi^GWAVES = A^T          tile transition
struct alignas(16) SecTab {
    float coef[5];
    int32_t hiq;             // 1: pole radius > 0.999 -> carry in FP64
    int32_t depth;           // look-back depth d: PhiT^d <= 2^-60, older tiles drop out (0 = none)
    int32_t pad;
    float fold[64][4];       // Phi^k, k = 0..63
    float psi[GWAVES][4];    // Psi^w, w < GWAVES
    float lb[9][4];          // PhiT^(2^j), j = 0..8
    double fold_d[64][4];
    double psi_d[GWAVES][4];
    double lb_d[9][4];
};

// The fp32 part of a SecTab (its leading members, same layout): what a
// workgroup copies into LDS for the sections it carries in fp32.
struct alignas(16) SecLds {
    float coef[5];
    int32_t hiq;
    int32_t depth;
    int32_t pad;
    float fold[64][4];
    float psi[GWAVES][4];
    float lb[9][4];
};
static_assert(offsetof(SecTab, lb) == offsetof(SecLds, lb), "SecLds must be the leading part of SecTab");
static_assert(sizeof(SecLds) <= offsetof(SecTab, fold_d), "SecLds must be the leading part of SecTab");
// The part of SecLds the cascade-level path reads (no look-back powers).
struct alignas(16) SecLdsC {
    float coef[5];
    int32_t hiq;
    int32_t depth;
    int32_t pad;
    float fold[64][4];
    float psi[GWAVES][4];
};
static_assert(offsetof(SecTab, psi) == offsetof(SecLdsC, psi), "SecLdsC must be the leading part of SecTab");
static_assert(sizeof(SecLdsC) % 16 == 0, "SecLdsC is copied in 16-byte pieces");
constexpr int LDS_SECTIONS = 32;  // sections staged in LDS at a time
constexpr int REC_WORDS = 4;      // 64-bit look-back words per (channel, tile, section)

// Cascades of up to CASC_MAX sections (without FP64-carry sections) carry
// their whole 2S-component state across tiles in one look-back per tile.
//
// Look-back depth: when every entry of the tile transition's d-th power is
// at most 2^-60 (about 1e-18), a tile d or more tiles back changes the
// state entering this tile by less than 2^-60 of its own state: 10^10 times
// below one fp32 rounding.  Such tiles are left out of the look-back, so
// for fast-decaying filters a tile needs only its d nearest predecessors'
// aggregates and never waits for a chain of inclusive prefixes.
constexpr double DEPTH_EPS = 8.673617379884035e-19;  // 2^-60
// Powers of the cascade's tile transition A_c^3072 (state order: section s
// at components 2s, 2s+1), zero-padded to 16 x 16.
constexpr int CASC_MAX = 8;
// LDS floats of a cascade look-back area for D = 2S components: T (3 D x D),
// one window weight per channel group (D x D), E and P per group (16 each).
__host__ __device__ constexpr int casc_floats(int D) { return (3 + GROUPS) * D * D + 2 * GROUPS * 16; }
struct alignas(16) CascTab {
    int32_t depth;       // look-back depth d <= 64 with max |Phi_T^d| <= 2^-60 (0 = none found)
    int32_t pad[3];
    float T[3][16][16];  // Phi_T, Phi_T^2, Phi_T^4
};
// Zero-input response of a cascade (chain path): with F the per-sample
// transition of the cascade state (D = 2S components) and c the row that
// maps the state to the cascade output under zero input, G[r] = c F^r.  The
// output of a tile is its zero-entering-state response plus
// G[r] . (F^(L k) P) at sample r of chunk k, P being the state entering the
// tile.  With k = 16 a + b, F^(L k) = F^(L b) F^(16 L a): Mb[i][j][b] =
// (F^(L b))[i][j] (b < 16) and MaT[a][j][i] = (F^(16 L a))[i][j] (a < 8),
// both with the lane's index (b, i) innermost: the kernel copies the rows
// j < 2S of both into LDS as they are.
constexpr int ZIR_B = 16, ZIR_A = GL / ZIR_B;
struct alignas(16) CascZir {
    float G[L][16];
    float Mb[16][16][ZIR_B];
    float MaT[ZIR_A][16][16];
};

// Matrix-core form of a cascade of up to CASC_MAX sections (chain path).
// With chunks of MC_LC = 32 samples, F the cascade's one-sample transition
// (D = 2S components), b its input column, c its output row and d the
// product of the b0s, a chunk with input x and entering state s gives
//     y  = Tc x + G s          Tc[r][m] = h[r - m] (h[0] = d, h[n] = c F^(n-1) b)
//     s' = Fc s + H x          G[r] = c F^r, H[:, m] = F^(31 - m) b, Fc = F^32.
// W stacks Tc (rows 0..31) over H (rows 32..47) as the A operand of the
// 16 x 16 x 4 fp32 matrix instruction, per lane: W[l][8 rb + t] is row
// 16 rb + (l & 15), column 8 (l >> 4) + t.  Gt[l][4 rb + k] is G's row
// 16 rb + (l & 15), column 4 (l >> 4) + k.  Fr[i][d] / Fsr[i][d] are row i
// of Fc / Fs = Fc^12 at the column the DPP rotation by d brings to lane i
// of a 16-lane row (mc_src).
// The matrix-core form runs cascades of MC_MIN_SECTIONS .. CASC_MAX sections:
// its cost hardly depends on the section count, while the cascade-level form
// with zero-input-response tables (up to ZIR_MAX sections) is faster for
// short cascades (measured on 8 x 5.76 M: equal at 6 sections, 17-25 %
// slower at 8).
constexpr int ZIR_MAX = 6;
constexpr int MC_MIN_SECTIONS = ZIR_MAX + 1;
constexpr int MC_LC = 32;            // samples per chunk
constexpr int MC_NCH = T / MC_LC;    // chunks per channel tile (96)
constexpr int MC_SEG = 12;           // chunks per recurrence segment
// lane whose value a row rotation by d (DPP row_ror:d) brings to lane i of
// a 16-lane row
__host__ __device__ constexpr int mc_src(int i, int d) { return (i - d) & 15; }
struct alignas(16) McTab {
    float W[64][24];
    float Gt[64][8];
    float Fr[16][16];
    float Fsr[16][16];
};

// Header words of a workspace: look-back error bit, look-back epoch, and
// whether any section needs the FP64 carry (the filter kernels come in two
// variants; the one that does not match this word exits at once).
enum { HDR_ERROR = 1, HDR_EPOCH = 2, HDR_HIQ = 3 };

// Pole radius of 1 + a1 z^-1 + a2 z^-2 above 0.999: the section's carry
// runs in FP64.
__host__ __device__ inline bool section_hiq(double a1, double a2) {
    const double disc = a1 * a1 - 4.0 * a2;
    double r;
    if (disc < 0.0) {
        r = sqrt(a2);
    } else {
        const double sq = sqrt(disc);
        const double r1 = fabs(0.5 * (-a1 + sq)), r2 = fabs(0.5 * (-a1 - sq));
        r = r1 > r2 ? r1 : r2;
    }
    return r > 0.999;
}

struct StageList {
    const float *ptr[MAX_STAGES];
    int32_t len[MAX_STAGES];
    int32_t n;
};

struct ChainPlan {
    const float *x;
    float *y;
    int64_t C, N, ldx, ldy;
    int32_t S;        // total sections
    int32_t fir_mode; // FirMode of the merged FIR
    int32_t cmp;      // tfx_compute of the FIR contraction (Toeplitz path)
    StageList sos;    // SOS stages in order (device pointers)
    StageList firs;   // FIR stages in order (merged when more than one)
    const float *state_in;
    float *state_out;
    float *ckpt;
    const float *hist_in;   // streaming: FIR inputs before the block, [C][M - 1] (null = zeros)
    float *hist_out;        // streaming: receives the last M - 1 inputs up to the block's end
    int64_t n_layout;       // block length the workspace layout was made for (0 = N)
    void *ws;
    size_t ws_bytes;
    hipStream_t stream;
};

// Workspace layout of a chain/SOS/FIR call.
struct WsLayout {
    size_t hdr, tab, recs, casc, zir, mc, taps, merge, twid, hspec, tw64, ttab, f16, total;
    int64_t ntiles, cpad;
};
WsLayout ws_layout(int64_t C, int64_t N, int32_t S, int32_t M_merged, int32_t n_fir, int32_t fir_mode);

// Sets the calling thread's tfx_last_error message and returns s (for entry
// points defined outside tfx_api.cpp).
tfx_status set_error(tfx_status s, const char *msg);

// The FIR form tfx_fir_autotune recorded for an fp32 call of this shape
// (false when there is none).
bool tuned_fir_algo(int32_t M, int64_t C, int64_t N, int32_t *algo, int32_t *cmp);

// Header words of a workspace (at least 256 bytes, else nothing) for a call
// that builds no tables.
hipError_t launch_header_init(void *ws, size_t ws_bytes, hipStream_t st);
// Status word of a workspace into *flags (tfx_workspace_status).
hipError_t launch_ws_status(void *ws, uint32_t *flags, int32_t clear, hipStream_t st);

// Tables + workspace initialisation (once per workspace and coefficients).
hipError_t launch_prepare(const ChainPlan &p);
// The filtering itself; may be repeated on a prepared workspace.
hipError_t launch_run(const ChainPlan &p);
// log2 of the block-order window K per XCD for the current device and a
// grid of npairs channel pairs per tile (0: block ids in order); see xcd_order
uint32_t xcd_window(int64_t npairs);

// Merged tap count of the FIR stages (each extra stage adds len - 1).
int32_t merged_taps(const StageList &f);
// The kernels of the prepare step into the workspace described by lay.
hipError_t launch_tables(const ChainPlan &p, const WsLayout &lay, const float *h, int32_t M);
// FIR part of a prepared chain alone over (in -> out): convolution with the
// merged taps, or correlation with them (the FIR adjoint) when correlate.
hipError_t launch_fir_pass(const ChainPlan &p, const WsLayout &lay, const float *in, int64_t ldin, float *out,
                           int64_t ldout, bool correlate);

// ---- matrix-core block-Toeplitz FIR (tfx_toeplitz.hip) --------------------------
int32_t toeplitz_lags(int32_t M);
size_t toeplitz_table_bytes(int32_t M, int32_t cmp);
hipError_t launch_toeplitz_prepare(const float *h, int32_t M, int32_t cmp, void *tab, hipStream_t st);
hipError_t launch_toeplitz(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy, int32_t M,
                           int32_t cmp, const void *tab, hipStream_t st, const float *hist = nullptr);

// ---- overlap-save FIR with 16384-point FFTs (tfx_fft16k.hip) --------------------
// Twiddle tables and tap spectrum of the 16384-point path.
size_t fft16k_table_bytes();
hipError_t launch_fft16k_prepare(const float *h, int32_t M, void *tab, hipStream_t st);
// FIR (or, with correlate, its adjoint correlation) x -> y; hist: streaming
// history [C][M - 1] before the block (convolution only), or null.
hipError_t launch_fft16k(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy, int32_t M,
                         const void *tab, bool correlate, const float *hist, hipStream_t st);

// ---- batched ragged clips (tfx_batched.hip) -------------------------------------
// Device descriptor of one clip, in processing order.  Blocks of the single
// launch are numbered clip by clip (blk0 = the clip's first block); within a
// clip they are tile-major over channel pairs, as in the chain kernel.
struct alignas(16) ClipDesc {
    const float *x;
    float *y;
    const float *sos;
    int64_t C, N, ldx, ldy;
    int64_t blk0, tab0, rec0;
    int64_t ntiles, cpad;
    int32_t S, vec;
};

struct BatchLayout {
    size_t hdr, desc, map, tab, recs, casc, mc, total;
    int64_t nblocks, nsec, nrec;
    int32_t smax;  // longest cascade of the batch
    bool casc_on;  // every cascade has at most CASC_MAX sections: one CascTab per clip
    bool mc_on;    // and the chunk length is L and smax >= MC_MIN_SECTIONS: one McTab per clip (matrix-core form)
};

// host-side clip record (mirrors the public tfx_clip)
struct ClipIn {
    const float *x;
    float *y;
    int64_t C, N, ldx, ldy;
    const float *sos;
    int32_t S;
};

// chunk lengths of the batched kernel
constexpr int BATCH_CHUNKS[3] = {16, 24, 32};

// Fills desc (processing order) and returns the layout for chunk length lc
// and clip order (0: as given, 1: longest first).
BatchLayout batch_plan(const ClipIn *clips, int32_t n, int lc, int order, ClipDesc *desc);
hipError_t upload_descriptors(const ClipDesc *desc, int32_t n, const BatchLayout &lay, void *ws, hipStream_t st);
hipError_t launch_batch_prepare(const BatchLayout &lay, int lc, int32_t nclips, void *ws, hipStream_t st);
hipError_t launch_batch_run(const BatchLayout &lay, int lc, int32_t nclips, void *ws, hipStream_t st);

// ---- short-time Fourier transform -------------------------------------------
struct StftPlan {
    int log2n;              // n_fft = 2^log2n, 4 .. 12
    int32_t hop, win_length, center, normalized;
    const float *win;       // [win_length] or NULL (ones)
    int64_t C, T;           // channels, frames per channel
    // forward
    const float *x;
    int64_t ldx, nx;
    float *spec;            // [C][T][n_fft/2+1] complex (re, im)
    // inverse
    const float *spec_in;
    float *y;
    int64_t length, ldy;
    hipStream_t stream;
};

hipError_t launch_stft(const StftPlan &sp);
hipError_t launch_istft(const StftPlan &sp);

// ---- adjoint -------------------------------------------------------------------
struct GradList {
    float *ptr[MAX_STAGES];
    int32_t len[MAX_STAGES];
    int32_t n;
};

struct BwdPlan {
    ChainPlan fwd;      // stages, x (ldx), C, N, ckpt, ws, stream of the forward
    const float *gy;    // gradient of the chain output
    float *gx;          // gradient of the chain input
    int64_t ldg, ldgx;
    GradList gsos;      // per SOS stage (ptr may be null), in stage order
    GradList gfir;      // per FIR stage (ptr may be null), in stage order
};

// Backward workspace: the forward layout, then the adjoint's buffers.
struct BwdLayout {
    WsLayout fwd;
    size_t part_sos, sos_sum, fbuf, gfbuf, part_gh, gh1, gH, obuf, twid, tw64, spec, total;
    int64_t nlag;
    // single-partition FFT FIR: tap-gradient spectra summed per workgroup
    // (spec_wg workgroups, spec_split of them per first-level sum)
    bool spec_path;
    int64_t spec_wg, spec_nsplit;
};
BwdLayout bwd_layout(int64_t C, int64_t N, int32_t S, int32_t M_merged, int32_t n_fir, int32_t fir_mode);
hipError_t launch_backward(const BwdPlan &p);

}  // namespace tfx
