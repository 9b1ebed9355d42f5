// Internal declarations shared by the kernel translation unit and the C ABI.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace tfx {

// ---- IIR tiling -------------------------------------------------------------
// A workgroup of WG lanes owns one tile of T = WG * L consecutive samples of one
// channel; lane i owns the chunk [i*L, (i+1)*L) of the tile and keeps it in
// registers for the whole chain (FIR output -> every section -> store).
constexpr int WG = 256;
constexpr int WAVES = WG / 64;
constexpr int L = 32;
constexpr int T = WG * L;

// ---- direct FIR tiling -----------------------------------------------------
constexpr int KB = 16;          // taps per register block
constexpr int KBLK_MAX = 1024;  // taps staged per LDS pass

constexpr int MAX_STAGES = 64;
constexpr int MAX_SECTIONS = 256;
constexpr int MAX_TAPS = 65536;

// Per-section tables built on the device from the fp32 coefficients (in FP64,
// then rounded).  2x2 matrices are row-major {m00, m01, m10, m11}.
//   A    = [[-a1, 1], [-a2, 0]]     one-sample state transition (TDF-II)
//   Phi  = A^L                       chunk transition
//   Psi  = Phi^64                    wave transition
//   PhiT = Psi^WAVES = A^T           tile transition
struct alignas(16) SecTab {
    float coef[5];
    int32_t hiq;             // 1: pole radius > 0.999 -> carry in FP64
    int32_t pad[2];
    float g[L][2];           // first row of A^t (zero-input response), t < L
    float fold[64][4];       // Phi^k, k = 0..63
    float psi[WAVES][4];     // Psi^w, w = 0..WAVES-1
    float lb[7][4];          // PhiT^(2^j), j = 0..5, and PhiT^64
    float apow[L][4];        // A^(t+1), t < L
    double fold_d[64][4];
    double psi_d[WAVES][4];
    double lb_d[7][4];
};

struct StageList {
    const float *ptr[MAX_STAGES];
    int32_t len[MAX_STAGES];
    int32_t n;
};

struct ChainPlan {
    const float *x;
    float *y;
    int64_t C, N, ldx, ldy;
    const float *h;   // merged taps (device), nullptr if no FIR
    int32_t M;
    int32_t S;        // total sections
    StageList sos;    // SOS stages in order (device pointers)
    StageList firs;   // FIR stages in order (merged when more than one)
    const float *state_in;
    float *state_out;
    float *ckpt;
    void *ws;
    size_t ws_bytes;
    hipStream_t stream;
};

// Workspace layout of a chain/SOS call.
struct WsLayout {
    size_t hdr, tab, flags, recs, taps, merge, total;
    int64_t ntiles;
};
WsLayout ws_layout(int64_t C, int64_t N, int32_t S, int32_t M_merged, int32_t n_fir);

// Tables + workspace initialisation (once per workspace and coefficients).
hipError_t launch_prepare(const ChainPlan &p);
// The filtering itself; may be repeated on a prepared workspace.
hipError_t launch_run(const ChainPlan &p);

}  // namespace tfx
