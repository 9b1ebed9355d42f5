// tfx_api.cpp -- the C ABI of libtfx: argument validation, status codes,
// workspace sizing and dispatch to the HIP kernels.  Everything here runs on
// the host; nothing is allocated and nothing synchronises.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "tfx.h"
#include "tfx_internal.h"

namespace {

thread_local std::string g_last_error;

tfx_status fail(tfx_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

tfx_status ok() {
    g_last_error.clear();
    return TFX_OK;
}

tfx_status hip_fail(hipError_t e, const char *where) {
    return fail(TFX_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + bbytes && pb < pa + abytes;
}

size_t span_bytes(int64_t C, int64_t N, int64_t ld) {
    if (C <= 0 || N <= 0) return 0;
    return (size_t)((C - 1) * ld + N) * sizeof(float);
}

tfx_status check_signal(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy) {
    if (C < 1) return fail(TFX_E_INVALID_ARG, "C must be >= 1 (got %lld)", (long long)C);
    if (N < 0 || N >= (int64_t(1) << 40)) return fail(TFX_E_INVALID_ARG, "N out of range (got %lld)", (long long)N);
    if (ldx < N || ldy < N) return fail(TFX_E_INVALID_ARG, "row strides must be >= N (ldx %lld, ldy %lld, N %lld)",
                                        (long long)ldx, (long long)ldy, (long long)N);
    if (N > 0 && (!x || !y)) return fail(TFX_E_INVALID_ARG, "x and y must be non-null");
    const int64_t ntiles = (N + tfx::T - 1) / tfx::T;
    if (C * ntiles >= (int64_t(1) << 31)) return fail(TFX_E_UNSUPPORTED, "C * ceil(N/%d) too large", tfx::T);
    if (N > 0 && overlaps(x, span_bytes(C, N, ldx), y, span_bytes(C, N, ldy)))
        return fail(TFX_E_ALIAS, "output overlaps the input");
    return TFX_OK;
}

tfx_status check_ws(void *ws, size_t ws_bytes, size_t need) {
    if (need == 0) return TFX_OK;
    if (!ws) return fail(TFX_E_WORKSPACE, "workspace of %zu bytes required, got NULL", need);
    if (ws_bytes < need) return fail(TFX_E_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(TFX_E_WORKSPACE, "workspace must be 256-byte aligned");
    return TFX_OK;
}

// Default fp32 FIR path by tap count: direct up to 48 taps, one 4096-point
// FFT per 3072-sample block up to 1025, one 16384-point FFT per 8192-sample
// block up to 8193, partitioned 4096-point FFTs beyond.
int32_t auto_fir_mode(int32_t M) {
    if (M <= 48) return tfx::FIR_DIRECT;
    if (M > tfx::FFT_PART && M <= tfx::FFT16_MAX_TAPS) return tfx::FIR_FFT16;
    return tfx::FIR_FFT;
}

// Validates the FIR request and picks the kernel path (*mode).  With
// `tuned` (FIR-only calls of shape C x N), an automatic fp32 choice takes the
// form tfx_fir_autotune recorded for this shape, if any.
tfx_status check_fir_mode(int32_t M, tfx_compute cmp, tfx_fir_algo algo, int32_t *mode, int64_t C = 0,
                          int64_t N = 0, bool tuned = false) {
    if (tuned && algo == TFX_FIR_AUTO && cmp == TFX_COMPUTE_F32 && M >= 1 && M <= tfx::MAX_TAPS) {
        int32_t ta = 0, tc = 0;
        if (tfx::tuned_fir_algo(M, C, N, &ta, &tc) && tc == TFX_COMPUTE_F32) algo = (tfx_fir_algo)ta;
    }
    if (M < 1 || M > tfx::MAX_TAPS) return fail(TFX_E_INVALID_ARG, "tap count M must be in [1, %d] (got %d)", tfx::MAX_TAPS, M);
    if (cmp < TFX_COMPUTE_F32 || cmp > TFX_COMPUTE_BF16X3) return fail(TFX_E_INVALID_ARG, "unknown compute mode %d", (int)cmp);
    if (algo < TFX_FIR_AUTO || algo > TFX_FIR_FFT16K) return fail(TFX_E_INVALID_ARG, "unknown FIR algorithm %d", (int)algo);
    if (cmp != TFX_COMPUTE_F32) {  // low-precision operands: only the matrix-core path
        if (algo == TFX_FIR_DIRECT || algo == TFX_FIR_FFT || algo == TFX_FIR_FFT16K)
            return fail(TFX_E_UNSUPPORTED, "the direct and FFT paths compute in fp32 only");
        *mode = tfx::FIR_TOEPLITZ;
        return TFX_OK;
    }
    if (algo == TFX_FIR_TOEPLITZ) return fail(TFX_E_UNSUPPORTED, "the Toeplitz path needs a bf16/fp16 compute mode");
    if (algo == TFX_FIR_FFT16K && M > tfx::FFT16_MAX_TAPS)
        return fail(TFX_E_UNSUPPORTED, "the 16384-point FFT path takes at most %d taps (got %d)", tfx::FFT16_MAX_TAPS, M);
    if (algo == TFX_FIR_DIRECT) *mode = tfx::FIR_DIRECT;
    else if (algo == TFX_FIR_FFT) *mode = tfx::FIR_FFT;
    else if (algo == TFX_FIR_FFT16K) *mode = tfx::FIR_FFT16;
    else *mode = auto_fir_mode(M);
    return TFX_OK;
}

struct Gathered {
    tfx::StageList firs{}, sos{};
    int32_t S = 0, Mtot = 0;
};

tfx_status gather(const tfx_stage *stages, int32_t nstages, Gathered &g) {
    if (nstages < 0 || nstages > tfx::MAX_STAGES)
        return fail(TFX_E_INVALID_ARG, "nstages must be in [0, %d]", tfx::MAX_STAGES);
    if (nstages > 0 && !stages) return fail(TFX_E_INVALID_ARG, "stages is NULL");
    for (int i = 0; i < nstages; ++i) {
        const tfx_stage &st = stages[i];
        if (!st.coef) return fail(TFX_E_INVALID_ARG, "stage %d has NULL coefficients", i);
        if (st.kind == TFX_STAGE_FIR) {
            if (st.len < 1 || st.len > tfx::MAX_TAPS) return fail(TFX_E_INVALID_ARG, "stage %d: bad tap count %d", i, st.len);
            g.firs.ptr[g.firs.n] = st.coef;
            g.firs.len[g.firs.n] = st.len;
            g.Mtot += (g.firs.n == 0) ? st.len : st.len - 1;
            g.firs.n++;
        } else if (st.kind == TFX_STAGE_SOS) {
            if (st.len < 0) return fail(TFX_E_INVALID_ARG, "stage %d: negative section count", i);
            if (st.len == 0) continue;
            g.sos.ptr[g.sos.n] = st.coef;
            g.sos.len[g.sos.n] = st.len;
            g.sos.n++;
            g.S += st.len;
        } else {
            return fail(TFX_E_INVALID_ARG, "stage %d: unknown kind %d", i, st.kind);
        }
    }
    if (g.S > tfx::MAX_SECTIONS) return fail(TFX_E_UNSUPPORTED, "more than %d sections in one chain", tfx::MAX_SECTIONS);
    if (g.Mtot > tfx::MAX_TAPS) return fail(TFX_E_UNSUPPORTED, "merged FIR longer than %d taps", tfx::MAX_TAPS);
    return TFX_OK;
}

tfx_status prepare(const tfx::ChainPlan &p) {
    const hipError_t e = tfx::launch_prepare(p);
    if (e != hipSuccess) return hip_fail(e, "table kernel launch");
    return ok();
}

tfx_status execute(const tfx::ChainPlan &p) {
    const hipError_t e = tfx::launch_run(p);
    if (e != hipSuccess) return hip_fail(e, "filter kernel launch");
    return ok();
}

tfx_status run(const tfx::ChainPlan &p) {
    tfx_status s = prepare(p);
    if (s) return s;
    return execute(p);
}

// Shared validation of the chain entry points; fills the plan's stage part.
tfx_status chain_plan(int64_t C, int64_t N, const tfx_stage *stages, int32_t nstages, tfx_compute cmp,
                      void *ws, size_t ws_bytes, void *stream, tfx::ChainPlan &p) {
    Gathered g;
    tfx_status s = gather(stages, nstages, g);
    if (s) return s;
    int32_t mode = tfx::FIR_NONE;
    if (g.firs.n > 0 && (s = check_fir_mode(g.Mtot, cmp, TFX_FIR_AUTO, &mode, C, N, g.S == 0))) return s;
    const tfx::WsLayout lay = tfx::ws_layout(C, N, g.S, g.Mtot, g.firs.n, mode);
    if ((s = check_ws(ws, ws_bytes, lay.total))) return s;
    p.fir_mode = mode;
    p.cmp = cmp;
    p.C = C;
    p.N = N;
    p.firs = g.firs;
    p.sos = g.sos;
    p.S = g.S;
    p.ws = ws;
    p.ws_bytes = ws_bytes;
    p.stream = static_cast<hipStream_t>(stream);
    return TFX_OK;
}

// Validation shared by the adjoint entry points; fills bp (all but the
// gradient lists).
tfx_status bwd_plan(const float *x, const float *gy, float *gx, int64_t C, int64_t N, int64_t ldx, int64_t ldg,
                    int64_t ldgx, const Gathered &g, int32_t mode, const float *ckpt, void *ws, size_t ws_bytes,
                    void *stream, tfx::BwdPlan &bp) {
    tfx_status s = check_signal(x, gx, C, N, ldx, ldgx);
    if (s) return s;
    if (ldg < N) return fail(TFX_E_INVALID_ARG, "ldg must be >= N");
    if (N > 0 && !gy) return fail(TFX_E_INVALID_ARG, "gy is NULL");
    if (N > 0 && overlaps(gy, span_bytes(C, N, ldg), gx, span_bytes(C, N, ldgx)))
        return fail(TFX_E_ALIAS, "gx overlaps gy");
    if (mode == tfx::FIR_TOEPLITZ) return fail(TFX_E_UNSUPPORTED, "the adjoint computes in fp32 only");
    if (g.S > tfx::BWD_MAX_SECTIONS)
        return fail(TFX_E_UNSUPPORTED, "the adjoint handles at most %d sections (got %d)", tfx::BWD_MAX_SECTIONS, g.S);
    if (g.S > 0 && N > 0 && !ckpt) return fail(TFX_E_INVALID_ARG, "ckpt (the forward's checkpoints) is required");
    const tfx::BwdLayout lay = tfx::bwd_layout(C, N, g.S, g.Mtot, g.firs.n, mode);
    if ((s = check_ws(ws, ws_bytes, lay.total))) return s;
    tfx::ChainPlan &p = bp.fwd;
    p.x = x;
    p.C = C;
    p.N = N;
    p.ldx = ldx;
    p.S = g.S;
    p.fir_mode = mode;
    p.sos = g.sos;
    p.firs = g.firs;
    p.ckpt = const_cast<float *>(ckpt);
    p.ws = ws;
    p.ws_bytes = ws_bytes;
    p.stream = static_cast<hipStream_t>(stream);
    bp.gy = gy;
    bp.gx = gx;
    bp.ldg = ldg;
    bp.ldgx = ldgx;
    return TFX_OK;
}

// ---- batched clips

tfx_status batch_clips(const tfx_clip *clips, int32_t n, tfx::ClipIn *out) {
    if (n < 0 || n > 65536) return fail(TFX_E_INVALID_ARG, "nclips must be in [0, 65536]");
    if (n > 0 && !clips) return fail(TFX_E_INVALID_ARG, "clips is NULL");
    for (int i = 0; i < n; ++i) {
        const tfx_clip &c = clips[i];
        tfx_status s = check_signal(c.x, c.y, c.C, c.N, c.ldx, c.ldy);
        if (s) return fail(s, "clip %d: %s", i, g_last_error.c_str());
        if (c.S < 0 || c.S > tfx::MAX_SECTIONS) return fail(TFX_E_INVALID_ARG, "clip %d: S must be in [0, %d]", i, tfx::MAX_SECTIONS);
        if (c.S > 0 && !c.sos) return fail(TFX_E_INVALID_ARG, "clip %d: sos is NULL", i);
        if (c.reserved != 0) return fail(TFX_E_INVALID_ARG, "clip %d: reserved must be 0", i);
        // 16-sample chunks give the most tiles
        if (c.C * ((c.N + 2047) / 2048) >= (int64_t(1) << 31)) return fail(TFX_E_UNSUPPORTED, "clip %d too large", i);
        out[i] = tfx::ClipIn{c.x, c.y, c.C, c.N, c.ldx, c.ldy, c.sos, c.S};
    }
    return TFX_OK;
}

tfx_status batch_config(const tfx_batch_config *cfg, int *lc, int *order) {
    *lc = 24;
    *order = 0;
    if (!cfg) return TFX_OK;
    if (cfg->chunk != 0 && cfg->chunk != 16 && cfg->chunk != 24 && cfg->chunk != 32)
        return fail(TFX_E_INVALID_ARG, "chunk must be 0, 16, 24 or 32 (got %d)", cfg->chunk);
    if (cfg->order != 0 && cfg->order != 1) return fail(TFX_E_INVALID_ARG, "order must be 0 or 1");
    if (cfg->chunk) *lc = cfg->chunk;
    *order = cfg->order;
    return TFX_OK;
}

size_t batch_ws_max(const tfx::ClipIn *c, int32_t n) {
    size_t m = 0;
    for (int lc : tfx::BATCH_CHUNKS) {
        const size_t t = tfx::batch_plan(c, n, lc, 0, nullptr).total;
        m = t > m ? t : m;
    }
    return m;
}

// Validates, and prepares (prep) and/or runs (run) one configuration.
tfx_status batch_do(const tfx_clip *clips, int32_t n, const tfx_batch_config *cfg, void *ws, size_t ws_bytes,
                    void *stream, bool prep, bool run) {
    std::vector<tfx::ClipIn> in(n > 0 ? n : 1);
    tfx_status s = batch_clips(clips, n, in.data());
    if (s) return s;
    int lc, order;
    if ((s = batch_config(cfg, &lc, &order))) return s;
    std::vector<tfx::ClipDesc> desc(n > 0 ? n : 1);
    const tfx::BatchLayout lay = tfx::batch_plan(in.data(), n, lc, order, desc.data());
    if ((s = check_ws(ws, ws_bytes, lay.total))) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    if (prep) {  // an empty batch still gets its header words written
        if (n > 0 && (e = tfx::upload_descriptors(desc.data(), n, lay, ws, st)) != hipSuccess)
            return hip_fail(e, "descriptor upload");
        if ((e = tfx::launch_batch_prepare(lay, lc, n, ws, st)) != hipSuccess) return hip_fail(e, "batch prepare");
    }
    if (run && n > 0 && (e = tfx::launch_batch_run(lay, lc, n, ws, st)) != hipSuccess)
        return hip_fail(e, "batch kernel launch");
    return ok();
}

tfx_status backward(const tfx::BwdPlan &bp) {
    const hipError_t e = tfx::launch_backward(bp);
    if (e != hipSuccess) return hip_fail(e, "adjoint kernel launch");
    return ok();
}

// Calls that synchronise (the tuners) are refused on a capturing stream.
tfx_status not_capturing(hipStream_t st, const char *what) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone)
        return fail(TFX_E_CAPTURE, "%s synchronises the stream and cannot run while it is being captured", what);
    return TFX_OK;
}

// STFT argument checks
int stft_log2(int32_t n_fft) {
    for (int l = 4; l <= 12; ++l)
        if (n_fft == (1 << l)) return l;
    return -1;
}

int64_t stft_count(int64_t N, int32_t n_fft, int32_t hop, int32_t center) {
    const int64_t np = center ? N + 2 * (int64_t)(n_fft / 2) : N;
    return np < n_fft ? 0 : 1 + (np - n_fft) / hop;
}

tfx_status stft_params(int32_t n_fft, int32_t hop, int32_t win_length, int *log2n) {
    *log2n = stft_log2(n_fft);
    if (*log2n < 0) return fail(TFX_E_UNSUPPORTED, "n_fft must be a power of two in [16, 4096] (got %d)", n_fft);
    if (hop < 1) return fail(TFX_E_INVALID_ARG, "hop must be >= 1 (got %d)", hop);
    if (win_length < 1 || win_length > n_fft)
        return fail(TFX_E_INVALID_ARG, "win_length must be in [1, n_fft] (got %d)", win_length);
    return TFX_OK;
}

}  // namespace

namespace tfx {
tfx_status set_error(tfx_status s, const char *msg) {
    g_last_error = msg;
    return s;
}
}  // namespace tfx

extern "C" {

const char *tfx_status_string(tfx_status s) {
    switch (s) {
        case TFX_OK: return "TFX_OK";
        case TFX_E_INVALID_ARG: return "TFX_E_INVALID_ARG";
        case TFX_E_UNSUPPORTED: return "TFX_E_UNSUPPORTED";
        case TFX_E_WORKSPACE: return "TFX_E_WORKSPACE";
        case TFX_E_UNSTABLE: return "TFX_E_UNSTABLE";
        case TFX_E_ALIAS: return "TFX_E_ALIAS";
        case TFX_E_CAPTURE: return "TFX_E_CAPTURE";
        case TFX_E_HIP: return "TFX_E_HIP";
        case TFX_E_DEVICE: return "TFX_E_DEVICE";
    }
    return "TFX_E_UNKNOWN";
}

const char *tfx_last_error(void) { return g_last_error.c_str(); }

int32_t tfx_version(void) { return 100; }

int64_t tfx_sos_tile_length(void) { return tfx::T; }

tfx_status tfx_sos_check_stable(const float *sos_host, int32_t S, int32_t *stable) {
    if (!stable || S < 0 || (S > 0 && !sos_host)) return fail(TFX_E_INVALID_ARG, "bad arguments");
    *stable = 1;
    for (int s = 0; s < S; ++s) {
        const double a1 = sos_host[5 * s + 3], a2 = sos_host[5 * s + 4];
        const double disc = a1 * a1 - 4.0 * a2;
        double r;
        if (disc < 0.0) {
            r = std::sqrt(a2);
        } else {
            const double sq = std::sqrt(disc);
            r = std::fmax(std::fabs(0.5 * (-a1 + sq)), std::fabs(0.5 * (-a1 - sq)));
        }
        if (!(r < 1.0)) {
            *stable = 0;
            return fail(TFX_E_UNSTABLE, "section %d has a pole of radius %.17g", s, r);
        }
    }
    return ok();
}

tfx_status tfx_workspace_status(const void *ws, size_t ws_bytes, uint32_t *flags, int32_t clear, void *stream) {
    if (!flags) return fail(TFX_E_INVALID_ARG, "flags is NULL");
    if (!ws || ws_bytes < 256) return ok();
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(TFX_E_WORKSPACE, "workspace must be 256-byte aligned");
    const hipError_t e = tfx::launch_ws_status(const_cast<void *>(ws), flags, clear ? 1 : 0,
                                               static_cast<hipStream_t>(stream));
    return e == hipSuccess ? ok() : hip_fail(e, "status kernel launch");
}

tfx_status tfx_fir_workspace_size(int64_t C, int64_t N, int32_t M, tfx_compute cmp, tfx_fir_algo algo,
                                  size_t *bytes) {
    if (!bytes) return fail(TFX_E_INVALID_ARG, "bytes is NULL");
    int32_t mode = 0;
    tfx_status s = check_fir_mode(M, cmp, algo, &mode, C, N, true);
    if (s) return s;
    if (C < 1 || N < 0) return fail(TFX_E_INVALID_ARG, "bad shape");
    *bytes = tfx::ws_layout(C, N, 0, M, 1, mode).total;
    return ok();
}

tfx_status tfx_sos_workspace_size(int64_t C, int64_t N, int32_t S, size_t *bytes) {
    if (!bytes) return fail(TFX_E_INVALID_ARG, "bytes is NULL");
    if (C < 1 || N < 0 || S < 0 || S > tfx::MAX_SECTIONS) return fail(TFX_E_INVALID_ARG, "bad shape");
    *bytes = tfx::ws_layout(C, N, S, 0, 0, tfx::FIR_NONE).total;
    return ok();
}

tfx_status tfx_chain_workspace_size(int64_t C, int64_t N, const tfx_stage *stages, int32_t nstages,
                                    tfx_compute cmp, size_t *bytes) {
    if (!bytes) return fail(TFX_E_INVALID_ARG, "bytes is NULL");
    if (C < 1 || N < 0) return fail(TFX_E_INVALID_ARG, "bad shape");
    Gathered g;
    tfx_status s = gather(stages, nstages, g);
    if (s) return s;
    int32_t mode = tfx::FIR_NONE;
    if (g.firs.n > 0 && (s = check_fir_mode(g.Mtot, cmp, TFX_FIR_AUTO, &mode, C, N, g.S == 0))) return s;
    *bytes = tfx::ws_layout(C, N, g.S, g.Mtot, g.firs.n, mode).total;
    return ok();
}

tfx_status tfx_fir(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy, const float *h,
                   int32_t M, tfx_compute cmp, tfx_fir_algo algo, void *ws, size_t ws_bytes, void *stream) {
    tfx_status s = check_signal(x, y, C, N, ldx, ldy);
    if (s) return s;
    int32_t mode = 0;
    if ((s = check_fir_mode(M, cmp, algo, &mode, C, N, true))) return s;
    if (!h) return fail(TFX_E_INVALID_ARG, "taps h is NULL");
    if ((s = check_ws(ws, ws_bytes, tfx::ws_layout(C, N, 0, M, 1, mode).total))) return s;
    tfx::ChainPlan p{};
    p.fir_mode = mode;
    p.cmp = cmp;
    p.x = x; p.y = y; p.C = C; p.N = N; p.ldx = ldx; p.ldy = ldy;
    p.firs.ptr[0] = h;
    p.firs.len[0] = M;
    p.firs.n = 1;
    p.S = 0;
    p.ws = ws;
    p.ws_bytes = ws_bytes;
    p.stream = static_cast<hipStream_t>(stream);
    return run(p);
}

tfx_status tfx_sos(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy, const float *sos,
                   int32_t S, const float *state_in, float *state_out, float *ckpt, void *ws, size_t ws_bytes,
                   void *stream) {
    tfx_status s = check_signal(x, y, C, N, ldx, ldy);
    if (s) return s;
    if (S < 0 || S > tfx::MAX_SECTIONS) return fail(TFX_E_INVALID_ARG, "S must be in [0, %d]", tfx::MAX_SECTIONS);
    if (S > 0 && !sos) return fail(TFX_E_INVALID_ARG, "sos is NULL");
    const tfx::WsLayout lay = tfx::ws_layout(C, N, S, 0, 0, tfx::FIR_NONE);
    if ((s = check_ws(ws, ws_bytes, lay.total))) return s;
    if (state_out && N > 0) {
        const size_t sb = (size_t)C * S * 2 * sizeof(float);
        if (overlaps(state_out, sb, x, span_bytes(C, N, ldx)) || overlaps(state_out, sb, y, span_bytes(C, N, ldy)))
            return fail(TFX_E_ALIAS, "state_out overlaps a signal");
    }
    tfx::ChainPlan p{};
    p.x = x; p.y = y; p.C = C; p.N = N; p.ldx = ldx; p.ldy = ldy;
    p.S = S;
    if (S > 0) {
        p.sos.ptr[0] = sos;
        p.sos.len[0] = S;
        p.sos.n = 1;
    }
    p.state_in = state_in;
    p.state_out = state_out;
    p.ckpt = ckpt;
    p.ws = ws;
    p.ws_bytes = ws_bytes;
    p.stream = static_cast<hipStream_t>(stream);
    return run(p);
}

tfx_status tfx_chain(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                     const tfx_stage *stages, int32_t nstages, tfx_compute cmp, float *ckpt, void *ws,
                     size_t ws_bytes, void *stream) {
    tfx_status s = check_signal(x, y, C, N, ldx, ldy);
    if (s) return s;
    tfx::ChainPlan p{};
    if ((s = chain_plan(C, N, stages, nstages, cmp, ws, ws_bytes, stream, p))) return s;
    p.x = x; p.y = y; p.ldx = ldx; p.ldy = ldy;
    p.ckpt = ckpt;
    return run(p);
}

tfx_status tfx_chain_prepare(int64_t C, int64_t N, const tfx_stage *stages, int32_t nstages, tfx_compute cmp,
                             void *ws, size_t ws_bytes, void *stream) {
    if (C < 1 || N < 0) return fail(TFX_E_INVALID_ARG, "bad shape");
    tfx::ChainPlan p{};
    tfx_status s = chain_plan(C, N, stages, nstages, cmp, ws, ws_bytes, stream, p);
    if (s) return s;
    return prepare(p);
}

tfx_status tfx_chain_run(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                         const tfx_stage *stages, int32_t nstages, tfx_compute cmp, float *ckpt, void *ws,
                         size_t ws_bytes, void *stream) {
    tfx_status s = check_signal(x, y, C, N, ldx, ldy);
    if (s) return s;
    tfx::ChainPlan p{};
    if ((s = chain_plan(C, N, stages, nstages, cmp, ws, ws_bytes, stream, p))) return s;
    p.x = x; p.y = y; p.ldx = ldx; p.ldy = ldy;
    p.ckpt = ckpt;
    return execute(p);
}

tfx_status tfx_chain_stream(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                            const tfx_stage *stages, int32_t nstages, tfx_compute cmp, int64_t n_max,
                            const float *hist_in, float *hist_out, const float *state_in, float *state_out,
                            void *ws, size_t ws_bytes, void *stream) {
    tfx_status s = check_signal(x, y, C, N, ldx, ldy);
    if (s) return s;
    if (N > n_max) return fail(TFX_E_INVALID_ARG, "the block (%lld samples) is longer than n_max (%lld)",
                                (long long)N, (long long)n_max);
    tfx::ChainPlan p{};
    if ((s = chain_plan(C, n_max, stages, nstages, cmp, ws, ws_bytes, stream, p))) return s;
    const int32_t M = tfx::merged_taps(p.firs);
    const size_t hb = M > 1 ? (size_t)C * (size_t)(M - 1) * sizeof(float) : 0;
    const size_t sb = (size_t)C * (size_t)p.S * 2 * sizeof(float);
    if (hb && hist_out) {
        if (overlaps(hist_out, hb, hist_in, hist_in ? hb : 0) || overlaps(hist_out, hb, x, span_bytes(C, N, ldx)) ||
            overlaps(hist_out, hb, y, span_bytes(C, N, ldy)))
            return fail(TFX_E_ALIAS, "hist_out overlaps hist_in or a signal");
    }
    if (hb && hist_in && overlaps(hist_in, hb, y, span_bytes(C, N, ldy)))
        return fail(TFX_E_ALIAS, "hist_in overlaps y");
    if (sb && state_out) {
        if (overlaps(state_out, sb, state_in, state_in ? sb : 0) || overlaps(state_out, sb, x, span_bytes(C, N, ldx)) ||
            overlaps(state_out, sb, y, span_bytes(C, N, ldy)))
            return fail(TFX_E_ALIAS, "state_out overlaps state_in or a signal");
    }
    p.N = N;
    p.n_layout = n_max;
    p.x = x; p.y = y; p.ldx = ldx; p.ldy = ldy;
    p.hist_in = hb ? hist_in : nullptr;
    p.hist_out = hb ? hist_out : nullptr;
    p.state_in = p.S > 0 ? state_in : nullptr;
    p.state_out = p.S > 0 ? state_out : nullptr;
    return execute(p);
}

tfx_status tfx_chain_backward_workspace_size(int64_t C, int64_t N, const tfx_stage *stages, int32_t nstages,
                                             tfx_compute cmp, size_t *bytes) {
    if (!bytes) return fail(TFX_E_INVALID_ARG, "bytes is NULL");
    if (C < 1 || N < 0) return fail(TFX_E_INVALID_ARG, "bad shape");
    Gathered g;
    tfx_status s = gather(stages, nstages, g);
    if (s) return s;
    int32_t mode = tfx::FIR_NONE;
    if (g.firs.n > 0 && (s = check_fir_mode(g.Mtot, cmp, TFX_FIR_AUTO, &mode, C, N, g.S == 0))) return s;
    *bytes = tfx::bwd_layout(C, N, g.S, g.Mtot, g.firs.n, mode).total;
    return ok();
}

tfx_status tfx_chain_backward(const float *x, const float *gy, float *gx, int64_t C, int64_t N, int64_t ldx,
                              int64_t ldg, int64_t ldgx, const tfx_stage *stages, int32_t nstages, tfx_compute cmp,
                              const float *ckpt, float *const *grads, void *ws, size_t ws_bytes, void *stream) {
    Gathered g;
    tfx_status s = gather(stages, nstages, g);
    if (s) return s;
    int32_t mode = tfx::FIR_NONE;
    if (g.firs.n > 0 && (s = check_fir_mode(g.Mtot, cmp, TFX_FIR_AUTO, &mode, C, N, g.S == 0))) return s;
    tfx::BwdPlan bp{};
    if ((s = bwd_plan(x, gy, gx, C, N, ldx, ldg, ldgx, g, mode, ckpt, ws, ws_bytes, stream, bp))) return s;
    // gradient pointers in the order of the gathered stage lists
    for (int i = 0; i < nstages; ++i) {
        const tfx_stage &st = stages[i];
        float *gp = grads ? grads[i] : nullptr;
        if (st.kind == TFX_STAGE_FIR) {
            bp.gfir.ptr[bp.gfir.n] = gp;
            bp.gfir.len[bp.gfir.n] = st.len;
            bp.gfir.n++;
        } else if (st.len > 0) {
            bp.gsos.ptr[bp.gsos.n] = gp;
            bp.gsos.len[bp.gsos.n] = st.len;
            bp.gsos.n++;
        }
    }
    return backward(bp);
}

tfx_status tfx_fir_backward_workspace_size(int64_t C, int64_t N, int32_t M, tfx_compute cmp, tfx_fir_algo algo,
                                           size_t *bytes) {
    if (!bytes) return fail(TFX_E_INVALID_ARG, "bytes is NULL");
    int32_t mode = 0;
    tfx_status s = check_fir_mode(M, cmp, algo, &mode, C, N, true);
    if (s) return s;
    if (C < 1 || N < 0) return fail(TFX_E_INVALID_ARG, "bad shape");
    *bytes = tfx::bwd_layout(C, N, 0, M, 1, mode).total;
    return ok();
}

tfx_status tfx_fir_backward(const float *x, const float *gy, float *gx, int64_t C, int64_t N, int64_t ldx,
                            int64_t ldg, int64_t ldgx, const float *h, int32_t M, float *gh, tfx_compute cmp,
                            tfx_fir_algo algo, void *ws, size_t ws_bytes, void *stream) {
    int32_t mode = 0;
    tfx_status s = check_fir_mode(M, cmp, algo, &mode, C, N, true);
    if (s) return s;
    if (!h) return fail(TFX_E_INVALID_ARG, "taps h is NULL");
    Gathered g;
    g.firs.ptr[0] = h;
    g.firs.len[0] = M;
    g.firs.n = 1;
    g.Mtot = M;
    tfx::BwdPlan bp{};
    if ((s = bwd_plan(x, gy, gx, C, N, ldx, ldg, ldgx, g, mode, nullptr, ws, ws_bytes, stream, bp))) return s;
    bp.gfir.ptr[0] = gh;
    bp.gfir.len[0] = M;
    bp.gfir.n = 1;
    return backward(bp);
}

tfx_status tfx_sos_backward_workspace_size(int64_t C, int64_t N, int32_t S, size_t *bytes) {
    if (!bytes) return fail(TFX_E_INVALID_ARG, "bytes is NULL");
    if (C < 1 || N < 0 || S < 0 || S > tfx::MAX_SECTIONS) return fail(TFX_E_INVALID_ARG, "bad shape");
    *bytes = tfx::bwd_layout(C, N, S, 0, 0, tfx::FIR_NONE).total;
    return ok();
}

tfx_status tfx_sos_backward(const float *x, const float *gy, float *gx, int64_t C, int64_t N, int64_t ldx,
                            int64_t ldg, int64_t ldgx, const float *sos, int32_t S, const float *ckpt, float *gsos,
                            void *ws, size_t ws_bytes, void *stream) {
    if (S < 0 || S > tfx::MAX_SECTIONS) return fail(TFX_E_INVALID_ARG, "S must be in [0, %d]", tfx::MAX_SECTIONS);
    if (S > 0 && !sos) return fail(TFX_E_INVALID_ARG, "sos is NULL");
    Gathered g;
    if (S > 0) {
        g.sos.ptr[0] = sos;
        g.sos.len[0] = S;
        g.sos.n = 1;
        g.S = S;
    }
    tfx::BwdPlan bp{};
    tfx_status s = bwd_plan(x, gy, gx, C, N, ldx, ldg, ldgx, g, tfx::FIR_NONE, ckpt, ws, ws_bytes, stream, bp);
    if (s) return s;
    if (S > 0) {
        bp.gsos.ptr[0] = gsos;
        bp.gsos.len[0] = S;
        bp.gsos.n = 1;
    }
    if (S == 0) {  // identity: gx = gy
        hipError_t e = tfx::launch_header_init(ws, ws_bytes, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "workspace header");
        if (N == 0) return ok();
        e = hipMemcpy2DAsync(gx, ldgx * sizeof(float), gy, ldg * sizeof(float), N * sizeof(float),
                                              C, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, "copy");
        return ok();
    }
    return backward(bp);
}

tfx_status tfx_sos_batched_workspace_size(const tfx_clip *clips, int32_t nclips, size_t *bytes) {
    if (!bytes) return fail(TFX_E_INVALID_ARG, "bytes is NULL");
    std::vector<tfx::ClipIn> in(nclips > 0 ? nclips : 1);
    tfx_status s = batch_clips(clips, nclips, in.data());
    if (s) return s;
    *bytes = batch_ws_max(in.data(), nclips);
    return ok();
}

tfx_status tfx_sos_batched_prepare(const tfx_clip *clips, int32_t nclips, const tfx_batch_config *cfg, void *ws,
                                   size_t ws_bytes, void *stream) {
    return batch_do(clips, nclips, cfg, ws, ws_bytes, stream, true, false);
}

tfx_status tfx_sos_batched_run(const tfx_clip *clips, int32_t nclips, const tfx_batch_config *cfg, void *ws,
                               size_t ws_bytes, void *stream) {
    return batch_do(clips, nclips, cfg, ws, ws_bytes, stream, false, true);
}

tfx_status tfx_sos_batched(const tfx_clip *clips, int32_t nclips, const tfx_batch_config *cfg, void *ws,
                           size_t ws_bytes, void *stream) {
    return batch_do(clips, nclips, cfg, ws, ws_bytes, stream, true, true);
}

tfx_status tfx_sos_batched_tune(const tfx_clip *clips, int32_t nclips, int32_t reps, void *ws, size_t ws_bytes,
                                void *stream, tfx_batch_config *best, float *best_ms) {
    if (!best) return fail(TFX_E_INVALID_ARG, "best is NULL");
    if (reps < 1 || reps > 1000) return fail(TFX_E_INVALID_ARG, "reps must be in [1, 1000]");
    hipStream_t st = static_cast<hipStream_t>(stream);
    tfx_status cs = not_capturing(st, "tfx_sos_batched_tune");
    if (cs) return cs;
    hipEvent_t e0, e1;
    hipError_t he;
    if ((he = hipEventCreate(&e0)) != hipSuccess) return hip_fail(he, "hipEventCreate");
    if ((he = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    tfx_status s = TFX_OK;
    float bms = -1.f;
    tfx_batch_config bc{24, 0};
    for (int lc : tfx::BATCH_CHUNKS) {
        for (int order = 0; order < 2 && !s; ++order) {
            const tfx_batch_config c{lc, order};
            if ((s = batch_do(clips, nclips, &c, ws, ws_bytes, stream, true, true))) break;  // prepare + warm-up
            if ((he = hipEventRecord(e0, st)) != hipSuccess) { s = hip_fail(he, "hipEventRecord"); break; }
            for (int r = 0; r < reps && !s; ++r) s = batch_do(clips, nclips, &c, ws, ws_bytes, stream, false, true);
            if (s) break;
            if ((he = hipEventRecord(e1, st)) != hipSuccess || (he = hipEventSynchronize(e1)) != hipSuccess) {
                s = hip_fail(he, "timing");
                break;
            }
            float ms = 0.f;
            if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { s = hip_fail(he, "hipEventElapsedTime"); break; }
            ms /= reps;
            if (bms < 0.f || ms < bms) {
                bms = ms;
                bc = c;
            }
        }
        if (s) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    *best = bc;
    if (best_ms) *best_ms = bms;
    return batch_do(clips, nclips, &bc, ws, ws_bytes, stream, true, false);
}


// ---- short-time Fourier transform ------------------------------------------------

tfx_status tfx_stft_frames(int64_t N, int32_t n_fft, int32_t hop, int32_t center, int64_t *T) {
    if (!T) return fail(TFX_E_INVALID_ARG, "T is NULL");
    int l;
    tfx_status s = stft_params(n_fft, hop, n_fft, &l);
    if (s) return s;
    if (N < 0 || N >= (int64_t(1) << 40)) return fail(TFX_E_INVALID_ARG, "N out of range");
    *T = stft_count(N, n_fft, hop, center);
    return ok();
}

tfx_status tfx_stft(const float *x, int64_t C, int64_t N, int64_t ldx, int32_t n_fft, int32_t hop,
                    const float *window, int32_t win_length, int32_t center, int32_t normalized, float *spec,
                    void *stream) {
    tfx::StftPlan sp{};
    tfx_status s = stft_params(n_fft, hop, win_length, &sp.log2n);
    if (s) return s;
    if (C < 1) return fail(TFX_E_INVALID_ARG, "C must be >= 1 (got %lld)", (long long)C);
    if (N < 0 || N >= (int64_t(1) << 40)) return fail(TFX_E_INVALID_ARG, "N out of range (got %lld)", (long long)N);
    if (ldx < N) return fail(TFX_E_INVALID_ARG, "ldx must be >= N");
    if (center && N > 0 && N <= n_fft / 2)
        return fail(TFX_E_INVALID_ARG, "centred frames reflect n_fft/2 samples: N must exceed %d (got %lld)",
                    n_fft / 2, (long long)N);
    const int64_t T = stft_count(N, n_fft, hop, center);
    if (T == 0 || N == 0) return ok();
    if (!x || !spec) return fail(TFX_E_INVALID_ARG, "x and spec must be non-null");
    const size_t sbytes = (size_t)C * (size_t)T * (size_t)(n_fft / 2 + 1) * 2 * sizeof(float);
    if (overlaps(x, span_bytes(C, N, ldx), spec, sbytes)) return fail(TFX_E_ALIAS, "spec overlaps x");
    sp.hop = hop;
    sp.win_length = win_length;
    sp.center = center ? 1 : 0;
    sp.normalized = normalized ? 1 : 0;
    sp.win = window;
    sp.C = C;
    sp.T = T;
    sp.x = x;
    sp.ldx = ldx;
    sp.nx = N;
    sp.spec = spec;
    sp.stream = static_cast<hipStream_t>(stream);
    hipError_t e = tfx::launch_stft(sp);
    return e == hipSuccess ? ok() : hip_fail(e, "stft kernel");
}

tfx_status tfx_istft(const float *spec, int64_t C, int64_t T, int32_t n_fft, int32_t hop, const float *window,
                     int32_t win_length, int32_t center, int32_t normalized, float *y, int64_t length, int64_t ldy,
                     void *stream) {
    tfx::StftPlan sp{};
    tfx_status s = stft_params(n_fft, hop, win_length, &sp.log2n);
    if (s) return s;
    if (C < 1 || T < 1) return fail(TFX_E_INVALID_ARG, "C and T must be >= 1");
    const int64_t total = (int64_t)n_fft + (int64_t)hop * (T - 1);
    if (total >= (int64_t(1) << 40)) return fail(TFX_E_INVALID_ARG, "T * hop out of range");
    if (length < 0) length = total - (center ? 2 * (int64_t)(n_fft / 2) : 0);
    if (length >= (int64_t(1) << 38)) return fail(TFX_E_UNSUPPORTED, "length must be below 2^38");
    if (ldy < length) return fail(TFX_E_INVALID_ARG, "ldy must be >= length");
    if (length == 0) return ok();
    if (!spec || !y) return fail(TFX_E_INVALID_ARG, "spec and y must be non-null");
    const size_t sbytes = (size_t)C * (size_t)T * (size_t)(n_fft / 2 + 1) * 2 * sizeof(float);
    if (overlaps(y, span_bytes(C, length, ldy), spec, sbytes)) return fail(TFX_E_ALIAS, "y overlaps spec");
    sp.hop = hop;
    sp.win_length = win_length;
    sp.center = center ? 1 : 0;
    sp.normalized = normalized ? 1 : 0;
    sp.win = window;
    sp.C = C;
    sp.T = T;
    sp.spec_in = spec;
    sp.y = y;
    sp.length = length;
    sp.ldy = ldy;
    sp.stream = static_cast<hipStream_t>(stream);
    hipError_t e = tfx::launch_istft(sp);
    return e == hipSuccess ? ok() : hip_fail(e, "istft kernel");
}

// ---- batched real FFT ------------------------------------------------------------
// Both run the STFT kernels: every row is one rectangular, uncentred frame
// (hop = n).  Rows that follow each other in memory (ld == n) form a single
// signal of B frames, so the kernels pair frames two to a complex FFT across
// rows; other strides give B channels of one frame each.

tfx_status tfx_rfft(const float *x, int64_t B, int32_t n, int64_t ldx, float *spec, void *stream) {
    tfx::StftPlan sp{};
    tfx_status s = stft_params(n, n, n, &sp.log2n);
    if (s) return s;
    if (B < 0 || B >= (int64_t(1) << 40) / n) return fail(TFX_E_INVALID_ARG, "B out of range (got %lld)", (long long)B);
    if (ldx < n) return fail(TFX_E_INVALID_ARG, "ldx must be >= n");
    if (B == 0) return ok();
    if (!x || !spec) return fail(TFX_E_INVALID_ARG, "x and spec must be non-null");
    const size_t sbytes = (size_t)B * (size_t)(n / 2 + 1) * 2 * sizeof(float);
    if (overlaps(x, span_bytes(B, n, ldx), spec, sbytes)) return fail(TFX_E_ALIAS, "spec overlaps x");
    const bool packed = ldx == n;
    sp.hop = n;
    sp.win_length = n;
    sp.center = 0;
    sp.normalized = 0;
    sp.win = nullptr;
    sp.C = packed ? 1 : B;
    sp.T = packed ? B : 1;
    sp.x = x;
    sp.nx = packed ? B * (int64_t)n : n;
    sp.ldx = packed ? sp.nx : ldx;
    sp.spec = spec;
    sp.stream = static_cast<hipStream_t>(stream);
    hipError_t e = tfx::launch_stft(sp);
    return e == hipSuccess ? ok() : hip_fail(e, "rfft kernel");
}

tfx_status tfx_irfft(const float *spec, int64_t B, int32_t n, float *y, int64_t ldy, void *stream) {
    tfx::StftPlan sp{};
    tfx_status s = stft_params(n, n, n, &sp.log2n);
    if (s) return s;
    if (B < 0 || B >= (int64_t(1) << 38) / n) return fail(TFX_E_INVALID_ARG, "B out of range (got %lld)", (long long)B);
    if (ldy < n) return fail(TFX_E_INVALID_ARG, "ldy must be >= n");
    if (B == 0) return ok();
    if (!spec || !y) return fail(TFX_E_INVALID_ARG, "spec and y must be non-null");
    const size_t sbytes = (size_t)B * (size_t)(n / 2 + 1) * 2 * sizeof(float);
    if (overlaps(y, span_bytes(B, n, ldy), spec, sbytes)) return fail(TFX_E_ALIAS, "y overlaps spec");
    const bool packed = ldy == n;
    sp.hop = n;
    sp.win_length = n;
    sp.center = 0;
    sp.normalized = 0;
    sp.win = nullptr;
    sp.C = packed ? 1 : B;
    sp.T = packed ? B : 1;
    sp.spec_in = spec;
    sp.y = y;
    sp.length = packed ? B * (int64_t)n : n;
    sp.ldy = packed ? sp.length : ldy;
    sp.stream = static_cast<hipStream_t>(stream);
    hipError_t e = tfx::launch_istft(sp);
    return e == hipSuccess ? ok() : hip_fail(e, "irfft kernel");
}

}  // extern "C"
