/*
 * tfx.h -- C ABI of the MI355X (gfx950) multichannel FIR / IIR-SOS filter
 * chain library (libtfx.so).
 *
 * What the library computes is the filtering that TorchFX (arXiv 2504.08624)
 * exposes: FIR filters and coefficient-driven IIR filters applied to
 * multichannel [channels x samples] signals (Sec. 3, "Design principles and
 * core features", and the multichannel focus stated in Sec. 1), chained in the
 * order written (the pipe-operator example of Sec. 3).  The paper gives no
 * equations; the operations are the textbook ones:
 *
 *   FIR  y[c,n] = sum_{k=0}^{min(M-1,n)} h[k] x[c,n-k]
 *        (causal, zero history, output length N, true convolution)
 *   SOS  cascade of second-order sections in transposed direct form II,
 *        coefficient rows [b0 b1 b2 a1 a2] with a0 == 1:
 *          y[n] = b0 x[n] + s1;  s1 = b1 x[n] - a1 y[n] + s2;  s2 = b2 x[n] - a2 y[n]
 *        H(z) = (b0 + b1 z^-1 + b2 z^-2) / (1 + a1 z^-1 + a2 z^-2), sections in
 *        array order, zero initial state unless a state is passed in.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Signals are fp32, row-major: channel c, sample n at  ptr[c*ld + n],
 *    ld >= N (elements).  Input and output must not overlap (TFX_E_ALIAS).
 *  - Pointers are DEVICE pointers unless the comment says "host".  The caller
 *    allocates and owns every buffer (signals, coefficients, states,
 *    checkpoints, gradients, workspace).  The library keeps no pointer after
 *    the call returns and allocates no device memory on these calls.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *    only enqueues work on that stream and returns; results are ready when the
 *    stream is synchronised.  The library never synchronises.
 *  - `ws`/`ws_bytes`: caller-owned device workspace, at least the size the
 *    matching *_workspace_size query returns (TFX_E_WORKSPACE otherwise);
 *    256-byte alignment required.  One workspace must not be used by two
 *    calls that may run concurrently.  Its contents need no initialisation
 *    and are undefined afterwards.
 *  - Coefficients are read on the device every call, so they may change
 *    between calls (learned filters) without any re-planning.
 *  - Errors: argument errors are detected on the host before anything is
 *    enqueued and return a non-zero tfx_status; tfx_last_error() then gives
 *    a message (thread-local).  A HIP launch failure returns TFX_E_HIP.
 *    Asynchronous device faults surface at the caller's next synchronisation,
 *    as with any HIP kernel.  Nothing aborts or throws across this ABI.
 *  - Results are bit-identical from run to run for fixed arguments (no
 *    floating-point atomics, fixed reduction orders).
 *
 * Limits: 1 <= C, 0 <= N < 2^40 (N == 0 is a no-op), 1 <= M <= 65536 taps,
 * 0 <= S <= 256 sections per cascade.
 */
#ifndef TFX_H
#define TFX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tfx_status {
    TFX_OK = 0,
    TFX_E_INVALID_ARG = 1, /* null pointer, negative size, ld < N, bad enum  */
    TFX_E_UNSUPPORTED = 2, /* valid request this build does not implement    */
    TFX_E_WORKSPACE = 3,   /* ws NULL / too small / misaligned               */
    TFX_E_UNSTABLE = 4,    /* host-checked filter with a pole on/outside |z|=1 */
    TFX_E_ALIAS = 5,       /* output overlaps an input                        */
    TFX_E_CAPTURE = 6,     /* call not allowed while the stream is captured   */
    TFX_E_HIP = 7,         /* a HIP runtime call failed                       */
    TFX_E_DEVICE = 8       /* a kernel flagged its result in a workspace's
                              status word (see tfx_workspace_status)          */
} tfx_status;

/* Arithmetic of the FIR contraction.  Signals stay fp32 in memory for every
 * mode; the IIR recursion is always fp32. */
typedef enum tfx_compute {
    TFX_COMPUTE_F32 = 0,    /* fp32 products, fp32 accumulation              */
    TFX_COMPUTE_BF16 = 1,   /* bf16 operands on MFMA, fp32 accumulation      */
    TFX_COMPUTE_F16 = 2,    /* fp16 operands on MFMA, fp32 accumulation      */
    TFX_COMPUTE_BF16X3 = 3  /* split bf16 hi+lo, 3 MFMA products (~fp32)     */
} tfx_compute;

typedef enum tfx_fir_algo {
    TFX_FIR_AUTO = 0,      /* pick by tap count and compute mode             */
    TFX_FIR_DIRECT = 1,    /* LDS-tiled direct convolution (fp32 only)       */
    TFX_FIR_TOEPLITZ = 2,  /* MFMA block-Toeplitz product (bf16/fp16/bf16x3) */
    TFX_FIR_FFT = 3,       /* overlap-save, 4096-point FFT per 3072 outputs;
                              taps beyond 1025 in partitions of 1025 (fp32) */
    TFX_FIR_FFT16K = 4     /* overlap-save, 16384-point FFT per 8192 outputs;
                              at most 8193 taps (fp32)                      */
} tfx_fir_algo;

typedef enum tfx_stage_kind { TFX_STAGE_FIR = 0, TFX_STAGE_SOS = 1 } tfx_stage_kind;

/* One stage of a chain (host array of these; `coef` is a device pointer).
 *   FIR: coef = h[len] taps, len = M.
 *   SOS: coef = [len][5] rows [b0 b1 b2 a1 a2], len = S sections. */
typedef struct tfx_stage {
    int32_t kind;
    int32_t len;
    const float *coef;
} tfx_stage;

/* ------------------------------------------------------------ diagnostics */

const char *tfx_status_string(tfx_status s);
/* Message of the last failing call on this host thread ("" if none). */
const char *tfx_last_error(void);
/* Library version as 10000*major + 100*minor + patch. */
int32_t tfx_version(void);
/* Samples per IIR tile: the granularity of checkpoints (see tfx_sos). */
int64_t tfx_sos_tile_length(void);

/* Host-side stability check of a cascade (host pointer, [S][5]): *stable = 1
 * when every section's poles lie strictly inside the unit circle.  The device
 * entry points cannot read coefficients on the host, so callers that need
 * TFX_E_UNSTABLE semantics check here first.  Returns TFX_E_UNSTABLE when not
 * stable. */
tfx_status tfx_sos_check_stable(const float *sos_host, int32_t S, int32_t *stable);

/* Device-side status of a workspace.  The IIR scan carries the state
 * entering each tile from its predecessors (Sec. 3's recursive filters run
 * as a chunked linear-recurrence scan): a workgroup waits, with a bounded
 * number of polls, for the tiles before it.  Workgroups are dispatched in
 * tile order, so the wait always ends; should the bound ever be reached the
 * kernel finishes with a wrong prefix and sets TFX_DEV_LOOKBACK_TIMEOUT in the
 * workspace's status word instead of hanging.  Every call that uses a
 * workspace of at least 256 bytes (forward, stream, adjoint, batched) clears
 * the word when it prepares the workspace; tfx_chain_run and
 * tfx_sos_batched_run only ever set bits, so the word covers every run since
 * the last prepare.
 *
 * tfx_workspace_status enqueues on `stream` one single-thread kernel that ORs
 * the status word of ws into *flags and, when `clear` is non-zero, zeroes the
 * word.  flags is a DEVICE pointer (or mapped pinned host memory, e.g. from
 * hipHostMalloc); its value is valid once the stream is synchronised.  The
 * call neither allocates nor synchronises, so it may be captured.  A NULL ws
 * or ws_bytes < 256 (a call that needed no workspace) leaves *flags
 * unchanged.  The caller reads *flags after synchronising and treats any set
 * bit as TFX_E_DEVICE for the calls that used ws. */
#define TFX_DEV_LOOKBACK_TIMEOUT 1u
tfx_status tfx_workspace_status(const void *ws, size_t ws_bytes, uint32_t *flags, int32_t clear, void *stream);

/* ------------------------------------------------------ workspace queries */

tfx_status tfx_fir_workspace_size(int64_t C, int64_t N, int32_t M, tfx_compute cmp,
                                  tfx_fir_algo algo, size_t *bytes);
tfx_status tfx_sos_workspace_size(int64_t C, int64_t N, int32_t S, size_t *bytes);
/* stages: host array as for tfx_chain. */
tfx_status tfx_chain_workspace_size(int64_t C, int64_t N, const tfx_stage *stages,
                                    int32_t nstages, tfx_compute cmp, size_t *bytes);

/* ---------------------------------------------------------------- forward */

/* FIR filter, every channel with the same taps h[M]. */
tfx_status tfx_fir(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                   const float *h, int32_t M, tfx_compute cmp, tfx_fir_algo algo,
                   void *ws, size_t ws_bytes, void *stream);

/* SOS cascade sos[S][5], every channel with the same cascade, by a chunked
 * parallel linear-recurrence scan.
 *   state_in  : NULL (zero state) or [C][S][2] = (s1, s2) per section
 *   state_out : NULL or [C][S][2], the state after sample N-1 (resume a
 *               stream by passing it as the next call's state_in)
 *   ckpt      : NULL or [C][ceil(N/T)][S][2] with T = tfx_sos_tile_length():
 *               the state entering each section at the start of every tile,
 *               used by tfx_sos_backward to recompute section signals.
 * S == 0 copies x to y. */
tfx_status tfx_sos(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                   const float *sos, int32_t S, const float *state_in, float *state_out,
                   float *ckpt, void *ws, size_t ws_bytes, void *stream);

/* Chain of stages applied left to right (replaces the paper's pipe
 * operator).  LTI stages with zero initial state commute, so the library may
 * regroup them: all FIR stages are merged into one tap vector (FP64 tap
 * convolution on the device) applied first, and all SOS stages are
 * concatenated into one cascade fused behind it in the same kernel.  Only
 * rounding differs from the written order.
 *   cmp  : arithmetic of the FIR part (TFX_COMPUTE_F32 for the plain chain)
 *   ckpt : NULL or as for tfx_sos with S = total sections (for the backward). */
tfx_status tfx_chain(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                     const tfx_stage *stages, int32_t nstages, tfx_compute cmp, float *ckpt,
                     void *ws, size_t ws_bytes, void *stream);

/* Two-phase form of tfx_chain for filters whose coefficients stay fixed over
 * many calls (serving loops, captured graphs).  tfx_chain_prepare builds the
 * per-section device tables (and the merged taps) into ws and initialises
 * it; tfx_chain_run then filters with them, any number of times.  Both take
 * the same C, N, stages and cmp; the stage coefficients must not change in
 * between (call prepare again if they do).  tfx_chain_run launches one kernel,
 * writes no memset and re-arms the workspace for the next run itself, so it
 * may be captured into a hipGraph and replayed; runs sharing one ws must not
 * overlap in time.  tfx_chain == prepare + run on the same stream. */
tfx_status tfx_chain_prepare(int64_t C, int64_t N, const tfx_stage *stages, int32_t nstages,
                             tfx_compute cmp, void *ws, size_t ws_bytes, void *stream);
tfx_status tfx_chain_run(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                         const tfx_stage *stages, int32_t nstages, tfx_compute cmp, float *ckpt,
                         void *ws, size_t ws_bytes, void *stream);

/* tfx_chain for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same computation and arguments as tfx_chain, with the workspace taken from
 * a scratch array the library holds on each device (TFX_NOALLOC_SCRATCH_BYTES,
 * kept until the process ends) instead of a caller-owned one.  The call
 * allocates nothing, frees nothing and does not synchronise.  A call whose
 * workspace (tfx_chain_workspace_size) exceeds the array returns
 * TFX_E_WORKSPACE before anything is enqueued.  Every call on a device
 * shares that device's array: calls that may overlap in time on one device
 * (two streams, two host threads) race and give wrong results; calls on one
 * stream are ordered and safe.  The array keeps the last call's contents;
 * each call initialises what it reads.
 *   flags : NULL, or a DEVICE word into which the array's status word is
 *           ORed after the run (as tfx_workspace_status with clear = 1),
 *           valid once the stream is synchronised. */
#define TFX_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
tfx_status tfx_chain_noalloc(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                             const tfx_stage *stages, int32_t nstages, tfx_compute cmp, float *ckpt,
                             uint32_t *flags, void *stream);

/* Streaming (block-by-block) form of tfx_chain (the real-time block
 * processing the paper's Sec. 5 names on its roadmap): y is the chain applied
 * to the block x[C][N] as the continuation of everything filtered before it.
 * The workspace is prepared once with tfx_chain_prepare(C, n_max, ...) for
 * the longest block; every block is then one call (one filter launch, plus a
 * small copy kernel for the history), N <= n_max, any N >= 0.
 *   hist_in   FIR history: the M - 1 inputs just before the block, [C][M - 1]
 *             row-major (M = the merged tap count); NULL = zeros (start of
 *             the stream).  Ignored without FIR stages or when M == 1.
 *   hist_out  receives the last M - 1 inputs up to the block's end (for the
 *             next call); NULL = not written.  Must not overlap hist_in, x
 *             or y.
 *   state_in  the cascade's TDF-II registers before the block, [C][S][2]
 *             (as for tfx_sos); NULL = zero.
 *   state_out receives them after the block's last sample; NULL = not
 *             written.  Must not overlap state_in, x or y.
 * Same stage and precision rules as tfx_chain (the bf16/fp16 matrix-core FIR
 * also takes its history); the coefficients must not change between the
 * prepare and the runs.  TFX_E_INVALID_ARG if N > n_max; TFX_E_WORKSPACE if
 * ws is smaller than the size for (C, n_max); TFX_E_ALIAS as listed. */
tfx_status tfx_chain_stream(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                            const tfx_stage *stages, int32_t nstages, tfx_compute cmp, int64_t n_max,
                            const float *hist_in, float *hist_out, const float *state_in, float *state_out,
                            void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------- tuning */

/* FIR algorithm tuner.  The FIR forms above compute the same convolution:
 * direct, overlap-save with 4096- or 16384-point FFTs (fp32), and the
 * matrix-core Toeplitz product in split bf16, fp16 or bf16 operands.  Each
 * has a stated accuracy, the per-channel relative RMS error it is held to:
 * fp32 forms 1e-5, split bf16 1e-4, fp16 and bf16 1e-2.  tfx_fir_autotune
 * times every form whose stated accuracy is within `tol` on the caller's
 * buffers (one untimed call each, then `reps` timed calls of tfx_fir with
 * HIP events; a form more than 4x slower than the best so far on its untimed
 * call is not timed further) and returns the fastest in *best_algo /
 * *best_cmp (its mean time per call in *best_ms if not NULL).  It records
 * the result in the process-wide tuning cache, keyed by (device architecture
 * and compute-unit count, M, C, floor(log2 N), tolerance class); from then on
 * an fp32 TFX_FIR_AUTO request of that key by tfx_fir, tfx_fir_backward and
 * FIR-only chains takes the recorded form (chains with sections keep the
 * fixed rule, under which the FIR fuses with the cascade).
 * Synchronises `stream` (TFX_E_CAPTURE, nothing enqueued, when the stream is
 * being captured); overwrites y.  ws: at least
 * tfx_fir_autotune_workspace_size bytes.  tol < 1e-5: TFX_E_UNSUPPORTED. */
tfx_status tfx_fir_autotune_workspace_size(int64_t C, int64_t N, int32_t M, double tol, size_t *bytes);
tfx_status tfx_fir_autotune(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                            const float *h, int32_t M, double tol, int32_t reps, void *ws, size_t ws_bytes,
                            void *stream, tfx_fir_algo *best_algo, tfx_compute *best_cmp, float *best_ms);
/* The cached form for (C, N, M, tol) on the current device, or
 * TFX_FIR_AUTO / TFX_COMPUTE_F32 when nothing is cached (host only). */
tfx_status tfx_fir_tuned(int64_t C, int64_t N, int32_t M, double tol, tfx_fir_algo *algo, tfx_compute *cmp);
/* Makes the tuning cache persistent in the text file `path` (host string):
 * entries already in the file are loaded now (lines of the form
 * "fir <arch> <M> <C> <log2 N> <class> <algo> <compute> <ms>"; arch "*"
 * matches any device), and the whole cache is rewritten there after every
 * tuning run.  NULL or "" keeps the cache in memory only.  Malformed lines
 * are skipped and reported as TFX_E_INVALID_ARG after the rest is loaded. */
tfx_status tfx_set_tuning_cache(const char *path);

/* ------------------------------------------------------- batched clips */

/* One clip of a ragged batch: its own channel count C, length N, strides and
 * SOS cascade sos[S][5] (device pointers, as for tfx_sos; zero initial
 * state).  x and y of one clip must not overlap; different clips must not
 * write overlapping outputs. */
typedef struct tfx_clip {
    const float *x;
    float *y;
    int64_t C, N, ldx, ldy;
    const float *sos;
    int32_t S;
    int32_t reserved; /* 0 */
} tfx_clip;

/* Launch shape of the batched kernel.
 *   chunk : samples per lane chunk, 16, 24 or 32 (tile = 128 chunk samples
 *           of one channel); 0 = 24
 *   order : 0 = clips in the given order, 1 = longest clip first */
typedef struct tfx_batch_config {
    int32_t chunk;
    int32_t order;
} tfx_batch_config;

/* Workspace for any configuration of this batch (host clips array). */
tfx_status tfx_sos_batched_workspace_size(const tfx_clip *clips, int32_t nclips, size_t *bytes);
/* Writes the clip descriptor table and every clip's section tables into ws
 * and initialises it (a few small kernels on `stream`).  Coefficients must
 * stay fixed until the next prepare.  cfg may be NULL (defaults). */
tfx_status tfx_sos_batched_prepare(const tfx_clip *clips, int32_t nclips, const tfx_batch_config *cfg,
                                   void *ws, size_t ws_bytes, void *stream);
/* Filters every clip of a prepared batch: ONE kernel launch over all clips
 * (plus a one-thread kernel that re-arms ws), no memset, so it may be
 * captured in a hipGraph and replayed.  clips, nclips and cfg must equal the
 * prepare call's. */
tfx_status tfx_sos_batched_run(const tfx_clip *clips, int32_t nclips, const tfx_batch_config *cfg,
                               void *ws, size_t ws_bytes, void *stream);
/* prepare + run. */
tfx_status tfx_sos_batched(const tfx_clip *clips, int32_t nclips, const tfx_batch_config *cfg, void *ws,
                           size_t ws_bytes, void *stream);
/* Autotuner: times every configuration (chunk 16/24/32 x both orders) on
 * this batch with HIP events, `reps` timed runs each after one warm-up, and
 * returns the fastest in *best (its mean time in *best_ms if not NULL).
 * Synchronises `stream`; overwrites the clips' outputs; leaves ws prepared
 * for *best.  Returns TFX_E_CAPTURE (nothing enqueued) when `stream` is
 * being captured into a graph. */
tfx_status tfx_sos_batched_tune(const tfx_clip *clips, int32_t nclips, int32_t reps, void *ws,
                                size_t ws_bytes, void *stream, tfx_batch_config *best, float *best_ms);

/* --------------------------------------------------------------- adjoint */

/* Gradients of a scalar loss L through the forward calls above, given
 * gy = dL/dy (fp32, [C][N], row stride ldg):
 *   gx    = dL/dx                      ([C][N], row stride ldgx; required)
 *   taps  dL/dh[k] = sum_{c,n} gy'[c,n] x[c,n-k]            (FIR stage)
 *   SOS   dL/d[b0 b1 b2 a1 a2] of every section, summed over channels
 * The FIR adjoint is the correlation gx[n] = sum_k h[k] g[n+k]; the SOS
 * adjoint runs the state-space adjoint recursion of each section in reverse
 * time (lambda_n = A^T lambda_{n+1} + (g_n, 0)), by the same chunked scan as
 * the forward with the transition transposed.  Section signals are rebuilt
 * tile by tile from the forward's checkpoints `ckpt` (the tile-entering
 * states written by the forward call with the same x, coefficients and
 * state_in), so nothing is stored per sample.  Coefficient gradients are
 * summed in fp32 within a chunk and over 16 neighbouring chunks, then in FP64,
 * always in a fixed order (bit-identical from run to run); gradient
 * buffers are overwritten, not accumulated into.  The gradient with respect
 * to state_in is not produced.
 * Limits: at most 16 sections in the cascade (TFX_E_UNSUPPORTED beyond). */
tfx_status tfx_chain_backward_workspace_size(int64_t C, int64_t N, const tfx_stage *stages,
                                             int32_t nstages, tfx_compute cmp, size_t *bytes);
/* grads: NULL (no coefficient gradients) or a host array of nstages device
 * pointers, grads[i] shaped like stages[i].coef (NULL entries are skipped). */
tfx_status tfx_chain_backward(const float *x, const float *gy, float *gx, int64_t C, int64_t N,
                              int64_t ldx, int64_t ldg, int64_t ldgx, const tfx_stage *stages,
                              int32_t nstages, tfx_compute cmp, const float *ckpt,
                              float *const *grads, void *ws, size_t ws_bytes, void *stream);

tfx_status tfx_fir_backward_workspace_size(int64_t C, int64_t N, int32_t M, tfx_compute cmp,
                                           tfx_fir_algo algo, size_t *bytes);
/* gh: NULL or [M] device buffer for dL/dh. */
tfx_status tfx_fir_backward(const float *x, const float *gy, float *gx, int64_t C, int64_t N,
                            int64_t ldx, int64_t ldg, int64_t ldgx, const float *h, int32_t M,
                            float *gh, tfx_compute cmp, tfx_fir_algo algo, void *ws,
                            size_t ws_bytes, void *stream);

tfx_status tfx_sos_backward_workspace_size(int64_t C, int64_t N, int32_t S, size_t *bytes);
/* ckpt: from the forward tfx_sos call (required when S > 0).  gsos: NULL or
 * [S][5] device buffer. */
tfx_status tfx_sos_backward(const float *x, const float *gy, float *gx, int64_t C, int64_t N,
                            int64_t ldx, int64_t ldg, int64_t ldgx, const float *sos, int32_t S,
                            const float *ckpt, float *gsos, void *ws, size_t ws_bytes,
                            void *stream);

/* ------------------------------------------------------------------ STFT */

/* Short-time Fourier transform, one of the signal-processing functions on
 * the roadmap of Sec. 5 (the textbook definition; the paper gives none):
 *
 *   X[c,t,k] = scale * sum_{n<n_fft} w[n] xp[c, t*hop + n] exp(-2 pi i k n / n_fft),
 *   k = 0 .. n_fft/2,   t = 0 .. T-1,
 *
 * xp = x, or with `center` x padded by n_fft/2 reflected samples on each
 * side (xp[-j] = x[j], xp[N-1+j] = x[N-1-j]); w = `window` (win_length
 * samples, or ones when window is NULL) placed in the middle of the frame
 * (offset (n_fft - win_length)/2, zeros elsewhere); scale = 1, or
 * n_fft^-1/2 with `normalized`.  T = 1 + (Np - n_fft)/hop (floor) with Np the
 * padded length (T = 0 when Np < n_fft: nothing is written).  These are the
 * conventions of torch.stft(onesided=True, pad_mode="reflect").
 *
 * n_fft: a power of two in [16, 4096] (TFX_E_UNSUPPORTED otherwise);
 * hop >= 1; 1 <= win_length <= n_fft; with `center`, N > n_fft/2.
 * x: [C][N] fp32, row stride ldx.  spec: [C][T][n_fft/2+1] complex as
 * interleaved (re, im) fp32, frame-major (contiguous; spec must not overlap
 * x).  Two frames share one complex FFT in LDS; no workspace. */
tfx_status tfx_stft_frames(int64_t N, int32_t n_fft, int32_t hop, int32_t center, int64_t *T);
tfx_status tfx_stft(const float *x, int64_t C, int64_t N, int64_t ldx, int32_t n_fft, int32_t hop,
                    const float *window, int32_t win_length, int32_t center, int32_t normalized, float *spec,
                    void *stream);

/* Inverse by weighted overlap-add (torch.istft's conventions):
 *   y[c, s] = sum_t w[p - t*hop] f_t[p - t*hop] / sum_t w[p - t*hop]^2,
 *   p = s + (center ? n_fft/2 : 0),
 * f_t = the real inverse DFT of spec[c,t,:] (imaginary parts of bins 0 and
 * n_fft/2 ignored), times n_fft^1/2 with `normalized`; the sums run over
 * the frames covering p.  length < 0 selects every covered sample less the
 * centre padding (n_fft + hop*(T-1) - 2*(n_fft/2 if center)); samples past
 * the covered range, and samples whose summed squared window is <= 1e-11,
 * are written as 0 (callers that need torch's error on a vanishing
 * envelope check the window themselves).  spec: [C][T][n_fft/2+1] complex,
 * T >= 1; y: [C][length], row stride ldy, not overlapping spec; length <
 * 2^38.  Each workgroup owns a segment of output samples, inverts the frames
 * that touch it and accumulates them in LDS, so nothing but y is written and
 * no workspace is needed. */
tfx_status tfx_istft(const float *spec, int64_t C, int64_t T, int32_t n_fft, int32_t hop, const float *window,
                     int32_t win_length, int32_t center, int32_t normalized, float *y, int64_t length, int64_t ldy,
                     void *stream);

/* ------------------------------------------------------------------- FFT */

/* Batched real FFT, the other transform on the roadmap of Sec. 5 (textbook
 * definition, numpy.fft.rfft / irfft conventions):
 *
 *   X[b,k] = sum_{m<n} x[b,m] exp(-2 pi i k m / n),  k = 0 .. n/2,
 *   y[b,m] = (1/n) (X[b,0] + X[b,n/2] (-1)^m
 *                   + 2 Re sum_{k=1}^{n/2-1} X[b,k] exp(+2 pi i k m / n)),
 *
 * the imaginary parts of bins 0 and n/2 ignored by the inverse.  n: a power
 * of two in [16, 4096] (TFX_E_UNSUPPORTED otherwise).  x / y: B rows of n
 * fp32 samples, row stride ldx / ldy >= n.  spec: [B][n/2+1] complex as
 * interleaved (re, im) fp32, contiguous, not overlapping x or y.  Both run
 * the STFT kernels with one rectangular frame per row (two rows share one
 * complex FFT when the rows are contiguous, ld == n); no workspace.  B == 0 is
 * a no-op. */
tfx_status tfx_rfft(const float *x, int64_t B, int32_t n, int64_t ldx, float *spec, void *stream);
tfx_status tfx_irfft(const float *spec, int64_t B, int32_t n, float *y, int64_t ldy, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TFX_H */
