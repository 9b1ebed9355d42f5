// tfx_tune.cpp -- the FIR algorithm tuner and its cache.
//
// Several FIR forms compute the same convolution (direct, overlap-save with
// 4096- or 16384-point FFTs, the matrix-core Toeplitz product in bf16 / fp16 /
// split bf16); which one is fastest depends on the tap count, the signal
// shape and the chip, and the low-precision forms are only admissible when
// the caller's error tolerance allows them.  tfx_fir_autotune times every
// admissible form on the caller's own buffers with HIP events and records the
// fastest in a process-wide cache keyed by (device architecture, M, C,
// floor(log2 N), tolerance class); TFX_FIR_AUTO with fp32 operands then takes
// the cached form for FIR-only calls.  tfx_set_tuning_cache makes the cache
// persistent in a text file (one entry per line, rewritten whole through a
// temporary file and a rename after every new entry).
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "tfx.h"
#include "tfx_internal.h"

namespace {

// Stated accuracy of each form (per-channel relative RMS error bound the
// library holds it to): fp32 FIR 1e-5, split bf16 1e-4, bf16 / fp16 1e-2.
struct Candidate {
    tfx_fir_algo algo;
    tfx_compute cmp;
    double stated;
};
constexpr Candidate CANDIDATES[] = {
    {TFX_FIR_DIRECT, TFX_COMPUTE_F32, 1e-5},    {TFX_FIR_FFT, TFX_COMPUTE_F32, 1e-5},
    {TFX_FIR_FFT16K, TFX_COMPUTE_F32, 1e-5},    {TFX_FIR_TOEPLITZ, TFX_COMPUTE_BF16X3, 1e-4},
    {TFX_FIR_TOEPLITZ, TFX_COMPUTE_F16, 1e-2},  {TFX_FIR_TOEPLITZ, TFX_COMPUTE_BF16, 1e-2},
};

// Tolerance class: the loosest stated accuracy the tolerance admits.
int tol_class(double tol) {
    if (tol >= 1e-2) return 2;
    if (tol >= 1e-4) return 1;
    if (tol >= 1e-5) return 0;
    return -1;
}

bool admissible(const Candidate &c, int32_t M, int cls) {
    if (cls < 0) return false;
    const double bound = cls == 2 ? 1e-2 : (cls == 1 ? 1e-4 : 1e-5);
    if (c.stated > bound) return false;
    if (c.algo == TFX_FIR_FFT16K && M > tfx::FFT16_MAX_TAPS) return false;
    return true;
}

int nlog2(int64_t N) {
    int l = 0;
    while (N > 1) {
        N >>= 1;
        ++l;
    }
    return l;
}

using Key = std::tuple<std::string, int32_t, int64_t, int32_t, int32_t>;  // arch, M, C, log2 N, tol class
struct Entry {
    int32_t algo, cmp;
    float ms;
};

std::mutex g_mu;
std::map<Key, Entry> g_cache;
std::string g_path;

// Architecture name of the current device ("" when there is none).
std::string device_arch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return std::string();
    static std::mutex mu;
    static std::map<int, std::string> names;
    std::lock_guard<std::mutex> lk(mu);
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return std::string();
    std::string a(p.gcnArchName);
    const size_t colon = a.find(':');
    if (colon != std::string::npos) a.resize(colon);
    a += "/" + std::to_string(p.multiProcessorCount) + "cu";
    names[dev] = a;
    return a;
}

bool save_locked(std::string *err) {
    if (g_path.empty()) return true;
    const std::string tmp = g_path + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) {
        *err = "cannot write " + tmp;
        return false;
    }
    fprintf(f, "# libtfx FIR tuning cache: fir <arch> <M> <C> <floor log2 N> <tol class> <algo> <compute> <ms>\n");
    for (const auto &kv : g_cache) {
        const Key &k = kv.first;
        fprintf(f, "fir %s %d %lld %d %d %d %d %.6g\n", std::get<0>(k).c_str(), std::get<1>(k),
                (long long)std::get<2>(k), std::get<3>(k), std::get<4>(k), kv.second.algo, kv.second.cmp,
                (double)kv.second.ms);
    }
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), g_path.c_str()) != 0) {
        *err = "cannot replace " + g_path;
        return false;
    }
    return true;
}

bool valid_entry(int32_t M, long long C, int lg, int cls, int algo, int cmp) {
    if (M < 1 || M > tfx::MAX_TAPS || C < 1 || lg < 0 || lg > 40 || cls < 0 || cls > 2) return false;
    for (const Candidate &c : CANDIDATES)
        if ((int)c.algo == algo && (int)c.cmp == cmp) return admissible(c, M, cls);
    return false;
}

}  // namespace

namespace tfx {

// Cached FIR form for an AUTO call (fp32 operands only reach class 0).
bool tuned_fir_algo(int32_t M, int64_t C, int64_t N, int32_t *algo, int32_t *cmp) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_cache.empty()) return false;
    const int lg = nlog2(N > 0 ? N : 1);
    const std::string arch = device_arch();
    for (const std::string &a : {arch, std::string("*")}) {
        if (a.empty()) continue;
        auto it = g_cache.find(Key(a, M, C, lg, 0));
        if (it != g_cache.end()) {
            *algo = it->second.algo;
            *cmp = it->second.cmp;
            return true;
        }
    }
    return false;
}

}  // namespace tfx

extern "C" {

tfx_status tfx_set_tuning_cache(const char *path) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_path = path ? std::string(path) : std::string();
    if (g_path.empty()) return TFX_OK;
    FILE *f = fopen(g_path.c_str(), "r");
    if (!f) return TFX_OK;  // created by the first tuning run
    char line[512];
    int bad = 0;
    while (fgets(line, sizeof(line), f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        char arch[128];
        int M, lg, cls, algo, cmp;
        long long C;
        float ms;
        if (sscanf(line, "fir %127s %d %lld %d %d %d %d %f", arch, &M, &C, &lg, &cls, &algo, &cmp, &ms) != 8 ||
            !valid_entry(M, C, lg, cls, algo, cmp)) {
            ++bad;
            continue;
        }
        g_cache[Key(arch, M, C, lg, cls)] = Entry{algo, cmp, ms};
    }
    fclose(f);
    if (bad) {
        char msg[160];
        snprintf(msg, sizeof(msg), "%d malformed line(s) in the tuning cache %s were skipped", bad, g_path.c_str());
        return tfx::set_error(TFX_E_INVALID_ARG, msg);
    }
    return TFX_OK;
}

tfx_status tfx_fir_tuned(int64_t C, int64_t N, int32_t M, double tol, tfx_fir_algo *algo, tfx_compute *cmp) {
    if (!algo || !cmp) return tfx::set_error(TFX_E_INVALID_ARG, "algo and cmp must be non-null");
    const int cls = tol_class(tol);
    if (cls < 0) return tfx::set_error(TFX_E_UNSUPPORTED, "no FIR form is held to a tolerance below 1e-5");
    std::lock_guard<std::mutex> lk(g_mu);
    const std::string arch = device_arch();
    for (const std::string &a : {arch, std::string("*")}) {
        if (a.empty()) continue;
        auto it = g_cache.find(Key(a, M, C, nlog2(N > 0 ? N : 1), cls));
        if (it != g_cache.end()) {
            *algo = (tfx_fir_algo)it->second.algo;
            *cmp = (tfx_compute)it->second.cmp;
            return TFX_OK;
        }
    }
    *algo = TFX_FIR_AUTO;
    *cmp = TFX_COMPUTE_F32;
    return TFX_OK;
}

tfx_status tfx_fir_autotune_workspace_size(int64_t C, int64_t N, int32_t M, double tol, size_t *bytes) {
    if (!bytes) return tfx::set_error(TFX_E_INVALID_ARG, "bytes is NULL");
    const int cls = tol_class(tol);
    if (cls < 0) return tfx::set_error(TFX_E_UNSUPPORTED, "no FIR form is held to a tolerance below 1e-5");
    size_t m = 0;
    for (const Candidate &c : CANDIDATES) {
        if (!admissible(c, M, cls)) continue;
        size_t b = 0;
        tfx_status s = tfx_fir_workspace_size(C, N, M, c.cmp, c.algo, &b);
        if (s) return s;
        m = b > m ? b : m;
    }
    *bytes = m;
    return TFX_OK;
}

tfx_status tfx_fir_autotune(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                            const float *h, int32_t M, double tol, int32_t reps, void *ws, size_t ws_bytes,
                            void *stream, tfx_fir_algo *best_algo, tfx_compute *best_cmp, float *best_ms) {
    if (!best_algo || !best_cmp) return tfx::set_error(TFX_E_INVALID_ARG, "best_algo and best_cmp must be non-null");
    if (reps < 1 || reps > 1000) return tfx::set_error(TFX_E_INVALID_ARG, "reps must be in [1, 1000]");
    const int cls = tol_class(tol);
    if (cls < 0) return tfx::set_error(TFX_E_UNSUPPORTED, "no FIR form is held to a tolerance below 1e-5");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess)
        return tfx::set_error(TFX_E_HIP, "hipStreamIsCapturing failed");
    if (cs != hipStreamCaptureStatusNone)
        return tfx::set_error(TFX_E_CAPTURE, "tfx_fir_autotune synchronises the stream and cannot run while it is "
                                             "being captured");
    size_t need = 0;
    tfx_status s = tfx_fir_autotune_workspace_size(C, N, M, tol, &need);
    if (s) return s;
    if (need > ws_bytes) {
        char msg[160];
        snprintf(msg, sizeof(msg), "the tuner needs a %zu-byte workspace (got %zu)", need, ws_bytes);
        return tfx::set_error(TFX_E_WORKSPACE, msg);
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return tfx::set_error(TFX_E_HIP, "hipEventCreate failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return tfx::set_error(TFX_E_HIP, "hipEventCreate failed");
    }
    float bms = -1.f;
    Candidate best{};
    for (const Candidate &c : CANDIDATES) {
        if (!admissible(c, M, cls)) continue;
        // one untimed call (with its own prepare), timed alone to prune forms
        // more than four times slower than the best so far
        float ms = 0.f;
        if (hipEventRecord(e0, st) != hipSuccess) { s = tfx::set_error(TFX_E_HIP, "hipEventRecord failed"); break; }
        if ((s = tfx_fir(x, y, C, N, ldx, ldy, h, M, c.cmp, c.algo, ws, ws_bytes, stream))) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            s = tfx::set_error(TFX_E_HIP, "timing failed");
            break;
        }
        if (bms >= 0.f && ms > 4.f * bms) continue;
        if (hipEventRecord(e0, st) != hipSuccess) { s = tfx::set_error(TFX_E_HIP, "hipEventRecord failed"); break; }
        for (int r = 0; r < reps && !s; ++r) s = tfx_fir(x, y, C, N, ldx, ldy, h, M, c.cmp, c.algo, ws, ws_bytes, stream);
        if (s) break;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            s = tfx::set_error(TFX_E_HIP, "timing failed");
            break;
        }
        ms /= reps;
        if (bms < 0.f || ms < bms) {
            bms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s) return s;
    *best_algo = best.algo;
    *best_cmp = best.cmp;
    if (best_ms) *best_ms = bms;
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[Key(device_arch(), M, C, nlog2(N > 0 ? N : 1), cls)] = Entry{best.algo, best.cmp, bms};
    std::string err;
    if (!save_locked(&err)) return tfx::set_error(TFX_E_INVALID_ARG, err.c_str());
    return TFX_OK;
}

}  // extern "C"
