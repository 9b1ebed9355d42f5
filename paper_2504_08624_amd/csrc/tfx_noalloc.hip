// tfx_noalloc.hip -- tfx_chain on a library-owned device scratch array, for
// callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid allocation).
//
// The array below is a file-scope device variable: every GPU the library
// runs on holds its own copy, at its own address, until the process ends.
// Host code never passes the array's name to a kernel (on the host that name
// is a stand-in, not a device address); the address of the current device's
// copy is looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "tfx.h"
#include "tfx_internal.h"

namespace {

constexpr size_t SCRATCH_BYTES = TFX_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device, with that device current).
tfx_status scratch_ptr(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return tfx::set_error(TFX_E_HIP, "hipGetDevice failed");
    if (dev < 0 || dev >= MAX_DEVICES) return tfx::set_error(TFX_E_UNSUPPORTED, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return tfx::set_error(TFX_E_HIP, "hipGetSymbolAddress(scratch) failed");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return TFX_OK;
}

}  // namespace

extern "C" {

tfx_status tfx_chain_noalloc(const float *x, float *y, int64_t C, int64_t N, int64_t ldx, int64_t ldy,
                             const tfx_stage *stages, int32_t nstages, tfx_compute cmp, float *ckpt, uint32_t *flags,
                             void *stream) {
    size_t need = 0;
    tfx_status s = tfx_chain_workspace_size(C, N, stages, nstages, cmp, &need);
    if (s) return s;
    if (need > SCRATCH_BYTES) {
        char msg[256];
        snprintf(msg, sizeof(msg),
                 "tfx_chain_noalloc: this call needs a %zu-byte workspace, more than the library's %zu-byte scratch "
                 "array; use tfx_chain with a caller-owned workspace",
                 need, SCRATCH_BYTES);
        return tfx::set_error(TFX_E_WORKSPACE, msg);
    }
    void *ws = nullptr;
    if ((s = scratch_ptr(&ws))) return s;
    if ((s = tfx_chain(x, y, C, N, ldx, ldy, stages, nstages, cmp, ckpt, ws, SCRATCH_BYTES, stream))) return s;
    // a call that needed no workspace did not write the array's header
    return (flags && need >= 256) ? tfx_workspace_status(ws, SCRATCH_BYTES, flags, 1, stream) : TFX_OK;
}

}  // extern "C"
