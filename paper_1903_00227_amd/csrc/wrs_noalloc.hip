// wrs_noalloc.hip -- wrs_alias_build_noalloc: the table construction of
// wrs_alias_build with its workspace in a fixed device array of this library
// instead of caller memory, for callers that cannot allocate.
//
// The array `scratch` is a file-scope device variable: every GPU the library
// runs on holds its own copy, at its own address, until the process ends.  In
// host code its name is only a stand-in, not a device address, so the host
// side never passes it anywhere: on a device's first call it looks up that
// device's address once (hipGetSymbolAddress, with the device current) and
// uses that pointer for every kernel argument.  Every call on one device
// shares the array and leaves the last call's contents in it; the build writes
// every word it later reads, so nothing needs clearing.  Calls that overlap on
// one device (on different streams, or from different threads without an
// ordering between their streams) race on the array.
#include <string.h>

#include <mutex>
#include <vector>

#include "wrs_internal.h"

namespace wrs {

static __device__ __align__(256) unsigned char scratch[WRS_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;  // per device: the address of `scratch`

// Device address of this device's `scratch`, looked up on its first use.
static void* scratch_ptr(int* err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0) {
        *err = (int)e;
        return nullptr;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = (int)(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// The build's status word, copied out for the caller.
__global__ void k_status_out(const BuildScalars* sc, int32_t* d_status) {
    if (threadIdx.x == 0) *d_status = sc->status;
}

}  // namespace wrs

using namespace wrs;

extern "C" int wrs_alias_build_noalloc(const float* d_w, int64_t n, wrs_entry* d_table, int32_t* d_status,
                                       void* stream) {
    clear_error();
    if (!d_w || !d_table) { set_error("wrs_alias_build_noalloc: null pointer"); return WRS_EINVAL; }
    if (n < 1 || n > 2147483647LL) {
        set_error("wrs_alias_build_noalloc: n = %lld out of [1, 2^31-1]", (long long)n);
        return WRS_EINVAL;
    }
    const size_t need = build_ws_bytes(n);  // the layout wrs_alias_build uses
    if (need > (size_t)WRS_NOALLOC_SCRATCH_BYTES) {
        set_error("wrs_alias_build_noalloc: n = %lld needs %zu bytes of workspace, above the %zu-byte scratch array",
                  (long long)n, need, (size_t)WRS_NOALLOC_SCRATCH_BYTES);
        return WRS_EINVAL;
    }
    if (((uintptr_t)d_table) & 7) { set_error("wrs_alias_build_noalloc: table not 8-byte aligned"); return WRS_EINVAL; }
    if (((uintptr_t)d_status) & 3) { set_error("wrs_alias_build_noalloc: status not 4-byte aligned"); return WRS_EINVAL; }
    int err = 0;
    void* ws = scratch_ptr(&err);
    if (!ws) {
        set_error("wrs_alias_build_noalloc: no address for the scratch array: %s", hipGetErrorString((hipError_t)err));
        return WRS_EDEVICE;
    }
    const hipStream_t st = (hipStream_t)stream;
    JobTable jt;
    memset(&jt, 0, sizeof jt);
    JobDesc& J = jt.one;
    J.w = d_w;
    J.table = d_table;
    build_ws_layout(J, ws, n);
    int64_t blocks[PH_COUNT];
    phase_blocks(J, blocks);
    hipError_t e = launch_build(jt, blocks, st);
    if (e == hipSuccess && d_status) {
        hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, st, (const BuildScalars*)J.sc, d_status);
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        set_error("wrs_alias_build_noalloc launch: %s", hipGetErrorString(e));
        return WRS_EDEVICE;
    }
    return WRS_OK;
}
