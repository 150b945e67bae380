// wrs_api.hip -- host side of the C ABI declared in include/wrs.h.
#include <stdarg.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "wrs_internal.h"

namespace wrs {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

static int dev_fail(const char* what, hipError_t e) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return WRS_EDEVICE;
}

static constexpr int64_t N_MAX = 2147483647LL;

}  // namespace wrs

using namespace wrs;

extern "C" const char* wrs_last_error(void) { return g_err; }

extern "C" size_t wrs_workspace_bytes(int op, int64_t n, int64_t k) {
    if (n < 1 || n > N_MAX || k < 0) return 0;
    if (op == WRS_OP_BUILD) return build_ws_bytes(n);
    if (op == WRS_OP_BUILD_PLUS) return plus_ws_bytes(n);
    if (op == WRS_OP_PERM) return perm_ws_bytes(n);
    if (op == WRS_OP_TWOLEVEL) return twolevel_ws_bytes(n);
    if (op == WRS_OP_WOR) return wor_ws_bytes(n, k);
    if (op == WRS_OP_OS) return k <= N_MAX ? os_ws_bytes(n, k) : 0;
    return 0;
}

extern "C" int wrs_alias_build(const float* d_w, int64_t n, wrs_entry* d_table, void* d_ws, size_t ws_bytes,
                               void* stream) {
    g_err[0] = 0;
    if (!d_w || !d_table || !d_ws) { set_error("wrs_alias_build: null pointer"); return WRS_EINVAL; }
    if (n < 1 || n > N_MAX) { set_error("wrs_alias_build: n = %lld out of [1, 2^31-1]", (long long)n); return WRS_EINVAL; }
    if (ws_bytes < build_ws_bytes(n)) { set_error("wrs_alias_build: workspace %zu < %zu bytes", ws_bytes, build_ws_bytes(n)); return WRS_EINVAL; }
    if (((uintptr_t)d_ws) & 255) { set_error("wrs_alias_build: workspace not 256-byte aligned"); return WRS_EINVAL; }
    if (((uintptr_t)d_table) & 7) { set_error("wrs_alias_build: table not 8-byte aligned"); return WRS_EINVAL; }
    JobTable jt;
    memset(&jt, 0, sizeof jt);
    JobDesc& J = jt.one;
    J.w = d_w;
    J.table = d_table;
    build_ws_layout(J, d_ws, n);
    int64_t blocks[PH_COUNT];
    phase_blocks(J, blocks);
    hipError_t e = launch_build(jt, blocks, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail("wrs_alias_build launch", e);
    return WRS_OK;
}

extern "C" int wrs_alias_build_plus(const float* d_w, int64_t n, wrs_entry* d_table, void* d_ws, size_t ws_bytes,
                                    void* stream) {
    g_err[0] = 0;
    if (!d_w || !d_table || !d_ws) { set_error("wrs_alias_build_plus: null pointer"); return WRS_EINVAL; }
    if (n < 1 || n > N_MAX) { set_error("wrs_alias_build_plus: n = %lld out of [1, 2^31-1]", (long long)n); return WRS_EINVAL; }
    if (ws_bytes < plus_ws_bytes(n)) { set_error("wrs_alias_build_plus: workspace %zu < %zu bytes", ws_bytes, plus_ws_bytes(n)); return WRS_EINVAL; }
    if (((uintptr_t)d_ws) & 255) { set_error("wrs_alias_build_plus: workspace not 256-byte aligned"); return WRS_EINVAL; }
    if (((uintptr_t)d_table) & 7) { set_error("wrs_alias_build_plus: table not 8-byte aligned"); return WRS_EINVAL; }
    const hipStream_t st = (hipStream_t)stream;
    // stage 0: total weight and grid (the reduction phases only)
    JobTable jt;
    memset(&jt, 0, sizeof jt);
    JobDesc& J = jt.one;
    J.w = d_w;
    J.table = d_table;
    build_ws_layout(J, d_ws, n);
    int64_t blocks[PH_COUNT];
    phase_blocks(J, blocks);
    for (int p = PH_TILE; p < PH_COUNT; ++p) blocks[p] = 0;
    hipError_t e = launch_build(jt, blocks, st);
    if (e != hipSuccess) return dev_fail("wrs_alias_build_plus launch", e);
    // stage 1: greedy blocks, their leftovers compacted into a list
    const PlusLayout P = plus_layout(d_ws, n);
    e = launch_greedy(J, P, st);
    if (e != hipSuccess) return dev_fail("wrs_alias_build_plus greedy launch", e);
    BuildScalars h;
    e = hipMemcpyAsync(&h, J.sc, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_fail("wrs_alias_build_plus leftover count", e);
    if (h.status != WRS_OK || h.nleft <= 0) return WRS_OK;  // status stays in the workspace
    if (h.nleft > n) { set_error("wrs_alias_build_plus: leftover count %lld > n", (long long)h.nleft); return WRS_EDEVICE; }
    // stage 2: the splitting construction over the list
    JobTable jl;
    memset(&jl, 0, sizeof jl);
    JobDesc& L = jl.one;
    L = J;
    L.w = P.lw;
    L.lidx = P.lidx;
    L.lres = P.res;
    L.PI = P.PI;
    build_list_layout(L, h.nleft);
    phase_blocks(L, blocks);
    e = launch_build(jl, blocks, st, true);
    if (e != hipSuccess) return dev_fail("wrs_alias_build_plus list launch", e);
    return WRS_OK;
}

extern "C" int wrs_permutation(const float* d_w, int64_t n, uint64_t seed, uint32_t stream_id, int32_t* d_out,
                               void* d_ws, size_t ws_bytes, void* stream) {
    g_err[0] = 0;
    if (!d_w || !d_out || !d_ws) { set_error("wrs_permutation: null pointer"); return WRS_EINVAL; }
    if (n < 1 || n > N_MAX) { set_error("wrs_permutation: n = %lld out of [1, 2^31-1]", (long long)n); return WRS_EINVAL; }
    if (ws_bytes < perm_ws_bytes(n)) { set_error("wrs_permutation: workspace %zu < %zu bytes", ws_bytes, perm_ws_bytes(n)); return WRS_EINVAL; }
    if (((uintptr_t)d_ws) & 255) { set_error("wrs_permutation: workspace not 256-byte aligned"); return WRS_EINVAL; }
    if (((uintptr_t)d_out) & 3) { set_error("wrs_permutation: output not 4-byte aligned"); return WRS_EINVAL; }
    const int e = launch_perm(d_w, n, seed, stream_id, d_out, d_ws, (hipStream_t)stream);
    if (e != 0) return dev_fail("wrs_permutation launch", (hipError_t)e);
    return WRS_OK;
}

extern "C" size_t wrs_os_bytes(int64_t n) { return (n < 1 || n > N_MAX) ? 0 : os_bytes(n); }

extern "C" int wrs_os_build(const float* d_w, int64_t n, void* d_os, size_t os_bytes_, void* d_ws, size_t ws_bytes,
                            void* stream) {
    g_err[0] = 0;
    if (!d_w || !d_os || !d_ws) { set_error("wrs_os_build: null pointer"); return WRS_EINVAL; }
    if (n < 1 || n > N_MAX) { set_error("wrs_os_build: n = %lld out of [1, 2^31-1]", (long long)n); return WRS_EINVAL; }
    if (os_bytes_ < os_bytes(n)) { set_error("wrs_os_build: structure %zu < %zu bytes", os_bytes_, os_bytes(n)); return WRS_EINVAL; }
    if (ws_bytes < os_ws_bytes(n, 0)) { set_error("wrs_os_build: workspace %zu < %zu bytes", ws_bytes, os_ws_bytes(n, 0)); return WRS_EINVAL; }
    if ((((uintptr_t)d_os) | ((uintptr_t)d_ws)) & 255) { set_error("wrs_os_build: structure or workspace not 256-byte aligned"); return WRS_EINVAL; }
    const int e = launch_os_build(d_w, n, d_os, d_ws, (hipStream_t)stream);
    if (e != 0) return dev_fail("wrs_os_build launch", (hipError_t)e);
    return WRS_OK;
}

extern "C" int wrs_os_sample(const void* d_os, int64_t n, int64_t k, uint64_t seed, int32_t* d_items,
                             int32_t* d_counts, int64_t* d_s, void* d_ws, size_t ws_bytes, void* stream) {
    g_err[0] = 0;
    if (!d_os || !d_s || !d_ws || (k > 0 && (!d_items || !d_counts))) { set_error("wrs_os_sample: null pointer"); return WRS_EINVAL; }
    if (n < 1 || n > N_MAX) { set_error("wrs_os_sample: n = %lld out of [1, 2^31-1]", (long long)n); return WRS_EINVAL; }
    if (k < 0 || k > N_MAX) { set_error("wrs_os_sample: k = %lld out of [0, 2^31-1]", (long long)k); return WRS_EINVAL; }
    if (ws_bytes < os_ws_bytes(n, k)) { set_error("wrs_os_sample: workspace %zu < %zu bytes", ws_bytes, os_ws_bytes(n, k)); return WRS_EINVAL; }
    if ((((uintptr_t)d_os) | ((uintptr_t)d_ws)) & 255) { set_error("wrs_os_sample: structure or workspace not 256-byte aligned"); return WRS_EINVAL; }
    if ((((uintptr_t)d_items) | ((uintptr_t)d_counts)) & 3 || ((uintptr_t)d_s) & 7) { set_error("wrs_os_sample: outputs misaligned"); return WRS_EINVAL; }
    const int e = launch_os_sample(d_os, n, k, seed, d_items, d_counts, d_s, d_ws, (hipStream_t)stream);
    if (e != 0) return dev_fail("wrs_os_sample launch", (hipError_t)e);
    return WRS_OK;
}

extern "C" int wrs_twolevel_build(const float* d_w, int64_t n, wrs_entry* d_table, wrs_entry* d_top, void* d_ws,
                                  size_t ws_bytes, void* stream) {
    g_err[0] = 0;
    if (!d_w || !d_table || !d_top || !d_ws) { set_error("wrs_twolevel_build: null pointer"); return WRS_EINVAL; }
    if (n < 1 || n > N_MAX) { set_error("wrs_twolevel_build: n = %lld out of [1, 2^31-1]", (long long)n); return WRS_EINVAL; }
    if (ws_bytes < twolevel_ws_bytes(n)) { set_error("wrs_twolevel_build: workspace %zu < %zu bytes", ws_bytes, twolevel_ws_bytes(n)); return WRS_EINVAL; }
    if (((uintptr_t)d_ws) & 255) { set_error("wrs_twolevel_build: workspace not 256-byte aligned"); return WRS_EINVAL; }
    if ((((uintptr_t)d_table) | ((uintptr_t)d_top)) & 7) { set_error("wrs_twolevel_build: tables not 8-byte aligned"); return WRS_EINVAL; }
    const hipStream_t st = (hipStream_t)stream;
    JobTable jt;
    memset(&jt, 0, sizeof jt);
    JobTable jtop;
    memset(&jtop, 0, sizeof jtop);
    TwoLayout T;
    JobDesc& J = jt.one;
    JobDesc& L = jtop.one;
    twolevel_layout(d_ws, n, J, L, T);
    J.w = d_w;
    J.table = d_table;
    L.table = d_top;
    // total weight and grid (the reduction phases of the main job)
    int64_t blocks[PH_COUNT];
    phase_blocks(J, blocks);
    for (int p = PH_TILE; p < PH_COUNT; ++p) blocks[p] = 0;
    hipError_t e = launch_build(jt, blocks, st);
    // the top job's scalars (n = G meta-items) on the items' grid: its sizes,
    // G times the blocks' exact sums, are integers of that grid
    if (e == hipSuccess) e = launch_finalize_on_grid(L, J.sc, st);
    // block tables and meta-items, then the top table (list mode)
    if (e == hipSuccess) e = launch_twolvl(J, T, st);
    if (e == hipSuccess) {
        phase_blocks(L, blocks);
        e = launch_build(jtop, blocks, st, true);
    }
    if (e != hipSuccess) return dev_fail("wrs_twolevel_build launch", e);
    return WRS_OK;
}

extern "C" int wrs_twolevel_sample(const wrs_entry* d_top, const wrs_entry* d_table, int64_t n, uint64_t seed,
                                   uint32_t stream_id, uint64_t first_counter, int64_t k, int32_t* d_out,
                                   void* stream) {
    g_err[0] = 0;
    if (!d_top || !d_table || (k > 0 && !d_out)) { set_error("wrs_twolevel_sample: null pointer"); return WRS_EINVAL; }
    if (n < 1 || n > N_MAX || k < 0) { set_error("wrs_twolevel_sample: bad n or k"); return WRS_EINVAL; }
    if (cdiv(k, 256 * 4) > 0x7fffffffLL) { set_error("wrs_twolevel_sample: k too large"); return WRS_EINVAL; }
    if ((((uintptr_t)d_table) | ((uintptr_t)d_top)) & 7) { set_error("wrs_twolevel_sample: tables not 8-byte aligned"); return WRS_EINVAL; }
    const hipError_t e = launch_sample2(d_top, d_table, n, seed, stream_id, first_counter, k, d_out, (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail("wrs_twolevel_sample launch", e);
    return WRS_OK;
}

extern "C" int wrs_plus_leftovers(const void* d_ws, void* stream, int64_t* nleft) {
    g_err[0] = 0;
    if (!d_ws || !nleft) { set_error("wrs_plus_leftovers: null pointer"); return WRS_EINVAL; }
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipMemcpy(nleft, (const char*)d_ws + offsetof(BuildScalars, nleft), sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_fail("wrs_plus_leftovers", e);
    return WRS_OK;
}

extern "C" int wrs_alias_sample(const wrs_entry* d_table, int64_t n, uint64_t seed, uint32_t stream_id,
                                uint64_t first_counter, int64_t k, int32_t* d_out, void* stream) {
    g_err[0] = 0;
    if (!d_table || (k > 0 && !d_out)) { set_error("wrs_alias_sample: null pointer"); return WRS_EINVAL; }
    if (n < 1 || n > N_MAX || k < 0) { set_error("wrs_alias_sample: bad n or k"); return WRS_EINVAL; }
    if (((uintptr_t)d_table) & 7) { set_error("wrs_alias_sample: table not 8-byte aligned"); return WRS_EINVAL; }
    if (k == 0) return WRS_OK;
    JobTable jt;
    memset(&jt, 0, sizeof jt);
    JobDesc& J = jt.one;
    set_sample_job(J, k);
    if (sample_blocks(J) > 0x7fffffffLL) { set_error("wrs_alias_sample: k too large"); return WRS_EINVAL; }
    J.table = const_cast<wrs_entry*>(d_table);
    J.n = n;
    J.seed = seed;
    J.stream_id = stream_id;
    J.first_counter = first_counter;
    J.out = d_out;
    J.sc = nullptr;
    hipError_t e = launch_sample(jt, sample_blocks(J), (hipStream_t)stream);
    if (e != hipSuccess) return dev_fail("wrs_alias_sample launch", e);
    return WRS_OK;
}

extern "C" int wrs_sample_wor(const float* d_w, int64_t n, int64_t k, uint64_t seed, uint32_t stream_id,
                              int32_t* d_out, void* d_ws, size_t ws_bytes, void* stream) {
    g_err[0] = 0;
    if (!d_w || !d_ws || (k > 0 && !d_out)) { set_error("wrs_sample_wor: null pointer"); return WRS_EINVAL; }
    if (n < 1 || n > N_MAX || k < 0) { set_error("wrs_sample_wor: bad n or k"); return WRS_EINVAL; }
    if (k > n) { set_error("wrs_sample_wor: k > n"); return WRS_EDOMAIN; }
    if (ws_bytes < wor_ws_bytes(n, k)) { set_error("wrs_sample_wor: workspace too small"); return WRS_EINVAL; }
    if (((uintptr_t)d_ws) & 255) { set_error("wrs_sample_wor: workspace not 256-byte aligned"); return WRS_EINVAL; }
    if (k == 0) {
        // status word: OK
        int ok = WRS_OK;
        hipError_t e = hipMemcpyAsync((char*)d_ws + wor_status_offset(), &ok, sizeof ok, hipMemcpyHostToDevice,
                                      (hipStream_t)stream);
        if (e != hipSuccess) return dev_fail("wrs_sample_wor", e);
        e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) return dev_fail("wrs_sample_wor", e);
        return WRS_OK;
    }
    int rc = launch_wor(d_w, n, k, seed, stream_id, d_out, d_ws, (hipStream_t)stream);
    if (rc != WRS_OK) return dev_fail("wrs_sample_wor launch", hipGetLastError());
    return WRS_OK;
}

static int read_ws(const void* d_ws, size_t off, void* dst, size_t bytes, void* stream) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return dev_fail("synchronize", e);
    e = hipMemcpy(dst, (const char*)d_ws + off, bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return dev_fail("read workspace", e);
    return WRS_OK;
}

extern "C" int wrs_status(const void* d_ws, void* stream, int* status_out) {
    g_err[0] = 0;
    if (!d_ws || !status_out) { set_error("wrs_status: null pointer"); return WRS_EINVAL; }
    // The build, PSA+, WOR and permutation workspaces all start with their status word.
    int s = 0;
    int rc = read_ws(d_ws, 0, &s, sizeof s, stream);
    if (rc) return rc;
    *status_out = s;
    return WRS_OK;
}

extern "C" int wrs_total_weight(const void* d_ws, void* stream, double* hi, double* lo) {
    g_err[0] = 0;
    if (!d_ws || !hi || !lo) { set_error("wrs_total_weight: null pointer"); return WRS_EINVAL; }
    BuildScalars S;
    int rc = read_ws(d_ws, 0, &S, sizeof S, stream);
    if (rc) return rc;
    *hi = S.W_hi;
    *lo = S.W_lo;
    return WRS_OK;
}

// ---------------------------------------------------------------------------
// Batches.  Workspace: [JobDesc x njobs][offsets PH_COUNT x (njobs+1)]
// [indices of the small jobs x njobs][BuildScalars x njobs][per-job build
// workspaces].  A small job (n <= FUSE_MAX) gets no block in the phase
// launches: the fused launch builds and samples it.
// ---------------------------------------------------------------------------
namespace wrs {

static inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchHeader {
    size_t jobs_off, off_off, small_off, sc_off, data_off, total;
};

static BatchHeader batch_header(int32_t njobs) {
    BatchHeader h;
    size_t o = 0;
    h.jobs_off = o; o = a256(o + sizeof(JobDesc) * njobs);
    h.off_off = o;  o = a256(o + sizeof(int64_t) * PH_COUNT * (njobs + 1));
    h.small_off = o; o = a256(o + sizeof(int32_t) * njobs);
    h.sc_off = o;   o = a256(o + sizeof(BuildScalars) * njobs);
    h.data_off = o;
    h.total = o;
    return h;
}

struct BatchPlan {
    std::vector<char> blob;          // the descriptors the graph's kernels read from the workspace
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    uint64_t last_use = 0;
};

static constexpr size_t MAX_PLANS = 64;  // recorded graphs kept; the least recently used goes first
static std::mutex g_batch_mu;
static std::unordered_map<std::string, BatchPlan*> g_plans;
static uint64_t g_plan_clock = 0;
static bool g_graph_mode = true;
static int32_t g_fuse_max = 0;  // batched jobs with n <= this go to the fused launch

static void destroy_plan(BatchPlan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
}

}  // namespace wrs

extern "C" size_t wrs_batch_workspace_bytes(const wrs_job* h_jobs, int32_t njobs) {
    if (!h_jobs || njobs < 1) return 0;
    BatchHeader h = batch_header(njobs);
    size_t total = h.data_off;
    for (int32_t j = 0; j < njobs; ++j) {
        if (h_jobs[j].n < 1 || h_jobs[j].n > N_MAX) return 0;
        total += a256(build_ws_bytes(h_jobs[j].n));
    }
    return total;
}

extern "C" int wrs_batch_graph_mode(int enable) {
    std::lock_guard<std::mutex> g(g_batch_mu);
    g_graph_mode = enable != 0;
    return WRS_OK;
}

extern "C" int wrs_batch_fuse_small(int32_t max_n) {
    static_assert(WRS_FUSE_MAX_N == FUSE_MAX, "the header's limit is the kernel's LDS table size");
    g_err[0] = 0;
    if (max_n < 0 || max_n > FUSE_MAX) {
        set_error("wrs_batch_fuse_small: max_n = %d out of [0, %d]", (int)max_n, FUSE_MAX);
        return WRS_EINVAL;
    }
    std::lock_guard<std::mutex> g(g_batch_mu);
    g_fuse_max = max_n;
    return WRS_OK;
}

static int batch_record(const wrs_job* h_jobs, int32_t njobs, void* d_ws, hipStream_t st, JobTable& jt,
                        int64_t* totals, std::vector<char>& host_blob, const int32_t** d_small, int32_t* nsmall) {
    BatchHeader h = batch_header(njobs);
    char* base = (char*)d_ws;
    std::vector<JobDesc> descs(njobs);
    std::vector<int64_t> off((size_t)PH_COUNT * (njobs + 1), 0);
    std::vector<int32_t> small;
    size_t o = h.data_off;
    for (int32_t j = 0; j < njobs; ++j) {
        JobDesc& J = descs[j];
        memset(&J, 0, sizeof J);
        J.w = h_jobs[j].d_w;
        J.table = h_jobs[j].d_table;
        J.out = h_jobs[j].d_out;
        set_sample_job(J, h_jobs[j].k);
        J.seed = h_jobs[j].seed;
        J.stream_id = h_jobs[j].stream_id;
        J.first_counter = 0;
        build_ws_layout(J, base + o, h_jobs[j].n);
        o += a256(build_ws_bytes(h_jobs[j].n));
        J.sc = (BuildScalars*)(base + h.sc_off) + j;  // statuses side by side
        int64_t b[PH_COUNT];
        phase_blocks(J, b);
        if (h_jobs[j].n <= g_fuse_max) {
            small.push_back(j);
            for (int p = 0; p < PH_COUNT; ++p) b[p] = 0;
        }
        for (int p = 0; p < PH_COUNT; ++p) off[(size_t)p * (njobs + 1) + j + 1] = off[(size_t)p * (njobs + 1) + j] + b[p];
    }
    for (int p = 0; p < PH_COUNT; ++p) totals[p] = off[(size_t)p * (njobs + 1) + njobs];
    host_blob.assign(h.data_off, 0);
    memcpy(host_blob.data() + h.jobs_off, descs.data(), sizeof(JobDesc) * njobs);
    memcpy(host_blob.data() + h.off_off, off.data(), sizeof(int64_t) * off.size());
    if (!small.empty()) memcpy(host_blob.data() + h.small_off, small.data(), sizeof(int32_t) * small.size());
    *d_small = (const int32_t*)(base + h.small_off);
    *nsmall = (int32_t)small.size();
    memset(&jt, 0, sizeof jt);
    jt.jobs = (const JobDesc*)(base + h.jobs_off);
    jt.off = (const int64_t*)(base + h.off_off);
    jt.njobs = njobs;
    (void)st;
    return WRS_OK;
}

extern "C" int wrs_batch_build_sample(const wrs_job* h_jobs, int32_t njobs, void* d_ws, size_t ws_bytes,
                                      void* stream) {
    g_err[0] = 0;
    if (!h_jobs || njobs < 1 || !d_ws) { set_error("wrs_batch_build_sample: bad arguments"); return WRS_EINVAL; }
    if (((uintptr_t)d_ws) & 255) { set_error("wrs_batch_build_sample: workspace not 256-byte aligned"); return WRS_EINVAL; }
    for (int32_t j = 0; j < njobs; ++j) {
        const wrs_job& q = h_jobs[j];
        if (!q.d_w || !q.d_table || q.n < 1 || q.n > N_MAX || q.k < 0 || (q.k > 0 && !q.d_out)) {
            set_error("wrs_batch_build_sample: job %d invalid", j);
            return WRS_EINVAL;
        }
        if (((uintptr_t)q.d_table) & 7) { set_error("wrs_batch_build_sample: job %d table misaligned", j); return WRS_EINVAL; }
    }
    const size_t need = wrs_batch_workspace_bytes(h_jobs, njobs);
    if (ws_bytes < need) { set_error("wrs_batch_build_sample: workspace %zu < %zu", ws_bytes, need); return WRS_EINVAL; }
    hipStream_t st = (hipStream_t)stream;
    JobTable jt;
    int64_t totals[PH_COUNT];
    std::vector<char> blob;
    const int32_t* d_small = nullptr;
    int32_t nsmall = 0;
    std::lock_guard<std::mutex> g(g_batch_mu);
    batch_record(h_jobs, njobs, d_ws, st, jt, totals, blob, &d_small, &nsmall);
    std::string key((const char*)h_jobs, sizeof(wrs_job) * njobs);
    key.append((const char*)&d_ws, sizeof d_ws);
    const uint64_t gen = tuning_generation();
    key.append((const char*)&gen, sizeof gen);
    key.append((const char*)&g_fuse_max, sizeof g_fuse_max);
    if (g_graph_mode) {
        auto it = g_plans.find(key);
        if (it != g_plans.end()) {
            // The workspace may hold another batch's descriptors since the
            // recording: upload this batch's again, ahead of the replay on the
            // same stream (the plan owns the host copy).
            BatchPlan* plan = it->second;
            plan->last_use = ++g_plan_clock;
            hipError_t e = hipMemcpyAsync(d_ws, plan->blob.data(), plan->blob.size(), hipMemcpyHostToDevice, st);
            if (e != hipSuccess) return dev_fail("upload batch descriptors", e);
            e = hipGraphLaunch(plan->exec, st);
            if (e != hipSuccess) return dev_fail("hipGraphLaunch", e);
            return WRS_OK;
        }
    }
    // Upload descriptors (synchronously: the host blob is temporary).
    hipError_t e = hipMemcpyAsync(d_ws, blob.data(), blob.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return dev_fail("upload batch descriptors", e);
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return dev_fail("upload batch descriptors", e);
    // The small jobs' launch runs beside the phase launches of the others, on
    // a library stream forked from the caller's and joined back (in a recorded
    // graph: a parallel branch).  It holds one workgroup per CU and waits on
    // its own barriers most of the time; alone on the stream it would add its
    // whole duration.
    static hipStream_t side = nullptr;
    static hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    if (nsmall > 0 && !side) {
        e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_join, hipEventDisableTiming);
        if (e != hipSuccess) return dev_fail("create the small-job stream", e);
    }
    auto launch_all = [&]() -> hipError_t {
        hipError_t r = hipSuccess;
        if (nsmall > 0) {
            r = hipEventRecord(ev_fork, st);
            if (r == hipSuccess) r = hipStreamWaitEvent(side, ev_fork, 0);
            if (r == hipSuccess) r = launch_fused_small(jt, d_small, nsmall, side);
            if (r == hipSuccess) r = hipEventRecord(ev_join, side);
            if (r != hipSuccess) return r;
        }
        r = launch_build(jt, totals, st);
        if (r == hipSuccess) r = launch_sample(jt, totals[PH_SAMPLE], st);
        if (r == hipSuccess && nsmall > 0) r = hipStreamWaitEvent(st, ev_join, 0);
        return r;
    };
    if (!g_graph_mode) {
        e = launch_all();
        if (e != hipSuccess) return dev_fail("batch launch", e);
        return WRS_OK;
    }
    // Record on a library stream (the caller's may be the legacy default
    // stream, which cannot be captured), replay on the caller's stream.
    static hipStream_t cap = nullptr;
    if (!cap) {
        e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e != hipSuccess) return dev_fail("create capture stream", e);
    }
    BatchPlan* plan = new BatchPlan();
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) { delete plan; return dev_fail("hipStreamBeginCapture", e); }
    const hipStream_t user_st = st;
    st = cap;
    hipError_t le = launch_all();
    st = user_st;
    e = hipStreamEndCapture(cap, &plan->graph);
    if (le != hipSuccess || e != hipSuccess) { delete plan; return dev_fail("batch capture", le != hipSuccess ? le : e); }
    e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(plan->graph); delete plan; return dev_fail("hipGraphInstantiate", e); }
    plan->blob = std::move(blob);
    plan->last_use = ++g_plan_clock;
    if (g_plans.size() >= MAX_PLANS) {
        // a graph may still run on some stream: wait before destroying one
        auto old = g_plans.begin();
        for (auto i = g_plans.begin(); i != g_plans.end(); ++i)
            if (i->second->last_use < old->second->last_use) old = i;
        e = hipDeviceSynchronize();
        if (e != hipSuccess) { destroy_plan(plan); return dev_fail("batch graph cache", e); }
        destroy_plan(old->second);
        g_plans.erase(old);
    }
    g_plans[key] = plan;
    e = hipGraphLaunch(plan->exec, st);
    if (e != hipSuccess) return dev_fail("hipGraphLaunch", e);
    return WRS_OK;
}

extern "C" int wrs_batch_status(const void* d_ws, int32_t njobs, void* stream, int* h_status) {
    g_err[0] = 0;
    if (!d_ws || njobs < 1 || !h_status) { set_error("wrs_batch_status: bad arguments"); return WRS_EINVAL; }
    BatchHeader h = batch_header(njobs);
    std::vector<BuildScalars> sc(njobs);
    int rc = read_ws(d_ws, h.sc_off, sc.data(), sizeof(BuildScalars) * njobs, stream);
    if (rc) return rc;
    for (int32_t j = 0; j < njobs; ++j) h_status[j] = sc[j].status;
    return WRS_OK;
}
