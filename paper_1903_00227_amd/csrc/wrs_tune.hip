// wrs_tune.hip -- launch-parameter tuning for the build and the sampler.
//
// Two launch parameters are free:
//   - tile events per pack block (4, 8, 16, 32): the merge is cut at tile
//     events and every block recomputes its start state from exact prefix
//     sums, so any split gives the same table;
//   - draws per sampler thread (1, 2, 4, 8): every draw is a function of its
//     counter alone.
// Both change speed only.  Values are kept per device kind (architecture name
// and CU count), operation and size class (ceil(log2 n) for the build,
// ceil(log2 k) for the sampler); a class without an entry takes a default
// derived from the size and the CU count.  Entries come from wrs_autotune
// (timed on the device), wrs_tune_set, or a JSON file (wrs_tune_load, or the
// file named by the environment variable WRS_TUNE_FILE at first use).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "wrs_device.h"

namespace wrs {

namespace {

struct DevInfo {
    std::string arch;
    int cus = 0;
    bool ok = false;
};

using Key = std::tuple<std::string, int, int, int>;  // arch, CUs, op, size class

struct Entry {
    int32_t value;
    double us;  // measured time of the winner (0 if set by hand)
};

std::mutex g_mu;
std::vector<DevInfo> g_dev;
std::map<Key, Entry> g_tab;
bool g_env_loaded = false;

const int32_t kBuildCand[] = {4, 8, 16, 32};
const int32_t kSampleCand[] = {1, 2, 4, 8};

bool valid_value(int op, int32_t v) {
    const int32_t* c = op == WRS_TUNE_BUILD ? kBuildCand : kSampleCand;
    for (int i = 0; i < 4; ++i)
        if (c[i] == v) return true;
    return false;
}

int size_class(int64_t x) {
    int c = 0;
    while (c < 62 && (int64_t(1) << c) < x) ++c;
    return c;
}

// caller holds g_mu
bool device_info(DevInfo& out) {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0) return false;
    if ((size_t)d >= g_dev.size()) g_dev.resize(d + 1);
    DevInfo& di = g_dev[d];
    if (!di.ok) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, d) != hipSuccess) return false;
        std::string a = p.gcnArchName;
        di.arch = a.substr(0, a.find(':'));
        di.cus = p.multiProcessorCount;
        di.ok = true;
    }
    out = di;
    return true;
}

// as many events per block as keeps four blocks per CU, between 4 and 16
int32_t default_pack_steps(int64_t n, int cus) {
    const int64_t events = 2 * cdiv(n, TILE);
    int32_t ps = 16;
    while (ps > PACK_STEPS_MIN && cdiv(events, ps) < 4LL * cus) ps >>= 1;
    return ps;
}

// as many draws per thread as keeps four blocks per CU, between 1 and 8
int32_t default_sample_unroll(int64_t k, int cus) {
    int32_t u = SAMPLE_UNROLL_MAX;
    while (u > 1 && cdiv(k, (int64_t)SAMPLE_TPB * u) < 4LL * cus) u >>= 1;
    return u;
}

// ---- JSON ------------------------------------------------------------------
// {"format": "wrs-tuning-1", "entries": [{"arch": "gfx950", "cus": 256,
//   "op": "build", "log2": 28, "value": 16, "us": 2900.5}, ...]}

bool json_str(const std::string& obj, const char* key, std::string& out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return false;
    p = obj.find('"', p);
    if (p == std::string::npos) return false;
    const size_t q = obj.find('"', p + 1);
    if (q == std::string::npos) return false;
    out = obj.substr(p + 1, q - p - 1);
    return true;
}

bool json_num(const std::string& obj, const char* key, double& out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return false;
    char* end = nullptr;
    out = strtod(obj.c_str() + p + 1, &end);
    return end != obj.c_str() + p + 1;
}

// caller holds g_mu
int load_locked(const char* path) {
    FILE* f = fopen(path, "rb");
    if (!f) {
        set_error("wrs_tune_load: cannot open %s", path);
        return WRS_EINVAL;
    }
    std::string s;
    char buf[4096];
    size_t r;
    while ((r = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, r);
    fclose(f);
    size_t p = s.find("\"entries\"");
    if (p == std::string::npos || s.find('[', p) == std::string::npos) {
        set_error("wrs_tune_load: %s has no entries array", path);
        return WRS_EINVAL;
    }
    p = s.find('[', p);
    const size_t end = s.find(']', p);
    if (end == std::string::npos) {
        set_error("wrs_tune_load: %s: unterminated entries array", path);
        return WRS_EINVAL;
    }
    std::map<Key, Entry> add;
    for (size_t a = s.find('{', p); a != std::string::npos && a < end; a = s.find('{', a + 1)) {
        const size_t b = s.find('}', a);
        if (b == std::string::npos || b > end) {
            set_error("wrs_tune_load: %s: unterminated entry", path);
            return WRS_EINVAL;
        }
        const std::string obj = s.substr(a, b - a + 1);
        std::string arch, op;
        double cus, cls, value, us = 0.0;
        if (!json_str(obj, "arch", arch) || !json_str(obj, "op", op) || !json_num(obj, "cus", cus) ||
            !json_num(obj, "log2", cls) || !json_num(obj, "value", value)) {
            set_error("wrs_tune_load: %s: entry without arch, op, cus, log2 or value", path);
            return WRS_EINVAL;
        }
        (void)json_num(obj, "us", us);
        const int o = op == "build" ? WRS_TUNE_BUILD : (op == "sample" ? WRS_TUNE_SAMPLE : 0);
        if (!o || !valid_value(o, (int32_t)value) || cls < 0 || cls > 62) {
            set_error("wrs_tune_load: %s: bad entry (op %s, value %g)", path, op.c_str(), value);
            return WRS_EINVAL;
        }
        add[Key(arch, (int)cus, o, (int)cls)] = Entry{(int32_t)value, us};
        a = b;
    }
    for (auto& kv : add) g_tab[kv.first] = kv.second;
    return WRS_OK;
}

// caller holds g_mu
void load_env_once() {
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char* p = getenv("WRS_TUNE_FILE");
    if (p && *p) (void)load_locked(p);  // a missing or bad file leaves the defaults
}

int32_t lookup(int op, int64_t size) {
    std::lock_guard<std::mutex> g(g_mu);
    load_env_once();
    DevInfo d;
    if (!device_info(d)) return op == WRS_TUNE_BUILD ? 16 : SAMPLE_UNROLL_MAX;
    auto it = g_tab.find(Key(d.arch, d.cus, op, size_class(size)));
    if (it != g_tab.end()) return it->second.value;
    return op == WRS_TUNE_BUILD ? default_pack_steps(size, d.cus) : default_sample_unroll(size, d.cus);
}

// ---- timing ------------------------------------------------------------------

// Synthetic weights for timing: uniform on (0, 1] from Philox counters.
__global__ void k_fill_uniform(float* w, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 x = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), 0x7475u, 0u), 0x6e65u, 0x7777u);
    w[i] = (float)((x.x >> 8) + 1u) * (1.0f / 16777216.0f);
}

struct Scratch {
    float* w = nullptr;
    wrs_entry* table = nullptr;
    void* ws = nullptr;
    int32_t* out = nullptr;
    ~Scratch() {
        if (w) (void)hipFree(w);
        if (table) (void)hipFree(table);
        if (ws) (void)hipFree(ws);
        if (out) (void)hipFree(out);
    }
};

hipError_t build_with(const Scratch& S, int64_t n, int32_t psteps, hipStream_t st) {
    JobTable jt;
    memset(&jt, 0, sizeof jt);
    JobDesc& J = jt.one;
    J.w = S.w;
    J.table = S.table;
    build_ws_layout(J, S.ws, n, psteps);
    int64_t blocks[PH_COUNT];
    phase_blocks(J, blocks);
    return launch_build(jt, blocks, st);
}

hipError_t sample_with(const Scratch& S, int64_t n, int64_t k, int32_t unroll, hipStream_t st) {
    JobTable jt;
    memset(&jt, 0, sizeof jt);
    JobDesc& J = jt.one;
    set_sample_job(J, k, unroll);
    J.table = S.table;
    J.n = n;
    J.seed = 1;
    J.out = S.out;
    return launch_sample(jt, sample_blocks(J), st);
}

}  // namespace

int32_t pack_steps_for(int64_t n) { return lookup(WRS_TUNE_BUILD, n); }
int32_t sample_unroll_for(int64_t k) { return k > 0 ? lookup(WRS_TUNE_SAMPLE, k) : 1; }

static uint64_t g_generation = 0;
uint64_t tuning_generation() {
    std::lock_guard<std::mutex> g(g_mu);
    return g_generation;
}

}  // namespace wrs

using namespace wrs;

static int tune_fail(const char* what, hipError_t e) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return WRS_EDEVICE;
}

extern "C" int wrs_tune_get(int op, int64_t size, int32_t* value) {
    if ((op != WRS_TUNE_BUILD && op != WRS_TUNE_SAMPLE) || size < 1 || !value) {
        set_error("wrs_tune_get: bad arguments");
        return WRS_EINVAL;
    }
    *value = lookup(op, size);
    return WRS_OK;
}

extern "C" int wrs_tune_set(int op, int64_t size, int32_t value) {
    if ((op != WRS_TUNE_BUILD && op != WRS_TUNE_SAMPLE) || size < 1 || (value != 0 && !valid_value(op, value))) {
        set_error("wrs_tune_set: bad arguments (op %d, size %lld, value %d)", op, (long long)size, value);
        return WRS_EINVAL;
    }
    std::lock_guard<std::mutex> g(g_mu);
    load_env_once();
    DevInfo d;
    if (!device_info(d)) {
        set_error("wrs_tune_set: no current device");
        return WRS_EDEVICE;
    }
    const Key key(d.arch, d.cus, op, size_class(size));
    if (value == 0) g_tab.erase(key);
    else g_tab[key] = Entry{value, 0.0};
    ++g_generation;
    return WRS_OK;
}

extern "C" int wrs_autotune(int op, int64_t n, int64_t k, void* stream, int32_t* best) {
    if ((op != WRS_TUNE_BUILD && op != WRS_TUNE_SAMPLE) || n < 1 || n > 2147483647LL ||
        (op == WRS_TUNE_SAMPLE && k < 1)) {
        set_error("wrs_autotune: bad arguments");
        return WRS_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    Scratch S;
    hipError_t e = hipMalloc(&S.w, sizeof(float) * n);
    if (e == hipSuccess) e = hipMalloc(&S.table, sizeof(wrs_entry) * n);
    if (e == hipSuccess) e = hipMalloc(&S.ws, build_ws_bytes(n));
    if (e == hipSuccess && op == WRS_TUNE_SAMPLE) e = hipMalloc(&S.out, sizeof(int32_t) * k);
    if (e != hipSuccess) {
        set_error("wrs_autotune: allocation failed: %s", hipGetErrorString(e));
        return WRS_ENOMEM;
    }
    hipLaunchKernelGGL(k_fill_uniform, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, S.w, n);
    if ((e = hipGetLastError()) != hipSuccess) return tune_fail("wrs_autotune fill", e);
    if (op == WRS_TUNE_SAMPLE && (e = build_with(S, n, 0, st)) != hipSuccess) return tune_fail("wrs_autotune build", e);
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return tune_fail("wrs_autotune event", e);
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return tune_fail("wrs_autotune event", e);
    }
    const int32_t* cand = op == WRS_TUNE_BUILD ? kBuildCand : kSampleCand;
    int32_t win = 0;
    float win_ms = 0.0f;
    for (int c = 0; c < 4 && e == hipSuccess; ++c) {
        const int32_t v = cand[c];
        auto run = [&]() { return op == WRS_TUNE_BUILD ? build_with(S, n, v, st) : sample_with(S, n, k, v, st); };
        e = run();  // warm-up
        float ms_min = 0.0f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = run();
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && (rep == 0 || ms < ms_min)) ms_min = ms;
        }
        if (e == hipSuccess && (win == 0 || ms_min < win_ms)) {
            win = v;
            win_ms = ms_min;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return tune_fail("wrs_autotune timing", e);
    {
        std::lock_guard<std::mutex> g(g_mu);
        load_env_once();
        DevInfo d;
        if (!device_info(d)) {
            set_error("wrs_autotune: no current device");
            return WRS_EDEVICE;
        }
        g_tab[Key(d.arch, d.cus, op, size_class(op == WRS_TUNE_BUILD ? n : k))] = Entry{win, 1000.0 * win_ms};
        ++g_generation;
    }
    if (best) *best = win;
    return WRS_OK;
}

extern "C" int wrs_tune_save(const char* path) {
    if (!path) {
        set_error("wrs_tune_save: null path");
        return WRS_EINVAL;
    }
    std::lock_guard<std::mutex> g(g_mu);
    FILE* f = fopen(path, "wb");
    if (!f) {
        set_error("wrs_tune_save: cannot write %s", path);
        return WRS_EINVAL;
    }
    fprintf(f, "{\"format\": \"wrs-tuning-1\", \"entries\": [");
    bool first = true;
    for (const auto& kv : g_tab) {
        fprintf(f, "%s\n  {\"arch\": \"%s\", \"cus\": %d, \"op\": \"%s\", \"log2\": %d, \"value\": %d, \"us\": %.1f}",
                first ? "" : ",", std::get<0>(kv.first).c_str(), std::get<1>(kv.first),
                std::get<2>(kv.first) == WRS_TUNE_BUILD ? "build" : "sample", std::get<3>(kv.first), kv.second.value,
                kv.second.us);
        first = false;
    }
    fprintf(f, "\n]}\n");
    const bool ok = fclose(f) == 0;
    if (!ok) {
        set_error("wrs_tune_save: write to %s failed", path);
        return WRS_EINVAL;
    }
    return WRS_OK;
}

extern "C" int wrs_tune_load(const char* path) {
    if (!path) {
        set_error("wrs_tune_load: null path");
        return WRS_EINVAL;
    }
    std::lock_guard<std::mutex> g(g_mu);
    load_env_once();
    const int rc = load_locked(path);
    if (rc == WRS_OK) ++g_generation;
    return rc;
}
