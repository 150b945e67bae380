// wrs_internal.h -- shared definitions of the HIP library (kernels + host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wrs.h"

namespace wrs {

typedef unsigned __int128 u128;
typedef __int128 i128;

// Launch geometry.  Every size below is a constant, so a table's result depends
// on its own n only (never on how jobs are batched).
constexpr int TILE = 1024;          // items per tile (classification and prefix sums)
constexpr int TILES_PER_AGG_BLOCK = 4;  // tile aggregation: one wave per tile
constexpr int TPB = 256;            // threads per block of the tile kernels
constexpr int IPT = TILE / TPB;     // items per thread in a tile
constexpr int PACK_STEPS_MIN = 4;   // tile events per pack block: tuned per size class
constexpr int PACK_STEPS_MAX = 32;
constexpr int RED_CHUNK = 65536;    // items per block of the total-weight reduction
constexpr int SCAN_SEG = 2048;      // tiles per segment of the tile scan
constexpr int SAMPLE_TPB = 256;     // threads per block of the sampler
constexpr int FUSE_MAX = 8192;      // batched tables up to this size: one workgroup per job, table in LDS
constexpr int FUSE_BLOCKS = 512;    // workgroups of that launch at most
constexpr int SAMPLE_UNROLL_MAX = 8;  // draws per thread of the sampler: tuned per size class (1..8)

// Per-table scalars written by the reduction, read by every later phase.
struct alignas(16) BuildScalars {
    int32_t status;   // WRS_OK or an error code (first word of every workspace)
    int32_t G;        // grid exponent
    int32_t pad[2];
    u128 Q;           // n-scaled bucket capacity on the grid 2^G: round(W / 2^G)
    double W_hi, W_lo;
    double Qd;        // Q as double
    double rQ;        // 1 / Qd
    double nscale;    // n * 2^-G
    uint64_t Qn;      // floor(Q / n): item i is light iff q_i <= Qn
    int64_t npos;     // number of positive weights
    int32_t kshift;   // merge keys are prefix sums >> kshift (64-bit)
    uint32_t wthr;    // bit pattern of the smallest heavy FP32 weight
    double tscale;    // 2^kshift / Q: key difference -> bucket fraction
    uint64_t Qk;      // Q >> kshift, rounded to nearest: bucket capacity in key units
    int64_t nleft;    // greedy construction: items its blocks left to the splitting stage
};

// Everything one table needs on the device.
struct JobDesc {
    const float* w;
    wrs_entry* table;
    int32_t* out;
    int64_t n;
    int64_t k;
    uint64_t seed;
    uint64_t first_counter;
    uint32_t stream_id;
    int32_t ntiles;       // C = ceil(n / TILE)
    int32_t nred;         // ceil(n / RED_CHUNK)
    int32_t nseg;         // ceil(C / SCAN_SEG)
    BuildScalars* sc;
    double2* red;         // [nred] partial sums (hi, lo)
    uint32_t* redinfo;    // [2 * nred] bad-value flag, positive count
    uint32_t* NL;         // [C+1] lights before tile c
    u128* DP;             // [C+1] light deficit before tile c
    u128* EP;             // [C+1] heavy excess before tile c
    uint64_t* DP64;       // [C+1] DP >> kshift (merge keys)
    uint64_t* EP64;       // [C+1] EP >> kshift
    int32_t* FH;          // [C+1] first heavy item in tiles >= c, -1 if none
    float* WP;            // [C * TILE] each tile's weights, its lights then its heavies
    uint16_t* PO;         // [C * TILE] offset inside the tile of each of those items
    int32_t* pstart;      // [npack] light events before each pack block's first event
    int32_t npack;        // pack blocks
    int32_t psteps;       // tile events per pack block
    int32_t sunroll;      // draws per sampler thread
    uint32_t* sNL;        // [nseg+1] segment totals / prefixes of the tile scan
    u128* sDP;
    u128* sEP;
    int32_t* sFH;
    // List mode (the splitting stage of the greedy construction): item p of
    // the job is original item lidx[p], w[p] is its weight, or a residual
    // marker (a NaN whose payload indexes lres, the exact n-scaled size of the
    // part of a heavy not yet placed).  Sizes are always n-scaled by nmul, the
    // original item count.
    const uint32_t* lidx;
    const u128* lres;
    // Optional, list mode: a marker's size as a double, for the light
    // threshold of a marker whose lres entry is a rounded small number (a
    // negative entry, or no array: the threshold comes from lres).
    const double* lresf;
    uint32_t* PI;         // [C * TILE] list mode: original index of each WP item
    uint32_t nmul;        // n of the size scaling (= n outside list mode)
    int32_t pad;
};

enum Phase { PH_RED = 0, PH_FIN, PH_TILE, PH_SEG, PH_TOP, PH_FIX, PH_SPLIT, PH_PACK, PH_SAMPLE, PH_COUNT };

// A launch covers one phase of one job (jobs == nullptr, description in `one`)
// or of many jobs (device array `jobs`, with block offsets per phase in
// off[phase * (njobs + 1) + j]).
struct JobTable {
    const JobDesc* jobs;
    const int64_t* off;
    int32_t njobs;
    int32_t phase;
    JobDesc one;
};

// Greedy blocks of the PSA+ construction: items per block, threads per block.
constexpr int GTILE = 2048;
constexpr int GTPB = 256;
constexpr int GIPT = GTILE / GTPB;
static_assert(GTILE == WRS_PSAPLUS_BLOCK, "greedy block size is part of the ABI");

// Residual marker: a NaN whose low 23 bits hold 1 + the greedy block.  Weights
// reach the kernels that test for it with the sign bit cleared (a valid weight
// is at most 0x7F7FFFFF), so no weight is taken for a marker.
__host__ __device__ inline uint32_t residual_marker(uint32_t g) { return 0x7F800000u | (g + 1u); }
__host__ __device__ inline bool is_residual_marker(uint32_t bits) { return bits > 0x7F800000u; }
__host__ __device__ inline uint32_t residual_slot(uint32_t bits) { return (bits & 0x7FFFFFu) - 1u; }

// Byte size of the per-table workspace and the pointer layout inside it.
size_t build_ws_bytes(int64_t n);
// psteps <= 0: the tuned (or default) value for n on the current device
void build_ws_layout(JobDesc& J, void* ws, int64_t n, int32_t psteps = 0);
// The same workspace reused by a list-mode job of m <= n items (tile arrays,
// scan arrays and pack starts are sized for n); counts and pack steps for m.
void build_list_layout(JobDesc& J, int64_t m);
// PSA+ workspace: the build workspace of n items, then the greedy stage's
// arrays; pointers into it.
struct PlusLayout {
    uint32_t* cnt;    // [G] items each greedy block left
    uint32_t* goff;   // [G] exclusive prefix of cnt
    uint32_t* part;   // [ceil(G / 512)] sums of cnt over parts of 512 blocks
    u128* res;        // [G] exact n-scaled size of each block's residual item
    uint32_t* sidx;   // [G * GTILE] left items of block g at g * GTILE (index)
    float* sw;        // [G * GTILE] ... (weight or residual marker)
    uint32_t* lidx;   // [n] left items, compacted in index order
    float* lw;        // [n]
    uint32_t* PI;     // [C * TILE] list-mode partitioned original indices
};
size_t plus_ws_bytes(int64_t n);
PlusLayout plus_layout(void* ws, int64_t n);

// 2-level tables: the main job (reduction only), the top-level list job over
// the G = ceil(n / GTILE) meta-items, and the meta-items themselves.
struct TwoLayout {
    uint32_t* lidx;  // [C_top * TILE] list item g is meta-item g
    float* lw;       // [C_top * TILE] residual markers
    u128* lres;      // [G] exact G-scaled size of each meta-item
    double* lresf;   // [G] the same size from the block's own grid, or -1
    uint32_t* PI;    // [C_top * TILE] list-mode partitioned indices
};
size_t twolevel_ws_bytes(int64_t n);
// J: main job over the n items; top: the list job over the meta-items (its
// scalars are its own, finalized from J's reduction partials).
void twolevel_layout(void* ws, int64_t n, JobDesc& J, JobDesc& top, TwoLayout& T);
void set_sample_job(JobDesc& J, int64_t k, int32_t sunroll = 0);
int64_t sample_blocks(const JobDesc& J);

// Launch parameters (result-neutral) for the current device: tuned values
// when present, else defaults derived from the size and the CU count.
int32_t pack_steps_for(int64_t n);
int32_t sample_unroll_for(int64_t k);
// Changes whenever a tuned value may have changed (recorded graphs keyed on it).
uint64_t tuning_generation();

// Blocks of every phase for one table (depends on n and k only).
void phase_blocks(const JobDesc& J, int64_t blocks[PH_COUNT]);

// Host launchers (stream-ordered).
// list = true: the list-mode kernels (splitting stage of the greedy construction)
hipError_t launch_build(const JobTable& jt, const int64_t* blocks, hipStream_t st, bool list = false);
// Greedy stage of PSA+ for one job (reduction already launched): greedy blocks,
// prefix of their leftover counts (into sc->nleft), compaction.
hipError_t launch_greedy(const JobDesc& J, const PlusLayout& P, hipStream_t st);
// The scalars of a job over meta-items on the grid (G, Q) of a finished job.
hipError_t launch_finalize_on_grid(const JobDesc& top, const BuildScalars* base, hipStream_t st);
hipError_t launch_twolvl(const JobDesc& J, const TwoLayout& T, hipStream_t st);
hipError_t launch_sample2(const wrs_entry* top, const wrs_entry* table, int64_t n, uint64_t seed, uint32_t sid,
                          uint64_t first, int64_t k, int32_t* out, hipStream_t st);
hipError_t launch_sample(const JobTable& jt, int64_t blocks, hipStream_t st);
// Jobs d_small[0, nsmall) of jt (each n <= FUSE_MAX), built and sampled in one launch.
hipError_t launch_fused_small(const JobTable& jt, const int32_t* d_small, int32_t nsmall, hipStream_t st);
// jt.jobs[j].sc->status -> d_dst[j] for every job (device memory, jobs on the device)
hipError_t launch_collect_status(const JobTable& jt, int32_t* d_dst, hipStream_t st);

// WOR
size_t wor_ws_bytes(int64_t n, int64_t k);
int launch_wor(const float* w, int64_t n, int64_t k, uint64_t seed, uint32_t sid, int32_t* out,
               void* ws, hipStream_t st);
int wor_status_offset();

// Weighted permutation (returns 0 or a hipError_t)
size_t perm_ws_bytes(int64_t n);
// Stable LSD radix passes (8-bit digits at bits first_shift + 8 p, p < passes)
// over the keys and 32-bit values that radix_inputs() locates in a workspace
// of perm_ws_bytes(n) bytes; *keys and *vals receive the sorted arrays.
void radix_inputs(void* ws, int64_t n, uint64_t** keys, uint32_t** vals);
int launch_radix(void* ws, int64_t n, int first_shift, int passes, hipStream_t st, const uint64_t** keys,
                 const uint32_t** vals);
int launch_perm(const float* w, int64_t n, uint64_t seed, uint32_t sid, int32_t* out, void* ws, hipStream_t st);

// Output-sensitive sampling with replacement (wrs_os.hip).
size_t os_bytes(int64_t n);
size_t os_ws_bytes(int64_t n, int64_t k);
int launch_os_build(const float* d_w, int64_t n, void* d_os, void* d_ws, hipStream_t st);
int launch_os_sample(const void* d_os, int64_t n, int64_t k, uint64_t seed, int32_t* d_items, int32_t* d_counts,
                     int64_t* d_s, void* d_ws, hipStream_t st);

// Error reporting for the C ABI (clear_error: empty this thread's text).
void set_error(const char* fmt, ...);
void clear_error();

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace wrs
