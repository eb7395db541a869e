// bh_internal.h - shared declarations of the libbh HIP sources: the context,
// device buffers, wavefront primitives for gfx950 (wave64) and the host-side
// launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bh.h"

namespace bh {

constexpr int kMaxLevel = 20;          // 60-bit keys: 20 levels of 3 bits (App. B)
constexpr int kLevels = kMaxLevel + 1;  // levels 0..20
constexpr uint32_t kQMax = (1u << 20) - 1u;
constexpr uint32_t kNone = 0xffffffffu;
constexpr int kWave = 64;

// Sort tiling: 256 threads x 8 keys per block.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// Tree-level tiling: one block of 256 threads handles 256 particles.
constexpr int kTreeTile = 256;

// Walk: one group per wavefront, 4 wavefronts per block.  A group holds at most
// kMaxGroup particles: a lane carries up to two (or three) of them.
constexpr int kWalkWaves = 4;
constexpr int kMaxGroup = 128;
constexpr int kStackCap = 1408;        // >= 21 levels x 64 ranges (see walk.hip)

// Per-cell record read by the walk: everything the opening test and a
// particle-cell interaction need, in one 64-byte line.
struct alignas(64) WalkCell {
    double cx, cy, cz;   // centre of mass (float64)
    float mass;          // cell mass (float32)
    float rcrit2;        // squared opening radius (float32): (l/theta + delta)^2 for
                         // Eq. (1), (l/theta)^2 for the minimum-distance test
    uint32_t link;       // first child (node) or first particle (leaf)
    uint32_t info;       // number of children (node) or count | 0x80000000 (leaf)
    float s3[6];         // 3 S: xx, yy, zz, xy, xz, yz (second moment about the centre of mass)
};
static_assert(sizeof(WalkCell) == 64, "walk record must be one 64-byte block");

// One cluster of a batch: its particles are [first, first + n) of the particle
// arrays (the same range before and after sorting), with its own opening angle,
// softening, leaf and group sizes and time step.  Set by the host.
struct DevCluster {
    double dt;           // leapfrog step
    float theta;         // opening angle of Eq. (1)
    float eps2;          // squared Plummer softening (float32 eps squared)
    uint32_t first;      // first particle
    uint32_t n;          // particles
    uint32_t nleaf;      // most particles in a leaf
    uint32_t ncrit;      // most particles in a group
    uint32_t chunk0;     // first chunk of the cluster in the chunk table
    uint32_t nchunk;     // chunks of the cluster
    uint32_t mac;        // opening test: 0 Eq. (1), 1 minimum distance
    uint32_t pad;
};
static_assert(sizeof(DevCluster) == 48, "cluster record layout");

// The cubic domain of one cluster (App. B), computed on the device at each build.
struct DevDomain {
    double lo[3];        // lower corner
    double L;            // cube side
    double scale;        // 2^20 / L
    double hi[3];        // upper corner: per-axis maximum of the build's positions
};

// A contiguous piece of one cluster's particles, processed by one block of the
// segmented kernels (bounding box, keys, energy).
struct Chunk {
    uint32_t cluster;
    uint32_t begin;
    uint32_t end;
    uint32_t pad;
};
constexpr int kChunk = 4096;           // particles per chunk
constexpr int kMaxBins = 16;           // time-step bins of the block scheme (levels 0..15)

// Small device-side scalars shared by the build and walk kernels.
struct DevMisc {
    // error bits, kept until the host reads and clears them: bit 0 non-finite
    // coordinate, bit 1 bad mass, bit 2 cell capacity, bit 3 index out of range
    uint32_t nonfinite;
    uint32_t pad0;
    uint32_t level_count[kLevels];
    uint32_t level_offset[kLevels + 1];
    uint32_t ncells;
    uint32_t nleaves;
    uint32_t ngroups;
    uint32_t depth;
    uint32_t walk_next;                // group work counter of the walk
    uint32_t levels_done;              // levels scanned in the current build (self-clearing)
    uint32_t nactive;                  // groups in the active list of a partial walk
    uint32_t walk_overflow;            // set if a per-wave list would overflow
    unsigned long long sum_npp;
    unsigned long long sum_npc;
    unsigned long long tot_npp;        // never reset: totals over all walks
    unsigned long long tot_npc;
    // block time-steps: the summed base of the particles a walk covered,
    // particles per time-step bin
    unsigned long long base_sum;
    uint32_t bin_count[kMaxBins];
    unsigned long long walked_groups;  // groups walked by the partial walks of a block step
};

}  // namespace bh

struct bh_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    bh_params p{};
    std::string err;

    int64_t n = 0;          // particles in the current system (all clusters)
    int64_t K = 0;          // clusters
    int64_t nchunks = 0;
    int max_nleaf = 16;     // largest leaf size over the clusters (LDS halo of the tree build)
    int64_t cap_n = 0;      // particle capacity of the buffers
    int64_t cap_c = 0;      // cell capacity
    int64_t cap_k = 0;      // cluster capacity
    int64_t cap_chunks = 0;
    int64_t bytes = 0;      // device bytes held
    int cur = 0;            // which particle buffer holds the current state
    bool built = false;
    bool have_forces = false;
    bool have_e0 = false;
    bool energy_current = false;  // e_out holds the sums of the current state
    bool any_eps0 = false;        // some cluster has zero softening (walk variant)
    int32_t mac = 0;              // opening test bh_build_tree gives its cluster
    bool moved = false;           // positions drifted since the last build or refit
    bool refitted = false;        // the cells' moments were refitted since the last build
    bool box_ready = false;       // bb_part holds the held positions' partials (a step's drift)
    bool rec_fresh = false;       // the walk records were written by the last moments pass with
                                  // the cluster table's current theta and opening test
    int64_t layout = 0;     // changes whenever buffers or the cluster table change

    // host copies of counts, refreshed at synchronisation points
    int64_t ncells = 0, ngroups = 0, nleaves = 0;
    int depth = 0;

    // ---- clusters ----
    bh::DevCluster *clus = nullptr;          // device [K]
    bh::DevCluster *clus_h = nullptr;        // pinned host staging of the table
    bh::DevDomain *dom = nullptr;            // device [K]
    bh::Chunk *chunks = nullptr;             // device [nchunks]
    bh::Chunk *chunks_h = nullptr;           // pinned host staging
    bool staging_busy = false;               // an upload from the staging may be in flight
    uint32_t *pcl = nullptr;                 // cluster of each particle position
    std::vector<double> e0_k;                // per-cluster energy at the first energy call
    std::vector<uint8_t> have_e0_k;
    double e0 = 0.0;                         // the same for the whole batch (bh_energy)
    std::vector<bh_cluster> host_clusters;   // the loaded cluster table as given
    std::vector<bh_tune_entry> tuning;       // leaf / group sizes per class of cluster
    bool capturing = false;                  // enqueueing into a graph: no event records

    // ---- particle buffers (sorted order) ----
    double4 *p4[2] = {nullptr, nullptr};     // x, y, z, mass
    double4 *v4[2] = {nullptr, nullptr};     // vx, vy, vz, m (the mass again, for the energy sums)
    uint32_t *pid[2] = {nullptr, nullptr};   // caller index
    float4 *acc4 = nullptr;                  // ax, ay, az, pot (sorted order)
    uint64_t *key[2] = {nullptr, nullptr};   // sort ping-pong
    uint32_t *val[2] = {nullptr, nullptr};
    uint64_t *splt = nullptr;                // a rebuild's sort: splitters, then candidates
    uint8_t *split = nullptr;                // level at which particle i leaves i-1's cell
    uint8_t *lam = nullptr;                  // level of the leaf holding particle i
    uint8_t *gflag = nullptr;                // group start flags
    uint32_t *blk = nullptr;                 // per-block counters (levels, sort digits, scans)
    int64_t blk_len = 0;
    uint32_t *scan_tmp = nullptr;
    int64_t scan_len = 0;

    // ---- cells (level-major, key order within a level) ----
    uint32_t *c_first = nullptr, *c_count = nullptr, *c_child = nullptr, *c_nchild = nullptr;
    uint32_t *c_parent = nullptr;
    uint32_t *c_end = nullptr;               // one past a cell's last particle (build only)
    uint32_t *c_cl = nullptr;                // the cell's cluster
    uint8_t *c_level = nullptr, *c_leaf = nullptr;
    double4 *c_com = nullptr;                // centre of mass, mass (float64)
    double *c_S = nullptr;                   // [c][6] float64 second moment
    float4 *c_q0 = nullptr, *c_q1 = nullptr; // float32 walk multipoles
    float *c_rcrit2 = nullptr;
    bh::WalkCell *c_rec = nullptr;           // per-cell walk record (walk.hip)
    double4 *c_geo = nullptr;                // geometric centre, half side (minimum-distance test)
    double *c_box = nullptr;                 // [c][6] tight box of a refitted cell: lo x, y, z, hi x, y, z
    uint8_t *bins = nullptr;                 // block time-step bin per particle (caller order)
    uint8_t *due = nullptr;                  // particles due for forces at a substep (caller order)
    uint32_t *pbase = nullptr;               // per particle (caller order): interactions of its group
                                             // in the last walk covering it on a freshly built tree
    bool pbase_valid = false;                // pbase recorded for the current system
    bool rebuild_next = false;               // a refitted tree's walk grew past the block-step limit
    uint32_t *walk_spill = nullptr;          // per-wave overflow of the walk stack
    unsigned long long *walk_part = nullptr; // per-workgroup interaction totals of a walk [blocks][2]
    int64_t walk_spill_waves = 0;

    // ---- groups ----
    uint32_t *g_first = nullptr, *g_count = nullptr, *g_npp = nullptr, *g_npc = nullptr;
    double4 *g_centre = nullptr;
    float4 *g_half = nullptr;

    // ---- scalars ----
    bh::DevMisc *misc = nullptr;             // device
    bh::DevMisc *misc_h = nullptr;           // pinned host mirror
    double *bb_part = nullptr;               // bounding-box chunk partials [nchunks][6]
    double *e_part = nullptr;                // energy chunk partials [nchunks][5]
    double *e_out = nullptr;                 // energy per cluster [K][5]
    double *e_out_h = nullptr;               // pinned host copy

    hipEvent_t ev[8] = {};
    bh_stats stats{};

    // start/end events around each walk-kernel launch, harvested lazily
    static constexpr int kWalkRing = 64;
    hipEvent_t wev[2 * kWalkRing] = {};
    int wring_head = 0, wring_count = 0;
    double walk_ms_total = 0.0, walk_ms_last = 0.0;
    int64_t walk_launches = 0;
    int64_t graph_launches = 0;
    int64_t graph_captures = 0;

    // captured leapfrog step, one per parity of the particle ping-pong buffers
    hipStream_t cap_stream = nullptr;        // capture only, never runs work
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    int64_t graph_layout = -1;
};

namespace bh {

// ---------------------------------------------------------------------------
// launchers (each returns hipSuccess or the first HIP error)

// build.hip: each takes the particles in the current buffers unless a caller
// array is given (initial load, caller order = cluster order)
hipError_t launch_domain(bh_ctx *c, const double *pos_aos);
hipError_t launch_keys(bh_ctx *c, const double *pos_aos);
hipError_t launch_reorder_from_caller(bh_ctx *c, const double *pos_aos, const double *mass,
                                      const double *vel, const uint32_t *perm);
hipError_t launch_reorder(bh_ctx *c, const uint32_t *perm);
hipError_t launch_tree(bh_ctx *c);
hipError_t launch_groups(bh_ctx *c);
hipError_t launch_group_boxes(bh_ctx *c);
hipError_t launch_moments(bh_ctx *c, bool boxes = false);   // boxes: also tight cell boxes (refit)
hipError_t launch_rcrit(bh_ctx *c);                 // per-cluster theta; also fills c_rec
hipError_t launch_cluster_ids(bh_ctx *c);           // pcl from the chunk table

// sort.hip
hipError_t radix_sort_pairs(bh_ctx *c);             // sorts key[0]/val[0] of n particles
                                                    // within clusters; result in key[0]/val[0]
// The same result for one cluster whose particles are held in the previous
// build's order (a rebuild); falls back to radix_sort_pairs where it does not apply.
hipError_t rebuild_sort_pairs(bh_ctx *c);
int rebuild_buckets(const bh_ctx *c);      // buckets of that sort (0: radix sort instead)
int rebuild_candidates(const bh_ctx *c);   // candidate keys the keys kernel writes for it
                                           // to splt + kRadix (0: none)
hipError_t compact_flags(bh_ctx *c, const uint8_t *flags, int64_t n, uint32_t *idx,
                         uint32_t *count);
int64_t sort_blk_words(int64_t n);
int64_t scan_tmp_words(int64_t n);

// walk.hip
hipError_t launch_walk(bh_ctx *c, bool timed, bool active_only = false);
hipError_t launch_active_groups(bh_ctx *c, const uint8_t *active);   // list for active_only
void walk_timer_harvest(bh_ctx *c, bool block);
hipEvent_t *walk_timer_slot(bh_ctx *c);
hipError_t launch_scatter(bh_ctx *c, float *acc, float *pot);
hipError_t launch_zero_acc(bh_ctx *c);
int64_t walk_spill_words(int64_t waves);
int64_t walk_grid_waves(bh_ctx *c);

// api.hip: context operations used by the serving loop (serve.hip)
int ctx_fail(bh_ctx *c, int code, const char *msg);
int ctx_hip_fail(bh_ctx *c, hipError_t e, const char *where);
int64_t ctx_bytes_for(bh_ctx *c, int64_t n, int64_t K, int nleaf_min);
int ctx_reserve(bh_ctx *c, int64_t n, int64_t K, int nleaf_min);
bool ctx_cells_fit(int64_t n, int64_t K, int nleaf_min);   // cell indices fit 29 bits
int ctx_check_clusters(bh_ctx *c, const bh_cluster *cl, int64_t K, std::vector<bh_cluster> &out,
                       int64_t *total);
int ctx_set_layout(bh_ctx *c, const std::vector<bh_cluster> &cl, int64_t n);
int ctx_update_params(bh_ctx *c, const std::vector<bh_cluster> &cl);
int ctx_step(bh_ctx *c, bool graph);
int ctx_sync_check(bh_ctx *c);
int ctx_log2_floor(int64_t n);
hipError_t ctx_enqueue_rebuild(bh_ctx *c);   // keys .. moments from the held particles
hipError_t ctx_enqueue_refit(bh_ctx *c);     // group boxes and moments of the existing cells
hipError_t ctx_enqueue_forces(bh_ctx *c);    // opening radii and the full walk
// buffers of a one-cluster context carved from caller-provided device memory
int64_t ctx_carve(bh_ctx *c, int64_t n, int nleaf_min, int64_t spill_waves, char *base,
                  int64_t bytes);
hipError_t ctx_enqueue_load(bh_ctx *c, const double *pos, const double *mass);
hipError_t ctx_enqueue_forces_out(bh_ctx *c, float *acc, float *pot);

// block.hip

// integrate.hip (per-cluster dt from the cluster table)
hipError_t launch_kick_drift(bh_ctx *c);
hipError_t launch_energy(bh_ctx *c);
hipError_t launch_kick_energy(bh_ctx *c);          // closing kick fused with the energy sums
hipError_t launch_drift(bh_ctx *c, double dt);                       // x += v dt, all particles
hipError_t launch_kick_masked(bh_ctx *c, double dt, const uint8_t *active);  // v += a dt
hipError_t launch_set_velocities(bh_ctx *c, const double *vel);
hipError_t launch_get_state(bh_ctx *c, double *pos, double *vel, float *acc, float *pot);
hipError_t launch_set_positions(bh_ctx *c, const double *pos, const double *vel);

}  // namespace bh

// ---------------------------------------------------------------------------
// wavefront primitives (wave64)

namespace bh {

__device__ __forceinline__ int lane_id()
{
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// number of set bits of mask below this lane
__device__ __forceinline__ int mask_rank(unsigned long long mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ unsigned long long ballot(bool p)
{
    return __ballot(p);
}

// Orders LDS traffic of one wavefront: writes issued before are visible to reads
// issued after, and the compiler may not move memory accesses across it.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum over the 64 lanes with DPP: shifts of 1, 2, 4, 8 lanes
// inside each row of 16 (lanes shifted in from outside the row read 0), then the
// last lane of row 0 / row 2 is broadcast into rows 1 / 3, then lane 31 into
// rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan_add(uint32_t v)
{
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return (uint32_t)x;
}

// value of lane i (i uniform across the wavefront)
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int i)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, i);
}

// sum over the 64 lanes, the same in every lane
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    return lane_value(wave_incl_scan_add(v), kWave - 1);
}

// The first kernel of a build clears the build's counts (the error bits stay
// until the host reads and clears them).
__device__ __forceinline__ void reset_build_counts(DevMisc *m)
{
    m->nleaves = 0;
    m->ngroups = 0;
    m->walk_next = 0;
    m->ncells = 0;
    m->levels_done = 0;
}

constexpr int kChunkThreads = 256;     // workgroup size of the per-chunk kernels

// A kChunkThreads workgroup's minima lo and maxima hi of the three axes into
// part[6 blockIdx.x + k] (k = 0..2 minima, 3..5 maxima); a non-finite
// coordinate seen by any thread (bad) sets bit 0 of the error flags.
__device__ __forceinline__ void box_partial(double lo[3], double hi[3], bool bad,
                                            double *__restrict__ part, DevMisc *m)
{
    __shared__ double s_v[6][kChunkThreads / kWave];
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double a = lo[k], b = hi[k];
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) {
            a = fmin(a, __shfl_xor(a, d, kWave));
            b = fmax(b, __shfl_xor(b, d, kWave));
        }
        if (l == 0) {
            s_v[k][w] = a;
            s_v[3 + k][w] = b;
        }
    }
    if (ballot(bad) && l == 0) atomicOr(&m->nonfinite, 1u);
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double a = s_v[k][0];
        for (int i = 1; i < kChunkThreads / kWave; ++i) a = k < 3 ? fmin(a, s_v[k][i]) : fmax(a, s_v[k][i]);
        part[6 * (int64_t)blockIdx.x + k] = a;
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ uint32_t readfirst(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

}  // namespace bh

#define BH_HIP_TRY(expr)                          \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return e_;          \
    } while (0)

#define BH_LAUNCH_CHECK() BH_HIP_TRY(hipGetLastError())
