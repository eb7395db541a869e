// block.hip - block time-steps (Sect. 5): between synchronisation points only the
// particles due for an update get new forces, walked on the tree whose moments
// are refitted to the current positions, and the tree is rebuilt once its walk
// has become considerably more expensive than on a freshly built tree.
//
// The paper gives neither the time-step criterion nor the schedule.  Here:
//  - each particle's step is dt_i = sqrt(2 eta l / |a_i|) rounded down to a
//    power-of-two fraction dt_max 2^-b of the block step, b in [0, B], decided
//    as (dt_max 2^-b)^4 |a|^2 <= (2 eta l)^2 in float64 from the float32
//    acceleration (no square root, no division: the same decision on any
//    IEEE machine); bins are assigned at the start of each block step, when
//    every particle is synchronised, and held for the block step;
//  - kick-drift-kick per bin: an opening half kick of every particle, then
//    2^B substeps of dt_max 2^-B; at the end of substep s the particles of the
//    bins with s a multiple of 2^(B - b) are due (every particle is first
//    drifted over the substeps since the previous force evaluation, in one step):
//    the groups holding a due particle are walked, and each due particle gets
//    its closing half kick and the opening half kick of its next step (a
//    substep at which no particle is due does nothing); at the last substep
//    every particle is due and every group is walked;
//  - the tree of each force evaluation: each particle carries a base, the
//    interaction count of its group in the last walk that covered it on a
//    freshly built tree.  A walk on a refitted tree is compared with the summed
//    base of the particles it covered: more than (1 + growth) times as many
//    interactions and the next force evaluation rebuilds the tree instead of
//    refitting it (growth <= 0: every force evaluation rebuilds, which with
//    B = 0 is exactly the leapfrog step).
#include <cmath>
#include <cstring>

#include "bh_internal.h"

#pragma clang fp contract(off)

using namespace bh;

namespace {

constexpr int kBlock = 256;
constexpr unsigned kBinsGrid = 512;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// bin of each particle from its float32 acceleration; histogram in misc (a
// small fixed grid: each workgroup adds its histogram to the device-wide one)
__global__ void __launch_bounds__(kBlock)
bins_kernel(int64_t n, const float4 *__restrict__ acc4, const uint32_t *__restrict__ pid,
            double dt_max, int levels, double k2, uint8_t *__restrict__ bins, DevMisc *m)
{
    __shared__ uint32_t hist[kMaxBins];
    if (threadIdx.x < kMaxBins) hist[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const float4 a = acc4[i];
        const double ax = (double)a.x, ay = (double)a.y, az = (double)a.z;
        const double a2 = (ax * ax + ay * ay) + az * az;
        int b = 0;
        for (; b < levels; ++b) {
            const double d = ldexp(dt_max, -b);
            const double d2 = d * d;
            if ((d2 * d2) * a2 <= k2) break;
        }
        bins[pid[i]] = (uint8_t)b;
        atomicAdd(&hist[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kMaxBins && hist[threadIdx.x]) atomicAdd(&m->bin_count[threadIdx.x], hist[threadIdx.x]);
}

__global__ void clear_bins_kernel(DevMisc *m)
{
    if (threadIdx.x < kMaxBins) m->bin_count[threadIdx.x] = 0;
    if (threadIdx.x == 0) m->walked_groups = 0;
}

__global__ void count_walked_kernel(DevMisc *m)
{
    if (threadIdx.x == 0) m->walked_groups += m->nactive;
}

// caller order: due[j] = the step of particle j ends at substep s
__global__ void __launch_bounds__(kBlock)
due_kernel(int64_t n, const uint8_t *__restrict__ bins, int64_t s, int levels,
           uint8_t *__restrict__ due)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int b = bins[j];
    due[j] = (uint8_t)((s & (((int64_t)1 << (levels - b)) - 1)) == 0);
}

// half kicks v += a dt_b / 2 with dt_b = dt_max 2^-bin.  s = 0: one half kick of
// every particle; s > 0: the particles due at substep s get two (the closing
// kick of the step that ends and the opening kick of the next).
__global__ void __launch_bounds__(kBlock)
kick_bins_kernel(int64_t n, const uint32_t *__restrict__ pid, const uint8_t *__restrict__ bins,
                 const float4 *__restrict__ acc4, double4 *__restrict__ v4, double dt_max,
                 int levels, int64_t s)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int b = bins[pid[i]];
    if (s > 0 && (s & (((int64_t)1 << (levels - b)) - 1)) != 0) return;
    const double h = 0.5 * ldexp(dt_max, -b);
    const float4 a = acc4[i];
    double4 v = v4[i];
    v.x = v.x + (double)a.x * h;
    v.y = v.y + (double)a.y * h;
    v.z = v.z + (double)a.z * h;
    if (s > 0) {
        v.x = v.x + (double)a.x * h;
        v.y = v.y + (double)a.y * h;
        v.z = v.z + (double)a.z * h;
    }
    v4[i] = v;
}

// base of the particles of the walked groups (the active list, or every group):
// their group's interaction count in the walk just finished on a fresh tree
__global__ void __launch_bounds__(kBlock)
base_record_kernel(const DevMisc *__restrict__ m, const uint32_t *__restrict__ glist,
                   const uint32_t *__restrict__ g_first, const uint32_t *__restrict__ g_count,
                   const uint32_t *__restrict__ g_npp, const uint32_t *__restrict__ g_npc,
                   const uint32_t *__restrict__ pid, uint32_t *__restrict__ pbase)
{
    const uint32_t ng = glist ? m->nactive : m->ngroups;
    for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < ng; k += gridDim.x * kBlock) {
        const uint32_t g = glist ? glist[k] : k;
        const uint32_t cnt = g_npp[g] + g_npc[g];
        const uint32_t s = g_first[g], e = s + g_count[g];
        for (uint32_t i = s; i < e; ++i) pbase[pid[i]] = cnt;
    }
}

__global__ void clear_base_sum_kernel(DevMisc *m)
{
    if (threadIdx.x == 0) m->base_sum = 0ull;
}

// summed base of the particles of the walked groups -> m->base_sum (a small
// fixed grid: one addition per workgroup)
__global__ void __launch_bounds__(kBlock)
base_sum_kernel(DevMisc *__restrict__ m, const uint32_t *__restrict__ glist,
                const uint32_t *__restrict__ g_first, const uint32_t *__restrict__ g_count,
                const uint32_t *__restrict__ pid, const uint32_t *__restrict__ pbase)
{
    __shared__ unsigned long long s_sum[kBlock / kWave];
    const uint32_t ng = glist ? m->nactive : m->ngroups;
    unsigned long long sum = 0;
    for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < ng; k += gridDim.x * kBlock) {
        const uint32_t g = glist ? glist[k] : k;
        const uint32_t s = g_first[g], e = s + g_count[g];
        for (uint32_t i = s; i < e; ++i) sum += pbase[pid[i]];
    }
    for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_down(sum, off, kWave);
    if (threadIdx.x % kWave == 0) s_sum[threadIdx.x / kWave] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < kBlock / kWave; ++i) t += s_sum[i];
        if (t) atomicAdd(&m->base_sum, t);
    }
}

bool bad_params(const bh_block_params *p)
{
    return !p || !(p->dt_max > 0.0) || !std::isfinite(p->dt_max) || !(p->eta > 0.0) ||
           !std::isfinite(p->eta) || !(p->length > 0.0) || !std::isfinite(p->length) ||
           p->max_level < 0 || p->max_level >= kMaxBins || !std::isfinite(p->growth);
}

double crit_k2(const bh_block_params *p)
{
    double k = 2.0 * p->eta * p->length;
    return k * k;
}

hipError_t enqueue_bins(bh_ctx *c, const bh_block_params *p)
{
    hipLaunchKernelGGL(clear_bins_kernel, dim3(1), dim3(64), 0, c->stream, c->misc);
    BH_HIP_TRY(hipGetLastError());
    const unsigned g = grid_for(c->n) < kBinsGrid ? grid_for(c->n) : kBinsGrid;
    hipLaunchKernelGGL(bins_kernel, dim3(g), dim3(kBlock), 0, c->stream, c->n, c->acc4,
                       c->pid[c->cur], p->dt_max, (int)p->max_level, crit_k2(p), c->bins, c->misc);
    return hipGetLastError();
}

hipError_t enqueue_kick(bh_ctx *c, const bh_block_params *p, int64_t s)
{
    hipLaunchKernelGGL(kick_bins_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n,
                       c->pid[c->cur], c->bins, c->acc4, c->v4[c->cur], p->dt_max,
                       (int)p->max_level, s);
    return hipGetLastError();
}

#define BTRY(expr)                                                  \
    do {                                                            \
        hipError_t e__ = (expr);                                    \
        if (e__ != hipSuccess) return ctx_hip_fail(c, e__, #expr);  \
    } while (0)

#define BTRY_ST(expr)              \
    do {                           \
        int st__ = (expr);         \
        if (st__) return st__;     \
    } while (0)

int check_state(bh_ctx *c, const bh_block_params *p)
{
    if (bad_params(p))
        return ctx_fail(c, BH_EINVAL,
                        "block parameters: dt_max, eta, length > 0 and finite, max_level in 0..15");
    if (!c->built) return ctx_fail(c, BH_ESTATE, "no particles loaded");
    if (!c->have_forces || c->moved)
        return ctx_fail(c, BH_ESTATE, "block steps need current forces of every particle");
    return BH_OK;
}

hipError_t enqueue_base_record(bh_ctx *c, bool active)
{
    hipLaunchKernelGGL(base_record_kernel, dim3(kBinsGrid), dim3(kBlock), 0, c->stream, c->misc,
                       active ? c->val[1] : nullptr, c->g_first, c->g_count, c->g_npp, c->g_npc,
                       c->pid[c->cur], c->pbase);
    return hipGetLastError();
}

hipError_t enqueue_base_sum(bh_ctx *c, bool active)
{
    hipLaunchKernelGGL(clear_base_sum_kernel, dim3(1), dim3(64), 0, c->stream, c->misc);
    BH_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(base_sum_kernel, dim3(kBinsGrid), dim3(kBlock), 0, c->stream, c->misc,
                       active ? c->val[1] : nullptr, c->g_first, c->g_count, c->pid[c->cur],
                       c->pbase);
    return hipGetLastError();
}

}  // namespace

extern "C" {

int bh_block_bins(bh_ctx *c, const bh_block_params *p, uint8_t *bins, int64_t *count)
{
    if (!c) return BH_EINVAL;
    BTRY_ST(check_state(c, p));
    BTRY(enqueue_bins(c, p));
    if (bins) BTRY(hipMemcpyAsync(bins, c->bins, (size_t)c->n, hipMemcpyDeviceToDevice, c->stream));
    BTRY_ST(ctx_sync_check(c));
    if (count)
        for (int b = 0; b < kMaxBins; ++b) count[b] = (int64_t)c->misc_h->bin_count[b];
    return BH_OK;
}

int bh_block_step(bh_ctx *c, const bh_block_params *p, bh_block_stats *out)
{
    if (!c) return BH_EINVAL;
    BTRY_ST(check_state(c, p));
    const int B = p->max_level;
    const int64_t S = (int64_t)1 << B;
    const double dtm = ldexp(p->dt_max, -B);
    const bool always = !(p->growth > 0.0f);
    const double limit = 1.0 + (double)p->growth;
    bh_block_stats st;
    memset(&st, 0, sizeof(st));
    st.substeps = S;

    // on a freshly built tree the counts of its last walk are every particle's base,
    // and nothing calls for a rebuild
    if (!c->pbase_valid || !c->refitted) {
        BTRY(enqueue_base_record(c, false));
        c->pbase_valid = true;
    }
    if (!c->refitted) c->rebuild_next = false;
    BTRY(enqueue_bins(c, p));
    BTRY(enqueue_kick(c, p, 0));
    // the occupied bins: a substep at which none of them is due does nothing
    BTRY_ST(ctx_sync_check(c));
    uint32_t occupied[kMaxBins];
    for (int b = 0; b < kMaxBins; ++b) occupied[b] = c->misc_h->bin_count[b];
    int64_t pending = 0;              // substeps since the last drift
    for (int64_t s = 1; s <= S; ++s) {
        ++pending;
        const bool last = s == S;     // every particle is due
        if (!last) {
            bool any = false;
            for (int b = 0; b <= B; ++b)
                any |= occupied[b] != 0 && (s & (((int64_t)1 << (B - b)) - 1)) == 0;
            if (!any) continue;
        }
        // velocities change only at force evaluations: one drift over the
        // substeps since the last one
        BTRY(launch_drift(c, (double)pending * dtm));
        pending = 0;
        c->energy_current = false;
        c->moved = true;              // until the step completes: forces are stale
        // the tree of this force evaluation: rebuilt, or refitted to the positions
        const bool fresh = always || c->rebuild_next;
        if (fresh) {
            BTRY(ctx_enqueue_rebuild(c));
            st.rebuilt += 1;
        } else {
            BTRY(ctx_enqueue_refit(c));
        }
        if (!last) {
            hipLaunchKernelGGL(due_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n,
                               c->bins, s, B, c->due);
            BTRY(hipGetLastError());
            BTRY(launch_rcrit(c));
            BTRY(launch_active_groups(c, c->due));
            BTRY(launch_walk(c, false, true));
            hipLaunchKernelGGL(count_walked_kernel, dim3(1), dim3(64), 0, c->stream, c->misc);
            BTRY(hipGetLastError());
        } else {
            BTRY(ctx_enqueue_forces(c));
        }
        // a fresh tree's counts become the walked particles' base; a refitted
        // tree's walk is judged against the base of the particles it covered
        if (fresh) {
            BTRY(enqueue_base_record(c, !last));
            c->rebuild_next = false;
        } else {
            BTRY(enqueue_base_sum(c, !last));
            BTRY_ST(ctx_sync_check(c));
            const DevMisc &m = *c->misc_h;
            c->rebuild_next = !always && (double)(m.sum_npp + m.sum_npc) > limit * (double)m.base_sum;
        }
        BTRY(enqueue_kick(c, p, last ? 0 : s));
    }
    c->moved = false;
    c->have_forces = true;
    // the mean base over all particles, then the statistics
    BTRY(enqueue_base_sum(c, false));
    BTRY_ST(ctx_sync_check(c));
    const DevMisc &m = *c->misc_h;
    st.sync_interactions = (double)(m.sum_npp + m.sum_npc) / (double)c->n;
    st.base_interactions = (double)m.base_sum / (double)c->n;
    for (int b = 0; b < kMaxBins; ++b) {
        st.bin_count[b] = (int64_t)m.bin_count[b];
        st.updates += st.bin_count[b] << b;
    }
    st.walked_groups = (int64_t)c->ngroups + (int64_t)m.walked_groups;
    if (out) *out = st;
    return BH_OK;
}

}  // extern "C"
