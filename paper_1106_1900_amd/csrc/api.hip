// api.hip - the C ABI declared in include/bh.h: context and device memory, the
// cluster table of a batch, the build / force / leapfrog sequences (eager, or
// captured once into a HIP graph and replayed), state copies, energy,
// statistics and the host export used to check the tree element by element.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "bh_internal.h"

using namespace bh;

namespace {

int fail(bh_ctx *c, int code, const char *msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(bh_ctx *c, hipError_t e, const char *where)
{
    (void)hipGetLastError();
    if (c) c->err = std::string(where) + ": " + hipGetErrorString(e);
    return BH_EDEVICE;
}

#define TRY_HIP(c, expr)                                             \
    do {                                                             \
        hipError_t e__ = (expr);                                     \
        if (e__ != hipSuccess) return hip_fail((c), e__, #expr);     \
    } while (0)

#define TRY_ST(expr)              \
    do {                          \
        int st__ = (expr);        \
        if (st__) return st__;    \
    } while (0)

// ---------------------------------------------------------------------------
// device memory

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

template <typename T>
void hfree(T *&p)
{
    if (p) (void)hipHostFree((void *)p);
    p = nullptr;
}

void drop_graphs(bh_ctx *c)
{
    for (int k = 0; k < 2; ++k) {
        if (c->graph_exec[k]) (void)hipGraphExecDestroy(c->graph_exec[k]);
        c->graph_exec[k] = nullptr;
    }
    c->graph_layout = -1;
}

void free_buffers(bh_ctx *c)
{
    drop_graphs(c);
    for (int i = 0; i < 2; ++i) {
        dfree(c->p4[i]);
        dfree(c->v4[i]);
        dfree(c->pid[i]);
        dfree(c->key[i]);
        dfree(c->val[i]);
    }
    dfree(c->splt);
    dfree(c->acc4);
    dfree(c->pcl);
    dfree(c->split);
    dfree(c->lam);
    dfree(c->gflag);
    dfree(c->blk);
    dfree(c->scan_tmp);
    dfree(c->c_first);
    dfree(c->c_count);
    dfree(c->c_end);
    dfree(c->c_cl);
    dfree(c->c_child);
    dfree(c->c_nchild);
    dfree(c->c_parent);
    dfree(c->c_level);
    dfree(c->c_leaf);
    dfree(c->c_com);
    dfree(c->c_S);
    dfree(c->c_q0);
    dfree(c->c_q1);
    dfree(c->c_rcrit2);
    dfree(c->c_rec);
    dfree(c->c_geo);
    dfree(c->c_box);
    dfree(c->bins);
    dfree(c->due);
    dfree(c->pbase);
    dfree(c->walk_spill);
    dfree(c->walk_part);
    dfree(c->g_first);
    dfree(c->g_count);
    dfree(c->g_npp);
    dfree(c->g_npc);
    dfree(c->g_centre);
    dfree(c->g_half);
    dfree(c->clus);
    dfree(c->dom);
    dfree(c->chunks);
    dfree(c->bb_part);
    dfree(c->e_part);
    dfree(c->e_out);
    hfree(c->clus_h);
    hfree(c->chunks_h);
    hfree(c->e_out_h);
    c->walk_spill_waves = 0;
    c->bytes = 0;
    c->cap_n = c->cap_c = c->cap_k = c->cap_chunks = 0;
    c->built = false;
    c->have_forces = false;
    c->layout += 1;
}

// Worst-case cell count of a forest of K trees over n particles whose smallest
// leaf size is nleaf: nodes hold more than nleaf particles and the nodes of one
// level are disjoint, so at most 20 n / (nleaf + 1) nodes below the roots; at
// most n leaves; K roots.
int64_t cell_bound(int64_t n, int64_t K, int nleaf)
{
    return n + (20 * n) / (nleaf + 1) + 2 * K + 2;
}

struct Sizes {
    int64_t n, K, chunks, cells, blk, scan, spill_waves;
};

Sizes sizes_for(bh_ctx *c, int64_t n, int64_t K, int nleaf_min)
{
    Sizes z;
    z.n = n;
    z.K = K;
    z.chunks = n / kChunk + K + 1;     // every layout with <= n particles, <= K clusters
    z.cells = cell_bound(n, K, nleaf_min);
    z.blk = std::max(sort_blk_words(n),
                     (int64_t)(kLevels + 1) * ((n + kTreeTile - 1) / kTreeTile) + kLevels + 1);
    z.scan = scan_tmp_words(n);
    z.spill_waves = walk_grid_waves(c);
    return z;
}

// Walks every device buffer of the context with its element size and count.
template <typename F>
hipError_t each_buffer(bh_ctx *c, const Sizes &z, F f)
{
    hipError_t e = hipSuccess;
#define B(ptr, cnt) \
    if (e == hipSuccess) e = f(&(ptr), sizeof(*(ptr)), (cnt))
    for (int i = 0; i < 2; ++i) {
        B(c->p4[i], z.n);
        B(c->v4[i], z.n);
        B(c->pid[i], z.n);
        B(c->key[i], z.n);
        B(c->val[i], z.n);
    }
    B(c->splt, (int64_t)kRadix * 5);
    B(c->acc4, z.n);
    B(c->pcl, z.n);
    B(c->split, z.n);
    B(c->lam, z.n);
    B(c->gflag, z.n);
    B(c->blk, z.blk);
    B(c->scan_tmp, z.scan);
    B(c->c_first, z.cells);
    B(c->c_count, z.cells);
    B(c->c_end, z.cells);
    B(c->c_cl, z.cells);
    B(c->c_child, z.cells);
    B(c->c_nchild, z.cells);
    B(c->c_parent, z.cells);
    B(c->c_level, z.cells);
    B(c->c_leaf, z.cells);
    B(c->c_com, z.cells);
    B(c->c_S, 6 * z.cells);
    B(c->c_q0, z.cells);
    B(c->c_q1, z.cells);
    B(c->c_rcrit2, z.cells);
    B(c->c_rec, z.cells);
    B(c->c_geo, z.cells);
    B(c->c_box, 6 * z.cells);
    B(c->bins, z.n);
    B(c->due, z.n);
    B(c->pbase, z.n);
    B(c->walk_spill, walk_spill_words(z.spill_waves));
    B(c->walk_part, 2 * z.spill_waves);
    B(c->g_first, z.n);
    B(c->g_count, z.n);
    B(c->g_npp, z.n);
    B(c->g_npc, z.n);
    B(c->g_centre, z.n);
    B(c->g_half, z.n);
    B(c->clus, z.K);
    B(c->dom, z.K);
    B(c->chunks, z.chunks);
    B(c->bb_part, 6 * z.chunks);
    B(c->e_part, 5 * z.chunks);
    B(c->e_out, 5 * z.K);
#undef B
    return e;
}

int64_t bytes_for(bh_ctx *c, const Sizes &z)
{
    int64_t total = 0;
    bh_ctx tmp;     // pointers only
    (void)each_buffer(&tmp, z, [&](auto **, size_t sz, int64_t cnt) {
        total += (int64_t)sz * std::max<int64_t>(cnt, 1);
        return hipSuccess;
    });
    (void)c;
    return total;
}

// Room for n particles in K clusters with the given smallest leaf size; keeps
// the buffers if they already fit.  Reallocation drops the loaded system.
int ensure_capacity(bh_ctx *c, int64_t n, int64_t K, int nleaf_min)
{
    const int64_t nchunks_max = n / kChunk + K + 1;
    if (n <= c->cap_n && K <= c->cap_k && nchunks_max <= c->cap_chunks &&
        cell_bound(n, K, nleaf_min) <= c->cap_c)
        return BH_OK;
    int64_t wn = std::max(n, c->p.max_n);
    int64_t wk = std::max(K, c->p.max_clusters);
    const int lmin = std::min(nleaf_min, (int)c->p.nleaf);
    Sizes z = sizes_for(c, wn, wk, lmin);
    if (c->p.hbm_budget_bytes > 0 && bytes_for(c, z) > c->p.hbm_budget_bytes) {
        z = sizes_for(c, n, K, nleaf_min);
        if (bytes_for(c, z) > c->p.hbm_budget_bytes)
            return fail(c, BH_ENOMEM, "particle count exceeds the context's memory budget");
    }
    // the walk stack packs a cell index into 29 bits
    if (z.cells >= (int64_t)1 << 29) {
        z = sizes_for(c, n, K, nleaf_min);
        if (z.cells >= (int64_t)1 << 29)
            return fail(c, BH_ENOMEM, "too many particles for 2^29 cells");
    }
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_buffers(c);
    hipError_t e = each_buffer(c, z, [&](auto **pp, size_t sz, int64_t cnt) {
        const int64_t bytes = (int64_t)sz * std::max<int64_t>(cnt, 1);
        hipError_t r = hipMalloc((void **)pp, (size_t)bytes);
        if (r == hipSuccess) c->bytes += bytes;
        return r;
    });
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->clus_h, sizeof(DevCluster) * (size_t)z.K, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->chunks_h, sizeof(Chunk) * (size_t)z.chunks, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->e_out_h, sizeof(double) * 5 * (size_t)z.K, hipHostMallocDefault);
    if (e != hipSuccess) {
        free_buffers(c);
        (void)hipGetLastError();
        return fail(c, BH_ENOMEM, "device allocation failed");
    }
    c->cap_n = z.n;
    c->cap_k = z.K;
    c->cap_chunks = z.chunks;
    c->cap_c = z.cells;
    c->walk_spill_waves = z.spill_waves;
    return BH_OK;
}

// ---------------------------------------------------------------------------
// host staging of the cluster table

// The pinned staging arrays may be rewritten only once earlier uploads from
// them have completed.
int staging_ready(bh_ctx *c)
{
    if (c->staging_busy) {
        TRY_HIP(c, hipStreamSynchronize(c->stream));
        c->staging_busy = false;
    }
    return BH_OK;
}

int upload_clusters(bh_ctx *c)
{
    TRY_HIP(c, hipMemcpyAsync(c->clus, c->clus_h, sizeof(DevCluster) * (size_t)c->K,
                              hipMemcpyHostToDevice, c->stream));
    c->staging_busy = true;
    return BH_OK;
}

bool bad_theta(float theta) { return !(theta > 0.0f && theta <= 1.0f); }
bool bad_eps(float eps) { return !(eps >= 0.0f) || !std::isfinite(eps); }

int log2_floor(int64_t n)
{
    int b = 0;
    while (n > 1) {
        n >>= 1;
        ++b;
    }
    return b;
}

const bh_tune_entry *tuned_for(bh_ctx *c, int64_t n, float theta)
{
    const int b = log2_floor(n);
    for (const auto &t : c->tuning)
        if (t.log2n == b && t.theta == theta) return &t;
    return nullptr;
}

// Checks a cluster table and resolves leaf / group sizes of 0 to the tuned
// values of the cluster's class, else the context's.
int check_clusters(bh_ctx *c, const bh_cluster *cl, int64_t K, std::vector<bh_cluster> &out,
                   int64_t *total)
{
    if (!cl) return fail(c, BH_EINVAL, "null cluster table");
    if (K < 1 || K > 0x7fffffffLL) return fail(c, BH_EINVAL, "number of clusters must be >= 1");
    out.assign(cl, cl + K);
    int64_t n = 0;
    for (auto &q : out) {
        if ((q.nleaf == 0 || q.ncrit == 0) && q.n >= 1) {
            const bh_tune_entry *t = tuned_for(c, q.n, q.theta);
            if (q.nleaf == 0) q.nleaf = t ? t->nleaf : c->p.nleaf;
            if (q.ncrit == 0) q.ncrit = t ? t->ncrit : c->p.ncrit;
        }
        if (q.n < 1) return fail(c, BH_EINVAL, "every cluster needs n >= 1");
        if (q.nleaf < 1 || q.nleaf > 64 || q.ncrit < 1 || q.ncrit > kMaxGroup)
            return fail(c, BH_EINVAL, "cluster nleaf must be in 1..64 and ncrit in 1..128");
        if (bad_theta(q.theta)) return fail(c, BH_EINVAL, "cluster theta must be in (0, 1]");
        if (bad_eps(q.eps)) return fail(c, BH_EINVAL, "cluster eps must be finite and >= 0");
        if (!std::isfinite(q.dt)) return fail(c, BH_EINVAL, "cluster dt must be finite");
        if (q.mac != BH_MAC_EQ1 && q.mac != BH_MAC_MIN_DIST)
            return fail(c, BH_EINVAL, "cluster mac must be BH_MAC_EQ1 or BH_MAC_MIN_DIST");
        n += q.n;
        if (n > 0x7fffffffLL) return fail(c, BH_EINVAL, "a batch holds fewer than 2^31 particles");
    }
    *total = n;
    return BH_OK;
}

bool any_zero_eps(const std::vector<bh_cluster> &cl)
{
    for (const auto &q : cl)
        if (!(q.eps > 0.0f) || !(q.eps * q.eps > 0.0f)) return true;
    return false;
}

void fill_params(DevCluster &d, const bh_cluster &q)
{
    d.dt = q.dt;
    d.theta = q.theta;
    const float e = q.eps;
    d.eps2 = e * e;
    d.mac = (uint32_t)q.mac;
}

// Writes the cluster and chunk tables of the (checked) batch to the staging
// arrays and uploads them.
int load_table(bh_ctx *c, const std::vector<bh_cluster> &cl, int64_t n)
{
    TRY_ST(staging_ready(c));
    const int64_t K = (int64_t)cl.size();
    int64_t first = 0, nch = 0;
    int lmax = 1;
    for (int64_t k = 0; k < K; ++k) {
        const bh_cluster &q = cl[k];
        DevCluster d;
        memset(&d, 0, sizeof(d));
        fill_params(d, q);
        d.first = (uint32_t)first;
        d.n = (uint32_t)q.n;
        d.nleaf = (uint32_t)q.nleaf;
        d.ncrit = (uint32_t)q.ncrit;
        d.chunk0 = (uint32_t)nch;
        for (int64_t b = 0; b < q.n; b += kChunk) {
            Chunk ch;
            ch.cluster = (uint32_t)k;
            ch.begin = (uint32_t)(first + b);
            ch.end = (uint32_t)(first + std::min<int64_t>(q.n, b + kChunk));
            ch.pad = 0;
            c->chunks_h[nch++] = ch;
        }
        d.nchunk = (uint32_t)(nch - d.chunk0);
        c->clus_h[k] = d;
        lmax = std::max(lmax, (int)q.nleaf);
        first += q.n;
    }
    c->n = n;
    c->K = K;
    c->nchunks = nch;
    c->max_nleaf = lmax;
    c->host_clusters = cl;
    c->rec_fresh = false;
    c->any_eps0 = any_zero_eps(cl);
    c->layout += 1;
    TRY_HIP(c, hipMemcpyAsync(c->chunks, c->chunks_h, sizeof(Chunk) * (size_t)nch,
                              hipMemcpyHostToDevice, c->stream));
    TRY_ST(upload_clusters(c));
    return BH_OK;
}

// Sets theta, eps and dt of clusters from a table (uploads only if any changed).
int update_params(bh_ctx *c, const std::vector<bh_cluster> &cl)
{
    bool changed = false, records = false;
    for (int64_t k = 0; k < c->K; ++k) {
        const bh_cluster &a = c->host_clusters[k], &b = cl[k];
        changed = changed || a.theta != b.theta || a.eps != b.eps || a.dt != b.dt || a.mac != b.mac;
        records = records || a.theta != b.theta || a.mac != b.mac;
    }
    if (!changed) return BH_OK;
    // the walk records hold the opening radii of the old theta or test
    if (records) c->rec_fresh = false;
    TRY_ST(staging_ready(c));
    for (int64_t k = 0; k < c->K; ++k) fill_params(c->clus_h[k], cl[k]);
    c->host_clusters = cl;
    const bool z = any_zero_eps(cl);
    if (z != c->any_eps0) {
        c->any_eps0 = z;
        c->layout += 1;     // the captured step holds the other walk variant
    }
    return upload_clusters(c);
}

// ---------------------------------------------------------------------------
// sequences

hipError_t rec(bh_ctx *c, int i)
{
    if (c->capturing || !c->ev[0]) return hipSuccess;     // no events: capture, or no-alloc
    return hipEventRecord(c->ev[i], c->stream);
}

hipError_t enqueue_finish_build(bh_ctx *c)
{
    BH_HIP_TRY(rec(c, 3));
    BH_HIP_TRY(launch_tree(c));
    BH_HIP_TRY(launch_groups(c));
    BH_HIP_TRY(launch_group_boxes(c));
    BH_HIP_TRY(rec(c, 4));
    BH_HIP_TRY(launch_moments(c));
    BH_HIP_TRY(rec(c, 5));
    return hipSuccess;
}

// Build from caller arrays in cluster order (first load of a system).
hipError_t enqueue_load(bh_ctx *c, const double *pos, const double *mass, const double *vel)
{
    c->cur = 0;
    c->refitted = false;
    BH_HIP_TRY(launch_cluster_ids(c));
    BH_HIP_TRY(rec(c, 0));
    BH_HIP_TRY(launch_domain(c, pos));
    BH_HIP_TRY(launch_keys(c, pos));
    BH_HIP_TRY(rec(c, 1));
    BH_HIP_TRY(radix_sort_pairs(c));
    BH_HIP_TRY(rec(c, 2));
    BH_HIP_TRY(launch_reorder_from_caller(c, pos, mass, vel, c->val[0]));
    return enqueue_finish_build(c);
}

// Rebuild from the particles held in the context (after a drift or set_state).
hipError_t enqueue_rebuild(bh_ctx *c)
{
    c->refitted = false;
    BH_HIP_TRY(rec(c, 0));
    BH_HIP_TRY(launch_domain(c, nullptr));
    BH_HIP_TRY(launch_keys(c, nullptr));
    BH_HIP_TRY(rec(c, 1));
    BH_HIP_TRY(rebuild_sort_pairs(c));
    BH_HIP_TRY(rec(c, 2));
    BH_HIP_TRY(launch_reorder(c, c->val[0]));
    return enqueue_finish_build(c);
}

hipError_t enqueue_forces(bh_ctx *c, float *acc, float *pot)
{
    BH_HIP_TRY(rec(c, 6));
    BH_HIP_TRY(launch_rcrit(c));
    BH_HIP_TRY(launch_walk(c, !c->capturing));
    BH_HIP_TRY(launch_scatter(c, acc, pot));
    BH_HIP_TRY(rec(c, 7));
    return hipSuccess;
}

// kick-drift-kick with each cluster's dt, then the energy and momentum sums of
// the new state (kept on the device until an energy call reads them)
hipError_t enqueue_step(bh_ctx *c)
{
    BH_HIP_TRY(launch_kick_drift(c));
    BH_HIP_TRY(enqueue_rebuild(c));
    BH_HIP_TRY(enqueue_forces(c, nullptr, nullptr));
    BH_HIP_TRY(launch_kick_energy(c));
    return hipSuccess;
}

// One step as a graph replay.  The particle buffers ping-pong once per step, so
// there is one captured graph per parity; both are recaptured when the buffers
// or the cluster layout change.  Capture runs on a private stream (the caller's
// may be the null stream, which cannot capture); the replay runs on the context
// stream.  No memset or event record is captured.
int step_graph(bh_ctx *c)
{
    if (c->graph_layout != c->layout) {
        TRY_HIP(c, hipStreamSynchronize(c->stream));
        drop_graphs(c);
        c->graph_layout = c->layout;
    }
    const int k = c->cur;
    if (!c->graph_exec[k]) {
        if (!c->cap_stream) TRY_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        c->capturing = true;
        hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
        hipError_t e_step = hipSuccess;
        hipGraph_t g = nullptr;
        if (e == hipSuccess) {
            e_step = enqueue_step(c);
            e = hipStreamEndCapture(c->stream, &g);
        }
        c->stream = user;
        c->capturing = false;
        c->cur = k;
        if (e_step != hipSuccess) e = e_step;
        if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec[k], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->graph_exec[k] = nullptr;
            return hip_fail(c, e, "capture of the leapfrog step");
        }
        c->graph_captures += 1;
    }
    TRY_HIP(c, hipGraphLaunch(c->graph_exec[k], c->stream));
    // the host-side effects of the captured step, which ran only at capture: the
    // step rebuilds the tree, so the cells are no longer refitted ones
    c->cur = k ^ 1;
    c->refitted = false;
    c->graph_launches += 1;
    return BH_OK;
}

// Drains the stream, refreshes the host copies of the device counts and
// reports (then clears) the error bits raised on the device since the last
// check.
int sync_check(bh_ctx *c)
{
    TRY_HIP(c, hipMemcpyAsync(c->misc_h, c->misc, sizeof(DevMisc), hipMemcpyDeviceToHost, c->stream));
    TRY_HIP(c, hipStreamSynchronize(c->stream));
    c->staging_busy = false;
    const DevMisc &m = *c->misc_h;
    c->ncells = m.ncells;
    c->ngroups = m.ngroups;
    c->nleaves = m.nleaves;
    c->depth = (int)m.depth;
    const uint32_t bits = m.nonfinite;
    const uint32_t over = m.walk_overflow;
    if (bits || over) {
        TRY_HIP(c, hipMemsetAsync(&c->misc->nonfinite, 0, sizeof(uint32_t), c->stream));
        TRY_HIP(c, hipMemsetAsync(&c->misc->walk_overflow, 0, sizeof(uint32_t), c->stream));
        TRY_HIP(c, hipStreamSynchronize(c->stream));
        c->built = false;
        c->have_forces = false;
        if (bits & 1u) return fail(c, BH_EINVAL, "non-finite particle coordinate");
        if (bits & 2u) return fail(c, BH_EINVAL, "particle mass must be finite and > 0");
        if (bits & 4u) return fail(c, BH_EDEVICE, "cell capacity exceeded");
        if (bits & 8u) return fail(c, BH_EDEVICE, "internal error: particle index out of range");
        return fail(c, BH_EDEVICE, "walk list overflow");
    }
    if (c->built && (c->ncells < c->K || c->ncells > c->cap_c || c->ngroups < c->K ||
                     c->ngroups > c->n)) {
        c->built = false;
        c->have_forces = false;
        return fail(c, BH_EDEVICE, "tree construction produced inconsistent counts");
    }
    return BH_OK;
}

void reset_e0(bh_ctx *c)
{
    c->have_e0 = false;
    c->have_e0_k.assign((size_t)c->K, 0);
    c->e0_k.assign((size_t)c->K, 0.0);
}

int load(bh_ctx *c, const std::vector<bh_cluster> &cl, int64_t n, const double *pos,
         const double *mass, const double *vel)
{
    int lmin = 64;
    for (auto &q : cl) lmin = std::min(lmin, (int)q.nleaf);
    TRY_ST(ensure_capacity(c, n, (int64_t)cl.size(), lmin));
    c->built = false;
    c->have_forces = false;
    c->energy_current = false;
    c->moved = false;
    c->pbase_valid = false;
    c->rebuild_next = false;
    TRY_ST(load_table(c, cl, n));
    reset_e0(c);
    TRY_HIP(c, enqueue_load(c, pos, mass, vel));
    c->built = true;
    return sync_check(c);
}

int run_forces(bh_ctx *c, float *acc, float *pot)
{
    if (!c->built) return fail(c, BH_ESTATE, "forces need a built tree");
    if (c->moved) return fail(c, BH_ESTATE, "positions moved: refit or rebuild before forces");
    TRY_HIP(c, enqueue_forces(c, acc, pot));
    c->have_forces = true;
    c->energy_current = false;
    return BH_OK;
}

int energies(bh_ctx *c)
{
    if (!c->have_forces) return fail(c, BH_ESTATE, "energy needs potentials from a force call");
    if (!c->energy_current) TRY_HIP(c, launch_energy(c));
    c->energy_current = true;
    TRY_HIP(c, hipMemcpyAsync(c->e_out_h, c->e_out, sizeof(double) * 5 * (size_t)c->K,
                              hipMemcpyDeviceToHost, c->stream));
    return sync_check(c);
}

void fill_energy(double *out, const double *s, double *e0, bool *have)
{
    const double T = s[0], W = s[1], E = T + W;
    if (!*have) {
        *e0 = E;
        *have = true;
    }
    out[0] = T;
    out[1] = W;
    out[2] = E;
    out[3] = s[2];
    out[4] = s[3];
    out[5] = s[4];
    out[6] = (*e0 != 0.0) ? (*e0 - E) / *e0 : 0.0;
}

}  // namespace

// ---------------------------------------------------------------------------
// entry points for the serving loop (serve.hip)

namespace bh {

int ctx_fail(bh_ctx *c, int code, const char *msg) { return fail(c, code, msg); }

int ctx_hip_fail(bh_ctx *c, hipError_t e, const char *where) { return hip_fail(c, e, where); }

int64_t ctx_bytes_for(bh_ctx *c, int64_t n, int64_t K, int nleaf_min)
{
    return bytes_for(c, sizes_for(c, n, K, nleaf_min));
}

bool ctx_cells_fit(int64_t n, int64_t K, int nleaf_min)
{
    return cell_bound(n, K, nleaf_min) < ((int64_t)1 << 29);
}

int ctx_reserve(bh_ctx *c, int64_t n, int64_t K, int nleaf_min)
{
    return ensure_capacity(c, n, K, nleaf_min);
}

int ctx_check_clusters(bh_ctx *c, const bh_cluster *cl, int64_t K, std::vector<bh_cluster> &out,
                       int64_t *total)
{
    return check_clusters(c, cl, K, out, total);
}

// Installs a new cluster table for particles already placed in the buffers of
// parity c->cur (a repacked batch); the next step rebuilds every tree.
int ctx_set_layout(bh_ctx *c, const std::vector<bh_cluster> &cl, int64_t n)
{
    TRY_ST(load_table(c, cl, n));
    TRY_HIP(c, launch_cluster_ids(c));
    c->built = true;
    c->have_forces = true;
    c->energy_current = false;
    return BH_OK;
}

int ctx_update_params(bh_ctx *c, const std::vector<bh_cluster> &cl) { return update_params(c, cl); }

int ctx_step(bh_ctx *c, bool graph)
{
    if (graph) TRY_ST(step_graph(c));
    else TRY_HIP(c, enqueue_step(c));
    c->energy_current = true;
    return BH_OK;
}

int ctx_sync_check(bh_ctx *c) { return sync_check(c); }

int ctx_log2_floor(int64_t n) { return log2_floor(n); }

hipError_t ctx_enqueue_rebuild(bh_ctx *c) { return enqueue_rebuild(c); }

hipError_t ctx_enqueue_refit(bh_ctx *c)
{
    c->refitted = true;
    BH_HIP_TRY(launch_group_boxes(c));
    return launch_moments(c, true);
}

hipError_t ctx_enqueue_forces(bh_ctx *c) { return enqueue_forces(c, nullptr, nullptr); }

// Points every device buffer of c (and its misc block) into [base, base + bytes)
// for n particles of one cluster with leaf size >= nleaf_min and a walk grid of
// spill_waves wavefronts, each buffer on a 256-byte boundary.  Returns the bytes
// the layout needs; with base == null (or too few bytes) nothing is assigned.
int64_t ctx_carve(bh_ctx *c, int64_t n, int nleaf_min, int64_t spill_waves, char *base,
                  int64_t bytes)
{
    Sizes z = sizes_for(c, n, 1, nleaf_min);
    z.spill_waves = spill_waves;
    auto round = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
    int64_t need = round((int64_t)sizeof(DevMisc));
    bh_ctx tmp;
    (void)each_buffer(&tmp, z, [&](auto **, size_t sz, int64_t cnt) {
        need += round((int64_t)sz * std::max<int64_t>(cnt, 1));
        return hipSuccess;
    });
    if (!base || need > bytes) return need;
    int64_t off = 0;
    c->misc = reinterpret_cast<DevMisc *>(base);
    off += round((int64_t)sizeof(DevMisc));
    (void)each_buffer(c, z, [&](auto **pp, size_t sz, int64_t cnt) {
        using T = std::remove_reference_t<decltype(**pp)>;
        *pp = reinterpret_cast<T *>(base + off);
        off += round((int64_t)sz * std::max<int64_t>(cnt, 1));
        return hipSuccess;
    });
    c->cap_n = z.n;
    c->cap_k = z.K;
    c->cap_chunks = z.chunks;
    c->cap_c = z.cells;
    c->walk_spill_waves = z.spill_waves;
    c->bytes = need;
    return need;
}

// Build from caller arrays (the sequence of bh_build_tree, enqueued only: the
// table, chunk and misc set-up is the caller's), and the walk with the outputs
// scattered to caller order (that of bh_compute_forces).
hipError_t ctx_enqueue_load(bh_ctx *c, const double *pos, const double *mass)
{
    return enqueue_load(c, pos, mass, nullptr);
}

hipError_t ctx_enqueue_forces_out(bh_ctx *c, float *acc, float *pot)
{
    return enqueue_forces(c, acc, pot);
}

}  // namespace bh

extern "C" {

int bh_drift(bh_ctx *c, double dt)
{
    if (!c) return BH_EINVAL;
    if (!std::isfinite(dt)) return fail(c, BH_EINVAL, "dt must be finite");
    if (!c->built) return fail(c, BH_ESTATE, "no particles loaded");
    TRY_HIP(c, launch_drift(c, dt));
    c->moved = true;
    c->energy_current = false;
    return BH_OK;
}

int bh_kick(bh_ctx *c, double dt, const uint8_t *active)
{
    if (!c) return BH_EINVAL;
    if (!std::isfinite(dt)) return fail(c, BH_EINVAL, "dt must be finite");
    if (!c->built || !c->have_forces) return fail(c, BH_ESTATE, "kick needs a prior force evaluation");
    TRY_HIP(c, launch_kick_masked(c, dt, active));
    c->energy_current = false;
    return BH_OK;
}

int bh_refit(bh_ctx *c)
{
    if (!c) return BH_EINVAL;
    if (!c->built) return fail(c, BH_ESTATE, "refit needs a built tree");
    TRY_HIP(c, rec(c, 3));
    TRY_HIP(c, launch_group_boxes(c));
    TRY_HIP(c, rec(c, 4));
    TRY_HIP(c, launch_moments(c, true));
    TRY_HIP(c, rec(c, 5));
    c->moved = false;
    c->refitted = true;
    return BH_OK;
}

int bh_compute_forces_active(bh_ctx *c, float theta, float eps, const uint8_t *active, float *acc,
                             float *pot)
{
    if (!c) return BH_EINVAL;
    if (!active) return fail(c, BH_EINVAL, "null active");
    if (bad_theta(theta) || bad_eps(eps))
        return fail(c, BH_EINVAL, "theta must be in (0, 1] and eps >= 0");
    if (!c->built) return fail(c, BH_ESTATE, "forces need a built tree");
    if (!c->have_forces)
        return fail(c, BH_ESTATE, "a full force evaluation must come first (inactive particles keep theirs)");
    if (c->moved) return fail(c, BH_ESTATE, "positions moved: refit or rebuild before forces");
    std::vector<bh_cluster> cl = c->host_clusters;
    for (auto &q : cl) {
        q.theta = theta;
        q.eps = eps;
    }
    TRY_ST(update_params(c, cl));
    TRY_HIP(c, rec(c, 6));
    TRY_HIP(c, launch_rcrit(c));
    TRY_HIP(c, launch_active_groups(c, active));
    TRY_HIP(c, launch_walk(c, true, true));
    TRY_HIP(c, launch_scatter(c, acc, pot));
    TRY_HIP(c, rec(c, 7));
    c->energy_current = false;
    return BH_OK;
}

int bh_default_params(bh_params *p)
{
    if (!p) return BH_EINVAL;
    p->nleaf = 16;
    p->ncrit = 64;
    p->max_n = 0;
    p->hbm_budget_bytes = 0;
    p->max_clusters = 0;
    return BH_OK;
}

int bh_create(bh_ctx **out, const bh_params *p, void *hip_stream)
{
    if (!out) return BH_EINVAL;
    *out = nullptr;
    bh_params q;
    bh_default_params(&q);
    if (p) q = *p;
    if (q.nleaf < 1 || q.nleaf > 64 || q.ncrit < 1 || q.ncrit > kMaxGroup || q.max_n < 0 ||
        q.hbm_budget_bytes < 0 || q.max_clusters < 0 || q.max_n > 0x7fffffffLL)
        return BH_EINVAL;
    bh_ctx *c = new (std::nothrow) bh_ctx();
    if (!c) return BH_ENOMEM;
    c->p = q;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipMalloc((void **)&c->misc, sizeof(DevMisc)) != hipSuccess ||
        hipHostMalloc((void **)&c->misc_h, sizeof(DevMisc), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        bh_destroy(c);
        return BH_EDEVICE;
    }
    for (int i = 0; i < 8; ++i) {
        if (hipEventCreate(&c->ev[i]) != hipSuccess) {
            (void)hipGetLastError();
            bh_destroy(c);
            return BH_EDEVICE;
        }
    }
    for (int i = 0; i < 2 * bh_ctx::kWalkRing; ++i) {
        if (hipEventCreate(&c->wev[i]) != hipSuccess) {
            (void)hipGetLastError();
            bh_destroy(c);
            return BH_EDEVICE;
        }
    }
    memset(c->misc_h, 0, sizeof(DevMisc));
    if (hipMemsetAsync(c->misc, 0, sizeof(DevMisc), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        bh_destroy(c);
        return BH_EDEVICE;
    }
    if (q.max_n > 0) {
        int st = ensure_capacity(c, q.max_n, std::max<int64_t>(1, q.max_clusters), q.nleaf);
        if (st) {
            bh_destroy(c);
            return st;
        }
    }
    *out = c;
    return BH_OK;
}

int bh_destroy(bh_ctx *c)
{
    if (!c) return BH_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    free_buffers(c);
    if (c->misc) (void)hipFree(c->misc);
    hfree(c->misc_h);
    for (int i = 0; i < 8; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    for (int i = 0; i < 2 * bh_ctx::kWalkRing; ++i)
        if (c->wev[i]) (void)hipEventDestroy(c->wev[i]);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    (void)hipGetLastError();
    delete c;
    return BH_OK;
}

int bh_build_tree(bh_ctx *c, const double *pos, const double *mass, int64_t n)
{
    if (!c) return BH_EINVAL;
    if (!pos || !mass) return fail(c, BH_EINVAL, "null pos or mass");
    if (n < 1 || n > 0x7fffffffLL) return fail(c, BH_EINVAL, "n must be in [1, 2^31)");
    bh_cluster one{};
    one.n = n;
    one.mac = c->mac;
    // theta, eps and dt are set by the force and step calls
    one.theta = c->K == 1 && !c->host_clusters.empty() ? c->host_clusters[0].theta : 0.75f;
    one.eps = c->K == 1 && !c->host_clusters.empty() ? c->host_clusters[0].eps : 0.0f;
    one.dt = c->K == 1 && !c->host_clusters.empty() ? c->host_clusters[0].dt : 0.0;
    one.nleaf = c->p.nleaf;
    one.ncrit = c->p.ncrit;
    return load(c, std::vector<bh_cluster>(1, one), n, pos, mass, nullptr);
}

int bh_batch_build(bh_ctx *c, const bh_cluster *clusters, int64_t k, const double *pos,
                   const double *mass, const double *vel)
{
    if (!c) return BH_EINVAL;
    if (!pos || !mass) return fail(c, BH_EINVAL, "null pos or mass");
    std::vector<bh_cluster> cl;
    int64_t n = 0;
    TRY_ST(check_clusters(c, clusters, k, cl, &n));
    return load(c, cl, n, pos, mass, vel);
}

int bh_batch_set_params(bh_ctx *c, const bh_cluster *clusters, int64_t k)
{
    if (!c) return BH_EINVAL;
    if (!c->built) return fail(c, BH_ESTATE, "no batch loaded");
    std::vector<bh_cluster> cl;
    int64_t n = 0;
    TRY_ST(check_clusters(c, clusters, k, cl, &n));
    if (k != c->K) return fail(c, BH_EINVAL, "cluster count differs from the loaded batch");
    for (int64_t i = 0; i < k; ++i) {
        const bh_cluster &a = c->host_clusters[i], &b = cl[i];
        if (a.n != b.n || a.nleaf != b.nleaf || a.ncrit != b.ncrit)
            return fail(c, BH_EINVAL, "n, nleaf and ncrit must match the loaded batch");
    }
    return update_params(c, cl);
}

int bh_set_mac(bh_ctx *c, int32_t mac)
{
    if (!c) return BH_EINVAL;
    if (mac != BH_MAC_EQ1 && mac != BH_MAC_MIN_DIST)
        return fail(c, BH_EINVAL, "mac must be BH_MAC_EQ1 or BH_MAC_MIN_DIST");
    c->mac = mac;
    if (!c->built) return BH_OK;
    std::vector<bh_cluster> cl = c->host_clusters;
    for (auto &q : cl) q.mac = mac;
    return update_params(c, cl);
}

int bh_set_velocities(bh_ctx *c, const double *vel)
{
    if (!c) return BH_EINVAL;
    if (!vel) return fail(c, BH_EINVAL, "null vel");
    if (!c->built) return fail(c, BH_ESTATE, "no particles loaded");
    TRY_HIP(c, launch_set_velocities(c, vel));
    reset_e0(c);
    c->energy_current = false;
    return BH_OK;
}

int bh_compute_forces(bh_ctx *c, float theta, float eps, float *acc, float *pot)
{
    if (!c) return BH_EINVAL;
    if (bad_theta(theta) || bad_eps(eps))
        return fail(c, BH_EINVAL, "theta must be in (0, 1] and eps >= 0");
    if (!c->built) return fail(c, BH_ESTATE, "compute_forces needs a built tree");
    std::vector<bh_cluster> cl = c->host_clusters;
    for (auto &q : cl) {
        q.theta = theta;
        q.eps = eps;
    }
    TRY_ST(update_params(c, cl));
    return run_forces(c, acc, pot);
}

int bh_batch_forces(bh_ctx *c, float *acc, float *pot)
{
    if (!c) return BH_EINVAL;
    return run_forces(c, acc, pot);
}

int bh_leapfrog_step(bh_ctx *c, double dt)
{
    if (!c) return BH_EINVAL;
    if (!std::isfinite(dt)) return fail(c, BH_EINVAL, "dt must be finite");
    if (!c->built || !c->have_forces)
        return fail(c, BH_ESTATE, "leapfrog_step needs a prior compute_forces");
    c->moved = false;       // the step rebuilds the tree
    std::vector<bh_cluster> cl = c->host_clusters;
    for (auto &q : cl) q.dt = dt;
    TRY_ST(update_params(c, cl));
    TRY_HIP(c, enqueue_step(c));
    c->energy_current = true;
    return BH_OK;
}

int bh_batch_run(bh_ctx *c, int32_t nsteps)
{
    if (!c) return BH_EINVAL;
    if (nsteps < 0) return fail(c, BH_EINVAL, "nsteps must be >= 0");
    if (!c->built || !c->have_forces)
        return fail(c, BH_ESTATE, "batch_run needs a prior force evaluation");
    c->moved = false;       // every step rebuilds the trees
    for (int32_t s = 0; s < nsteps; ++s) {
        TRY_ST(step_graph(c));
        c->energy_current = true;
    }
    return BH_OK;
}

int bh_get_state(bh_ctx *c, double *pos, double *vel, float *acc, float *pot)
{
    if (!c) return BH_EINVAL;
    if (!c->built) return fail(c, BH_ESTATE, "no particles loaded");
    if ((acc || pot) && !c->have_forces) return fail(c, BH_ESTATE, "no forces computed yet");
    TRY_HIP(c, launch_get_state(c, pos, vel, acc, pot));
    return BH_OK;
}

int bh_set_state(bh_ctx *c, const double *pos, const double *vel)
{
    if (!c) return BH_EINVAL;
    if (!pos || !vel) return fail(c, BH_EINVAL, "null pos or vel");
    if (!c->built) return fail(c, BH_ESTATE, "no particles loaded");
    TRY_HIP(c, launch_set_positions(c, pos, vel));
    reset_e0(c);
    c->have_forces = false;
    c->energy_current = false;
    c->moved = false;
    c->pbase_valid = false;
    c->rebuild_next = false;
    TRY_HIP(c, enqueue_rebuild(c));
    return sync_check(c);
}

int bh_energy(bh_ctx *c, double out[7])
{
    if (!c) return BH_EINVAL;
    if (!out) return fail(c, BH_EINVAL, "null out");
    TRY_ST(energies(c));
    double s[5] = {0, 0, 0, 0, 0};
    for (int64_t k = 0; k < c->K; ++k)
        for (int j = 0; j < 5; ++j) s[j] += c->e_out_h[5 * k + j];
    fill_energy(out, s, &c->e0, &c->have_e0);
    return BH_OK;
}

int bh_batch_energy(bh_ctx *c, double *out)
{
    if (!c) return BH_EINVAL;
    if (!out) return fail(c, BH_EINVAL, "null out");
    TRY_ST(energies(c));
    for (int64_t k = 0; k < c->K; ++k) {
        bool have = c->have_e0_k[k] != 0;
        fill_energy(out + 7 * k, c->e_out_h + 5 * k, &c->e0_k[k], &have);
        c->have_e0_k[k] = have ? 1 : 0;
    }
    return BH_OK;
}

int bh_stats_get(bh_ctx *c, bh_stats *out)
{
    if (!c) return BH_EINVAL;
    if (!out) return fail(c, BH_EINVAL, "null out");
    const int st = sync_check(c);
    bh_stats s;
    memset(&s, 0, sizeof(s));
    s.n = c->n;
    s.ncells = c->ncells;
    s.nleaves = c->nleaves;
    s.ngroups = c->ngroups;
    s.depth = c->depth;
    s.lanes_per_group_max = kWave;
    s.sum_npp = (int64_t)c->misc_h->sum_npp;
    s.sum_npc = (int64_t)c->misc_h->sum_npc;
    float ms = 0.f;
    if (c->built) {
        if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) s.ms_keys = ms;
        if (hipEventElapsedTime(&ms, c->ev[1], c->ev[2]) == hipSuccess) s.ms_sort = ms;
        if (hipEventElapsedTime(&ms, c->ev[2], c->ev[3]) == hipSuccess) s.ms_move = ms;
        if (hipEventElapsedTime(&ms, c->ev[3], c->ev[4]) == hipSuccess) s.ms_tree = ms;
        if (hipEventElapsedTime(&ms, c->ev[4], c->ev[5]) == hipSuccess) s.ms_moments = ms;
    }
    if (c->have_forces && hipEventElapsedTime(&ms, c->ev[6], c->ev[7]) == hipSuccess) s.ms_walk = ms;
    (void)hipGetLastError();
    s.device_bytes = c->bytes;
    walk_timer_harvest(c, true);
    s.ms_walk_kernel = c->walk_ms_last;
    s.walk_kernel_ms_total = c->walk_ms_total;
    s.walk_kernel_launches = c->walk_launches;
    s.total_npp = (int64_t)c->misc_h->tot_npp;
    s.total_npc = (int64_t)c->misc_h->tot_npc;
    s.nclusters = c->K;
    s.graph_launches = c->graph_launches;
    s.graph_captures = c->graph_captures;
    *out = s;
    return st;
}

int bh_export_tree(bh_ctx *c, const bh_tree_host *o)
{
    if (!c) return BH_EINVAL;
    if (!o) return fail(c, BH_EINVAL, "null out");
    if (!c->built) return fail(c, BH_ESTATE, "no tree");
    TRY_ST(sync_check(c));
    const int64_t n = c->n, nc = c->ncells, ng = c->ngroups;
    auto get = [&](auto *dst, const auto *src, int64_t cnt) -> hipError_t {
        return hipMemcpy(dst, src, sizeof(*src) * (size_t)cnt, hipMemcpyDeviceToHost);
    };
    if (o->key) TRY_HIP(c, get(o->key, c->key[0], n));
    if (o->perm) {
        std::vector<uint32_t> v(n);
        TRY_HIP(c, get(v.data(), c->pid[c->cur], n));
        for (int64_t i = 0; i < n; ++i) o->perm[i] = v[i];
    }
    std::vector<uint32_t> first(nc), cnt(nc), child(nc), nchild(nc), parent(nc);
    std::vector<uint8_t> level(nc), leaf(nc);
    TRY_HIP(c, get(first.data(), c->c_first, nc));
    TRY_HIP(c, get(cnt.data(), c->c_count, nc));
    TRY_HIP(c, get(child.data(), c->c_child, nc));
    TRY_HIP(c, get(nchild.data(), c->c_nchild, nc));
    TRY_HIP(c, get(parent.data(), c->c_parent, nc));
    TRY_HIP(c, get(level.data(), c->c_level, nc));
    TRY_HIP(c, get(leaf.data(), c->c_leaf, nc));
    std::vector<uint64_t> skey(n);
    if (o->prefix) TRY_HIP(c, get(skey.data(), c->key[0], n));
    for (int64_t i = 0; i < nc; ++i) {
        if (o->level) o->level[i] = level[i];
        if (o->first) o->first[i] = first[i];
        if (o->count) o->count[i] = cnt[i];
        if (o->is_leaf) o->is_leaf[i] = leaf[i];
        if (o->parent) o->parent[i] = parent[i] == kNone ? -1 : (int64_t)parent[i];
        if (o->child) o->child[i] = leaf[i] ? -1 : (int64_t)child[i];
        if (o->nchild) o->nchild[i] = leaf[i] ? 0 : (int32_t)nchild[i];
        if (o->prefix)
            o->prefix[i] = first[i] < (uint32_t)n ? (skey[first[i]] >> (3 * (kMaxLevel - level[i]))) : 0;
    }
    if (o->mass || o->com) {
        std::vector<double4> com(nc);
        TRY_HIP(c, get(com.data(), c->c_com, nc));
        for (int64_t i = 0; i < nc; ++i) {
            if (o->mass) o->mass[i] = com[i].w;
            if (o->com) {
                o->com[3 * i] = com[i].x;
                o->com[3 * i + 1] = com[i].y;
                o->com[3 * i + 2] = com[i].z;
            }
        }
    }
    if (o->S) TRY_HIP(c, get(o->S, c->c_S, 6 * nc));
    if (o->rcrit2) TRY_HIP(c, get(o->rcrit2, c->c_rcrit2, nc));
    if (o->gfirst || o->gcount || o->gcentre || o->ghalf || o->npp || o->npc) {
        std::vector<uint32_t> gf(ng), gcn(ng), npp(ng), npc(ng);
        std::vector<double4> gce(ng);
        std::vector<float4> gha(ng);
        TRY_HIP(c, get(gf.data(), c->g_first, ng));
        TRY_HIP(c, get(gcn.data(), c->g_count, ng));
        TRY_HIP(c, get(gce.data(), c->g_centre, ng));
        TRY_HIP(c, get(gha.data(), c->g_half, ng));
        TRY_HIP(c, get(npp.data(), c->g_npp, ng));
        TRY_HIP(c, get(npc.data(), c->g_npc, ng));
        for (int64_t g = 0; g < ng; ++g) {
            if (o->gfirst) o->gfirst[g] = gf[g];
            if (o->gcount) o->gcount[g] = gcn[g];
            if (o->gcentre) {
                o->gcentre[3 * g] = gce[g].x;
                o->gcentre[3 * g + 1] = gce[g].y;
                o->gcentre[3 * g + 2] = gce[g].z;
            }
            if (o->ghalf) {
                o->ghalf[3 * g] = gha[g].x;
                o->ghalf[3 * g + 1] = gha[g].y;
                o->ghalf[3 * g + 2] = gha[g].z;
            }
            if (o->npp) o->npp[g] = npp[g];
            if (o->npc) o->npc[g] = npc[g];
        }
    }
    return BH_OK;
}

const char *bh_last_error(bh_ctx *c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

}  // extern "C"
