// api.hip - the C ABI declared in include/bh.h: context and device memory, the
// build / force / leapfrog sequences, state copies, energy, statistics and the
// host export used to check the tree element by element.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "bh_internal.h"

namespace bh {
int64_t energy_words();
}

using namespace bh;

namespace {

int fail(bh_ctx *c, int code, const char *msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(bh_ctx *c, hipError_t e, const char *where)
{
    if (c) {
        c->err = std::string(where) + ": " + hipGetErrorString(e);
    }
    return BH_EDEVICE;
}

#define TRY_HIP(c, expr)                                   \
    do {                                                   \
        hipError_t e__ = (expr);                           \
        if (e__ != hipSuccess) return hip_fail((c), e__, #expr); \
    } while (0)

template <typename T>
hipError_t dalloc(bh_ctx *c, T **p, int64_t count)
{
    const int64_t bytes = (int64_t)sizeof(T) * (count > 0 ? count : 1);
    hipError_t e = hipMalloc((void **)p, (size_t)bytes);
    if (e == hipSuccess) c->bytes += bytes;
    return e;
}

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

void free_buffers(bh_ctx *c)
{
    for (int i = 0; i < 2; ++i) {
        dfree(c->p4[i]);
        dfree(c->v4[i]);
        dfree(c->pid[i]);
        dfree(c->key[i]);
        dfree(c->val[i]);
    }
    dfree(c->acc4);
    dfree(c->split);
    dfree(c->lam);
    dfree(c->gflag);
    dfree(c->blk);
    dfree(c->scan_tmp);
    dfree(c->c_first);
    dfree(c->c_count);
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
    dfree(c->walk_spill);
    c->walk_spill_waves = 0;
    dfree(c->g_first);
    dfree(c->g_count);
    dfree(c->g_npp);
    dfree(c->g_npc);
    dfree(c->g_centre);
    dfree(c->g_half);
    dfree(c->red);
    c->bytes = 0;
    c->cap_n = 0;
    c->cap_c = 0;
}

// Worst-case cell count: nodes hold more than nleaf particles and nodes of one
// level are disjoint, so at most 20 n / (nleaf + 1) nodes; at most n leaves.
int64_t cell_bound(int64_t n, int nleaf)
{
    return n + (20 * n) / (nleaf + 1) + 2;
}

int64_t bytes_for(int64_t n, int nleaf)
{
    const int64_t nc = cell_bound(n, nleaf);
    const int64_t per_p = 2 * 32 + 2 * 32 + 2 * 4 + 16 + 2 * 8 + 2 * 4 + 3 + 64;
    const int64_t per_c = 5 * 4 + 2 + 32 + 48 + 32 + 4 + 64;
    const int64_t blk_words = std::max(sort_blk_words(n), (int64_t)kLevels * ((n + kTreeTile - 1) / kTreeTile) + kLevels);
    return n * per_p + nc * per_c + 4 * (blk_words + scan_tmp_words(n)) + 8 * energy_words();
}

int ensure_capacity(bh_ctx *c, int64_t n)
{
    if (n <= c->cap_n) return BH_OK;
    int64_t want = n;
    if (c->p.max_n > want) want = c->p.max_n;
    if (c->p.hbm_budget_bytes > 0 && bytes_for(want, c->p.nleaf) > c->p.hbm_budget_bytes) {
        if (bytes_for(n, c->p.nleaf) > c->p.hbm_budget_bytes)
            return fail(c, BH_ENOMEM, "particle count exceeds the context's memory budget");
        want = n;
    }
    free_buffers(c);
    const int64_t nc = cell_bound(want, c->p.nleaf);
    c->blk_len = std::max(sort_blk_words(want),
                          (int64_t)kLevels * ((want + kTreeTile - 1) / kTreeTile) + kLevels);
    c->scan_len = scan_tmp_words(want);
    c->red_len = energy_words();
    hipError_t e = hipSuccess;
#define A(ptr, cnt) \
    if (e == hipSuccess) e = dalloc(c, &(ptr), (cnt))
    for (int i = 0; i < 2; ++i) {
        A(c->p4[i], want);
        A(c->v4[i], want);
        A(c->pid[i], want);
        A(c->key[i], want);
        A(c->val[i], want);
    }
    A(c->acc4, want);
    A(c->split, want);
    A(c->lam, want);
    A(c->gflag, want);
    A(c->blk, c->blk_len);
    A(c->scan_tmp, c->scan_len);
    A(c->c_first, nc);
    A(c->c_count, nc);
    A(c->c_child, nc);
    A(c->c_nchild, nc);
    A(c->c_parent, nc);
    A(c->c_level, nc);
    A(c->c_leaf, nc);
    A(c->c_com, nc);
    A(c->c_S, 6 * nc);
    A(c->c_q0, nc);
    A(c->c_q1, nc);
    A(c->c_rcrit2, nc);
    A(c->c_rec, nc);
    A(c->g_first, want);
    A(c->g_count, want);
    A(c->g_npp, want);
    A(c->g_npc, want);
    A(c->g_centre, want);
    A(c->g_half, want);
    A(c->red, c->red_len);
#undef A
    if (e != hipSuccess) {
        free_buffers(c);
        (void)hipGetLastError();
        return fail(c, BH_ENOMEM, "device allocation failed");
    }
    c->cap_n = want;
    c->cap_c = nc;
    return BH_OK;
}

// Read the device scalars back (synchronous) and check the build's flags.
int read_misc(bh_ctx *c)
{
    TRY_HIP(c, hipMemcpyAsync(c->misc_h, c->misc, sizeof(DevMisc), hipMemcpyDeviceToHost, c->stream));
    TRY_HIP(c, hipStreamSynchronize(c->stream));
    return BH_OK;
}

// Tree, groups and moments from the particles now in key order.
int finish_build(bh_ctx *c)
{
    const int64_t n = c->n;
    TRY_HIP(c, hipEventRecord(c->ev[3], c->stream));
    TRY_HIP(c, launch_tree(c, n));
    TRY_HIP(c, launch_groups(c, n));
    int st = read_misc(c);
    if (st) return st;
    const DevMisc &m = *c->misc_h;
    if (m.nonfinite & 1u) {
        c->built = false;
        return fail(c, BH_EINVAL, "non-finite particle coordinate");
    }
    if (m.nonfinite & 2u) {
        c->built = false;
        return fail(c, BH_EINVAL, "particle mass must be finite and > 0");
    }
    if (m.nonfinite & 4u) {
        c->built = false;
        return fail(c, BH_EDEVICE, "cell capacity exceeded");
    }
    c->ncells = m.ncells;
    c->ngroups = m.ngroups;
    c->nleaves = m.nleaves;
    c->depth = (int)m.depth;
    if (c->ncells < 1 || c->ncells > c->cap_c || c->ngroups < 1 || c->ngroups > n) {
        c->built = false;
        return fail(c, BH_EDEVICE, "tree construction produced inconsistent counts");
    }
    TRY_HIP(c, launch_group_boxes(c, c->ngroups));
    TRY_HIP(c, hipEventRecord(c->ev[4], c->stream));
    TRY_HIP(c, launch_moments(c, c->ncells));
    TRY_HIP(c, hipEventRecord(c->ev[5], c->stream));
    c->built = true;
    c->have_forces = false;
    return BH_OK;
}

// Rebuild from the particles held in the context (after a drift or set_state).
int rebuild(bh_ctx *c)
{
    const int64_t n = c->n;
    TRY_HIP(c, hipEventRecord(c->ev[0], c->stream));
    TRY_HIP(c, launch_bbox(c, nullptr, n));
    TRY_HIP(c, launch_keys(c, nullptr, n));
    TRY_HIP(c, hipEventRecord(c->ev[1], c->stream));
    TRY_HIP(c, radix_sort_pairs(c, n));
    TRY_HIP(c, hipEventRecord(c->ev[2], c->stream));
    TRY_HIP(c, launch_reorder(c, c->val[0], n));
    return finish_build(c);
}

int forces(bh_ctx *c, float theta, float eps, float *acc, float *pot)
{
    TRY_HIP(c, hipEventRecord(c->ev[6], c->stream));
    TRY_HIP(c, launch_rcrit(c, c->ncells, theta));
    TRY_HIP(c, launch_walk(c, theta, eps));
    TRY_HIP(c, launch_scatter(c, acc, pot));
    TRY_HIP(c, hipEventRecord(c->ev[7], c->stream));
    c->theta = theta;
    c->eps = eps;
    c->have_forces = true;
    return BH_OK;
}

bool bad_theta_eps(float theta, float eps)
{
    return !(theta > 0.0f && theta <= 1.0f) || !(eps >= 0.0f) || !std::isfinite(eps);
}

}  // namespace

extern "C" {

int bh_default_params(bh_params *p)
{
    if (!p) return BH_EINVAL;
    p->nleaf = 16;
    p->ncrit = 64;
    p->max_n = 0;
    p->hbm_budget_bytes = 0;
    return BH_OK;
}

int bh_create(bh_ctx **out, const bh_params *p, void *hip_stream)
{
    if (!out) return BH_EINVAL;
    *out = nullptr;
    bh_params q;
    bh_default_params(&q);
    if (p) q = *p;
    if (q.nleaf < 1 || q.nleaf > 64 || q.ncrit < 1 || q.ncrit > 64 || q.max_n < 0 ||
        q.hbm_budget_bytes < 0)
        return BH_EINVAL;
    bh_ctx *c = new (std::nothrow) bh_ctx();
    if (!c) return BH_ENOMEM;
    c->p = q;
    c->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipMalloc((void **)&c->misc, sizeof(DevMisc)) != hipSuccess ||
        hipMalloc((void **)&c->bb_part, 6 * 1024 * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void **)&c->misc_h, sizeof(DevMisc), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->red_h, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        if (c->misc) (void)hipFree(c->misc);
        if (c->bb_part) (void)hipFree(c->bb_part);
        if (c->misc_h) (void)hipHostFree(c->misc_h);
        if (c->red_h) (void)hipHostFree(c->red_h);
        delete c;
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
        int st = ensure_capacity(c, q.max_n);
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
    if (c->bb_part) (void)hipFree(c->bb_part);
    if (c->misc_h) (void)hipHostFree(c->misc_h);
    if (c->red_h) (void)hipHostFree(c->red_h);
    for (int i = 0; i < 8; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    for (int i = 0; i < 2 * bh_ctx::kWalkRing; ++i)
        if (c->wev[i]) (void)hipEventDestroy(c->wev[i]);
    delete c;
    return BH_OK;
}

int bh_build_tree(bh_ctx *c, const double *pos, const double *mass, int64_t n)
{
    if (!c) return BH_EINVAL;
    if (!pos || !mass) return fail(c, BH_EINVAL, "null pos or mass");
    if (n < 1 || n > 0x7fffffffLL) return fail(c, BH_EINVAL, "n must be in [1, 2^31)");
    int st = ensure_capacity(c, n);
    if (st) return st;
    c->n = n;
    c->cur = 0;
    c->built = false;
    c->have_forces = false;
    c->have_e0 = false;
    TRY_HIP(c, hipEventRecord(c->ev[0], c->stream));
    TRY_HIP(c, launch_bbox(c, pos, n));
    TRY_HIP(c, launch_keys(c, pos, n));
    TRY_HIP(c, hipEventRecord(c->ev[1], c->stream));
    TRY_HIP(c, radix_sort_pairs(c, n));
    TRY_HIP(c, hipEventRecord(c->ev[2], c->stream));
    TRY_HIP(c, launch_reorder_from_caller(c, pos, mass, c->val[0], n));
    return finish_build(c);
}

int bh_set_velocities(bh_ctx *c, const double *vel)
{
    if (!c) return BH_EINVAL;
    if (!vel) return fail(c, BH_EINVAL, "null vel");
    if (!c->built) return fail(c, BH_ESTATE, "no particles loaded");
    TRY_HIP(c, launch_set_velocities(c, vel));
    c->have_e0 = false;
    return BH_OK;
}

int bh_compute_forces(bh_ctx *c, float theta, float eps, float *acc, float *pot)
{
    if (!c) return BH_EINVAL;
    if (bad_theta_eps(theta, eps)) return fail(c, BH_EINVAL, "theta must be in (0, 1] and eps >= 0");
    if (!c->built) return fail(c, BH_ESTATE, "compute_forces needs a built tree");
    return forces(c, theta, eps, acc, pot);
}

int bh_leapfrog_step(bh_ctx *c, double dt)
{
    if (!c) return BH_EINVAL;
    if (!std::isfinite(dt)) return fail(c, BH_EINVAL, "dt must be finite");
    if (!c->built || !c->have_forces) return fail(c, BH_ESTATE, "leapfrog_step needs a prior compute_forces");
    const float theta = c->theta, eps = c->eps;
    TRY_HIP(c, launch_kick_drift(c, 0.5 * dt, dt));
    int st = rebuild(c);
    if (st) return st;
    st = forces(c, theta, eps, nullptr, nullptr);
    if (st) return st;
    TRY_HIP(c, launch_kick(c, 0.5 * dt));
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
    c->have_e0 = false;
    return rebuild(c);
}

int bh_energy(bh_ctx *c, double out[7])
{
    if (!c) return BH_EINVAL;
    if (!out) return fail(c, BH_EINVAL, "null out");
    if (!c->have_forces) return fail(c, BH_ESTATE, "energy needs potentials from compute_forces");
    TRY_HIP(c, launch_energy(c));
    TRY_HIP(c, hipMemcpyAsync(c->red_h, c->red + (c->red_len - 8), 5 * sizeof(double),
                              hipMemcpyDeviceToHost, c->stream));
    TRY_HIP(c, hipStreamSynchronize(c->stream));
    const double T = c->red_h[0], W = c->red_h[1];
    const double E = T + W;
    if (!c->have_e0) {
        c->e0 = E;
        c->have_e0 = true;
    }
    out[0] = T;
    out[1] = W;
    out[2] = E;
    out[3] = c->red_h[2];
    out[4] = c->red_h[3];
    out[5] = c->red_h[4];
    out[6] = (c->e0 != 0.0) ? (c->e0 - E) / c->e0 : 0.0;
    return BH_OK;
}

int bh_stats_get(bh_ctx *c, bh_stats *out)
{
    if (!c) return BH_EINVAL;
    if (!out) return fail(c, BH_EINVAL, "null out");
    int st = read_misc(c);
    if (st) return st;
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
    *out = s;
    if (c->misc_h->walk_overflow) return fail(c, BH_EDEVICE, "walk list overflow");
    return BH_OK;
}

int bh_export_tree(bh_ctx *c, const bh_tree_host *o)
{
    if (!c) return BH_EINVAL;
    if (!o) return fail(c, BH_EINVAL, "null out");
    if (!c->built) return fail(c, BH_ESTATE, "no tree");
    TRY_HIP(c, hipStreamSynchronize(c->stream));
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
        if (o->prefix) o->prefix[i] = first[i] < (uint32_t)n ? (skey[first[i]] >> (3 * (kMaxLevel - level[i]))) : 0;
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
