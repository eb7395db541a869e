// tune.hip - autotuning of the leaf size and the group size per class of cluster
// (floor(log2 n), theta): each class of the loaded batch is stepped in a private
// context for every candidate pair and the fastest pair is kept.
#include <algorithm>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

#include "bh_internal.h"

using namespace bh;

namespace {

constexpr int kBlock = 256;
constexpr int32_t kLeafSizes[] = {8, 16, 32};
constexpr int32_t kGroupSizes[] = {32, 64, 128};

// positions and masses of the loaded batch in the caller's order
__global__ void __launch_bounds__(kBlock)
caller_order_kernel(int64_t n, const double4 *__restrict__ p4, const uint32_t *__restrict__ pid,
                    double *__restrict__ pos, double *__restrict__ mass)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double4 p = p4[i];
    const size_t o = pid[i];
    pos[3 * o] = p.x;
    pos[3 * o + 1] = p.y;
    pos[3 * o + 2] = p.z;
    mass[o] = p.w;
}

struct Scratch {
    double *pos = nullptr, *mass = nullptr, *spos = nullptr, *smass = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bh_ctx *tmp = nullptr;
    ~Scratch()
    {
        if (tmp) bh_destroy(tmp);
        for (double *p : {pos, mass, spos, smass})
            if (p) (void)hipFree(p);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        (void)hipGetLastError();
    }
};

// Milliseconds per dt = 0 step of the class's clusters with one (nleaf, ncrit).
int time_pair(bh_ctx *c, Scratch &w, std::vector<bh_cluster> cl, int64_t n, int32_t nleaf,
              int32_t ncrit, int32_t reps, double *ms)
{
    for (auto &q : cl) {
        q.nleaf = nleaf;
        q.ncrit = ncrit;
        q.dt = 0.0;
    }
    int st = bh_batch_build(w.tmp, cl.data(), (int64_t)cl.size(), w.spos, w.smass, nullptr);
    if (!st) st = bh_batch_forces(w.tmp, nullptr, nullptr);
    // two warm-up steps capture the graphs of both buffer parities, so no capture
    // or instantiation falls inside the timed steps
    if (!st) st = bh_batch_run(w.tmp, 2);
    if (st) return ctx_fail(c, st, bh_last_error(w.tmp));
    hipError_t e = hipEventRecord(w.ev[0], c->stream);
    if (e == hipSuccess) st = bh_batch_run(w.tmp, reps);
    if (st) return ctx_fail(c, st, bh_last_error(w.tmp));
    if (e == hipSuccess) e = hipEventRecord(w.ev[1], c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(w.ev[1]);
    float f = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, w.ev[0], w.ev[1]);
    if (e != hipSuccess) return ctx_hip_fail(c, e, "autotune timing");
    *ms = (double)f / reps;
    (void)n;
    return BH_OK;
}

}  // namespace

extern "C" {

int bh_autotune(bh_ctx *c, int32_t reps, bh_tune_entry *out, int64_t cap, int64_t *count)
{
    if (!c) return BH_EINVAL;
    if (!count) return ctx_fail(c, BH_EINVAL, "null count");
    if (reps < 1) return ctx_fail(c, BH_EINVAL, "reps must be >= 1");
    if (cap < 0 || (cap > 0 && !out)) return ctx_fail(c, BH_EINVAL, "bad output table");
    if (!c->built) return ctx_fail(c, BH_ESTATE, "autotune needs a loaded batch");
    int st = ctx_sync_check(c);
    if (st) return st;
    const int64_t n = c->n;
    Scratch w;
    hipError_t e = hipMalloc((void **)&w.pos, sizeof(double) * 3 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc((void **)&w.mass, sizeof(double) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc((void **)&w.spos, sizeof(double) * 3 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc((void **)&w.smass, sizeof(double) * (size_t)n);
    if (e == hipSuccess) e = hipEventCreate(&w.ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&w.ev[1]);
    if (e != hipSuccess) return ctx_hip_fail(c, e, "autotune scratch");
    hipLaunchKernelGGL(caller_order_kernel, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, c->stream, n, c->p4[c->cur], c->pid[c->cur], w.pos, w.mass);
    if ((e = hipGetLastError()) != hipSuccess) return ctx_hip_fail(c, e, "autotune gather");
    bh_params tp = c->p;
    tp.max_n = 0;
    tp.max_clusters = 0;
    tp.hbm_budget_bytes = 0;
    st = bh_create(&w.tmp, &tp, (void *)c->stream);
    if (st) return ctx_fail(c, st, "autotune context");

    // classes in order of first appearance
    std::vector<std::pair<int, float>> keys;
    std::map<std::pair<int, float>, std::vector<int64_t>> members;
    std::vector<int64_t> first(c->K);
    int64_t f = 0;
    for (int64_t k = 0; k < c->K; ++k) {
        first[k] = f;
        f += c->host_clusters[k].n;
        const auto key = std::make_pair(ctx_log2_floor(c->host_clusters[k].n), c->host_clusters[k].theta);
        if (!members.count(key)) keys.push_back(key);
        members[key].push_back(k);
    }
    std::vector<bh_tune_entry> table;
    for (const auto &key : keys) {
        std::vector<bh_cluster> cl;
        int64_t m = 0;
        for (int64_t k : members[key]) {
            const bh_cluster &q = c->host_clusters[k];
            e = hipMemcpyAsync(w.spos + 3 * m, w.pos + 3 * first[k], sizeof(double) * 3 * (size_t)q.n,
                               hipMemcpyDeviceToDevice, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(w.smass + m, w.mass + first[k], sizeof(double) * (size_t)q.n,
                                   hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) return ctx_hip_fail(c, e, "autotune copy");
            cl.push_back(q);
            m += q.n;
        }
        bh_tune_entry best;
        memset(&best, 0, sizeof(best));
        best.log2n = key.first;
        best.theta = key.second;
        best.ms = -1.0;
        best.ms_default = -1.0;
        for (int32_t nl : kLeafSizes) {
            for (int32_t nc : kGroupSizes) {
                double ms = 0.0;
                st = time_pair(c, w, cl, m, nl, nc, reps, &ms);
                if (st) return st;
                if (best.ms < 0.0 || ms < best.ms) {
                    best.ms = ms;
                    best.nleaf = nl;
                    best.ncrit = nc;
                }
                if (nl == c->p.nleaf && nc == c->p.ncrit) best.ms_default = ms;
            }
        }
        if (best.ms_default < 0.0) {
            st = time_pair(c, w, cl, m, c->p.nleaf, c->p.ncrit, reps, &best.ms_default);
            if (st) return st;
        }
        table.push_back(best);
    }
    c->tuning = table;
    *count = (int64_t)table.size();
    for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)table.size()); ++i) out[i] = table[i];
    return BH_OK;
}

int bh_set_tuning(bh_ctx *c, const bh_tune_entry *entries, int64_t count)
{
    if (!c) return BH_EINVAL;
    if (count < 0 || (count > 0 && !entries)) return ctx_fail(c, BH_EINVAL, "bad tuning table");
    for (int64_t i = 0; i < count; ++i) {
        const bh_tune_entry &t = entries[i];
        if (t.nleaf < 1 || t.nleaf > 64 || t.ncrit < 1 || t.ncrit > kMaxGroup || !(t.theta > 0.0f) ||
            t.log2n < 0 || t.log2n > 31)
            return ctx_fail(c, BH_EINVAL, "tuning entry out of range");
    }
    c->tuning.assign(entries, entries + count);
    return BH_OK;
}

}  // extern "C"
