// serve.hip - the serving loop declared in include/bh.h: requests (one system
// each: a force evaluation, then leapfrog steps) queue for admission by the
// memory budget, live as clusters of one resident batch, and advance together
// one unit per iteration; the batch is repacked on the device whenever requests
// join or leave.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "bh_internal.h"

using namespace bh;

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Copies one resident cluster's particles from one buffer parity to the other,
// renumbering the caller indices to the cluster's new first position.  The
// accelerations move through a staging array (they have a single buffer).
__global__ void __launch_bounds__(kBlock)
move_kernel(const double4 *__restrict__ p4s, const double4 *__restrict__ v4s,
            const uint32_t *__restrict__ pids, const float4 *__restrict__ accs, uint32_t src,
            double4 *__restrict__ p4d, double4 *__restrict__ v4d, uint32_t *__restrict__ pidd,
            float4 *__restrict__ accd, uint32_t dst, uint32_t n, DevMisc *m)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t q = pids[src + i];
    // a cluster's caller indices are its own positions; anything else is an
    // internal error (bit 3), reported by the next check
    if (q < src || q - src >= n) atomicOr(&m->nonfinite, 8u);
    p4d[dst + i] = p4s[src + i];
    v4d[dst + i] = v4s[src + i];
    pidd[dst + i] = (q < src || q - src >= n) ? dst + i : q - src + dst;
    accd[dst + i] = accs[src + i];
}

// Loads a new request's arrays (its own order, checked at admission) at position
// dst; accelerations start at zero (its first unit is a step with dt = 0, i.e. a
// force evaluation).
__global__ void __launch_bounds__(kBlock)
load_kernel(const double *__restrict__ pos, const double *__restrict__ mass,
            const double *__restrict__ vel, double4 *__restrict__ p4, double4 *__restrict__ v4,
            uint32_t *__restrict__ pid, float4 *__restrict__ accd, uint32_t dst, uint32_t n)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    p4[dst + i] = make_double4(pos[3 * (size_t)i], pos[3 * (size_t)i + 1], pos[3 * (size_t)i + 2],
                               mass[i]);
    v4[dst + i] = vel ? make_double4(vel[3 * (size_t)i], vel[3 * (size_t)i + 1], vel[3 * (size_t)i + 2], mass[i])
                      : make_double4(0.0, 0.0, 0.0, mass[i]);     // w: the mass
    pid[dst + i] = dst + i;
    accd[dst + i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// Sets flag[0] if any coordinate, velocity or mass of a request is unusable.
__global__ void __launch_bounds__(kBlock)
check_kernel(const double *__restrict__ pos, const double *__restrict__ mass,
             const double *__restrict__ vel, uint32_t n, uint32_t *__restrict__ flag)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    if (i < n) {
        const double ms = mass[i];
        bad = !(ms > 0.0) || !isfinite(ms);
        for (int k = 0; k < 3; ++k) {
            bad |= !isfinite(pos[3 * (size_t)i + k]);
            if (vel) bad |= !isfinite(vel[3 * (size_t)i + k]);
        }
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(flag, 1u);
}

__global__ void __launch_bounds__(kBlock) clear_u32_kernel(uint32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void __launch_bounds__(kBlock)
copy_f4_kernel(const float4 *__restrict__ a, float4 *__restrict__ b, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// One cluster's state in its request's own order.
__global__ void __launch_bounds__(kBlock)
cluster_out_kernel(const double4 *__restrict__ p4, const double4 *__restrict__ v4,
                   const uint32_t *__restrict__ pid, const float4 *__restrict__ acc4,
                   uint32_t first, uint32_t n, double *__restrict__ pos, double *__restrict__ vel,
                   float *__restrict__ acc, float *__restrict__ pot, DevMisc *m)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const size_t s = first + i;
    const uint32_t q = pid[s];
    if (q < first || q - first >= n) {     // internal error (bit 3): never write outside
        atomicOr(&m->nonfinite, 8u);
        return;
    }
    const size_t o = q - first;
    if (pos) {
        const double4 p = p4[s];
        pos[3 * o] = p.x;
        pos[3 * o + 1] = p.y;
        pos[3 * o + 2] = p.z;
    }
    if (vel) {
        const double4 v = v4[s];
        vel[3 * o] = v.x;
        vel[3 * o + 1] = v.y;
        vel[3 * o + 2] = v.z;
    }
    const float4 a = acc4[s];
    if (acc) {
        acc[3 * o] = a.x;
        acc[3 * o + 1] = a.y;
        acc[3 * o + 2] = a.z;
    }
    if (pot) pot[o] = a.w;
}

struct Req {
    bh_request r;
    int64_t ticket;
    int state = BH_REQ_QUEUED;
    int units_done = 0;
    bool placed = false;     // its particles are in the batch buffers
    uint32_t first = 0;      // then its first position there
    double arrival = 0, admitted = -1, completed = -1;
    double e0 = 0;
    double energy[7] = {0, 0, 0, 0, 0, 0, 0};
};

double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)std::floor(pos), hi = std::min(v.size() - 1, lo + 1);
    const double f = pos - (double)lo;
    return v[lo] * (1.0 - f) + v[hi] * f;
}

}  // namespace

struct bh_server {
    bh_server_params p{};
    bh_ctx *ctx = nullptr;
    std::string err;
    std::chrono::steady_clock::time_point t0;
    int64_t cap_n = 0;                   // resident particle capacity
    int64_t next_ticket = 1;
    std::unordered_map<int64_t, Req> reqs;
    std::deque<int64_t> queue;           // tickets waiting for admission
    std::vector<int64_t> resident;       // tickets in cluster order
    int64_t resident_n = 0;
    bool layout_dirty = false;
    bool stable = false;                 // layout unchanged since the last iteration
    std::vector<double> latencies, waits;
    bh_server_stats st{};
    uint32_t *bad = nullptr;             // device [max_requests] input-check flags
    uint32_t *bad_h = nullptr;           // pinned host copy

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

int sfail(bh_server *s, int code, const std::string &msg)
{
    s->err = msg;
    return code;
}

int ctx_err(bh_server *s, int code)
{
    s->err = bh_last_error(s->ctx);
    return code;
}

#define S_TRY(s, expr)                       \
    do {                                     \
        int st__ = (expr);                   \
        if (st__) return ctx_err((s), st__); \
    } while (0)

#define S_HIP(s, expr)                                                       \
    do {                                                                     \
        hipError_t e__ = (expr);                                             \
        if (e__ != hipSuccess) {                                             \
            (void)hipGetLastError();                                         \
            return sfail((s), BH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e__)); \
        }                                                                    \
    } while (0)

bh_cluster cluster_of(const Req &q)
{
    bh_cluster c{};
    c.n = q.r.n;
    c.mac = q.r.mac;
    c.theta = q.r.theta;
    c.eps = q.r.eps;
    // the first unit of a request is its force evaluation: a step with dt = 0
    c.dt = q.units_done == 0 ? 0.0 : q.r.dt;
    c.nleaf = q.r.nleaf;
    c.ncrit = q.r.ncrit;
    return c;
}

// Admits queued requests in arrival order while they fit.  Their arrays are
// checked on the device first; a request with a non-finite value or a mass that
// is not positive is rejected (BH_REQ_FAILED) and never joins the batch.
int admit(bh_server *s, double t)
{
    bh_ctx *c = s->ctx;
    std::vector<int64_t> cand;
    int64_t n = s->resident_n;
    size_t k = s->resident.size();
    for (int64_t tk : s->queue) {
        const Req &q = s->reqs[tk];
        if (n + q.r.n > s->cap_n || (int64_t)k >= s->p.max_requests) break;
        // the working-set limit, which a lone request may exceed
        if (s->p.max_resident > 0 && n > 0 && n + q.r.n > s->p.max_resident) break;
        cand.push_back(tk);
        n += q.r.n;
        k += 1;
    }
    if (cand.empty()) return BH_OK;
    hipLaunchKernelGGL(clear_u32_kernel, dim3(grid_for((int64_t)cand.size())), dim3(kBlock), 0,
                       c->stream, s->bad, (int64_t)cand.size());
    S_HIP(s, hipGetLastError());
    for (size_t j = 0; j < cand.size(); ++j) {
        const Req &q = s->reqs[cand[j]];
        hipLaunchKernelGGL(check_kernel, dim3(grid_for(q.r.n)), dim3(kBlock), 0, c->stream, q.r.pos,
                           q.r.mass, q.r.vel, (uint32_t)q.r.n, s->bad + j);
        S_HIP(s, hipGetLastError());
    }
    S_HIP(s, hipMemcpyAsync(s->bad_h, s->bad, sizeof(uint32_t) * cand.size(), hipMemcpyDeviceToHost,
                            c->stream));
    S_HIP(s, hipStreamSynchronize(c->stream));
    for (size_t j = 0; j < cand.size(); ++j) {
        s->queue.pop_front();
        Req &q = s->reqs[cand[j]];
        q.admitted = t;
        s->waits.push_back(q.admitted - q.arrival);
        if (s->bad_h[j]) {
            q.state = BH_REQ_FAILED;
            q.completed = t;
            s->st.rejected += 1;
            continue;
        }
        q.state = BH_REQ_RUNNING;
        s->resident.push_back(q.ticket);
        s->resident_n += q.r.n;
        s->layout_dirty = true;
        s->st.admitted += 1;
    }
    return BH_OK;
}

// Places the resident requests contiguously in cluster order in the other
// buffer parity: survivors move from the ranges they hold, new ones load from
// their arrays.
int repack(bh_server *s)
{
    bh_ctx *c = s->ctx;
    const int src = c->cur, dst = src ^ 1;
    // accelerations move through the group-centre array (rebuilt by every step)
    float4 *acc_stage = reinterpret_cast<float4 *>(c->g_centre);
    uint32_t pos = 0;
    for (int64_t t : s->resident) {
        Req &q = s->reqs[t];
        const uint32_t n = (uint32_t)q.r.n;
        if (q.placed) {
            hipLaunchKernelGGL(move_kernel, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, c->p4[src],
                               c->v4[src], c->pid[src], c->acc4, q.first, c->p4[dst], c->v4[dst],
                               c->pid[dst], acc_stage, pos, n, c->misc);
        } else {
            hipLaunchKernelGGL(load_kernel, dim3(grid_for(n)), dim3(kBlock), 0, c->stream, q.r.pos,
                               q.r.mass, q.r.vel, c->p4[dst], c->v4[dst], c->pid[dst], acc_stage,
                               pos, n);
        }
        S_HIP(s, hipGetLastError());
        q.placed = true;
        q.first = pos;
        pos += n;
    }
    if (pos > 0) {
        hipLaunchKernelGGL(copy_f4_kernel, dim3(grid_for(pos)), dim3(kBlock), 0, c->stream, acc_stage,
                           c->acc4, (int64_t)pos);
        S_HIP(s, hipGetLastError());
    }
    c->cur = dst;
    return BH_OK;
}

}  // namespace

extern "C" {

int bh_server_create(bh_server **out, const bh_server_params *p, void *hip_stream)
{
    if (!out || !p) return BH_EINVAL;
    *out = nullptr;
    if (p->hbm_budget_bytes <= 0 || p->max_requests < 1 || p->max_requests > (1 << 20) ||
        p->nleaf < 1 || p->nleaf > 64 || p->ncrit < 1 || p->ncrit > kMaxGroup || p->min_nleaf < 0 ||
        p->min_nleaf > p->nleaf || p->max_resident < 0)
        return BH_EINVAL;
    bh_server *s = new (std::nothrow) bh_server();
    if (!s) return BH_ENOMEM;
    s->p = *p;
    if (s->p.min_nleaf == 0) s->p.min_nleaf = std::min(8, p->nleaf);
    const int lmin = s->p.min_nleaf;
    s->t0 = std::chrono::steady_clock::now();
    bh_params cp;
    bh_default_params(&cp);
    cp.nleaf = p->nleaf;
    cp.ncrit = p->ncrit;
    cp.hbm_budget_bytes = p->hbm_budget_bytes;
    int st = bh_create(&s->ctx, &cp, hip_stream);
    if (st) {
        delete s;
        return st;
    }
    // the largest resident particle count whose buffers fit the budget, with the
    // smallest leaf size a request may choose, and whose cell indices fit the walk
    int64_t lo = 0, hi = 0x7fffffffLL;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (ctx_cells_fit(mid, p->max_requests, lmin) &&
            ctx_bytes_for(s->ctx, mid, p->max_requests, lmin) <= p->hbm_budget_bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    if (lo < 1) {
        bh_destroy(s->ctx);
        delete s;
        return BH_ENOMEM;
    }
    st = ctx_reserve(s->ctx, lo, p->max_requests, lmin);
    if (st == BH_OK &&
        (hipMalloc((void **)&s->bad, sizeof(uint32_t) * (size_t)p->max_requests) != hipSuccess ||
         hipHostMalloc((void **)&s->bad_h, sizeof(uint32_t) * (size_t)p->max_requests,
                       hipHostMallocDefault) != hipSuccess)) {
        (void)hipGetLastError();
        st = BH_ENOMEM;
    }
    if (st) {
        bh_server_destroy(s);
        return st;
    }
    s->cap_n = lo;
    *out = s;
    return BH_OK;
}

int bh_server_destroy(bh_server *s)
{
    if (!s) return BH_OK;
    bh_destroy(s->ctx);
    if (s->bad) (void)hipFree(s->bad);
    if (s->bad_h) (void)hipHostFree(s->bad_h);
    delete s;
    return BH_OK;
}

int bh_server_submit(bh_server *s, const bh_request *r, int64_t *ticket)
{
    if (!s) return BH_EINVAL;
    if (!r || !ticket) return sfail(s, BH_EINVAL, "null request or ticket");
    if (!r->pos || !r->mass) return sfail(s, BH_EINVAL, "null pos or mass");
    if (r->nsteps < 0) return sfail(s, BH_EINVAL, "nsteps must be >= 0");
    bh_cluster c{};
    c.n = r->n;
    c.mac = r->mac;
    c.theta = r->theta;
    c.eps = r->eps;
    c.dt = r->dt;
    c.nleaf = r->nleaf;
    c.ncrit = r->ncrit;
    std::vector<bh_cluster> chk;
    int64_t total = 0;
    S_TRY(s, ctx_check_clusters(s->ctx, &c, 1, chk, &total));
    if (r->n > s->cap_n) return sfail(s, BH_ENOMEM, "request larger than the server's capacity");
    if (chk[0].nleaf < s->p.min_nleaf)
        return sfail(s, BH_EINVAL, "request leaf size below the server's min_nleaf");
    Req q;
    q.r = *r;
    q.r.nleaf = chk[0].nleaf;
    q.r.ncrit = chk[0].ncrit;
    q.ticket = s->next_ticket++;
    q.arrival = r->arrival >= 0.0 ? r->arrival : s->now();
    s->reqs.emplace(q.ticket, q);
    s->queue.push_back(q.ticket);
    s->st.submitted += 1;
    *ticket = q.ticket;
    return BH_OK;
}

int bh_server_step(bh_server *s, int64_t *resident)
{
    if (!s) return BH_EINVAL;
    const double t_in = s->now();
    bh_ctx *c = s->ctx;
    {
        const int st = admit(s, t_in);
        if (st) return st;
    }
    if (resident) *resident = (int64_t)s->resident.size();
    if (s->resident.empty()) {
        s->st.busy_seconds += s->now() - t_in;
        return BH_OK;
    }
    std::vector<bh_cluster> table;
    table.reserve(s->resident.size());
    for (int64_t t : s->resident) table.push_back(cluster_of(s->reqs[t]));
    bool graph = false;
    if (s->layout_dirty) {
        S_TRY(s, ctx_sync_check(c));
        int st = repack(s);
        if (st) return st;
        S_TRY(s, ctx_set_layout(c, table, s->resident_n));
        s->layout_dirty = false;
        s->stable = false;
    } else {
        S_TRY(s, ctx_update_params(c, table));
        // replay the captured step once the layout has held for an iteration
        graph = s->stable;
        s->stable = true;
    }
    S_TRY(s, ctx_step(c, graph));
    // outputs of the requests that finish with this unit
    std::vector<int64_t> finishing;
    for (int64_t t : s->resident) {
        Req &q = s->reqs[t];
        const uint32_t n = (uint32_t)q.r.n;
        const uint32_t first = q.first;
        if (q.units_done + 1 >= 1 + q.r.nsteps) {
            finishing.push_back(t);
            if (q.r.out_pos || q.r.out_vel || q.r.out_acc || q.r.out_pot) {
                hipLaunchKernelGGL(cluster_out_kernel, dim3(grid_for(n)), dim3(kBlock), 0, c->stream,
                                   c->p4[c->cur], c->v4[c->cur], c->pid[c->cur], c->acc4, first, n,
                                   q.r.out_pos, q.r.out_vel, q.r.out_acc, q.r.out_pot, c->misc);
                S_HIP(s, hipGetLastError());
            }
        }
    }
    const int64_t K = (int64_t)s->resident.size();
    S_HIP(s, hipMemcpyAsync(c->e_out_h, c->e_out, sizeof(double) * 5 * (size_t)K,
                            hipMemcpyDeviceToHost, c->stream));
    S_TRY(s, ctx_sync_check(c));
    const double t_out = s->now();
    for (int64_t k = 0; k < K; ++k) {
        Req &q = s->reqs[s->resident[k]];
        const double *e = c->e_out_h + 5 * k;
        const double T = e[0], W = e[1], E = T + W;
        if (q.units_done == 0) q.e0 = E;
        q.energy[0] = T;
        q.energy[1] = W;
        q.energy[2] = E;
        q.energy[3] = e[2];
        q.energy[4] = e[3];
        q.energy[5] = e[4];
        q.energy[6] = q.e0 != 0.0 ? (q.e0 - E) / q.e0 : 0.0;
        q.units_done += 1;
    }
    if (!finishing.empty()) {
        for (int64_t t : finishing) {
            Req &q = s->reqs[t];
            q.state = BH_REQ_DONE;
            q.completed = t_out;
            s->latencies.push_back(q.completed - q.arrival);
            s->st.completed += 1;
            s->st.particle_evals += q.r.n * (1 + (int64_t)q.r.nsteps);
            s->resident_n -= q.r.n;
        }
        std::vector<int64_t> keep;
        for (int64_t t : s->resident)
            if (s->reqs[t].state != BH_REQ_DONE) keep.push_back(t);
        s->resident.swap(keep);
        s->layout_dirty = true;
    }
    s->st.iterations += 1;
    s->st.busy_seconds += s->now() - t_in;
    return BH_OK;
}

int bh_server_poll(bh_server *s, int64_t ticket, bh_request_status *out)
{
    if (!s) return BH_EINVAL;
    if (!out) return sfail(s, BH_EINVAL, "null out");
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(s, BH_EINVAL, "unknown ticket");
    const Req &q = it->second;
    out->state = q.state;
    out->units_done = q.units_done;
    out->arrival = q.arrival;
    out->admitted = q.admitted;
    out->completed = q.completed;
    for (int j = 0; j < 7; ++j) out->energy[j] = q.energy[j];
    return BH_OK;
}

int bh_server_release(bh_server *s, int64_t ticket)
{
    if (!s) return BH_EINVAL;
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return sfail(s, BH_EINVAL, "unknown ticket");
    const int state = it->second.state;
    if (state != BH_REQ_DONE && state != BH_REQ_FAILED)
        return sfail(s, BH_ESTATE, "request still queued or running");
    s->reqs.erase(it);
    return BH_OK;
}

int bh_server_stats_get(bh_server *s, bh_server_stats *out)
{
    if (!s) return BH_EINVAL;
    if (!out) return sfail(s, BH_EINVAL, "null out");
    bh_server_stats r = s->st;
    r.queued = (int64_t)s->queue.size();
    r.resident_requests = (int64_t)s->resident.size();
    r.resident_particles = s->resident_n;
    r.capacity_particles = s->cap_n;
    r.latency_p50 = percentile(s->latencies, 0.50);
    r.latency_p99 = percentile(s->latencies, 0.99);
    r.latency_max = s->latencies.empty() ? 0.0 : *std::max_element(s->latencies.begin(), s->latencies.end());
    r.queue_wait_p50 = percentile(s->waits, 0.50);
    r.queue_wait_p99 = percentile(s->waits, 0.99);
    *out = r;
    return BH_OK;
}

int bh_server_set_tuning(bh_server *s, const bh_tune_entry *entries, int64_t count)
{
    if (!s) return BH_EINVAL;
    for (int64_t i = 0; entries && i < count; ++i)
        if (entries[i].nleaf < s->p.min_nleaf)
            return sfail(s, BH_EINVAL, "tuned leaf size below the server's min_nleaf");
    S_TRY(s, bh_set_tuning(s->ctx, entries, count));
    return BH_OK;
}

int bh_server_now(bh_server *s, double *t)
{
    if (!s || !t) return BH_EINVAL;
    *t = s->now();
    return BH_OK;
}

const char *bh_server_last_error(bh_server *s)
{
    if (!s) return "null server";
    return s->err.c_str();
}

}  // extern "C"
