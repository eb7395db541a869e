// walk.hip - the group walk and force evaluation (Sect. 2.2, 3.3).
//
// One wavefront (64 lanes) takes one group of at most 128 particles.  It walks
// the tree from the root: up to 64 cells are tested at a time, one per lane,
// with the cluster's opening test (Eq. (1), or the minimum distance between the
// group's box and the cell's cube, the alternative of Sect. 3.3; both in float32
// on offsets from the group centre).  An accepted cell goes to the cell list, an
// opened leaf to the particle list, an opened node pushes its contiguous
// children.  As soon as a list holds a full tile it is evaluated: the sources
// are staged in LDS as float32 offsets from the group's box centre and every
// lane accumulates them on its particles.  A lane carries M particles of the
// group (M = 1, 2 or 3, whichever needs the fewest loop trips per tile; groups
// of more than 64 particles need M >= 2): P = ceil(g / M) particle slots,
// k = floor(64 / P) lanes per slot (the paper uses up to 4 threads per
// particle).  Lane (p, s) takes sources s, s + k, s + 2k, ... of each tile and
// the k partial sums are added at the end.  A full tile of cells holds
// k ceil(64 / k) entries, so that no lane runs a padded trip; a tile of
// particles holds 64.
//
// Per wavefront, in LDS:
//   stack : pending cell ranges (first cell, count <= 8) packed in 32 bits, used
//           last-in first-out.  A pop takes up to 64 cells from the top; each pop
//           pushes at most 64 ranges, all deeper than anything popped before them
//           that is still held, so at most 64 ranges per level (21 levels, 1344)
//           can be on it.  The first 128 entries live in LDS; deeper entries go to
//           a per-wavefront region in device memory (a Plummer sphere of 2^20
//           particles needs about 50 at theta = 0.75 and 140 at theta = 0.4).
//   cells : the cell list, already staged as float32 tiles (offset from the
//           group centre, mass, second moment): a lane that accepts a cell writes
//           its entry from the record it just read for the opening test, so no
//           cell record is read twice.  Fewer than 64 entries between
//           evaluations, plus padding (far away, zero mass) behind the evaluated
//           tile so that every lane runs the same number of iterations.
//   pp    : opened leaves as (first particle, count) ranges (< 64 particles
//           pending between evaluations, so < 128 ranges).
//   tile  : 64 staged particles plus padding.
//
// Every pair goes through float32 arithmetic on group-centred offsets; a lane's
// terms are summed in plain float32 over at most 64 terms (one tile with one
// lane per particle, several smaller tiles otherwise), and these partial sums are
// added to the particle's totals with an error-free two-sum (compensated
// accumulation).
//
// Groups are handed out in Morton order (a wavefront's first group is its own
// index, the rest come from one device-wide counter), so at any
// moment all 256 CUs work on neighbouring groups whose interaction lists overlap:
// the active part of the tree stays small and shared in the Infinity Cache.
// (Splitting the groups into per-XCD ranges, so that each XCD's L2 sees one
// region, measured 17% slower at N = 2^20.)
#include "bh_internal.h"

#pragma clang fp contract(off)

namespace bh {
namespace {

constexpr int kWalkBlock = kWalkWaves * kWave;
constexpr int kPpCap = 128;
constexpr int kLdsStack = 128;
constexpr int kSpillPerWave = kStackCap - kLdsStack;
// Lane (p, s) reads tile entries s + t k for t < ceil(cnt / k): at most 83 past
// the tile's first entry for cnt <= 64 and k = floor(64 / g); the tail is padding.
constexpr int kTileReach = 84;
// Cell tiles: with BH_WALK_FLEX_TILE a full tile holds k ceil(64 / k) cells (at
// most 84, for k = 21), so that every lane's trips read real cells; otherwise 64
// cells and padding.  The cell list holds fewer than a full tile between
// evaluations plus at most 64 from one pop (< 148 entries); the last, partial
// tile of fewer than 84 cells is read up to 83 + 20 past its start.
// Particle tiles of k floor(64 / k) particles for k lanes per particle slot.
#ifndef BH_WALK_PP_FULL
#define BH_WALK_PP_FULL 1
#endif
// Stack reads and pushes that stay within the LDS part use LDS instructions only.
#ifndef BH_WALK_LDS_FAST
#define BH_WALK_LDS_FAST 1
#endif
#ifndef BH_WALK_FLEX_TILE
#define BH_WALK_FLEX_TILE 1
#endif
constexpr int kPcCap = 148;
constexpr float kFar = 1.0e30f;
#ifndef BH_WALK_UNROLL
#define BH_WALK_UNROLL 4
#endif
#ifndef BH_WALK_WAVES_PER_EU
#define BH_WALK_WAVES_PER_EU 4
#endif
constexpr int kUnroll = BH_WALK_UNROLL;   // tile entries per loop trip
// Workgroups of the persistent grid per CU: as many as are resident at once (LDS
// and registers allow four).  A larger grid leaves workgroups waiting for a slot,
// and the groups those hold from the start (each wavefront's first group is its
// own index) are then walked only at the end, after the rest of the tree has
// left the caches.
#ifndef BH_WALK_BLOCKS_PER_CU
#define BH_WALK_BLOCKS_PER_CU 4
#endif

struct WalkArgs {
    const DevCluster *clus;   // per-cluster softening
    const uint32_t *g_first;
    const uint32_t *g_count;
    const double4 *g_centre;  // box centre; w: the group's cluster (its root cell)
    const float4 *g_half;
    const double4 *p4;        // sources and targets: x, y, z, mass (sorted order)
    const WalkCell *rec;      // per-cell walk records
    const double4 *geo;       // per-cell geometric centre, half side (minimum-distance test)
    float4 *acc4;             // out: ax, ay, az, pot (sorted order)
    uint32_t *g_npp;
    uint32_t *g_npc;
    uint32_t *spill;          // kSpillPerWave entries per wavefront of the grid
    unsigned long long *part; // out: per-workgroup interaction totals (p-p, p-c)
    DevMisc *misc;            // group and cell counts, work counter, interaction totals
    const uint32_t *glist;    // groups to walk (misc->nactive of them), or null: all
};

struct WaveLds {
    uint32_t stack[kLdsStack];
    uint2 pp[kPpCap];
    // the cell list, staged as it is built
    float4 ca[kPcCap];        // offset x, y, z; mass
    float4 cb[kPcCap];        // 3Sxx, 3Syy, 3Szz, 3Sxy
    float4 cc[kPcCap];        // 3Sxz, 3Syz, tr(S)/2, 3 tr(S)/2
    union {
        float4 ta[kTileReach];  // particle tile: offset x, y, z; mass
        int mark[kWave];        // scratch of pop64 (never live during a particle tile)
    };
};
static_assert(4 * sizeof(WaveLds) * 4 <= 160 * 1024, "four blocks of four wavefronts per CU");

// Running sums of the M particles a lane carries, with their compensations, and
// the plain float32 partial sums of the tiles evaluated since the last
// compensated addition (trips: terms per partial so far, the same in every lane).
template <int M>
struct Acc {
    float ax[M], ay[M], az[M], ph[M];
    float cx[M], cy[M], cz[M], cp[M];
    float px[M], py[M], pz[M], pp[M];
    int trips;
};

// A partial is added to the compensated totals before it could hold more than
// this many plain float32 terms (64: the terms of one tile with one lane per
// particle).  BH_WALK_COMP_EVERY_TILE: after every tile instead.
#ifndef BH_WALK_COMP_EVERY_TILE
#define BH_WALK_COMP_EVERY_TILE 0
#endif
constexpr int kPlainTerms = 64;

// s + t with the rounding error of the addition carried in c (two-sum).
__device__ __forceinline__ void comp_add(float &s, float &c, float t)
{
    const float r = s + t;
    const float bp = r - s;
    const float err = (s - (r - bp)) + (t - bp);
    s = r;
    c = c + err;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Pop up to cap <= 64 elements (cap the same in every lane) from a list of
// ranges kept as a stack.  Lane j receives element j of the popped run in *elem;
// returns how many were popped.
template <class List>
__device__ __forceinline__ int pop64(List list, int &top, int *mark, uint32_t &elem,
                                     int cap = kWave)
{
    const int lane = lane_id();
    const int m = top < kWave ? top : kWave;
    uint32_t f = 0, cnt = 0;
    // a stack whose entries all lie in LDS is read with LDS loads only (top is
    // the same in every lane, so the branch is uniform)
    if (BH_WALK_LDS_FAST && list.all_lds(top)) {
        if (lane < m) list.get_lds(top - 1 - lane, f, cnt);
    } else {
        if (lane < m) list.get(top - 1 - lane, f, cnt);
    }
    const uint32_t incl = wave_incl_scan_add(cnt);
    const uint32_t excl = incl - cnt;
    uint32_t take = 0;
    if (lane < m && excl < (uint32_t)cap) {
        const uint32_t room = (uint32_t)cap - excl;
        take = cnt < room ? cnt : room;
    }
    const bool full = lane < m && take == cnt;
    const int nfull = __popcll(ballot(full));
    const uint32_t total = lane_value(incl, m - 1);
    const int got = uniform(total < (uint32_t)cap ? (int)total : cap);
    // the lanes that take a range form a prefix with strictly increasing starts,
    // so the range that output slot `lane` comes from is the number of range
    // starts at or below it, minus one
    mark[lane] = 0;
    wave_sync();
    if (take > 0) mark[excl] = 1;
    wave_sync();
    const unsigned long long starts = ballot(mark[lane] != 0);
    int src = mask_rank(starts) + (int)((starts >> lane) & 1ull) - 1;
    src = src < 0 ? 0 : src;
    const uint32_t fs = __shfl(f, src, kWave);
    const uint32_t es = __shfl(excl, src, kWave);
    elem = fs + ((uint32_t)lane - es);
    if (lane == nfull && lane < m && take > 0 && take < cnt) {
        if (BH_WALK_LDS_FAST && list.all_lds(top)) list.set_lds(top - 1 - lane, f + take, cnt - take);
        else list.set(top - 1 - lane, f + take, cnt - take);
    }
    // only an access to the device part needs its stores waited for
    const bool lds_only = BH_WALK_LDS_FAST && list.all_lds(top);
    top -= nfull;
    if (lds_only) wave_sync();
    else list.sync();
    return got;
}

// Cell ranges packed as first << 3 | (count - 1); LDS first, then device memory.
struct CellStack {
    uint32_t *s;
    volatile uint32_t *spill;
    __device__ bool all_lds(int n) const { return n <= kLdsStack; }
    __device__ void get(int i, uint32_t &f, uint32_t &c) const
    {
        const uint32_t v = i < kLdsStack ? s[i] : spill[i - kLdsStack];
        f = v >> 3;
        c = (v & 7u) + 1u;
    }
    __device__ void get_lds(int i, uint32_t &f, uint32_t &c) const
    {
        const uint32_t v = s[i];
        f = v >> 3;
        c = (v & 7u) + 1u;
    }
    __device__ void set_lds(int i, uint32_t f, uint32_t c) const { s[i] = (f << 3) | (c - 1u); }
    __device__ void set(int i, uint32_t f, uint32_t c) const
    {
        const uint32_t v = (f << 3) | (c - 1u);
        if (i < kLdsStack) s[i] = v;
        else spill[i - kLdsStack] = v;
    }
    // stores to device memory must have landed before another lane reads them
    __device__ void sync() const
    {
        __builtin_amdgcn_s_waitcnt(0);
        wave_sync();
    }
};

struct LeafList {
    uint2 *s;
    __device__ bool all_lds(int) const { return true; }
    __device__ void get(int i, uint32_t &f, uint32_t &c) const
    {
        const uint2 v = s[i];
        f = v.x;
        c = v.y;
    }
    __device__ void get_lds(int i, uint32_t &f, uint32_t &c) const { get(i, f, c); }
    __device__ void set_lds(int i, uint32_t f, uint32_t c) const { set(i, f, c); }
    __device__ void set(int i, uint32_t f, uint32_t c) const { s[i] = make_uint2(f, c); }
    __device__ void sync() const { wave_sync(); }
};

// particle j on the lane's target (offsets o from the group centre)
template <bool kEps0>
__device__ __forceinline__ void pp_term(const float4 s, float ox, float oy, float oz, float eps2,
                                        float &ax, float &ay, float &az, float &ph)
{
    const float dx = s.x - ox, dy = s.y - oy, dz = s.z - oz;
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, __builtin_fmaf(dz, dz, eps2)));
    float ri = __builtin_amdgcn_rsqf(r2);
    if (kEps0) ri = r2 > 0.0f ? ri : 0.0f;
    const float mr = s.w * ri;
    const float ri2 = ri * ri;
    const float mr3 = mr * ri2;
    ax = __builtin_fmaf(mr3, dx, ax);
    ay = __builtin_fmaf(mr3, dy, ay);
    az = __builtin_fmaf(mr3, dz, az);
    ph = ph - mr;
}

// cell (A = offset of its centre of mass, mass; B, C = 3S and trace terms) on the
// lane's target: monopole plus quadrupole with softened inverse distance rho,
//   phi = -M rho - 3/2 r.S.r rho^5 + 1/2 tr(S) rho^3,   a = -grad phi.
template <bool kEps0>
__device__ __forceinline__ void pc_term(const float4 A, const float4 B, const float4 C, float ox,
                                        float oy, float oz, float eps2, float &ax, float &ay,
                                        float &az, float &ph)
{
    const float rx = ox - A.x, ry = oy - A.y, rz = oz - A.z;
    const float r2 = __builtin_fmaf(rx, rx, __builtin_fmaf(ry, ry, __builtin_fmaf(rz, rz, eps2)));
    float rho = __builtin_amdgcn_rsqf(r2);
    if (kEps0) rho = r2 > 0.0f ? rho : 0.0f;
    const float rho2 = rho * rho;
    const float rho3 = rho2 * rho;
    const float rho5 = rho3 * rho2;
    const float sx = __builtin_fmaf(B.x, rx, __builtin_fmaf(B.w, ry, C.x * rz));
    const float sy = __builtin_fmaf(B.w, rx, __builtin_fmaf(B.y, ry, C.y * rz));
    const float sz = __builtin_fmaf(C.x, rx, __builtin_fmaf(C.y, ry, B.z * rz));
    const float u = __builtin_fmaf(rx, sx, __builtin_fmaf(ry, sy, rz * sz));   // 3 r.S.r
    const float w1 = rho2 * u;
    const float tp = __builtin_fmaf(-0.5f, w1, C.z);
    const float ip = __builtin_fmaf(rho2, tp, -A.w);
    ph = __builtin_fmaf(rho, ip, ph);
    const float ta = __builtin_fmaf(-2.5f, w1, C.w);
    const float f = __builtin_fmaf(rho2, ta, -A.w);
    const float g = rho3 * f;
    ax = __builtin_fmaf(g, rx, ax);
    ay = __builtin_fmaf(g, ry, ay);
    az = __builtin_fmaf(g, rz, az);
    ax = __builtin_fmaf(rho5, sx, ax);
    ay = __builtin_fmaf(rho5, sy, ay);
    az = __builtin_fmaf(rho5, sz, az);
}

// The lane's share of a group of g particles: P = ceil(g / M) particle slots,
// k = floor(64 / P) lanes per slot; lane = slot + sub P.  Slot p carries the
// particles p, p + P, ..., p + (M - 1) P that exist (offsets from the group
// centre); lane (p, sub) takes sources sub, sub + k, sub + 2k, ... of a tile.
template <int M>
struct Target {
    float ox[M], oy[M], oz[M];
    int sub, k;
    int tmax;    // trips of the largest tile (cells or particles)
};

// sources per loop trip: fewer when the lane carries more particles (registers)
#ifndef BH_WALK_UNROLL2
#define BH_WALK_UNROLL2 1
#endif
template <int M>
constexpr int unroll_for() { return M == 1 ? kUnroll : (M == 2 ? BH_WALK_UNROLL2 : 1); }

// the partials into the compensated totals (two-sum), partials cleared
template <int M>
__device__ __forceinline__ void acc_flush(Acc<M> &acc)
{
#pragma unroll
    for (int m = 0; m < M; ++m) {
        comp_add(acc.ax[m], acc.cx[m], acc.px[m]);
        comp_add(acc.ay[m], acc.cy[m], acc.py[m]);
        comp_add(acc.az[m], acc.cz[m], acc.pz[m]);
        comp_add(acc.ph[m], acc.cp[m], acc.pp[m]);
        acc.px[m] = acc.py[m] = acc.pz[m] = acc.pp[m] = 0.f;
    }
    acc.trips = 0;
}

// after a tile of T trips: flush when the next tile (at most tmax trips) could
// take a partial past kPlainTerms terms
template <int M>
__device__ __forceinline__ void acc_tile_done(Acc<M> &acc, int T, int tmax)
{
    acc.trips += T;
    if (BH_WALK_COMP_EVERY_TILE || acc.trips + tmax > kPlainTerms) acc_flush<M>(acc);
}

template <bool kEps0, int M>
__device__ __forceinline__ void run_pc(const WaveLds &L, int base, int cnt, const Target<M> &t,
                                       float eps2, Acc<M> &acc)
{
    constexpr int U = unroll_for<M>();
    float *ax = acc.px, *ay = acc.py, *az = acc.pz, *ph = acc.pp;
    const int k = t.k;
    const int T = uniform((cnt + k - 1) / k);
    int j = base + t.sub;
    int it = 0;
    for (; it + U <= T; it += U) {
        float4 A[U], B[U], C[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            A[u] = L.ca[j + u * k];
            B[u] = L.cb[j + u * k];
            C[u] = L.cc[j + u * k];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int m = 0; m < M; ++m)
                pc_term<kEps0>(A[u], B[u], C[u], t.ox[m], t.oy[m], t.oz[m], eps2, ax[m], ay[m],
                               az[m], ph[m]);
        j += U * k;
    }
    for (; it < T; ++it) {
        const float4 A = L.ca[j], B = L.cb[j], C = L.cc[j];
#pragma unroll
        for (int m = 0; m < M; ++m)
            pc_term<kEps0>(A, B, C, t.ox[m], t.oy[m], t.oz[m], eps2, ax[m], ay[m], az[m], ph[m]);
        j += k;
    }
}

template <bool kEps0, int M>
__device__ __forceinline__ void run_pp(const WaveLds &L, int cnt, const Target<M> &t, float eps2,
                                       Acc<M> &acc)
{
    constexpr int U = unroll_for<M>();
    float *ax = acc.px, *ay = acc.py, *az = acc.pz, *ph = acc.pp;
    const int k = t.k;
    const int T = uniform((cnt + k - 1) / k);
    int j = t.sub;
    int it = 0;
    for (; it + U <= T; it += U) {
        float4 S[U];
#pragma unroll
        for (int u = 0; u < U; ++u) S[u] = L.ta[j + u * k];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int m = 0; m < M; ++m)
                pp_term<kEps0>(S[u], t.ox[m], t.oy[m], t.oz[m], eps2, ax[m], ay[m], az[m], ph[m]);
        j += U * k;
    }
    for (; it < T; ++it) {
        const float4 S = L.ta[j];
#pragma unroll
        for (int m = 0; m < M; ++m)
            pp_term<kEps0>(S, t.ox[m], t.oy[m], t.oz[m], eps2, ax[m], ay[m], az[m], ph[m]);
        j += k;
    }
}

// evaluate cnt <= 64 cells of the staged cell list from entry base: the entries
// a lane may read past them are set to padding (far away, zero mass) first
template <bool kEps0, int M>
__device__ __forceinline__ void eval_pc(WaveLds &L, int base, int cnt, const Target<M> &t,
                                        float eps2, Acc<M> &acc)
{
    const int lane = lane_id();
    // the lanes read entries up to k ceil(cnt / k) past base
    const int reach = t.k * uniform((cnt + t.k - 1) / t.k);
    for (int i = base + cnt + lane; i < base + reach; i += kWave) {
        L.ca[i] = make_float4(kFar, kFar, kFar, 0.0f);
        L.cb[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        L.cc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    wave_sync();
    if (t.sub < t.k) run_pc<kEps0, M>(L, base, cnt, t, eps2, acc);
    acc_tile_done<M>(acc, reach / t.k, t.tmax);
    wave_sync();
}

// stage up to 64 particles (lane j holds particle index idx) and evaluate them
template <bool kEps0, int M>
__device__ __forceinline__ void eval_pp(const WalkArgs &a, WaveLds &L, uint32_t idx, int cnt,
                                        const double4 gc, const Target<M> &t, float eps2,
                                        Acc<M> &acc)
{
    const int lane = lane_id();
    if (lane < cnt) {
        const double4 p = a.p4[idx];
        L.ta[lane] = make_float4((float)(p.x - gc.x), (float)(p.y - gc.y), (float)(p.z - gc.z), (float)p.w);
    } else {
        L.ta[lane] = make_float4(kFar, kFar, kFar, 0.0f);
    }
    wave_sync();
    if (t.sub < t.k) run_pp<kEps0, M>(L, cnt, t, eps2, acc);
    acc_tile_done<M>(acc, uniform((cnt + t.k - 1) / t.k), t.tmax);
    wave_sync();
}

// the next group after the current one: from the device-wide counter, offset by
// the W wavefronts of the grid (wavefront w starts with group w, so the launch
// does not begin with W fetches at one address)
__device__ __forceinline__ uint32_t next_slot(const WalkArgs &a, uint32_t waves)
{
    uint32_t v = 0;
    if (lane_id() == 0) v = atomicAdd(&a.misc->walk_next, 1u);
    return waves + readfirst(v);
}

// The opening test of a cell (record w) for the group of centre gc and half-sizes
// gh: the distance from the group's box to the cell's centre of mass (Eq. (1)),
// or to the cell's cube (the minimum-distance test), against the cell's radius;
// o receives the cell's centre of mass relative to the group centre.
__device__ __forceinline__ bool mac_accept(const WalkArgs &a, const WalkCell &w, uint32_t cell,
                                           const double4 gc, const float4 gh, bool mindist,
                                           float &ox, float &oy, float &oz)
{
    ox = (float)(w.cx - gc.x);
    oy = (float)(w.cy - gc.y);
    oz = (float)(w.cz - gc.z);
    float dx, dy, dz;
    if (mindist) {
        const double4 q = a.geo[cell];
        const float h = (float)q.w;
        dx = (fabsf((float)(q.x - gc.x)) - gh.x) - h;
        dy = (fabsf((float)(q.y - gc.y)) - gh.y) - h;
        dz = (fabsf((float)(q.z - gc.z)) - gh.z) - h;
    } else {
        dx = fabsf(ox) - gh.x;
        dy = fabsf(oy) - gh.y;
        dz = fabsf(oz) - gh.z;
    }
    const float ux = dx > 0.0f ? dx : 0.0f;
    const float uy = dy > 0.0f ? dy : 0.0f;
    const float uz = dz > 0.0f ? dz : 0.0f;
    const float d2 = (ux * ux + uy * uy) + uz * uz;
    return d2 > w.rcrit2;
}

// One group: walk its cluster's tree from the root, evaluate its lists, and
// write its particles' accelerations and potentials.  M: particles per lane.
template <bool kEps0, int M>
__device__ __forceinline__ void walk_group(const WalkArgs &a, WaveLds &L, CellStack &stack,
                                           LeafList &leaves, uint32_t ncells, uint32_t gs, int gn,
                                           const double4 gc, const float4 gh, uint32_t cid,
                                           float eps2, bool mindist, uint32_t &npp_out,
                                           uint32_t &npc_out, bool &overflow_out)
{
    const int lane = lane_id();
    const int P = (gn + M - 1) / M;
    Target<M> t;
    t.k = uniform(kWave / P);
    const int p = lane % P;
    t.sub = lane / P;
    float mi[M];
    Acc<M> acc;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        t.ox[m] = t.oy[m] = t.oz[m] = 0.f;
        mi[m] = 0.f;
        acc.ax[m] = acc.ay[m] = acc.az[m] = acc.ph[m] = 0.f;
        acc.cx[m] = acc.cy[m] = acc.cz[m] = acc.cp[m] = 0.f;
        acc.px[m] = acc.py[m] = acc.pz[m] = acc.pp[m] = 0.f;
        const int q = p + m * P;
        if (t.sub < t.k && q < gn) {
            const double4 x = a.p4[gs + q];
            t.ox[m] = (float)(x.x - gc.x);
            t.oy[m] = (float)(x.y - gc.y);
            t.oz[m] = (float)(x.z - gc.z);
            mi[m] = (float)x.w;
        }
    }

    // cells per full tile (uniform); trips of the largest tile
    const int tsz = BH_WALK_FLEX_TILE ? t.k * ((kWave + t.k - 1) / t.k) : kWave;
    t.tmax = (tsz + t.k - 1) / t.k;
    // particles per full particle tile: k floor(64 / k), every trip full
    const int psz = BH_WALK_PP_FULL ? t.k * (kWave / t.k) : kWave;
    acc.trips = 0;
    int top = 1;
    {
        // The cluster's root holds the group, so the opening test opens it (it
        // is tested all the same, with the loop's arithmetic): its children then
        // start the stack, which saves the traversal's one-cell first pass.
        const WalkCell rw = a.rec[cid];
        float rx, ry, rz;
        const bool racc = mac_accept(a, rw, cid, gc, gh, mindist, rx, ry, rz);
        const bool rleaf = (rw.info >> 31) != 0u;
        if (lane == 0) {
            if (!racc && !rleaf) stack.set(0, rw.link, rw.info);
            else stack.set(0, cid, 1u);
        }
    }
    wave_sync();
    int pc_n = 0, pp_n = 0;
    uint32_t pend = 0, npp = 0, npc = 0;
    bool overflow = false;
    uint32_t iters = 0;

    while (top > 0) {
        // Traversal (pop, opening test, list appends) runs at a raised wave
        // priority and evaluation at the normal one: a wavefront's next loads then
        // issue ahead of the arithmetic of the other wavefronts on its SIMD, which
        // hides more of the traversal's latency behind that arithmetic.
        __builtin_amdgcn_s_setprio(1);
        // a correct tree visits each cell at most once per group
        if (++iters > ncells + 1u) {
            overflow = true;
            break;
        }
        uint32_t cell;
        const int got = pop64(stack, top, L.mark, cell);
        const bool has = lane < got && cell < ncells;
        bool acc_cell = false, leaf = false;
        uint32_t link = 0, info = 0;
        WalkCell w;
        float ox = 0.f, oy = 0.f, oz = 0.f;
        if (has) {
            w = a.rec[cell];
            link = w.link;
            info = w.info;
            acc_cell = mac_accept(a, w, cell, gc, gh, mindist, ox, oy, oz);
            leaf = (info >> 31) != 0u;
        }
        // accepted cells -> cell list, staged for evaluation at once (offset
        // from the group centre, mass, 3 S and the trace terms)
        const unsigned long long bpc = ballot(has && acc_cell);
        if (has && acc_cell) {
            const int i = pc_n + mask_rank(bpc);
            const float tr3 = (w.s3[0] + w.s3[1]) + w.s3[2];     // 3 tr(S)
            L.ca[i] = make_float4(ox, oy, oz, w.mass);
            L.cb[i] = make_float4(w.s3[0], w.s3[1], w.s3[2], w.s3[3]);
            L.cc[i] = make_float4(w.s3[4], w.s3[5], tr3 * (1.0f / 6.0f), tr3 * 0.5f);
        }
        pc_n += __popcll(bpc);
        npc += (uint32_t)__popcll(bpc);
        // opened leaves -> particle list
        const bool isl = has && !acc_cell && leaf;
        const unsigned long long bpp = ballot(isl);
        const uint32_t lc = isl ? (info & 0x7fffffffu) : 0u;
        if (isl) L.pp[pp_n + mask_rank(bpp)] = make_uint2(link, lc);
        pp_n += __popcll(bpp);
        if (bpp) {      // uniform: some lane opened a leaf
            const uint32_t lsum = wave_sum_u32(lc);
            pend += lsum;
            npp += lsum;
        }
        // opened nodes -> children onto the stack
        const bool isn = has && !acc_cell && !leaf;
        const unsigned long long bn = ballot(isn);
        const int nn = __popcll(bn);
        if (top + nn > kStackCap) {
            overflow = true;
            wave_sync();
        } else {
            if (BH_WALK_LDS_FAST && stack.all_lds(top + nn)) {
                if (isn) stack.set_lds(top + mask_rank(bn), link, info);
                top += nn;
                wave_sync();
            } else {
                if (isn) stack.set(top + mask_rank(bn), link, info);
                top += nn;
                stack.sync();
            }
        }
        if (pc_n >= tsz) {       // pc_n < tsz + 64: one tile of the last tsz entries
            __builtin_amdgcn_s_setprio(0);
            eval_pc<kEps0, M>(L, pc_n - tsz, tsz, t, eps2, acc);
            pc_n -= tsz;
        }
        while (pend >= (uint32_t)psz) {
            uint32_t idx;
            const int n = pp_n > 0 ? pop64(leaves, pp_n, L.mark, idx, psz) : 0;
            if (n <= 0) {   // inconsistent bookkeeping: never spin
                overflow = true;
                pend = 0;
                break;
            }
            __builtin_amdgcn_s_setprio(0);
            eval_pp<kEps0, M>(a, L, idx, n, gc, t, eps2, acc);
            pend -= (uint32_t)n;
        }
        if (overflow) break;
    }
    __builtin_amdgcn_s_setprio(0);
    if (pc_n > 0) eval_pc<kEps0, M>(L, 0, pc_n, t, eps2, acc);
    while (pend > 0) {
        uint32_t idx;
        const int n = pp_n > 0 ? pop64(leaves, pp_n, L.mark, idx, psz) : 0;
        if (n <= 0) {
            overflow = true;
            break;
        }
        eval_pp<kEps0, M>(a, L, idx, n, gc, t, eps2, acc);
        pend -= (uint32_t)n < pend ? (uint32_t)n : pend;
    }

    if (acc.trips > 0) acc_flush<M>(acc);
    // add the k partial sums of each particle: halving steps over the sub-lane
    // index, in a fixed order
    float ax[M], ay[M], az[M], ph[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        ax[m] = acc.ax[m] + acc.cx[m];
        ay[m] = acc.ay[m] + acc.cy[m];
        az[m] = acc.az[m] + acc.cz[m];
        ph[m] = acc.ph[m] + acc.cp[m];
    }
    for (int kk = t.k; kk > 1;) {
        const int h = (kk + 1) >> 1;
        const int src = lane + h * P;
        const int srcl = src < kWave ? src : lane;
        const bool take = t.sub + h < kk;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const float bx = __shfl(ax[m], srcl, kWave);
            const float by = __shfl(ay[m], srcl, kWave);
            const float bz = __shfl(az[m], srcl, kWave);
            const float bp = __shfl(ph[m], srcl, kWave);
            if (take) {
                ax[m] += bx;
                ay[m] += by;
                az[m] += bz;
                ph[m] += bp;
            }
        }
        kk = h;
    }
    if (t.sub == 0 && lane < P) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int q = p + m * P;
            if (q >= gn) continue;
            // the particle met itself once in the particle list: with eps > 0
            // that term added -m/eps to the potential and nothing to the
            // acceleration
            float phm = ph[m];
            if (!kEps0 || eps2 > 0.0f) phm = phm + mi[m] * __builtin_amdgcn_rsqf(eps2);
            a.acc4[gs + q] = make_float4(ax[m], ay[m], az[m], phm);
        }
    }
    npp_out = npp;
    npc_out = npc;
    overflow_out = overflow;
}

// Particles per lane for a group of g: the M in {1, .., kMaxPerLane} with the
// fewest loop trips per 64-source tile, M ceil(64 / floor(64 / ceil(g / M)));
// ties go to the smaller M.  M must leave at most 64 particle slots (groups of
// up to 128 particles need M >= 2).
#ifndef BH_WALK_MAX_PER_LANE
#define BH_WALK_MAX_PER_LANE 3
#endif
constexpr int kMaxPerLane = BH_WALK_MAX_PER_LANE;
static_assert(kMaxPerLane >= 2 && kMaxPerLane * kWave >= kMaxGroup,
              "a group of kMaxGroup particles must fit one wavefront");

__device__ __forceinline__ int lanes_mode(int g)
{
    int best = kMaxPerLane, cost = 1 << 30;
    for (int m = 1; m <= kMaxPerLane; ++m) {
        const int P = (g + m - 1) / m;
        if (P > kWave) continue;
        const int k = kWave / P;
        const int c = m * ((kWave + k - 1) / k);
        if (c < cost) {
            cost = c;
            best = m;
        }
    }
    return best;
}

// kEps0: some cluster of the launch has zero softening, so pairs at zero
// distance (a particle with itself) must be skipped explicitly.
template <bool kEps0>
__global__ void __launch_bounds__(kWalkBlock)
__attribute__((amdgpu_waves_per_eu(BH_WALK_WAVES_PER_EU))) walk_kernel(WalkArgs a)
{
    const uint32_t ngroups = readfirst(a.glist ? a.misc->nactive : a.misc->ngroups);
    const uint32_t ncells = readfirst(a.misc->ncells);
    __shared__ WaveLds s_lds[kWalkWaves];
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    WaveLds &L = s_lds[w];
    const int64_t wave_global = (int64_t)blockIdx.x * kWalkWaves + w;
    CellStack stack{L.stack, a.spill + wave_global * kSpillPerWave};
    LeafList leaves{L.pp};

    // particle tile padding beyond its 64 staged entries: far away, zero mass
    for (int i = kWave + lane; i < kTileReach; i += kWave) L.ta[i] = make_float4(kFar, kFar, kFar, 0.0f);
    wave_sync();

    unsigned long long wave_pp = 0, wave_pc = 0;   // interaction totals of this wavefront
    bool wave_overflow = false;
    const uint32_t waves = gridDim.x * kWalkWaves;
    for (uint32_t slot = readfirst((uint32_t)wave_global); slot < ngroups;
         slot = next_slot(a, waves)) {
        const uint32_t g = a.glist ? readfirst(a.glist[slot]) : slot;
        const uint32_t gs = a.g_first[g];
        const int gn = uniform((int)a.g_count[g]);
        const double4 gc = a.g_centre[g];
        const float4 gh = a.g_half[g];
        // the group's cluster: its root is the cluster's level-0 cell
        const uint32_t cid = readfirst((uint32_t)gc.w);
        const float eps2 = a.clus[cid].eps2;
        const bool mindist = uniform((int)a.clus[cid].mac) != 0;
        uint32_t npp = 0, npc = 0;
        bool overflow = false;
        switch (uniform(lanes_mode(gn))) {
        case 1:
            walk_group<kEps0, 1>(a, L, stack, leaves, ncells, gs, gn, gc, gh, cid, eps2, mindist,
                                 npp, npc, overflow);
            break;
        case 2:
            walk_group<kEps0, 2>(a, L, stack, leaves, ncells, gs, gn, gc, gh, cid, eps2, mindist,
                                 npp, npc, overflow);
            break;
        default:
            if (kMaxPerLane >= 3)
                walk_group<kEps0, (kMaxPerLane >= 3 ? 3 : 1)>(a, L, stack, leaves, ncells, gs, gn,
                                                              gc, gh, cid, eps2, mindist, npp,
                                                              npc, overflow);
            break;
        }
        if (lane == 0) {
            a.g_npp[g] = npp;
            a.g_npc[g] = npc;
        }
        wave_pp += (unsigned long long)npp * (unsigned long long)gn;
        wave_pc += (unsigned long long)npc * (unsigned long long)gn;
        wave_overflow |= overflow;
        wave_sync();
    }
    // the block's totals go to its own slot (summed by walk_sum_kernel): thousands
    // of workgroups adding to one address at the end of the kernel serialise
    __shared__ unsigned long long s_tot[kWalkWaves][2];
    __shared__ uint32_t s_over[kWalkWaves];
    if (lane == 0) {
        s_tot[w][0] = wave_pp;
        s_tot[w][1] = wave_pc;
        s_over[w] = wave_overflow ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long pp = 0, pc = 0;
        uint32_t over = 0;
        for (int i = 0; i < kWalkWaves; ++i) {
            pp += s_tot[i][0];
            pc += s_tot[i][1];
            over |= s_over[i];
        }
        a.part[2 * (int64_t)blockIdx.x] = pp;
        a.part[2 * (int64_t)blockIdx.x + 1] = pc;
        if (over) atomicOr(&a.misc->walk_overflow, 1u);
    }
}

// the walk's interaction totals from its per-workgroup slots (fixed order)
__global__ void __launch_bounds__(256)
walk_sum_kernel(const unsigned long long *__restrict__ part, int blocks, DevMisc *m)
{
    __shared__ unsigned long long s[2][256];
    unsigned long long pp = 0, pc = 0;
    for (int b = threadIdx.x; b < blocks; b += 256) {
        pp += part[2 * b];
        pc += part[2 * b + 1];
    }
    s[0][threadIdx.x] = pp;
    s[1][threadIdx.x] = pc;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            s[0][threadIdx.x] += s[0][threadIdx.x + d];
            s[1][threadIdx.x] += s[1][threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        m->sum_npp = s[0][0];
        m->sum_npc = s[1][0];
        m->tot_npp += s[0][0];
        m->tot_npc += s[1][0];
        m->walk_next = 0;       // the next walk hands out its groups from 0 again
    }
}


__global__ void __launch_bounds__(256) zero_f4_kernel(int64_t n, float4 *__restrict__ p)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void __launch_bounds__(256)
scatter_kernel(int64_t n, const float4 *__restrict__ acc4, const uint32_t *__restrict__ pid,
               float *__restrict__ acc, float *__restrict__ pot)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float4 v = acc4[i];
    const int64_t o = pid[i];
    if (acc) {
        acc[3 * o] = v.x;
        acc[3 * o + 1] = v.y;
        acc[3 * o + 2] = v.z;
    }
    if (pot) pot[o] = v.w;
}

}  // namespace

// Harvest finished walk timings; with block == true wait for all of them.
void walk_timer_harvest(bh_ctx *c, bool block)
{
    while (c->wring_count > 0) {
        hipEvent_t *ev = &c->wev[2 * c->wring_head];
        if (!block && hipEventQuery(ev[1]) != hipSuccess) break;
        if (block) (void)hipEventSynchronize(ev[1]);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) {
            c->walk_ms_total += ms;
            c->walk_ms_last = ms;
            c->walk_launches += 1;
        }
        c->wring_head = (c->wring_head + 1) % bh_ctx::kWalkRing;
        c->wring_count -= 1;
    }
    (void)hipGetLastError();
}

// Next free pair of timing events (the oldest is harvested if the ring is full).
hipEvent_t *walk_timer_slot(bh_ctx *c)
{
    if (!c->wev[0]) return nullptr;
    walk_timer_harvest(c, false);
    if (c->wring_count == bh_ctx::kWalkRing) {
        hipEvent_t *old = &c->wev[2 * c->wring_head];
        (void)hipEventSynchronize(old[1]);
        walk_timer_harvest(c, false);
    }
    const int slot = (c->wring_head + c->wring_count) % bh_ctx::kWalkRing;
    c->wring_count += 1;
    return &c->wev[2 * slot];
}

int64_t walk_spill_words(int64_t waves) { return waves * kSpillPerWave; }

// wavefronts of the persistent walk grid
int64_t walk_grid_waves(bh_ctx *c)
{
    int dev_cus = 256;
    if (hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
        hipSuccess) {
        (void)hipGetLastError();
        dev_cus = 256;
    }
    return (int64_t)dev_cus * BH_WALK_BLOCKS_PER_CU * kWalkWaves;
}

// The work counter starts at zero (set when the context's device scalars are
// cleared and at the start of every build) and walk_sum_kernel clears it after
// each walk; the interaction sums are written by walk_sum_kernel.
// Flags the groups that hold at least one active particle (flags[g], zero for
// g >= ngroups up to n so that the flags can be compacted over n entries).
__global__ void __launch_bounds__(256)
mark_active_groups_kernel(const DevMisc *__restrict__ m, const uint32_t *__restrict__ g_first,
                          const uint32_t *__restrict__ g_count, const uint32_t *__restrict__ pid,
                          const uint8_t *__restrict__ active, int64_t n, uint8_t *__restrict__ flags)
{
    const uint32_t ngroups = m->ngroups;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n;
         g += (int64_t)gridDim.x * 256) {
        uint8_t f = 0;
        if (g < (int64_t)ngroups) {
            const uint32_t s = g_first[g], e = s + g_count[g];
            for (uint32_t i = s; i < e && !f; ++i) f = active[pid[i]] != 0;
        }
        flags[g] = f;
    }
}

hipError_t launch_active_groups(bh_ctx *c, const uint8_t *active)
{
    int g = (int)((c->n + 255) / 256);
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(mark_active_groups_kernel, dim3(g), dim3(256), 0, c->stream, c->misc,
                       c->g_first, c->g_count, c->pid[c->cur], active, c->n, c->gflag);
    BH_LAUNCH_CHECK();
    // the active group list goes to the sort's spare value buffer
    return compact_flags(c, c->gflag, c->n, c->val[1], &c->misc->nactive);
}

hipError_t launch_walk(bh_ctx *c, bool timed, bool active_only)
{
    int64_t blocks = walk_grid_waves(c) / kWalkWaves;
    if (blocks * kWalkWaves > c->walk_spill_waves) blocks = c->walk_spill_waves / kWalkWaves;
    if (blocks < 1) return hipErrorInvalidValue;
    WalkArgs a;
    a.clus = c->clus;
    a.g_first = c->g_first;
    a.g_count = c->g_count;
    a.g_centre = c->g_centre;
    a.g_half = c->g_half;
    a.p4 = c->p4[c->cur];
    a.rec = c->c_rec;
    a.geo = c->c_geo;
    a.acc4 = c->acc4;
    a.g_npp = c->g_npp;
    a.g_npc = c->g_npc;
    a.spill = c->walk_spill;
    a.part = c->walk_part;
    a.misc = c->misc;
    a.glist = active_only ? c->val[1] : nullptr;
    hipEvent_t *ev = timed ? walk_timer_slot(c) : nullptr;
    if (ev) BH_HIP_TRY(hipEventRecord(ev[0], c->stream));
    if (c->any_eps0)
        hipLaunchKernelGGL(walk_kernel<true>, dim3((unsigned)blocks), dim3(kWalkBlock), 0, c->stream, a);
    else
        hipLaunchKernelGGL(walk_kernel<false>, dim3((unsigned)blocks), dim3(kWalkBlock), 0, c->stream, a);
    BH_LAUNCH_CHECK();
    if (ev) BH_HIP_TRY(hipEventRecord(ev[1], c->stream));
    hipLaunchKernelGGL(walk_sum_kernel, dim3(1), dim3(256), 0, c->stream, c->walk_part,
                       (int)blocks, c->misc);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_zero_acc(bh_ctx *c)
{
    hipLaunchKernelGGL(zero_f4_kernel, dim3((unsigned)((c->n + 255) / 256)), dim3(256), 0, c->stream,
                       c->n, c->acc4);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_scatter(bh_ctx *c, float *acc, float *pot)
{
    if (!acc && !pot) return hipSuccess;
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((c->n + 255) / 256)), dim3(256), 0, c->stream,
                       c->n, c->acc4, c->pid[c->cur], acc, pot);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

}  // namespace bh
