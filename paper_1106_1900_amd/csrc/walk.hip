// walk.hip - the group walk and force evaluation (Sect. 2.2, 3.3).
//
// One wavefront (64 lanes) takes one group of at most 64 particles.  It walks
// the tree breadth-first from the root: up to 64 cells are tested at a time,
// one per lane, with the opening test of Eq. (1).  An accepted cell goes to the
// cell list, an opened leaf to the particle list, an opened node pushes its
// contiguous children.  As soon as a list holds 64 entries it is evaluated: the
// 64 sources are staged in LDS as float32 offsets from the group's box centre
// and every lane accumulates them on its particle.  Groups of at most 32, 21 or
// 16 particles use 2, 3 or 4 lanes per particle, each lane taking every k-th
// source, and the lanes are summed at the end (the paper's several threads per
// particle).
//
// Per wavefront, in LDS:
//   stack : pending cell ranges (first cell, count <= 8) packed in 32 bits.  A
//           pop takes up to 64 cells from the top; each pop pushes at most 64
//           ranges, all deeper than anything popped before them that is still on
//           the stack, so at most 64 ranges per level (21 levels) are ever held.
//   pc    : accepted cells (< 64 between evaluations, 128 entries).
//   pp    : opened leaves as (first particle, count) ranges (< 64 particles
//           pending between evaluations, so < 128 ranges).
//   tile  : 64 staged sources (3 x float4 for a cell, 1 x float4 for a particle).
//
// Every pair goes through float32 arithmetic on group-centred offsets; each
// 64-source tile is summed in plain float32 and the tile sums are added to the
// particle's totals with an error-free two-sum (compensated accumulation).
#include "bh_internal.h"

#pragma clang fp contract(off)

namespace bh {
namespace {

constexpr int kWalkBlock = kWalkWaves * kWave;
constexpr int kPcCap = 128;
constexpr int kPpCap = 128;

struct WalkArgs {
    int64_t ngroups;
    uint32_t ncells;
    const uint32_t *g_first;
    const uint32_t *g_count;
    const double4 *g_centre;
    const float4 *g_half;
    const double4 *p4;        // sources and targets: x, y, z, mass (sorted order)
    const double4 *c_com;     // centre of mass, mass
    const float4 *c_q0;       // 3Sxx, 3Syy, 3Szz, 3Sxy
    const float4 *c_q1;       // 3Sxz, 3Syz, tr(S)/2, 3 tr(S)/2
    const uint4 *c_walk;      // first child or particle, nchild or count|leaf bit, rcrit2 bits
    float4 *acc4;             // out: ax, ay, az, pot (sorted order)
    uint32_t *g_npp;
    uint32_t *g_npc;
    DevMisc *misc;
    float eps2;
};

struct WaveLds {
    uint32_t stack[kStackCap];
    uint32_t pc[kPcCap];
    uint2 pp[kPpCap];
    int mark[kWave];
    float4 tile[3 * kWave];
};

struct Acc {
    float ax, ay, az, ph;     // running sums
    float cx, cy, cz, cp;     // running compensations
};

// s + t with the rounding error of the addition carried in c (two-sum).
__device__ __forceinline__ void comp_add(float &s, float &c, float t)
{
    const float r = s + t;
    const float bp = r - s;
    const float err = (s - (r - bp)) + (t - bp);
    s = r;
    c = c + err;
}

// Pop up to 64 elements from a list of ranges kept as a stack in LDS.  Lane j
// receives element j of the popped run in *elem; returns how many were popped.
template <class List>
__device__ __forceinline__ int pop64(List list, int &top, int *mark, uint32_t &elem)
{
    const int lane = lane_id();
    const int m = top < kWave ? top : kWave;
    uint32_t f = 0, cnt = 0;
    if (lane < m) list.get(top - 1 - lane, f, cnt);
    const uint32_t incl = wave_incl_scan_add(cnt);
    const uint32_t excl = incl - cnt;
    uint32_t take = 0;
    if (lane < m && excl < (uint32_t)kWave) {
        const uint32_t room = (uint32_t)kWave - excl;
        take = cnt < room ? cnt : room;
    }
    const bool full = lane < m && take == cnt;
    const int nfull = __popcll(ballot(full));
    const uint32_t total = __shfl(incl, m - 1, kWave);
    const int got = total < (uint32_t)kWave ? (int)total : kWave;
    mark[lane] = -1;
    wave_sync();
    if (take > 0) mark[excl] = lane;
    wave_sync();
    int src = wave_incl_scan_max(mark[lane]);
    src = src < 0 ? 0 : src;
    const uint32_t fs = __shfl(f, src, kWave);
    const uint32_t es = __shfl(excl, src, kWave);
    elem = fs + ((uint32_t)lane - es);
    if (lane == nfull && lane < m && take > 0 && take < cnt) list.set(top - 1 - lane, f + take, cnt - take);
    top -= nfull;
    wave_sync();
    return got;
}

struct CellStack {
    uint32_t *s;
    __device__ void get(int i, uint32_t &f, uint32_t &c) const
    {
        const uint32_t v = s[i];
        f = v >> 3;
        c = (v & 7u) + 1u;
    }
    __device__ void set(int i, uint32_t f, uint32_t c) const { s[i] = (f << 3) | (c - 1u); }
};

struct LeafList {
    uint2 *s;
    __device__ void get(int i, uint32_t &f, uint32_t &c) const
    {
        const uint2 v = s[i];
        f = v.x;
        c = v.y;
    }
    __device__ void set(int i, uint32_t f, uint32_t c) const { s[i] = make_uint2(f, c); }
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
    // 3 S r with B = (3Sxx, 3Syy, 3Szz, 3Sxy), C = (3Sxz, 3Syz, trS/2, 3trS/2)
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

template <bool kEps0>
__device__ __forceinline__ void eval_pc(const WalkArgs &a, WaveLds &L, const uint32_t *list, int cnt,
                                        const double4 gc, bool tact, int sub, int k, float ox,
                                        float oy, float oz, Acc &acc)
{
    const int lane = lane_id();
    if (lane < cnt) {
        const uint32_t c = list[lane];
        const double4 cm = a.c_com[c];
        L.tile[lane] = make_float4((float)(cm.x - gc.x), (float)(cm.y - gc.y), (float)(cm.z - gc.z),
                                   (float)cm.w);
        L.tile[kWave + lane] = a.c_q0[c];
        L.tile[2 * kWave + lane] = a.c_q1[c];
    }
    wave_sync();
    if (tact) {
        float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
        for (int j = sub; j < cnt; j += k)
            pc_term<kEps0>(L.tile[j], L.tile[kWave + j], L.tile[2 * kWave + j], ox, oy, oz, a.eps2,
                           ax, ay, az, ph);
        comp_add(acc.ax, acc.cx, ax);
        comp_add(acc.ay, acc.cy, ay);
        comp_add(acc.az, acc.cz, az);
        comp_add(acc.ph, acc.cp, ph);
    }
    wave_sync();
}

template <bool kEps0>
__device__ __forceinline__ void eval_pp(const WalkArgs &a, WaveLds &L, uint32_t idx, int cnt,
                                        const double4 gc, bool tact, int sub, int k, float ox,
                                        float oy, float oz, Acc &acc)
{
    const int lane = lane_id();
    if (lane < cnt) {
        const double4 p = a.p4[idx];
        L.tile[lane] = make_float4((float)(p.x - gc.x), (float)(p.y - gc.y), (float)(p.z - gc.z),
                                   (float)p.w);
    }
    wave_sync();
    if (tact) {
        float ax = 0.f, ay = 0.f, az = 0.f, ph = 0.f;
        for (int j = sub; j < cnt; j += k) pp_term<kEps0>(L.tile[j], ox, oy, oz, a.eps2, ax, ay, az, ph);
        comp_add(acc.ax, acc.cx, ax);
        comp_add(acc.ay, acc.cy, ay);
        comp_add(acc.az, acc.cz, az);
        comp_add(acc.ph, acc.cp, ph);
    }
    wave_sync();
}

template <bool kEps0>
__global__ void __launch_bounds__(kWalkBlock) walk_kernel(WalkArgs a)
{
    __shared__ WaveLds s_lds[kWalkWaves];
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    WaveLds &L = s_lds[w];
    CellStack stack{L.stack};
    LeafList leaves{L.pp};

    for (;;) {
        uint32_t gnext = 0;
        if (lane == 0) gnext = atomicAdd(&a.misc->walk_next, 1u);
        const uint32_t g = readfirst(gnext);
        if ((int64_t)g >= a.ngroups) break;

        const uint32_t gs = a.g_first[g];
        const int gn = (int)a.g_count[g];
        const double4 gc = a.g_centre[g];
        const float4 gh = a.g_half[g];
        int k = kWave / gn;
        k = k > 4 ? 4 : k;
        const int p = lane % gn;
        const int sub = lane / gn;
        const bool tact = sub < k;
        float ox = 0.f, oy = 0.f, oz = 0.f, mi = 0.f;
        if (tact) {
            const double4 q = a.p4[gs + p];
            ox = (float)(q.x - gc.x);
            oy = (float)(q.y - gc.y);
            oz = (float)(q.z - gc.z);
            mi = (float)q.w;
        }
        Acc acc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

        int top = 0;
        if (lane == 0) stack.set(0, 0u, 1u);   // the root
        top = 1;
        int pc_n = 0, pp_n = 0;
        uint32_t pend = 0, npp = 0, npc = 0;
        bool overflow = false;
        wave_sync();

        uint32_t iters = 0;
        while (top > 0) {
            // a correct tree visits each cell at most once per group
            if (++iters > a.ncells + 1u) {
                overflow = true;
                break;
            }
            uint32_t cell;
            const int got = pop64(stack, top, L.mark, cell);
            const bool has = lane < got && cell < a.ncells;
            bool acc_cell = false, leaf = false;
            uint4 wk = make_uint4(0, 0, 0, 0);
            if (has) {
                const double4 cm = a.c_com[cell];
                wk = a.c_walk[cell];
                const float dx = fabsf((float)(cm.x - gc.x)) - gh.x;
                const float dy = fabsf((float)(cm.y - gc.y)) - gh.y;
                const float dz = fabsf((float)(cm.z - gc.z)) - gh.z;
                const float ux = dx > 0.0f ? dx : 0.0f;
                const float uy = dy > 0.0f ? dy : 0.0f;
                const float uz = dz > 0.0f ? dz : 0.0f;
                const float d2 = (ux * ux + uy * uy) + uz * uz;
                acc_cell = d2 > __uint_as_float(wk.z);
                leaf = (wk.y >> 31) != 0u;
            }
            // accepted cells -> cell list
            const unsigned long long bpc = ballot(has && acc_cell);
            if (has && acc_cell) L.pc[pc_n + mask_rank(bpc)] = cell;
            pc_n += __popcll(bpc);
            npc += (uint32_t)__popcll(bpc);
            // opened leaves -> particle list
            const bool isl = has && !acc_cell && leaf;
            const unsigned long long bpp = ballot(isl);
            const uint32_t lc = isl ? (wk.y & 0x7fffffffu) : 0u;
            if (isl) L.pp[pp_n + mask_rank(bpp)] = make_uint2(wk.x, lc);
            pp_n += __popcll(bpp);
            const uint32_t lsum = wave_sum(lc);
            pend += lsum;
            npp += lsum;
            // opened nodes -> children onto the stack
            const bool isn = has && !acc_cell && !leaf;
            const unsigned long long bn = ballot(isn);
            const int nn = __popcll(bn);
            if (top + nn > kStackCap) {
                overflow = true;
            } else {
                if (isn) stack.set(top + mask_rank(bn), wk.x, wk.y);
                top += nn;
            }
            wave_sync();
            while (pc_n >= kWave) {
                eval_pc<kEps0>(a, L, L.pc + (pc_n - kWave), kWave, gc, tact, sub, k, ox, oy, oz, acc);
                pc_n -= kWave;
            }
            while (pend >= (uint32_t)kWave) {
                uint32_t idx;
                const int n = pp_n > 0 ? pop64(leaves, pp_n, L.mark, idx) : 0;
                if (n <= 0) {   // inconsistent bookkeeping: never spin
                    overflow = true;
                    pend = 0;
                    break;
                }
                eval_pp<kEps0>(a, L, idx, n, gc, tact, sub, k, ox, oy, oz, acc);
                pend -= (uint32_t)n;
            }
            if (overflow) break;
        }
        if (pc_n > 0) eval_pc<kEps0>(a, L, L.pc, pc_n, gc, tact, sub, k, ox, oy, oz, acc);
        while (pend > 0) {
            uint32_t idx;
            const int n = pp_n > 0 ? pop64(leaves, pp_n, L.mark, idx) : 0;
            if (n <= 0) {
                overflow = true;
                break;
            }
            eval_pp<kEps0>(a, L, idx, n, gc, tact, sub, k, ox, oy, oz, acc);
            pend -= (uint32_t)n < pend ? (uint32_t)n : pend;
        }

        // combine the k lanes of each particle
        float ax = acc.ax + acc.cx, ay = acc.ay + acc.cy, az = acc.az + acc.cz, ph = acc.ph + acc.cp;
        for (int s = 1; s < k; ++s) {
            const int srcl = lane + s * gn;
            const float bx = __shfl(ax, srcl < kWave ? srcl : lane, kWave);
            const float by = __shfl(ay, srcl < kWave ? srcl : lane, kWave);
            const float bz = __shfl(az, srcl < kWave ? srcl : lane, kWave);
            const float bp = __shfl(ph, srcl < kWave ? srcl : lane, kWave);
            if (sub == 0) {
                ax += bx;
                ay += by;
                az += bz;
                ph += bp;
            }
        }
        if (sub == 0 && lane < gn) {
            // the particle met itself once in the particle list: with eps > 0 that
            // term added -m/eps to the potential and nothing to the acceleration
            if (!kEps0) ph = ph + mi * __builtin_amdgcn_rsqf(a.eps2);
            a.acc4[gs + lane] = make_float4(ax, ay, az, ph);
        }
        if (lane == 0) {
            a.g_npp[g] = npp;
            a.g_npc[g] = npc;
            atomicAdd(&a.misc->sum_npp, (unsigned long long)npp * (unsigned long long)gn);
            atomicAdd(&a.misc->sum_npc, (unsigned long long)npc * (unsigned long long)gn);
            if (overflow) atomicOr(&a.misc->walk_overflow, 1u);
        }
        wave_sync();
    }
}

__global__ void walk_reset_kernel(DevMisc *m)
{
    if (threadIdx.x == 0) {
        m->walk_next = 0;
        m->walk_overflow = 0;
        m->sum_npp = 0;
        m->sum_npc = 0;
    }
}

// per-cell walk record: (first child, nchild) for nodes, (first particle, count |
// leaf bit) for leaves, and the float32 opening radius squared
__global__ void __launch_bounds__(256)
pack_walk_kernel(int64_t ncells, const uint8_t *__restrict__ c_leaf,
                 const uint32_t *__restrict__ c_first, const uint32_t *__restrict__ c_count,
                 const uint32_t *__restrict__ c_child, const uint32_t *__restrict__ c_nchild,
                 const float *__restrict__ rcrit2, uint4 *__restrict__ c_walk)
{
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= ncells) return;
    const bool leaf = c_leaf[c] != 0;
    const uint32_t x = leaf ? c_first[c] : c_child[c];
    const uint32_t y = leaf ? (c_count[c] | 0x80000000u) : c_nchild[c];
    c_walk[c] = make_uint4(x, y, __float_as_uint(rcrit2[c]), 0u);
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

hipError_t launch_walk(bh_ctx *c, float theta, float eps)
{
    (void)theta;
    const int64_t nc = c->ncells;
    uint4 *cw = c->c_walk;
    hipLaunchKernelGGL(pack_walk_kernel, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, c->stream,
                       nc, c->c_leaf, c->c_first, c->c_count, c->c_child, c->c_nchild, c->c_rcrit2,
                       cw);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(walk_reset_kernel, dim3(1), dim3(64), 0, c->stream, c->misc);
    BH_LAUNCH_CHECK();
    WalkArgs a;
    a.ngroups = c->ngroups;
    a.ncells = (uint32_t)c->ncells;
    a.g_first = c->g_first;
    a.g_count = c->g_count;
    a.g_centre = c->g_centre;
    a.g_half = c->g_half;
    a.p4 = c->p4[c->cur];
    a.c_com = c->c_com;
    a.c_q0 = c->c_q0;
    a.c_q1 = c->c_q1;
    a.c_walk = cw;
    a.acc4 = c->acc4;
    a.g_npp = c->g_npp;
    a.g_npc = c->g_npc;
    a.misc = c->misc;
    a.eps2 = eps * eps;
    int dev_cus = 256;
    if (hipDeviceGetAttribute(&dev_cus, hipDeviceAttributeMultiprocessorCount, c->device) !=
        hipSuccess)
        dev_cus = 256;
    int64_t blocks = (int64_t)dev_cus * 8;
    const int64_t need = (c->ngroups + kWalkWaves - 1) / kWalkWaves;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    if (a.eps2 > 0.0f)
        hipLaunchKernelGGL(walk_kernel<false>, dim3((unsigned)blocks), dim3(kWalkBlock), 0, c->stream, a);
    else
        hipLaunchKernelGGL(walk_kernel<true>, dim3((unsigned)blocks), dim3(kWalkBlock), 0, c->stream, a);
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
