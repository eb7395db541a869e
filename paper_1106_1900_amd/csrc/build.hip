// build.hip - tree construction on the device: bounding box, integer map and
// Morton keys (App. B), particle reordering ("moving", Sect. 4.1), the cell array
// (Sect. 2.1), links, groups (Sect. 2.2), float64 multipole moments (Sect. 3.2)
// and the opening radius of Eq. (1) (Sect. 3.3).
//
// Every kernel works on a batch of K independent clusters held back to back in
// the particle arrays (K = 1 for a single system).  Each cluster keeps its own
// domain, keys, tree and groups; the cell array holds the cells of all clusters,
// level-major, and within a level in particle order, so each cluster's cells form
// exactly its own (level, key) ordered array, interleaved by level with the
// others.  Level 0 holds the K roots in cluster order.
//
// The paper forms cells level by level: it masks the keys of particles not yet in
// a leaf, groups equal masked keys by compaction, marks cells of at most N_leaf
// particles as leaves and repeats down to the deepest level, then links parents
// and children with binary searches and atomics.  The same cell array is built
// here with a fixed number of launches, independent of the depth:
//
//   split(i)  = first level at which sorted particles i-1 and i fall in
//               different cells (from the common key prefix; 21 if equal keys;
//               0 at the first particle of a cluster);
//   leaf(i)   = the level of the leaf holding particle i: the first level at
//               which the run of particles sharing i's key prefix is at most
//               N_leaf long, or 20 (found from split() within +-N_leaf of i);
//   particle i starts exactly the cells of the levels split(i) .. leaf(i).
//
// Counting those starts per level and block, one scan per level gives every
// cell its position in the (level, key) order, its parent and first child come
// from the per-level ranks of the same particle, and a cell's end is the first
// start after it at the same or a shallower level.  The result is the paper's
// cell array exactly, in its order.
//
// No kernel here needs a count on the host: cell, group and level counts stay in
// device memory and the kernels that depend on them loop over fixed grids, so a
// whole build can be captured in a HIP graph.
#include <algorithm>

#include "bh_internal.h"

#pragma clang fp contract(off)

namespace bh {

namespace {

constexpr int kBlock = 256;
static_assert(kBlock == kChunkThreads, "per-chunk kernels share box_partial");
constexpr int kFixedGrid = 2048;       // grid of the kernels that read their size on the device

__device__ __forceinline__ uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0xFFFFFu;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint32_t compact3(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10C30C30C30C30C3ull;
    x = (x ^ (x >> 4)) & 0x100F00F00F00F00Full;
    x = (x ^ (x >> 8)) & 0x001F0000FF0000FFull;
    x = (x ^ (x >> 16)) & 0x001F00000000FFFFull;
    x = (x ^ (x >> 32)) & 0x1FFFFFull;
    return (uint32_t)x;
}

__device__ __forceinline__ uint32_t coord_to_int(double x, double lo, double scale)
{
    double d = x - lo;
    double f = d * scale;
    return f >= (double)kQMax ? kQMax : (uint32_t)f;
}

inline int grid_for(int64_t n, int block) { return (int)((n + block - 1) / block); }

// ---------------------------------------------------------------------------


struct AosSrc {
    const double *p;
    __device__ void get3(int64_t i, double *v) const
    {
        v[0] = p[3 * i];
        v[1] = p[3 * i + 1];
        v[2] = p[3 * i + 2];
    }
};
struct P4Src {
    const double4 *p;
    __device__ void get3(int64_t i, double *v) const
    {
        const double4 q = p[i];
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
    }
};

// cluster of every particle position, from the chunk table
__global__ void __launch_bounds__(kBlock)
cluster_ids_kernel(const Chunk *__restrict__ chunks, uint32_t *__restrict__ pcl)
{
    const Chunk ch = chunks[blockIdx.x];
    for (uint32_t i = ch.begin + threadIdx.x; i < ch.end; i += kBlock) pcl[i] = ch.cluster;
}

// Per-chunk minima and maxima of each axis: part[6 b + k], k = 0..2 minima, 3..5
// maxima.  A non-finite coordinate sets bit 0 of the misc flags.  (A leapfrog
// step's kick-drift kernel writes the same partials of the drifted positions.)
template <typename Src>
__global__ void __launch_bounds__(kBlock)
bbox_kernel(Src src, const Chunk *__restrict__ chunks, double *__restrict__ part, DevMisc *m)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) reset_build_counts(m);
    const Chunk ch = chunks[blockIdx.x];
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    for (uint32_t i = ch.begin + threadIdx.x; i < ch.end; i += kBlock) {
        double v[3];
        src.get3(i, v);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            bad |= !isfinite(v[k]);
            lo[k] = fmin(lo[k], v[k]);
            hi[k] = fmax(hi[k], v[k]);
        }
    }
    box_partial(lo, hi, bad, part, m);
}

// One block per cluster: reduce its chunk partials; cube side = largest extent
// (1 if all extents vanish); scale = 2^20 / side.
__global__ void __launch_bounds__(kBlock)
domain_kernel(const double *__restrict__ part, const DevCluster *__restrict__ clus,
              DevDomain *__restrict__ dom)
{
    const DevCluster &cl = clus[blockIdx.x];
    const uint32_t b0 = cl.chunk0, b1 = cl.chunk0 + cl.nchunk;
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += kBlock) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[k] = fmin(v[k], part[6 * (int64_t)b + k]);
            v[3 + k] = fmax(v[3 + k], part[6 * (int64_t)b + 3 + k]);
        }
    }
    __shared__ double s_v[6][kBlock / kWave];
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double a = v[k];
#pragma unroll
        for (int d = kWave / 2; d > 0; d >>= 1) {
            const double o = __shfl_xor(a, d, kWave);
            a = k < 3 ? fmin(a, o) : fmax(a, o);
        }
        if (l == 0) s_v[k][w] = a;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = s_v[k][0];
        hi[k] = s_v[3 + k][0];
        for (int i = 1; i < kBlock / kWave; ++i) {
            lo[k] = fmin(lo[k], s_v[k][i]);
            hi[k] = fmax(hi[k], s_v[3 + k][i]);
        }
    }
    DevDomain d;
    double side = 0.0;
    for (int k = 0; k < 3; ++k) {
        d.lo[k] = lo[k];
        d.hi[k] = hi[k];
        const double e = hi[k] - lo[k];
        if (e > side) side = e;
    }
    if (side == 0.0) side = 1.0;
    d.L = side;
    d.scale = 1048576.0 / side;
    dom[blockIdx.x] = d;
}

// Keys of the particles, written in caller order: the pair of the particle at
// position i goes to slot pid[i] (its caller index; pid == null: the positions
// are the caller order, a first load) with value i.  The stable sort that
// follows then orders equal keys by caller index, on a first load and on every
// rebuild alike (App. A: the split primitive keeps the input order).  With
// held != 0 the pair goes to slot i instead (a rebuild's bucket sort, which
// orders equal keys by pid itself).  With ncand > 0 the keys at positions
// (c + 1) cstride, c < ncand, are also written to cand[c] (the candidate
// splitters of that sort).
template <typename Src>
__global__ void __launch_bounds__(kBlock)
keys_kernel(Src src, const Chunk *__restrict__ chunks, const DevDomain *__restrict__ dom,
            const uint32_t *__restrict__ pid, uint32_t n, uint64_t *__restrict__ key,
            uint32_t *__restrict__ val, uint32_t held, uint64_t *__restrict__ cand,
            uint32_t ncand, uint32_t cstride, DevMisc *m)
{
    const Chunk ch = chunks[blockIdx.x];
    const DevDomain &cl = dom[ch.cluster];
    const double lx = cl.lo[0], ly = cl.lo[1], lz = cl.lo[2], scale = cl.scale;
    // kKeyBatch elements per thread at a time: all their loads are issued before
    // the scattered stores, which the compiler may not move loads across
    constexpr int kKeyBatch = 8;
    for (uint32_t i0 = ch.begin + threadIdx.x; i0 < ch.end; i0 += kKeyBatch * kBlock) {
        double v[kKeyBatch][3];
        uint32_t o[kKeyBatch];
#pragma unroll
        for (int u = 0; u < kKeyBatch; ++u) {
            const uint32_t i = i0 + (uint32_t)u * kBlock;
            if (i < ch.end) {
                src.get3(i, v[u]);
                o[u] = pid && !held ? pid[i] : i;
            }
        }
#pragma unroll
        for (int u = 0; u < kKeyBatch; ++u) {
            const uint32_t i = i0 + (uint32_t)u * kBlock;
            if (i >= ch.end) continue;
            const uint32_t qx = coord_to_int(v[u][0], lx, scale);
            const uint32_t qy = coord_to_int(v[u][1], ly, scale);
            const uint32_t qz = coord_to_int(v[u][2], lz, scale);
            uint32_t dst = o[u];
            if (dst >= n) {     // caller indices are a permutation of [0, n)
                atomicOr(&m->nonfinite, 8u);
                dst = i;
            }
            const uint64_t k = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
            key[dst] = k;
            val[dst] = i;
            if (ncand) {
                const uint32_t q = (uint32_t)(((double)i + 0.5) / (double)cstride);
                if (q >= 1u && q <= ncand && q * cstride == i) cand[q - 1] = k;
            }
        }
    }
}

__global__ void __launch_bounds__(kBlock)
reorder_from_caller_kernel(const double *__restrict__ pos, const double *__restrict__ mass,
                           const double *__restrict__ vel, const uint32_t *__restrict__ perm,
                           int64_t n, double4 *__restrict__ p4, double4 *__restrict__ v4,
                           uint32_t *__restrict__ pid, DevMisc *m)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t s = perm[i];
    const double ms = mass[s];
    if (!(ms > 0.0) || !isfinite(ms)) atomicOr(&m->nonfinite, 2u);
    p4[i] = make_double4(pos[3 * s], pos[3 * s + 1], pos[3 * s + 2], ms);
    // the velocity record carries the mass too (read by the energy sums)
    v4[i] = vel ? make_double4(vel[3 * s], vel[3 * s + 1], vel[3 * s + 2], ms)
                : make_double4(0.0, 0.0, 0.0, ms);
    pid[i] = (uint32_t)s;
}

__global__ void __launch_bounds__(kBlock)
reorder_kernel(const double4 *__restrict__ p4i, const double4 *__restrict__ v4i,
               const uint32_t *__restrict__ pidi, const uint32_t *__restrict__ perm, int64_t n,
               double4 *__restrict__ p4o, double4 *__restrict__ v4o, uint32_t *__restrict__ pido,
               DevMisc *m)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t s = perm[i];
    if (s >= (uint64_t)n) {     // only after an internal error (bit 3 already set)
        atomicOr(&m->nonfinite, 8u);
        s = (uint32_t)i;
    }
    p4o[i] = p4i[s];
    v4o[i] = v4i[s];
    pido[i] = pidi[s];
}

// ---------------------------------------------------------------------------
// cells

__device__ __forceinline__ int wave_min_i32(int v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const int o = __shfl_xor(v, d, kWave);
        v = o < v ? o : v;
    }
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const int o = __shfl_xor(v, d, kWave);
        v = o > v ? o : v;
    }
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ uint8_t split_level(uint64_t a, uint64_t b)
{
    uint64_t x = a ^ b;
    if (x == 0) return (uint8_t)(kMaxLevel + 1);
    // keys use 60 bits: 4 leading zero bits are not part of the key
    int lz = __clzll((long long)x) - 4;
    return (uint8_t)(1 + lz / 3);
}

// Per particle: split level, leaf level; per block and level: number of cells
// starting in the block.  blk layout: [level][block], then a row of the leaves
// starting in each block.  H is the largest leaf size
// of the batch (the halo); each particle uses its own cluster's leaf size.
__global__ void __launch_bounds__(kTreeTile)
split_leaf_kernel(const uint64_t *__restrict__ key, const uint32_t *__restrict__ pcl, int64_t n,
                  int H, const DevCluster *__restrict__ clus, uint8_t *__restrict__ split,
                  uint8_t *__restrict__ lam, uint8_t *__restrict__ gflag, uint32_t *__restrict__ blk,
                  int nblk, DevMisc *__restrict__ m)
{
    extern __shared__ uint8_t s_dyn[];
    const int W = kTreeTile + 2 * H;              // split values held in LDS
    uint8_t *s_split = s_dyn;                     // [W]
    uint8_t *s_pl = s_dyn + ((W + 15) & ~15);     // [H][kTreeTile] left prefix minima
    __shared__ uint32_t s_cnt[kLevels];
    __shared__ uint32_t s_leaves;

    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kTreeTile;
    if (t < kLevels) s_cnt[t] = 0;
    if (t == 0) s_leaves = 0;
    // split of global index j, with split = 0 at the first particle of a cluster
    // and at n
    for (int u = t; u < W; u += kTreeTile) {
        int64_t j = base - H + u;
        uint8_t v;
        if (j <= 0 || j >= n || pcl[j] != pcl[j - 1]) v = 0;
        else v = split_level(key[j - 1], key[j]);
        s_split[u] = v;
    }
    __syncthreads();

    const int64_t i = base + t;
    const bool valid = i < n;
    uint8_t sp = 0, lm = 0;
    if (valid) {
        const int h = (int)clus[pcl[i]].nleaf;
        sp = s_split[H + t];
        // left prefix minima PL[a] = min split(i - a'), a' = 0..a
        uint8_t run = 255;
        for (int a = 0; a < h; ++a) {
            uint8_t v = (i - a <= 0) ? (uint8_t)0 : s_split[H + t - a];
            run = v < run ? v : run;
            s_pl[a * kTreeTile + t] = run;
        }
        // right prefix minima PR[b] over split(i + b'), b' = 1..b, combined with
        // PL[h - b]: leaf level = min_b max(PL[h - b], PR[b])
        uint8_t best = 255;
        run = 255;
        for (int b = 1; b <= h; ++b) {
            uint8_t v = (i + b >= n) ? (uint8_t)0 : s_split[H + t + b];
            run = v < run ? v : run;
            uint8_t pl = s_pl[(h - b) * kTreeTile + t];
            uint8_t mx = pl > run ? pl : run;
            best = mx < best ? mx : best;
        }
        lm = best > kMaxLevel ? (uint8_t)kMaxLevel : best;
        split[i] = sp;
        lam[i] = lm;
        gflag[i] = 0;       // group starts are flagged later by cell_finish_kernel
    }
    // count starts per level (only the levels where some particle of the
    // wavefront starts a cell)
    const int l = t % kWave;
    const bool starts = valid && sp <= lm;
    const int lo = wave_min_i32(starts ? (int)sp : kLevels);
    const int hi = wave_max_i32(starts ? (int)lm : -1);
    for (int lev = lo; lev <= hi; ++lev) {
        unsigned long long b = ballot(valid && sp <= lev && lev <= lm);
        if (l == 0 && b) atomicAdd(&s_cnt[lev], (uint32_t)__popcll(b));
    }
    {
        unsigned long long b = ballot(valid && sp <= lm);
        if (l == 0 && b) atomicAdd(&s_leaves, (uint32_t)__popcll(b));
    }
    __syncthreads();
    if (t < kLevels) blk[(int64_t)t * nblk + blockIdx.x] = s_cnt[t];
    // leaves started in this block: one more row of the count table, summed by
    // scan_levels_kernel (a device-wide atomic per block serialises at one address)
    if (t == 0) blk[(int64_t)kLevels * nblk + blockIdx.x] = s_leaves;
}

// level counts -> level offsets (level-major order), total cells, depth.
__device__ void level_finalize(const uint32_t *__restrict__ tot, DevMisc *m, int64_t cap_c)
{
    uint64_t off = 0;
    uint32_t depth = 0;
    uint32_t cnt[kLevels];
    for (int l = 0; l < kLevels; ++l) {
        cnt[l] = __hip_atomic_load(&tot[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        m->level_offset[l] = (uint32_t)off;
        m->level_count[l] = cnt[l];
        if (cnt[l]) depth = (uint32_t)l;
        off += cnt[l];
    }
    if (off > (uint64_t)cap_c) {
        // cannot happen for a consistent tree; keep every later write in bounds
        m->nonfinite |= 4u;
        for (int l = 0; l < kLevels; ++l) m->level_count[l] = 0;
        off = 0;
    }
    m->level_offset[kLevels] = (uint32_t)off;
    m->ncells = (uint32_t)off;
    m->depth = depth;
    m->nleaves = __hip_atomic_load(&tot[kLevels], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// one block per level (and one for the leaf row): exclusive scan of the row's
// block counts in place; the last block to finish derives the level offsets
constexpr int kScanLevelsBlock = 1024;

__global__ void __launch_bounds__(kScanLevelsBlock)
scan_levels_kernel(uint32_t *__restrict__ blk, int nblk, uint32_t *__restrict__ tot, DevMisc *m,
                   int64_t cap_c)
{
    constexpr int kWaves = kScanLevelsBlock / kWave;
    __shared__ uint32_t s_tmp[kWaves];
    uint32_t *row = blk + (int64_t)blockIdx.x * nblk;
    uint32_t run = 0;
    const int t = threadIdx.x, w = t / kWave, l = t % kWave;
    for (int b0 = 0; b0 < nblk; b0 += kScanLevelsBlock) {
        int b = b0 + t;
        uint32_t v = b < nblk ? row[b] : 0u;
        uint32_t inc = wave_incl_scan_add(v);
        if (l == kWave - 1) s_tmp[w] = inc;
        __syncthreads();
        uint32_t off = 0, totw = 0;
        for (int k = 0; k < kWaves; ++k) {
            const uint32_t x = s_tmp[k];
            if (k < w) off += x;
            totw += x;
        }
        __syncthreads();
        if (b < nblk) row[b] = run + off + inc - v;
        run += totw;
    }
    if (t == 0) {
        __hip_atomic_store(&tot[blockIdx.x], run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // release this level's total, then count the finished levels
        const uint32_t done = __hip_atomic_fetch_add(&m->levels_done, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            level_finalize(tot, m, cap_c);
            m->levels_done = 0;      // ready for the next build
        }
    }
}

// For every level, the index of the cell of that level holding particle i
// (valid up to lam(i)): level offset + number of starts at that level up to i,
// minus one.  Computed with wavefront ballots and the scanned block counts.
struct Ranks {
    uint32_t anc[kLevels];
};

// Only the levels lo..hi (wavefront-uniform) get their ranks; the starts of every
// level are counted, as other wavefronts of the block may need them.
__device__ __forceinline__ void level_ranks(bool valid, uint8_t sp, uint8_t lm,
                                            const uint32_t *__restrict__ blk_scanned, int nblk,
                                            const DevMisc *__restrict__ m, uint32_t (*s_wc)[kLevels],
                                            int lo, int hi, Ranks &r)
{
    const int t = threadIdx.x, w = t / kWave, l = t % kWave;
    unsigned long long balls[kLevels];
#pragma unroll
    for (int lev = 0; lev < kLevels; ++lev) {
        balls[lev] = ballot(valid && sp <= lev && lev <= lm);
        if (l == 0) s_wc[w][lev] = (uint32_t)__popcll(balls[lev]);
    }
    __syncthreads();
    const unsigned long long le = (l == kWave - 1) ? ~0ull : ((2ull << l) - 1ull);
#pragma unroll
    for (int lev = 0; lev < kLevels; ++lev) {
        if (lev < lo || lev > hi) continue;
        uint32_t off = blk_scanned[(int64_t)lev * nblk + blockIdx.x];
        for (int ww = 0; ww < w; ++ww) off += s_wc[ww][lev];
        uint32_t incl = off + (uint32_t)__popcll(balls[lev] & le);
        r.anc[lev] = m->level_offset[lev] + incl - 1u;
    }
}

// Every cell a particle starts: its first particle, level, leaf flag, parent and
// first child.  The last particle of a cell (the next particle starts a cell at
// the same or a shallower level, or lies beyond the cluster) writes the cell's
// end; the last particle of a node also writes one past the node's last child
// (the child holding that particle).  Counts follow as end - first.
__global__ void __launch_bounds__(kTreeTile)
emit_cells_kernel(const uint8_t *__restrict__ split, const uint8_t *__restrict__ lam, int64_t n,
                  const uint32_t *__restrict__ blk_scanned, int nblk, const DevMisc *__restrict__ m,
                  uint32_t *__restrict__ c_first, uint8_t *__restrict__ c_level,
                  uint8_t *__restrict__ c_leaf, uint32_t *__restrict__ c_parent,
                  uint32_t *__restrict__ c_child, uint32_t *__restrict__ c_end,
                  uint32_t *__restrict__ c_cend, const uint32_t *__restrict__ pcl,
                  uint32_t *__restrict__ c_cl)
{
    __shared__ uint32_t s_wc[kTreeTile / kWave][kLevels];
    const int64_t i = (int64_t)blockIdx.x * kTreeTile + threadIdx.x;
    const bool valid = i < n;
    const uint8_t sp = valid ? split[i] : (uint8_t)255;
    const uint8_t lm = valid ? lam[i] : (uint8_t)0;
    // split of the next particle: 0 past the end (and at a cluster's first particle)
    const uint8_t sn = (valid && i + 1 < n) ? split[i + 1] : (uint8_t)0;
    // the levels whose ranks this particle uses: from the parent of its first
    // start or end up to its leaf (none if it starts and ends nothing)
    const int first_lev = sp < sn ? sp : sn;
    const bool used = valid && first_lev <= lm;
    const int lo = wave_min_i32(used ? (first_lev > 0 ? first_lev - 1 : 0) : kLevels);
    const int hi = wave_max_i32(used ? (int)lm : -1);
    Ranks r;
    level_ranks(valid, sp, lm, blk_scanned, nblk, m, s_wc, lo, hi, r);
    const uint32_t ncells = m->ncells;
    if (!valid || ncells == 0) return;
    const uint32_t cluster = sp <= lm ? pcl[i] : 0u;
#pragma unroll
    for (int lev = 0; lev < kLevels; ++lev) {
        if (lev < lo || lev > hi) continue;      // wavefront-uniform
        if (lev > lm) continue;
        const uint32_t c = r.anc[lev];
        if (c >= ncells) continue;
        if (lev >= sp) {
            c_first[c] = (uint32_t)i;
            c_cl[c] = cluster;
            c_level[c] = (uint8_t)lev;
            c_leaf[c] = (uint8_t)(lev == lm);
            c_parent[c] = lev > 0 ? r.anc[lev > 0 ? lev - 1 : 0] : kNone;
            c_child[c] = lev < lm ? r.anc[lev < kMaxLevel ? lev + 1 : kMaxLevel] : kNone;
        }
        if (lev >= sn) {
            // particle i is the last of its level-lev cell
            c_end[c] = (uint32_t)(i + 1);
            if (lev < lm) {
                const uint32_t last = r.anc[lev < kMaxLevel ? lev + 1 : kMaxLevel];
                c_cend[c] = last + 1u;
            }
        }
    }
}

// Per cell: count = end - first, children = one past the last child - first
// child (0 for a leaf), and the group starts (Sect. 2.2): a cell of at most
// ncrit particles whose parent holds more (or the root) starts a group at its
// first particle; a leaf still larger than ncrit is cut into runs of ncrit
// particles.  Reads the ends of a cell's parent, never its converted fields.
__global__ void __launch_bounds__(kBlock)
cell_finish_kernel(DevMisc *__restrict__ m, const uint32_t *__restrict__ pcl,
                   const DevCluster *__restrict__ clus, const uint32_t *__restrict__ c_first,
                   const uint32_t *__restrict__ c_end, const uint8_t *__restrict__ c_leaf,
                   const uint8_t *__restrict__ c_level, const uint32_t *__restrict__ c_parent,
                   const uint32_t *__restrict__ c_child, uint32_t *__restrict__ c_count,
                   uint32_t *__restrict__ c_nchild, uint8_t *__restrict__ gflag, int64_t n)
{
    const uint32_t ncells = m->ncells;
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < ncells; c += gridDim.x * kBlock) {
        const uint32_t f = c_first[c];
        uint32_t e = c_end[c];
        const bool leaf = c_leaf[c] != 0;
        const uint32_t nc = leaf ? 0u : c_nchild[c] - c_child[c];
        // never for a consistent tree; keeps every later access in bounds
        if (f >= (uint64_t)n || e <= f || e > (uint64_t)n || (!leaf && (nc < 1u || nc > 8u))) {
            c_count[c] = 0;
            c_nchild[c] = 0;
            atomicOr(&m->nonfinite, 8u);
            continue;
        }
        const uint32_t cnt = e - f;
        c_count[c] = cnt;
        c_nchild[c] = nc;
        const uint32_t ncrit = clus[pcl[f]].ncrit;
        bool top = c_level[c] == 0;
        if (!top) {
            const uint32_t p = c_parent[c];
            top = p < ncells && c_end[p] - c_first[p] > ncrit;
        }
        if (cnt <= ncrit && top) gflag[f] = 1;
        if (leaf && cnt > ncrit)
            for (uint32_t o = 0; o < cnt; o += ncrit) gflag[f + o] = 1;
    }
}

// group counts and tight boxes: 16 lanes per group, grid-stride over the groups
// counted on the device
__global__ void __launch_bounds__(kBlock)
group_boxes_kernel(const uint32_t *__restrict__ g_first, const DevMisc *__restrict__ m, int64_t n,
                   const double4 *__restrict__ p4, const uint32_t *__restrict__ pcl,
                   uint32_t *__restrict__ g_count, double4 *__restrict__ g_centre,
                   float4 *__restrict__ g_half)
{
    constexpr int kSeg = 16;                       // lanes per group
    const int64_t ngroups = m->ngroups;
    const int l = threadIdx.x % kSeg;
    for (int64_t g0 = (int64_t)blockIdx.x * (kBlock / kSeg); g0 < ngroups;
         g0 += (int64_t)gridDim.x * (kBlock / kSeg)) {
        const int64_t g = g0 + threadIdx.x / kSeg;
        const bool valid = g < ngroups;
        const uint32_t s = valid ? g_first[g] : 0u;
        const uint32_t e = valid ? ((g + 1 < ngroups) ? g_first[g + 1] : (uint32_t)n) : 0u;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (uint32_t j = s + l; j < e; j += kSeg) {
            const double4 p = p4[j];
            lo[0] = fmin(lo[0], p.x); hi[0] = fmax(hi[0], p.x);
            lo[1] = fmin(lo[1], p.y); hi[1] = fmax(hi[1], p.y);
            lo[2] = fmin(lo[2], p.z); hi[2] = fmax(hi[2], p.z);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int d = kSeg / 2; d > 0; d >>= 1) {
                lo[k] = fmin(lo[k], __shfl_xor(lo[k], d, kWave));
                hi[k] = fmax(hi[k], __shfl_xor(hi[k], d, kWave));
            }
        }
        if (valid && l == 0) {
            g_count[g] = e - s;
            // w: the group's cluster, whose root is the level-0 cell of that index
            g_centre[g] = make_double4(0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]),
                                       0.5 * (lo[2] + hi[2]), (double)pcl[s]);
            g_half[g] = make_float4((float)(0.5 * (hi[0] - lo[0])), (float)(0.5 * (hi[1] - lo[1])),
                                    (float)(0.5 * (hi[2] - lo[2])), 0.0f);
        }
    }
}

// ---------------------------------------------------------------------------
// moments: float64 monopole and second moment, level by level from the deepest
// (Sect. 3.2): a leaf from its particles, a node from its children (one level
// deeper, finished by the previous launch), both in array order.

// Where the opening radii and walk records go, and what they are computed from.
struct RecOut {
    const DevCluster *clus;
    const DevDomain *dom;
    const uint8_t *c_level;
    const uint32_t *c_cl;     // cluster of each cell
    const uint64_t *skey;     // sorted keys
    float *rcrit2;
    WalkCell *rec;
    double4 *geo;
};

// Eq. (1): r_crit = l/theta + delta with l = L 2^-level and delta the distance of
// the centre of mass from the cell's geometric centre (a refitted cell whose
// particles left it: its tight box's centre and side); stored as float32 r_crit^2,
// together with the rest of the cell's walk record.  theta, the opening test and
// the domain are those of the cell's cluster k; for the minimum-distance test
// r_crit = l/theta and the cube (centre, half side) goes to geo.  f: the cell's
// first particle (its key gives the key prefix); box: the cell's tight box (lo x,
// y, z, hi x, y, z) after a refit, else null.
__device__ __forceinline__ void cell_record(uint32_t c, uint32_t f, int lev, uint32_t k, bool leaf,
                                            uint32_t link, uint32_t info, const double4 cm,
                                            const float4 a, const float4 b, const double *blo,
                                            const double *bhi, const RecOut &ro)
{
    const DevDomain &cl = ro.dom[k];
    const float theta = ro.clus[k].theta;
    const double l = ldexp(cl.L, -lev);
    const uint64_t pre = ro.skey[f] >> (3 * (kMaxLevel - lev));
    const double gx = cl.lo[0] + ((double)compact3(pre) + 0.5) * l;
    const double gy = cl.lo[1] + ((double)compact3(pre >> 1) + 0.5) * l;
    const double gz = cl.lo[2] + ((double)compact3(pre >> 2) + 0.5) * l;
    // After a refit a cell whose particles all still lie in its key cell keeps
    // this geometry; any other cell takes its box's centre and side
    // max(l, largest extent), so that the cube of the opening tests holds every
    // particle of the cell.  The integer map is monotone, so the particles keep
    // the key cell exactly when the box's two ends do.
    double side = l, cx = gx, cy = gy, cz = gz;
    if (blo) {
        const int sh = kMaxLevel - lev;
        const uint32_t cell[3] = {compact3(pre), compact3(pre >> 1), compact3(pre >> 2)};
        bool inside = true;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            inside = inside && blo[q] >= cl.lo[q] && bhi[q] <= cl.hi[q] &&
                     (coord_to_int(blo[q], cl.lo[q], cl.scale) >> sh) == cell[q] &&
                     (coord_to_int(bhi[q], cl.lo[q], cl.scale) >> sh) == cell[q];
        }
        if (!inside) {
            double ext = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) ext = bhi[q] - blo[q] > ext ? bhi[q] - blo[q] : ext;
            side = ext > l ? ext : l;
            cx = 0.5 * (blo[0] + bhi[0]);
            cy = 0.5 * (blo[1] + bhi[1]);
            cz = 0.5 * (blo[2] + bhi[2]);
        }
    }
    double r;
    if (ro.clus[k].mac) {
        // minimum-distance test: the cube (geometric centre, half side) must lie
        // beyond side / theta of the group's box
        r = side / (double)theta;
        ro.geo[c] = make_double4(cx, cy, cz, 0.5 * side);
    } else {
        const double dx = cm.x - cx, dy = cm.y - cy, dz = cm.z - cz;
        const double delta = sqrt((dx * dx + dy * dy) + dz * dz);
        r = side / (double)theta + delta;
    }
    const float r2 = (float)(r * r);
    ro.rcrit2[c] = r2;
    WalkCell w;
    w.cx = cm.x;
    w.cy = cm.y;
    w.cz = cm.z;
    w.mass = (float)cm.w;
    w.rcrit2 = r2;
    w.link = link;
    w.info = leaf ? (info | 0x80000000u) : info;
    w.s3[0] = a.x;
    w.s3[1] = a.y;
    w.s3[2] = a.z;
    w.s3[3] = a.w;
    w.s3[4] = b.x;
    w.s3[5] = b.y;
    ro.rec[c] = w;
}

__device__ __forceinline__ void store_walk_multipole(uint32_t c, const double *S,
                                                     float4 *__restrict__ q0, float4 *__restrict__ q1,
                                                     float4 &a, float4 &b)
{
    const double tr = (S[0] + S[1]) + S[2];
    a = make_float4((float)(3.0 * S[0]), (float)(3.0 * S[1]), (float)(3.0 * S[2]),
                    (float)(3.0 * S[3]));
    b = make_float4((float)(3.0 * S[4]), (float)(3.0 * S[5]), (float)(0.5 * tr), (float)(1.5 * tr));
    q0[c] = a;
    q1[c] = b;
}

// Moments of cell c: a leaf from its particles, a node from its children (one
// level deeper, already done), both in array order.  Each pass over the members
// loads a run of kRun of them at once (indices past the end repeat the last
// member and are left out of the sums), so a pass costs one memory latency per
// run instead of one per member; the sums keep the members' order.
constexpr int kRun = 8;
// leaves of up to kLeafFast particles load them once for all three sums
#ifndef BH_LEAF_FAST
#define BH_LEAF_FAST 8
#endif
constexpr int kLeafFast = BH_LEAF_FAST;

template <bool kLeaf, bool kBox>
__device__ __forceinline__ void cell_moments(uint32_t c, const uint32_t *__restrict__ c_first,
                                             const uint32_t *__restrict__ c_count,
                                             const uint32_t *__restrict__ c_child,
                                             const uint32_t *__restrict__ c_nchild,
                                             const double4 *__restrict__ p4,
                                             double4 *__restrict__ c_com, double *__restrict__ c_S,
                                             float4 *__restrict__ q0, float4 *__restrict__ q1,
                                             double2 *__restrict__ box, const RecOut &ro)
{
    // members [s, s + n): particles of a leaf (position, mass) or children of a
    // node (centre of mass, mass; second moments in c_S)
    const uint32_t s = kLeaf ? c_first[c] : c_child[c];
    const uint32_t n = kLeaf ? c_count[c] : c_nchild[c];
    // the walk record's inputs, loaded with the cell's own record
    const int lev = ro.c_level[c];
    const uint32_t kc = ro.c_cl[c];
    const uint32_t rlink = kLeaf ? s : c_child[c];
    const double4 *__restrict__ src = kLeaf ? p4 : c_com;
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    double S[6] = {0, 0, 0, 0, 0, 0};
    // kBox: the tight box of the cell's particles (min and max are exact, so the
    // order of the members does not matter): a leaf's from its particles, a
    // node's as the union of its children's
    double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (kLeaf && n >= 1u && n <= (uint32_t)kLeafFast) {
        // one run: its members are loaded once and serve all three passes, with
        // the operations of the general path below in the same order
        double4 q[kLeafFast];
#pragma unroll
        for (int k = 0; k < kLeafFast; ++k) q[k] = src[s + min((uint32_t)k, n - 1u)];
#pragma unroll
        for (int k = 0; k < kLeafFast; ++k)
            if ((uint32_t)k < n) M = M + q[k].w;
        if (kBox) {
#pragma unroll
            for (int k = 0; k < kLeafFast; ++k) {
                blo[0] = fmin(blo[0], q[k].x); bhi[0] = fmax(bhi[0], q[k].x);
                blo[1] = fmin(blo[1], q[k].y); bhi[1] = fmax(bhi[1], q[k].y);
                blo[2] = fmin(blo[2], q[k].z); bhi[2] = fmax(bhi[2], q[k].z);
            }
        }
#pragma unroll
        for (int k = 0; k < kLeafFast; ++k) {
            if ((uint32_t)k < n) {
                sx = sx + q[k].w * q[k].x;
                sy = sy + q[k].w * q[k].y;
                sz = sz + q[k].w * q[k].z;
            }
        }
        const double cx = sx / M, cy = sy / M, cz = sz / M;
#pragma unroll
        for (int k = 0; k < kLeafFast; ++k) {
            if ((uint32_t)k < n) {
                const double dx = q[k].x - cx, dy = q[k].y - cy, dz = q[k].z - cz;
                const double w = q[k].w;
                S[0] += w * dx * dx; S[1] += w * dy * dy; S[2] += w * dz * dz;
                S[3] += w * dx * dy; S[4] += w * dx * dz; S[5] += w * dy * dz;
            }
        }
        c_com[c] = make_double4(cx, cy, cz, M);
        if (kBox) {
            double2 *b = box + 3 * (int64_t)c;
            b[0] = make_double2(blo[0], blo[1]);
            b[1] = make_double2(blo[2], bhi[0]);
            b[2] = make_double2(bhi[1], bhi[2]);
        }
        double2 *out = reinterpret_cast<double2 *>(c_S + 6 * (int64_t)c);
        out[0] = make_double2(S[0], S[1]);
        out[1] = make_double2(S[2], S[3]);
        out[2] = make_double2(S[4], S[5]);
        float4 qa, qb;
        store_walk_multipole(c, S, q0, q1, qa, qb);
        cell_record(c, s, lev, kc, kLeaf, rlink, n, make_double4(cx, cy, cz, M), qa, qb,
                    kBox ? blo : nullptr, kBox ? bhi : nullptr, ro);
        return;
    }
    // masses and first moments in one pass (each sum in the members' order)
    for (uint32_t r = 0; r < n; r += kRun) {
        double4 q[kRun];
#pragma unroll
        for (int k = 0; k < kRun; ++k) q[k] = src[s + min(r + k, n - 1)];
#pragma unroll
        for (int k = 0; k < kRun; ++k)
            if (r + k < n) M = M + q[k].w;
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            if (r + k < n) {
                sx = sx + q[k].w * q[k].x;
                sy = sy + q[k].w * q[k].y;
                sz = sz + q[k].w * q[k].z;
            }
        }
        if (kBox && kLeaf) {
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                blo[0] = fmin(blo[0], q[k].x); bhi[0] = fmax(bhi[0], q[k].x);
                blo[1] = fmin(blo[1], q[k].y); bhi[1] = fmax(bhi[1], q[k].y);
                blo[2] = fmin(blo[2], q[k].z); bhi[2] = fmax(bhi[2], q[k].z);
            }
        }
        if (kBox && !kLeaf) {
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const double2 *b = box + 3 * (int64_t)(s + min(r + k, n - 1));
                const double2 b0 = b[0], b1 = b[1], b2 = b[2];   // lo x, y; lo z, hi x; hi y, z
                blo[0] = fmin(blo[0], b0.x); blo[1] = fmin(blo[1], b0.y);
                blo[2] = fmin(blo[2], b1.x); bhi[0] = fmax(bhi[0], b1.y);
                bhi[1] = fmax(bhi[1], b2.x); bhi[2] = fmax(bhi[2], b2.y);
            }
        }
    }
    const double cx = sx / M, cy = sy / M, cz = sz / M;
    for (uint32_t r = 0; r < n; r += kRun) {
        double4 q[kRun];
#pragma unroll
        for (int k = 0; k < kRun; ++k) q[k] = src[s + min(r + k, n - 1)];
        if (kLeaf) {
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                if (r + k < n) {
                    const double dx = q[k].x - cx, dy = q[k].y - cy, dz = q[k].z - cz;
                    const double w = q[k].w;
                    S[0] += w * dx * dx; S[1] += w * dy * dy; S[2] += w * dz * dz;
                    S[3] += w * dx * dy; S[4] += w * dx * dz; S[5] += w * dy * dz;
                }
            }
        } else {
            double2 Sk[kRun][3];
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                const double2 *p = reinterpret_cast<const double2 *>(c_S + 6 * (int64_t)(s + min(r + k, n - 1)));
                Sk[k][0] = p[0];
                Sk[k][1] = p[1];
                Sk[k][2] = p[2];
            }
#pragma unroll
            for (int k = 0; k < kRun; ++k) {
                if (r + k < n) {
                    const double ex = q[k].x - cx, ey = q[k].y - cy, ez = q[k].z - cz;
                    const double w = q[k].w;
                    S[0] += Sk[k][0].x + w * ex * ex; S[1] += Sk[k][0].y + w * ey * ey;
                    S[2] += Sk[k][1].x + w * ez * ez; S[3] += Sk[k][1].y + w * ex * ey;
                    S[4] += Sk[k][2].x + w * ex * ez; S[5] += Sk[k][2].y + w * ey * ez;
                }
            }
        }
    }
    c_com[c] = make_double4(cx, cy, cz, M);
    if (kBox) {
        double2 *b = box + 3 * (int64_t)c;
        b[0] = make_double2(blo[0], blo[1]);
        b[1] = make_double2(blo[2], bhi[0]);
        b[2] = make_double2(bhi[1], bhi[2]);
    }
    double2 *out = reinterpret_cast<double2 *>(c_S + 6 * (int64_t)c);
    out[0] = make_double2(S[0], S[1]);
    out[1] = make_double2(S[2], S[3]);
    out[2] = make_double2(S[4], S[5]);
    float4 qa, qb;
    store_walk_multipole(c, S, q0, q1, qa, qb);
    cell_record(c, s, lev, kc, kLeaf, rlink, n, make_double4(cx, cy, cz, M), qa, qb,
                kBox ? blo : nullptr, kBox ? bhi : nullptr, ro);
}

// Moments of node c from its n <= 8 children [s, s + n) (one level deeper,
// already done), with the same operations in the same order as cell_moments:
// every child's centre of mass, second moment (and box) is loaded up front in
// one batch, so a node costs one round of dependent loads after its own record.
template <bool kBox>
__device__ __forceinline__ void node_moments(uint32_t c, uint32_t s, uint32_t n, uint32_t f, int lev,
                                             uint32_t k, double4 *__restrict__ c_com,
                                             double *__restrict__ c_S, float4 *__restrict__ q0,
                                             float4 *__restrict__ q1, double2 *__restrict__ box,
                                             const RecOut &ro)
{
    if (n < 1u || n > 8u) return;      // a node has 1..8 children (checked when the tree is built)
    double4 q[8];
    double2 Sk[8][3];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t j = s + min((uint32_t)k, n - 1u);
        q[k] = c_com[j];
        const double2 *p = reinterpret_cast<const double2 *>(c_S + 6 * (int64_t)j);
        Sk[k][0] = p[0];
        Sk[k][1] = p[1];
        Sk[k][2] = p[2];
    }
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if ((uint32_t)k < n) M = M + q[k].w;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if ((uint32_t)k < n) {
            sx = sx + q[k].w * q[k].x;
            sy = sy + q[k].w * q[k].y;
            sz = sz + q[k].w * q[k].z;
        }
    }
    const double cx = sx / M, cy = sy / M, cz = sz / M;
    double S[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if ((uint32_t)k < n) {
            const double ex = q[k].x - cx, ey = q[k].y - cy, ez = q[k].z - cz;
            const double w = q[k].w;
            S[0] += Sk[k][0].x + w * ex * ex; S[1] += Sk[k][0].y + w * ey * ey;
            S[2] += Sk[k][1].x + w * ez * ez; S[3] += Sk[k][1].y + w * ex * ey;
            S[4] += Sk[k][2].x + w * ex * ez; S[5] += Sk[k][2].y + w * ey * ez;
        }
    }
    c_com[c] = make_double4(cx, cy, cz, M);
    double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (kBox) {
        // the union of the children's boxes (refits only: a second round of
        // loads keeps the registers of the common path free)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            // lo x, y; lo z, hi x; hi y, z (repeated members change no min or max)
            const double2 *bp = box + 3 * (int64_t)(s + min((uint32_t)k, n - 1u));
            const double2 b0 = bp[0], b1 = bp[1], b2 = bp[2];
            blo[0] = fmin(blo[0], b0.x); blo[1] = fmin(blo[1], b0.y);
            blo[2] = fmin(blo[2], b1.x); bhi[0] = fmax(bhi[0], b1.y);
            bhi[1] = fmax(bhi[1], b2.x); bhi[2] = fmax(bhi[2], b2.y);
        }
        double2 *b = box + 3 * (int64_t)c;
        b[0] = make_double2(blo[0], blo[1]);
        b[1] = make_double2(blo[2], bhi[0]);
        b[2] = make_double2(bhi[1], bhi[2]);
    }
    double2 *out = reinterpret_cast<double2 *>(c_S + 6 * (int64_t)c);
    out[0] = make_double2(S[0], S[1]);
    out[1] = make_double2(S[2], S[3]);
    out[2] = make_double2(S[4], S[5]);
    float4 qa, qb;
    store_walk_multipole(c, S, q0, q1, qa, qb);
    cell_record(c, f, lev, k, false, s, n, make_double4(cx, cy, cz, M), qa, qb, kBox ? blo : nullptr,
                kBox ? bhi : nullptr, ro);
}

// kLeaves: every leaf of the tree (any level); otherwise the nodes of one level.
// kBox: also the cells' tight boxes (refits).
template <bool kLeaves, bool kBox>
__global__ void __launch_bounds__(kBlock)
moments_kernel(int level, const DevMisc *__restrict__ m, const uint8_t *__restrict__ c_leaf,
               const uint32_t *__restrict__ c_first, const uint32_t *__restrict__ c_count,
               const uint32_t *__restrict__ c_child, const uint32_t *__restrict__ c_nchild,
               const double4 *__restrict__ p4, double4 *__restrict__ c_com,
               double *__restrict__ c_S, float4 *__restrict__ q0, float4 *__restrict__ q1,
               double2 *__restrict__ box, RecOut ro)
{
    const uint32_t begin = kLeaves ? 0u : m->level_offset[level];
    const uint32_t count = kLeaves ? m->ncells : m->level_count[level];
    for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < count; t += gridDim.x * kBlock) {
        const uint32_t c = begin + t;
        const bool leaf = c_leaf[c] != 0;
        if (kLeaves) {
            if (leaf)
                cell_moments<true, kBox>(c, c_first, c_count, c_child, c_nchild, p4, c_com, c_S,
                                         q0, q1, box, ro);
        } else {
            // the node's own record, loaded with its leaf flag in one round
            const uint32_t ch = c_child[c], nc = c_nchild[c], f = c_first[c], k = ro.c_cl[c];
            const int lev = ro.c_level[c];
            if (!leaf) node_moments<kBox>(c, ch, nc, f, lev, k, c_com, c_S, q0, q1, box, ro);
        }
    }
}

// The nodes of levels hi down to lo in one workgroup of kThreads, a barrier
// between levels: for the levels below the tree's expected depth, which normally
// hold no cells, and for the small levels next to the root, where a launch per
// level would cost more than the work.
constexpr int kLevelsBlock = 256;
constexpr int kTopBlock = 512;
constexpr uint32_t kTopCells = 512;     // top levels of at most this many cells share a launch

template <bool kBox, int kThreads>
__global__ void __launch_bounds__(kThreads)
moments_levels_kernel(int hi, int lo, const DevMisc *__restrict__ m,
                      const uint8_t *__restrict__ c_leaf, const uint32_t *__restrict__ c_first,
                      const uint32_t *__restrict__ c_count, const uint32_t *__restrict__ c_child,
                      const uint32_t *__restrict__ c_nchild, const double4 *__restrict__ p4,
                      double4 *__restrict__ c_com, double *__restrict__ c_S,
                      float4 *__restrict__ q0, float4 *__restrict__ q1, double2 *__restrict__ box,
                      RecOut ro)
{
    for (int level = hi; level >= lo; --level) {
        const uint32_t begin = m->level_offset[level];
        const uint32_t count = m->level_count[level];
        for (uint32_t t = threadIdx.x; t < count; t += kThreads) {
            const uint32_t c = begin + t;
            const uint32_t ch = c_child[c], nc = c_nchild[c], f = c_first[c], k = ro.c_cl[c];
            if (c_leaf[c] == 0)
                node_moments<kBox>(c, ch, nc, f, level, k, c_com, c_S, q0, q1, box, ro);
        }
        __syncthreads();
    }
}

// The opening radii and walk records of every cell from its stored moments (the
// moments kernels write them as they go; this pass serves force calls whose
// theta or opening test differ from those the moments saw).  See cell_record.
__global__ void __launch_bounds__(kBlock)
rcrit_kernel(DevMisc *__restrict__ m, RecOut ro, const uint32_t *__restrict__ c_first,
             const uint32_t *__restrict__ c_count, const uint32_t *__restrict__ c_child,
             const uint32_t *__restrict__ c_nchild, const uint8_t *__restrict__ c_leaf,
             const double4 *__restrict__ c_com, const float4 *__restrict__ q0,
             const float4 *__restrict__ q1, const double2 *__restrict__ box)
{
    const uint32_t ncells = m->ncells;
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < ncells; c += gridDim.x * kBlock) {
        const uint32_t f = c_first[c];
        const bool leaf = c_leaf[c] != 0;
        double blo[3], bhi[3];
        if (box) {
            const double2 b0 = box[3 * (int64_t)c], b1 = box[3 * (int64_t)c + 1],
                          b2 = box[3 * (int64_t)c + 2];
            blo[0] = b0.x; blo[1] = b0.y; blo[2] = b1.x;
            bhi[0] = b1.y; bhi[1] = b2.x; bhi[2] = b2.y;
        }
        cell_record(c, f, ro.c_level[c], ro.c_cl[c], leaf, leaf ? f : c_child[c],
                    leaf ? c_count[c] : c_nchild[c], c_com[c], q0[c], q1[c], box ? blo : nullptr,
                    box ? bhi : nullptr, ro);
    }
}

}  // namespace

// ---------------------------------------------------------------------------

hipError_t launch_cluster_ids(bh_ctx *c)
{
    hipLaunchKernelGGL(cluster_ids_kernel, dim3((unsigned)c->nchunks), dim3(kBlock), 0, c->stream,
                       c->chunks, c->pcl);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_domain(bh_ctx *c, const double *pos_aos)
{
    if (!pos_aos && c->box_ready) {
        // the partials of the held positions came with the step's drift
        c->box_ready = false;
    } else if (pos_aos)
        hipLaunchKernelGGL(bbox_kernel<AosSrc>, dim3((unsigned)c->nchunks), dim3(kBlock), 0,
                           c->stream, AosSrc{pos_aos}, c->chunks, c->bb_part, c->misc);
    else
        hipLaunchKernelGGL(bbox_kernel<P4Src>, dim3((unsigned)c->nchunks), dim3(kBlock), 0,
                           c->stream, P4Src{c->p4[c->cur]}, c->chunks, c->bb_part, c->misc);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(domain_kernel, dim3((unsigned)c->K), dim3(kBlock), 0, c->stream, c->bb_part,
                       c->clus, c->dom);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_keys(bh_ctx *c, const double *pos_aos)
{
    if (pos_aos)
        hipLaunchKernelGGL(keys_kernel<AosSrc>, dim3((unsigned)c->nchunks), dim3(kBlock), 0,
                           c->stream, AosSrc{pos_aos}, c->chunks, c->dom, nullptr, (uint32_t)c->n,
                           c->key[0], c->val[0], 0u, nullptr, 0u, 0u, c->misc);
    else {
        // a rebuild: held-order pairs and the candidate splitters for its bucket
        // sort, at a fixed stride (or caller-order pairs for the radix sort)
        const uint32_t held = rebuild_buckets(c) > 0 ? 1u : 0u;
        const uint32_t ncand = (uint32_t)rebuild_candidates(c);
        const uint32_t cstride = ncand ? (uint32_t)(c->n / (ncand + 1)) : 0u;
        hipLaunchKernelGGL(keys_kernel<P4Src>, dim3((unsigned)c->nchunks), dim3(kBlock), 0,
                           c->stream, P4Src{c->p4[c->cur]}, c->chunks, c->dom, c->pid[c->cur],
                           (uint32_t)c->n, c->key[0], c->val[0], held, c->splt + kRadix, ncand,
                           cstride, c->misc);
    }
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_reorder_from_caller(bh_ctx *c, const double *pos_aos, const double *mass,
                                      const double *vel, const uint32_t *perm)
{
    hipLaunchKernelGGL(reorder_from_caller_kernel, dim3(grid_for(c->n, kBlock)), dim3(kBlock), 0,
                       c->stream, pos_aos, mass, vel, perm, c->n, c->p4[c->cur], c->v4[c->cur],
                       c->pid[c->cur], c->misc);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_reorder(bh_ctx *c, const uint32_t *perm)
{
    const int s = c->cur, d = c->cur ^ 1;
    hipLaunchKernelGGL(reorder_kernel, dim3(grid_for(c->n, kBlock)), dim3(kBlock), 0, c->stream,
                       c->p4[s], c->v4[s], c->pid[s], perm, c->n, c->p4[d], c->v4[d], c->pid[d],
                       c->misc);
    BH_LAUNCH_CHECK();
    c->cur = d;
    return hipSuccess;
}

hipError_t launch_tree(bh_ctx *c)
{
    const int64_t n = c->n;
    const int nblk = grid_for(n, kTreeTile);
    uint32_t *blk = c->blk;                       // [kLevels + 1][nblk]
    uint32_t *tot = c->blk + (int64_t)(kLevels + 1) * nblk;
    const int H = c->max_nleaf;
    const size_t lds = (size_t)((kTreeTile + 2 * H + 15) & ~15) + (size_t)kTreeTile * H;
    hipLaunchKernelGGL(split_leaf_kernel, dim3(nblk), dim3(kTreeTile), lds, c->stream, c->key[0],
                       c->pcl, n, H, c->clus, c->split, c->lam, c->gflag, blk, nblk, c->misc);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(scan_levels_kernel, dim3(kLevels + 1), dim3(kScanLevelsBlock), 0, c->stream,
                       blk, nblk, tot,
                       c->misc, c->cap_c);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(emit_cells_kernel, dim3(nblk), dim3(kTreeTile), 0, c->stream, c->split,
                       c->lam, n, blk, nblk, c->misc, c->c_first, c->c_level, c->c_leaf,
                       c->c_parent, c->c_child, c->c_end, c->c_nchild, c->pcl, c->c_cl);
    BH_LAUNCH_CHECK();
    int g = grid_for(c->cap_c, kBlock);
    if (g > kFixedGrid) g = kFixedGrid;
    hipLaunchKernelGGL(cell_finish_kernel, dim3(g), dim3(kBlock), 0, c->stream, c->misc, c->pcl,
                       c->clus, c->c_first, c->c_end, c->c_leaf, c->c_level, c->c_parent,
                       c->c_child, c->c_count, c->c_nchild, c->gflag, n);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_groups(bh_ctx *c)
{
    return compact_flags(c, c->gflag, c->n, c->g_first, &c->misc->ngroups);
}

hipError_t launch_group_boxes(bh_ctx *c)
{
    int g = grid_for(c->n, kBlock / 16);
    if (g > kFixedGrid) g = kFixedGrid;
    hipLaunchKernelGGL(group_boxes_kernel, dim3(g), dim3(kBlock), 0, c->stream, c->g_first, c->misc,
                       c->n, c->p4[c->cur], c->pcl, c->g_count, c->g_centre, c->g_half);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

template <bool kBox>
hipError_t moments_launches(bh_ctx *c, double2 *box)
{
    int g = grid_for(c->cap_c, kBlock);
    if (g > kFixedGrid) g = kFixedGrid;
    // every cell's opening radius and walk record are written with its moments
    const RecOut ro{c->clus, c->dom, c->c_level, c->c_cl, c->key[0], c->c_rcrit2, c->c_rec, c->c_geo};
    // every leaf, whatever its level, from its particles
    hipLaunchKernelGGL((moments_kernel<true, kBox>), dim3(g), dim3(kBlock), 0, c->stream, 0, c->misc,
                       c->c_leaf, c->c_first, c->c_count, c->c_child, c->c_nchild, c->p4[c->cur],
                       c->c_com, c->c_S, c->c_q0, c->c_q1, box, ro);
    BH_LAUNCH_CHECK();
    // nodes from their children, deepest level first (level 20 holds only leaves).
    // The level sizes are known on the device only; the host takes those seen at
    // its last synchronisation as hints: levels below the hinted depth (normally
    // empty; a tree that grew deeper since) share one workgroup, and so do the
    // levels next to the root while each holds at most kTopCells cells; every
    // other level gets a launch of its own with a grid sized for twice its hinted
    // count.  The kernels read the true counts and loop over them, so any tree is
    // handled whatever the hints.
    const DevMisc &hint = *c->misc_h;
    const int deep = hint.depth ? std::min(kMaxLevel - 1, (int)hint.depth) : kMaxLevel - 1;
    if (deep < kMaxLevel - 1) {
        hipLaunchKernelGGL((moments_levels_kernel<kBox, kLevelsBlock>), dim3(1), dim3(kLevelsBlock),
                           0, c->stream, kMaxLevel - 1, deep + 1, c->misc, c->c_leaf, c->c_first,
                           c->c_count, c->c_child, c->c_nchild, c->p4[c->cur], c->c_com, c->c_S,
                           c->c_q0, c->c_q1, box, ro);
        BH_LAUNCH_CHECK();
    }
    // the small levels next to the root: 0 .. top
    int top = -1;
    if (hint.depth)
        while (top < deep && hint.level_count[top + 1] <= kTopCells) ++top;
    for (int lev = deep; lev > top; --lev) {
        int gl = g;
        if (hint.depth && hint.level_count[lev])
            gl = (int)std::min<int64_t>(g, grid_for(2 * (int64_t)hint.level_count[lev], kBlock));
        hipLaunchKernelGGL((moments_kernel<false, kBox>), dim3(gl), dim3(kBlock), 0, c->stream, lev,
                           c->misc, c->c_leaf, c->c_first, c->c_count, c->c_child, c->c_nchild,
                           c->p4[c->cur], c->c_com, c->c_S, c->c_q0, c->c_q1, box, ro);
        BH_LAUNCH_CHECK();
    }
    if (top >= 0) {
        hipLaunchKernelGGL((moments_levels_kernel<kBox, kTopBlock>), dim3(1), dim3(kTopBlock), 0,
                           c->stream, top, 0, c->misc, c->c_leaf, c->c_first, c->c_count,
                           c->c_child, c->c_nchild, c->p4[c->cur], c->c_com, c->c_S, c->c_q0,
                           c->c_q1, box, ro);
        BH_LAUNCH_CHECK();
    }
    c->rec_fresh = true;
    return hipSuccess;
}

hipError_t launch_moments(bh_ctx *c, bool boxes)
{
    if (boxes) return moments_launches<true>(c, reinterpret_cast<double2 *>(c->c_box));
    return moments_launches<false>(c, nullptr);
}

hipError_t launch_rcrit(bh_ctx *c)
{
    // the moments pass wrote the records with the current table already
    if (c->rec_fresh) return hipSuccess;
    int g = grid_for(c->cap_c, kBlock);
    if (g > kFixedGrid) g = kFixedGrid;
    const RecOut ro{c->clus, c->dom, c->c_level, c->c_cl, c->key[0], c->c_rcrit2, c->c_rec, c->c_geo};
    hipLaunchKernelGGL(rcrit_kernel, dim3(g), dim3(kBlock), 0, c->stream, c->misc, ro, c->c_first,
                       c->c_count, c->c_child, c->c_nchild, c->c_leaf, c->c_com, c->c_q0, c->c_q1,
                       c->refitted ? reinterpret_cast<const double2 *>(c->c_box) : nullptr);
    BH_LAUNCH_CHECK();
    c->rec_fresh = true;
    return hipSuccess;
}

}  // namespace bh
