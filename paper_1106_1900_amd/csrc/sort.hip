// sort.hip - scan, compaction and the stable LSD radix sort of (key, index)
// pairs (App. A: count, scan offsets, place; radix sort by stable passes from the
// least significant digit up).
//
// The paper splits one bit per pass; here each pass places an 8-bit digit, which
// is the same stable partition done for 256 buckets at once: 8 passes over the
// 60-bit keys.  For a batch of clusters, further stable passes on the cluster of
// each element follow, so the keys end up sorted within each cluster and the
// clusters keep their places.  Each pass is reduce-then-scan (no inter-block
// waiting):
//   1. hist:    per-block digit counts, stored digit-major;
//   2. scan:    one block per digit scans that digit's counts over blocks;
//   3. scatter: each block ranks its keys stably (wavefront match on the digit
//               bits), stages them in LDS in digit order and writes them out
//               coalesced at digit base + block offset + rank.
#include "bh_internal.h"

#include <algorithm>

namespace bh {
namespace {

// digit of an element: from its key, or (cl != NULL) from the cluster of the
// position it came from
__device__ __forceinline__ uint32_t digit_of(uint64_t k, uint32_t v, const uint32_t *cl, int shift)
{
    return cl ? ((cl[v] >> shift) & (kRadix - 1)) : ((uint32_t)(k >> shift) & (kRadix - 1));
}

// bucket of a key among kRadix - 1 ascending splitters (unused ones are ~0):
// the number of splitters below it, so equal keys share a bucket and buckets
// follow key order
__device__ __forceinline__ uint32_t bucket_of(uint64_t k, const uint64_t *spl)
{
    uint32_t b = 0;
#pragma unroll
    for (uint32_t step = kRadix / 2; step > 0; step >>= 1)
        if (spl[b + step - 1] < k) b += step;
    return b;
}

// The lanes of the wavefront that are valid and hold the same 8-bit digit as
// this lane: one ballot per digit bit, collecting the lanes that differ.
__device__ __forceinline__ unsigned long long match_digit(uint32_t d, bool valid)
{
    const unsigned long long v = ballot(valid);
    uint32_t dlo = ~(uint32_t)v, dhi = ~(uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const uint32_t s = (uint32_t)((int32_t)(d << (31 - b)) >> 31);   // ~0 if bit b is set
        const unsigned long long m = ballot(s != 0u);
        dlo |= (uint32_t)m ^ s;
        dhi |= (uint32_t)(m >> 32) ^ s;
    }
    return ~(((unsigned long long)dhi << 32) | dlo);
}

// OR and AND of a 64-bit value over the wavefront (every lane gets the result)
__device__ __forceinline__ unsigned long long wave_or_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) v |= __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ unsigned long long wave_and_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) v &= __shfl_xor(v, off);
    return v;
}

// Exclusive scan of one value per thread over a 256-thread block.  Returns the
// exclusive prefix; *total receives the block sum (same in every thread).
__device__ uint32_t block_excl_scan_256(uint32_t v, uint32_t *s_tmp, uint32_t *total)
{
    const int t = threadIdx.x, w = t / kWave, l = t % kWave;
    uint32_t inc = wave_incl_scan_add(v);
    if (l == kWave - 1) s_tmp[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t x = s_tmp[i];
        if (i < w) off += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

constexpr int kSplitOver = 4;           // candidate keys per bucket of a rebuild's sort
constexpr int kCand = kRadix * kSplitOver;

// The digit of a pass is a radix digit of the key (or of the element's cluster),
// or, with splitters (spl != NULL: kRadix - 1 ascending keys, unused ones ~0),
// the key's bucket.
__global__ void __launch_bounds__(kSortThreads)
hist_kernel(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
            const uint32_t *__restrict__ cl, const uint64_t *__restrict__ spl, int64_t n,
            int shift, uint32_t *__restrict__ hist, int nblk)
{
    __shared__ uint32_t cnt[kRadix];
    __shared__ uint64_t s_spl[kRadix];
    const int t = threadIdx.x;
    cnt[t] = 0;
    if (spl && t < kRadix - 1) s_spl[t] = spl[t];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int64_t i = base + (int64_t)k * kSortThreads + t;
        if (i < n) {
            const uint64_t key = keys[i];
            const uint32_t d = spl ? bucket_of(key, s_spl)
                                   : digit_of(key, cl ? vals[i] : 0u, cl, shift);
            atomicAdd(&cnt[d], 1u);
        }
    }
    __syncthreads();
    hist[(int64_t)t * nblk + blockIdx.x] = cnt[t];
}

// One block per digit: exclusive scan of hist[d][0..nblk) in place, total -> tot[d].
__global__ void __launch_bounds__(256)
scan_digit_kernel(uint32_t *__restrict__ hist, int nblk, uint32_t *__restrict__ tot)
{
    __shared__ uint32_t s_tmp[4];
    uint32_t *row = hist + (int64_t)blockIdx.x * nblk;
    uint32_t run = 0;
    for (int b0 = 0; b0 < nblk; b0 += 256) {
        int b = b0 + threadIdx.x;
        uint32_t v = b < nblk ? row[b] : 0u;
        uint32_t sum;
        uint32_t ex = block_excl_scan_256(v, s_tmp, &sum);
        if (b < nblk) row[b] = run + ex;
        run += sum;
    }
    if (threadIdx.x == 0) tot[blockIdx.x] = run;
}

__global__ void __launch_bounds__(kSortThreads)
scatter_kernel(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
               uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
               const uint32_t *__restrict__ cl, const uint64_t *__restrict__ spl, int64_t n,
               int shift, const uint32_t *__restrict__ hist,
               const uint32_t *__restrict__ tot, int nblk)
{
    __shared__ uint32_t s_wcnt[kSortThreads / kWave][kRadix];  // per-wave digit counts
    __shared__ uint32_t s_base[kRadix];                         // global digit base
    __shared__ uint32_t s_local[kRadix];                        // block-local digit start
    __shared__ uint32_t s_tmp[4];
    __shared__ uint64_t s_spl[kRadix];
    __shared__ uint64_t s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint8_t s_dig[kSortTile];

    const int t = threadIdx.x, w = t / kWave, l = t % kWave;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int tile_n = (int)((n - base) < kSortTile ? (n - base) : kSortTile);

    for (int d = t; d < kRadix; d += kSortThreads) {
#pragma unroll
        for (int i = 0; i < kSortThreads / kWave; ++i) s_wcnt[i][d] = 0;
    }
    {
        uint32_t sum;
        uint32_t ex = block_excl_scan_256(tot[t], s_tmp, &sum);
        s_base[t] = ex;
    }
    if (spl && t < kRadix - 1) s_spl[t] = spl[t];
    __syncthreads();

    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rank[kSortItems];
    uint32_t dig[kSortItems];
    const int wbase = w * kWave * kSortItems;  // this wave's contiguous sub-tile
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int p = wbase + k * kWave + l;
        bool valid = p < tile_n;
        key[k] = valid ? kin[base + p] : 0ull;
        val[k] = valid ? vin[base + p] : 0u;
        uint32_t d = 0;
        if (valid) d = spl ? bucket_of(key[k], s_spl) : digit_of(key[k], val[k], cl, shift);
        dig[k] = d;
        const unsigned long long peers = match_digit(d, valid);
        uint32_t before = s_wcnt[w][d];
        int r = mask_rank(peers);
        rank[k] = before + (uint32_t)r;
        wave_sync();
        if (valid && r == 0) s_wcnt[w][d] = before + (uint32_t)__popcll(peers);
        wave_sync();
    }
    __syncthreads();

    // wave offsets within the block, block totals, block-local digit starts
    {
        const int d = t;
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < kSortThreads / kWave; ++i) {
            uint32_t c = s_wcnt[i][d];
            s_wcnt[i][d] = run;
            run += c;
        }
        uint32_t sum;
        uint32_t ex = block_excl_scan_256(run, s_tmp, &sum);
        s_local[d] = ex;
    }
    __syncthreads();

#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int p = wbase + k * kWave + l;
        if (p < tile_n) {
            const uint32_t d = dig[k];
            uint32_t lp = s_local[d] + s_wcnt[w][d] + rank[k];
            s_key[lp] = key[k];
            s_val[lp] = val[k];
            s_dig[lp] = (uint8_t)d;
        }
    }
    __syncthreads();

    for (int p = t; p < tile_n; p += kSortThreads) {
        uint64_t k = s_key[p];
        const uint32_t d = s_dig[p];
        int64_t g = (int64_t)s_base[d] + hist[(int64_t)d * nblk + blockIdx.x] + (p - s_local[d]);
        kout[g] = k;
        vout[g] = s_val[p];
    }
}

__global__ void __launch_bounds__(256)
copy_pairs_kernel(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                  uint64_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        kout[i] = kin[i];
        vout[i] = vin[i];
    }
}

// ---------------------------------------------------------------------------
// generic exclusive scan of u32 / compaction of u8 flags

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__global__ void __launch_bounds__(kScanThreads)
scan_reduce_kernel(const T *__restrict__ in, int64_t n, uint32_t *__restrict__ part)
{
    __shared__ uint32_t s_tmp[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += (uint32_t)in[base + k];
    uint32_t sum;
    block_excl_scan_256(s, s_tmp, &sum);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

// Writes the positions of set flags, in order, to idx[0..count).  Each block
// adds up the counts of the blocks before it (part: per-block counts from
// scan_reduce_kernel); the last block also writes the total to *count.
__global__ void __launch_bounds__(kScanThreads)
compact_down_kernel(const uint8_t *__restrict__ flags, int64_t n, const uint32_t *__restrict__ part,
                    uint32_t *__restrict__ idx, uint32_t *__restrict__ count)
{
    __shared__ uint32_t s_tmp[4];
    uint32_t before = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kScanThreads) before += part[b];
    uint32_t sum;
    block_excl_scan_256(before, s_tmp, &sum);
    before = sum;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? (uint32_t)(flags[base + k] != 0) : 0u;
        s += v[k];
    }
    uint32_t run = before + block_excl_scan_256(s, s_tmp, &sum);
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *count = before + sum;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (v[k]) idx[run++] = (uint32_t)(base + k);
    }
}


// ---------------------------------------------------------------------------
// Sort of a rebuild.  The particles are held in the previous build's key order
// and move little between builds, so the new keys taken at regular positions of
// that order (the candidates, written by the keys kernel) split the new key
// range into buckets of similar size.  One stable pass places the pairs by
// bucket (the same three kernels as a radix pass, with the bucket as the digit),
// and one workgroup per bucket sorts it by key, stably.  The pairs arrive in the
// held order (the keys kernel writes them without the scatter to caller order);
// a bucket holding equal keys orders them by caller index, so the result is the
// stable radix sort's of the pairs in caller order, bit for bit.

constexpr int kBucketTarget = 4096;     // mean bucket size the bucket count aims at
constexpr int kBucketCap = 12288;       // largest bucket sorted in LDS
constexpr int kBucketThreads = 1024;
constexpr int kBucketWaves = kBucketThreads / kWave;

// Splitters of nspl + 1 buckets: the ncand candidate keys in sorted order, every
// kSplitOver-th kept, kRadix - 1 values with the unused ones ~0.  Each workgroup
// ranks kSplitOver candidates against all of them (ties by index: ranks are a
// permutation) and the candidate of rank (b + 1) kSplitOver - 1 becomes splitter
// b; the grid has kRadix workgroups.
__global__ void __launch_bounds__(kCand)
splitter_kernel(const uint64_t *__restrict__ cand, int ncand, int nspl, uint64_t *__restrict__ spl)
{
    __shared__ uint32_t s_cnt[kSplitOver][kCand / kWave];
    const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
    const uint64_t mine = t < ncand ? cand[t] : 0ull;
#pragma unroll
    for (int q = 0; q < kSplitOver; ++q) {
        const int c = blockIdx.x * kSplitOver + q;      // the candidate ranked
        uint32_t below = 0;
        if (c < ncand && t < ncand) {
            const uint64_t v = cand[c];
            below = (mine < v || (mine == v && t < c)) ? 1u : 0u;
        }
        below = wave_sum_u32(below);
        if (lane == 0) s_cnt[q][w] = below;
    }
    __syncthreads();
    if (t < kSplitOver) {
        const int c = blockIdx.x * kSplitOver + t;
        if (c < ncand) {
            uint32_t r = 0;
            for (int q = 0; q < kCand / kWave; ++q) r += s_cnt[t][q];
            if ((r + 1) % kSplitOver == 0 && (int)(r / kSplitOver) < nspl)
                spl[r / kSplitOver] = cand[c];
        }
    }
    if (blockIdx.x == 0)
        for (int b = nspl + t; b < kRadix - 1; b += kCand) spl[b] = ~0ull;
}

// One workgroup per bucket: the bucket's pairs (k1, v1)[lo, lo + L) are sorted
// stably by key into (k0, v0)[lo, lo + L).  With pid == NULL the pairs arrive in
// caller order; otherwise in the held order (value = held position, pid[value] =
// caller index), and equal keys are put in caller order explicitly.  Up to
// kBucketCap pairs are sorted in LDS by stable 8-bit passes (keys and positions
// move, values are gathered at the end), skipping the digits every key of the
// bucket shares; a bucket holding equal keys is then sorted again, by caller index
// first and by key after it.  A larger bucket (many equal or clustered keys) is
// sorted by the workgroup with the same passes through (k0, v0) and back.
__global__ void __launch_bounds__(kBucketThreads)
bucket_sort_kernel(uint64_t *__restrict__ k1, uint32_t *__restrict__ v1, uint64_t *__restrict__ k0,
                   uint32_t *__restrict__ v0, const uint32_t *__restrict__ tot,
                   const uint32_t *__restrict__ pid)
{
    constexpr int kItems = kBucketCap / kBucketThreads;   // most pairs per thread in LDS
    __shared__ uint64_t s_k[kBucketCap];
    __shared__ uint16_t s_x[kBucketCap];
    __shared__ uint32_t s_wcnt[kBucketWaves][kRadix];
    __shared__ uint32_t s_wcnt2[kBucketWaves][kRadix];     // the next LDS pass's counts
    __shared__ uint32_t s_off[kRadix];
    __shared__ uint32_t s_ctot[kRadix];
    __shared__ uint32_t s_tmp[kBucketWaves];
    __shared__ uint32_t s_lo;
    __shared__ unsigned long long s_or, s_and;
    const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
    const int b = blockIdx.x;
    if (w == 0) {       // the bucket's first position: the sizes of the buckets before it
        uint32_t x = 0;
        for (int d = lane; d < b; d += kWave) x += tot[d];
        x = wave_sum_u32(x);
        if (lane == 0) s_lo = x;
    }
    __syncthreads();
    const int64_t lo = s_lo;
    const uint32_t L = tot[b];

    if (L <= (uint32_t)kBucketCap) {
        const int items = (int)((L + kBucketThreads - 1) / kBucketThreads);
        const uint32_t sub = (uint32_t)items * kWave;      // a wavefront's positions
        uint32_t(*cur)[kRadix] = s_wcnt;       // counts of a pass (zero at its start)
        uint32_t(*nxt)[kRadix] = s_wcnt2;      // cleared during a pass for the next one
        // s_k[i] = v[j] for positions i = j kBucketThreads + t < L, s_x[i] = i, with
        // every load of the thread in flight at once; returns the bits in which
        // the values differ
        auto load = [&](const uint64_t(&v)[kItems]) -> uint64_t {
            __syncthreads();        // earlier readers of s_k, s_x, s_or and s_and are done
            unsigned long long o = 0ull, a = ~0ull;
#pragma unroll
            for (int j = 0; j < kItems; ++j) {
                const uint32_t i = (uint32_t)(j * kBucketThreads + t);
                if (i < L) {
                    s_k[i] = v[j];
                    s_x[i] = (uint16_t)i;
                    o |= v[j];
                    a &= v[j];
                }
            }
            o = wave_or_u64(o);
            a = wave_and_u64(a);
            if (t == 0) {
                s_or = 0ull;
                s_and = ~0ull;
            }
            for (int q = t; q < kBucketWaves * kRadix; q += kBucketThreads) (&cur[0][0])[q] = 0;
            __syncthreads();
            if (lane == 0) {
                atomicOr(&s_or, o);
                atomicAnd(&s_and, a);
            }
            __syncthreads();
            return s_or ^ s_and;
        };
        // stable 8-bit passes over the bytes of s_k in which vary has bits
        auto passes = [&](uint64_t vary) {
            for (int pass = 0; pass < 8; ++pass) {
                const int shift = pass * kRadixBits;
                if (((vary >> shift) & (kRadix - 1)) == 0) continue;    // one digit: order kept
                // thread (w, lane) takes positions w sub + j kWave + lane: position
                // order is (wavefront, j, lane) order, which the ranks below keep
                uint64_t key[kItems];
                uint32_t idx[kItems], rank[kItems], dg[kItems];
#pragma unroll
                for (int j = 0; j < kItems; ++j) {
                    if (j < items) {    // uniform
                        const uint32_t p = w * sub + (uint32_t)(j * kWave + lane);
                        const bool valid = p < L;
                        key[j] = valid ? s_k[p] : 0ull;
                        idx[j] = valid ? s_x[p] : 0u;
                        const uint32_t d = (uint32_t)(key[j] >> shift) & (kRadix - 1);
                        dg[j] = d;
                        const unsigned long long peers = match_digit(d, valid);
                        const int r = mask_rank(peers);
                        const uint32_t before = j == 0 ? 0u : cur[w][d];
                        rank[j] = before + (uint32_t)r;
                        wave_sync();
                        if (valid && r == 0) cur[w][d] = before + (uint32_t)__popcll(peers);
                        wave_sync();
                    }
                }
                for (int q = t; q < kBucketWaves * kRadix; q += kBucketThreads) (&nxt[0][0])[q] = 0;
                __syncthreads();
                uint32_t cnt = 0, inc = 0;
                if (t < kRadix) {   // wavefronts before each one, per digit; digit totals
                    uint32_t x[kBucketWaves];
#pragma unroll
                    for (int q = 0; q < kBucketWaves; ++q) x[q] = cur[q][t];
                    uint32_t run = 0;
#pragma unroll
                    for (int q = 0; q < kBucketWaves; ++q) {
                        cur[q][t] = run;
                        run += x[q];
                    }
                    cnt = run;
                    inc = wave_incl_scan_add(cnt);
                    if (lane == kWave - 1) s_tmp[w] = inc;
                }
                __syncthreads();
                if (t < kRadix) {
                    uint32_t before = 0;
                    for (int q = 0; q < w; ++q) before += s_tmp[q];
                    s_off[t] = before + inc - cnt;    // first position of digit t
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < kItems; ++j) {
                    const uint32_t p = w * sub + (uint32_t)(j * kWave + lane);
                    if (j < items && p < L) {
                        const uint32_t d = dg[j];
                        const uint32_t np = s_off[d] + cur[w][d] + rank[j];
                        s_k[np] = key[j];
                        s_x[np] = (uint16_t)idx[j];
                    }
                }
                __syncthreads();
                uint32_t(*tmp)[kRadix] = cur;
                cur = nxt;
                nxt = tmp;
            }
        };

        uint64_t v[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t i = (uint32_t)(j * kBucketThreads + t);
            v[j] = i < L ? k1[lo + i] : 0ull;
        }
        passes(load(v));
        if (pid) {
            // equal keys, if any, are still in the held order
            bool tie = false;
            for (uint32_t i = t; i + 1 < L; i += kBucketThreads) tie |= s_k[i] == s_k[i + 1];
            if (__syncthreads_or(tie)) {
#pragma unroll
                for (int j = 0; j < kItems; ++j) {
                    const uint32_t i = (uint32_t)(j * kBucketThreads + t);
                    v[j] = i < L ? (uint64_t)pid[v1[lo + i]] : 0ull;
                }
                passes(load(v));        // by caller index
#pragma unroll
                for (int j = 0; j < kItems; ++j) {
                    const uint32_t i = (uint32_t)(j * kBucketThreads + t);
                    v[j] = i < L ? k1[lo + s_x[i]] : 0ull;
                }
                uint16_t x[kItems];
#pragma unroll
                for (int j = 0; j < kItems; ++j) {
                    const uint32_t i = (uint32_t)(j * kBucketThreads + t);
                    x[j] = i < L ? s_x[i] : 0;
                }
                const uint64_t vary = load(v);      // keys in caller-index order ...
#pragma unroll
                for (int j = 0; j < kItems; ++j) {  // ... with their own positions
                    const uint32_t i = (uint32_t)(j * kBucketThreads + t);
                    if (i < L) s_x[i] = x[j];
                }
                __syncthreads();
                passes(vary);           // then by key
            }
        }
        // every value gather of a thread in flight at once
        uint32_t vout[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t i = (uint32_t)(j * kBucketThreads + t);
            vout[j] = i < L ? v1[lo + s_x[i]] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t i = (uint32_t)(j * kBucketThreads + t);
            if (i < L) {
                k0[lo + i] = s_k[i];
                v0[lo + i] = vout[j];
            }
        }
        return;
    }

    // Large bucket: stable passes through device memory, (k1, v1) -> (k0, v0) ->
    // (k1, v1) ...: with pid, three passes on the caller index (below 2^24) first,
    // then eight on the 60-bit keys; the result is copied to (k0, v0) if it ends in
    // (k1, v1).
    uint64_t *ks = k1, *kd = k0;
    uint32_t *vs = v1, *vd = v0;
    const int npid = pid ? 3 : 0;
    for (int pass = 0; pass < npid + 8; ++pass) {
        const bool by_pid = pass < npid;
        const int shift = (by_pid ? pass : pass - npid) * kRadixBits;
        auto digit = [&](uint64_t key, uint32_t val) -> uint32_t {
            return by_pid ? (pid[val] >> shift) & (kRadix - 1)
                          : (uint32_t)(key >> shift) & (kRadix - 1);
        };
        if (t < kRadix) s_off[t] = 0;
        __syncthreads();
        for (uint32_t i = t; i < L; i += kBucketThreads)
            atomicAdd(&s_off[digit(ks[lo + i], vs[lo + i])], 1u);
        __syncthreads();
        uint32_t cnt = 0, inc = 0;
        if (t < kRadix) {
            cnt = s_off[t];
            inc = wave_incl_scan_add(cnt);
            if (lane == kWave - 1) s_tmp[w] = inc;
        }
        __syncthreads();
        if (t < kRadix) {
            uint32_t before = 0;
            for (int q = 0; q < w; ++q) before += s_tmp[q];
            s_off[t] = before + inc - cnt;        // first output slot of digit t
        }
        __syncthreads();
        for (uint32_t c0 = 0; c0 < L; c0 += kBucketThreads) {
            const uint32_t i = c0 + t;
            const bool valid = i < L;
            const uint64_t key = valid ? ks[lo + i] : 0ull;
            const uint32_t val = valid ? vs[lo + i] : 0u;
            const uint32_t d = valid ? digit(key, val) : 0u;
            const unsigned long long peers = match_digit(d, valid);
            const int r = mask_rank(peers);
            for (int q = t; q < kBucketWaves * kRadix; q += kBucketThreads) (&s_wcnt[0][0])[q] = 0;
            __syncthreads();
            if (valid && r == 0) s_wcnt[w][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            if (t < kRadix) {   // wavefronts before each one, per digit
                uint32_t x[kBucketWaves];
#pragma unroll
                for (int q = 0; q < kBucketWaves; ++q) x[q] = s_wcnt[q][t];
                uint32_t run = 0;
#pragma unroll
                for (int q = 0; q < kBucketWaves; ++q) {
                    s_wcnt[q][t] = run;
                    run += x[q];
                }
                s_ctot[t] = run;
            }
            __syncthreads();
            if (valid) {
                const uint32_t pos = s_off[d] + s_wcnt[w][d] + (uint32_t)r;
                kd[lo + pos] = key;
                vd[lo + pos] = val;
            }
            __syncthreads();
            if (t < kRadix) s_off[t] += s_ctot[t];
            __syncthreads();
        }
        uint64_t *kt = ks;
        ks = kd;
        kd = kt;
        uint32_t *vt = vs;
        vs = vd;
        vd = vt;
    }
    if (ks != k0) {
        for (uint32_t i = t; i < L; i += kBucketThreads) {
            k0[lo + i] = ks[lo + i];
            v0[lo + i] = vs[lo + i];
        }
    }
}

}  // namespace

hipError_t radix_sort_pairs(bh_ctx *c)
{
    const int64_t n = c->n;
    const int nblk = (int)((n + kSortTile - 1) / kSortTile);
    uint32_t *hist = c->blk;                 // kRadix * nblk
    uint32_t *tot = c->blk + (int64_t)kRadix * nblk;
    int cluster_passes = 0;
    for (int64_t k = c->K - 1; k > 0; k >>= kRadixBits) ++cluster_passes;
    const int passes = 8 + cluster_passes;
    int src = 0;
    for (int pass = 0; pass < passes; ++pass) {
        const bool by_cluster = pass >= 8;
        const int shift = by_cluster ? (pass - 8) * kRadixBits : pass * kRadixBits;
        const uint32_t *cl = by_cluster ? c->pcl : nullptr;
        hipLaunchKernelGGL(hist_kernel, dim3(nblk), dim3(kSortThreads), 0, c->stream,
                           c->key[src], c->val[src], cl, nullptr, n, shift, hist, nblk);
        BH_LAUNCH_CHECK();
        hipLaunchKernelGGL(scan_digit_kernel, dim3(kRadix), dim3(256), 0, c->stream, hist, nblk,
                           tot);
        BH_LAUNCH_CHECK();
        hipLaunchKernelGGL(scatter_kernel, dim3(nblk), dim3(kSortThreads), 0, c->stream,
                           c->key[src], c->val[src], c->key[src ^ 1], c->val[src ^ 1], cl, nullptr,
                           n, shift, hist, tot, nblk);
        BH_LAUNCH_CHECK();
        src ^= 1;
    }
    if (src != 0) {
        // keep the result in buffer 0 whatever the number of passes
        hipLaunchKernelGGL(copy_pairs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                           c->stream, c->key[1], c->val[1], c->key[0], c->val[0], n);
        BH_LAUNCH_CHECK();
    }
    return hipSuccess;
}

hipError_t rebuild_sort_pairs(bh_ctx *c)
{
    const int64_t n = c->n;
    if (!rebuild_buckets(c)) return radix_sort_pairs(c);
    const int nb = rebuild_buckets(c);
    const int nblk = (int)((n + kSortTile - 1) / kSortTile);
    uint32_t *hist = c->blk;
    uint32_t *tot = c->blk + (int64_t)kRadix * nblk;
    const uint64_t *cand = c->splt + kRadix;    // written by the keys kernel
    hipLaunchKernelGGL(splitter_kernel, dim3(kRadix), dim3(kCand), 0, c->stream, cand,
                       rebuild_candidates(c), nb - 1, c->splt);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(hist_kernel, dim3(nblk), dim3(kSortThreads), 0, c->stream, c->key[0],
                       c->val[0], nullptr, c->splt, n, 0, hist, nblk);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(scan_digit_kernel, dim3(kRadix), dim3(256), 0, c->stream, hist, nblk, tot);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(scatter_kernel, dim3(nblk), dim3(kSortThreads), 0, c->stream, c->key[0],
                       c->val[0], c->key[1], c->val[1], nullptr, c->splt, n, 0, hist, tot, nblk);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(bucket_sort_kernel, dim3(nb), dim3(kBucketThreads), 0, c->stream, c->key[1],
                       c->val[1], c->key[0], c->val[0], tot, c->pid[c->cur]);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

int rebuild_buckets(const bh_ctx *c)
{
    // one cluster, and few enough particles for at most kRadix buckets
    if (c->K != 1 || c->n < 2 || c->n > (int64_t)kRadix * kBucketTarget) return 0;
    return (int)((c->n + kBucketTarget - 1) / kBucketTarget);
}

int rebuild_candidates(const bh_ctx *c)
{
    const int nb = rebuild_buckets(c);
    return nb > 1 ? nb * kSplitOver - 1 : 0;
}

hipError_t compact_flags(bh_ctx *c, const uint8_t *flags, int64_t n, uint32_t *idx,
                         uint32_t *count)
{
    // one block at least, so that the count is written for n = 0 too
    const int nblk = std::max(1, (int)((n + kScanTile - 1) / kScanTile));
    uint32_t *part = c->scan_tmp;
    hipLaunchKernelGGL(scan_reduce_kernel<uint8_t>, dim3(nblk), dim3(kScanThreads), 0, c->stream,
                       flags, n, part);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(compact_down_kernel, dim3(nblk), dim3(kScanThreads), 0, c->stream, flags, n,
                       part, idx, count);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

int64_t sort_blk_words(int64_t n)
{
    const int64_t nblk = (n + kSortTile - 1) / kSortTile;
    return (int64_t)kRadix * nblk + kRadix;
}

int64_t scan_tmp_words(int64_t n)
{
    return (n + kScanTile - 1) / kScanTile + 1;
}

}  // namespace bh
