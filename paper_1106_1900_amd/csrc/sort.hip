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

namespace bh {
namespace {

// digit of an element: from its key, or (cl != NULL) from the cluster of the
// position it came from
__device__ __forceinline__ uint32_t digit_of(uint64_t k, uint32_t v, const uint32_t *cl, int shift)
{
    return cl ? ((cl[v] >> shift) & (kRadix - 1)) : ((uint32_t)(k >> shift) & (kRadix - 1));
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

__global__ void __launch_bounds__(kSortThreads)
hist_kernel(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
            const uint32_t *__restrict__ cl, int64_t n, int shift, uint32_t *__restrict__ hist,
            int nblk)
{
    __shared__ uint32_t cnt[kRadix];
    const int t = threadIdx.x;
    cnt[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int64_t i = base + (int64_t)k * kSortThreads + t;
        if (i < n) atomicAdd(&cnt[digit_of(keys[i], cl ? vals[i] : 0u, cl, shift)], 1u);
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
               const uint32_t *__restrict__ cl, int64_t n, int shift,
               const uint32_t *__restrict__ hist, const uint32_t *__restrict__ tot, int nblk)
{
    __shared__ uint32_t s_wcnt[kSortThreads / kWave][kRadix];  // per-wave digit counts
    __shared__ uint32_t s_base[kRadix];                         // global digit base
    __shared__ uint32_t s_local[kRadix];                        // block-local digit start
    __shared__ uint32_t s_tmp[4];
    __shared__ uint64_t s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];

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
    __syncthreads();

    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t rank[kSortItems];
    const int wbase = w * kWave * kSortItems;  // this wave's contiguous sub-tile
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
        int p = wbase + k * kWave + l;
        bool valid = p < tile_n;
        key[k] = valid ? kin[base + p] : 0ull;
        val[k] = valid ? vin[base + p] : 0u;
        uint32_t d = valid ? digit_of(key[k], val[k], cl, shift) : 0u;
        unsigned long long peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            bool bit = (d >> b) & 1u;
            unsigned long long m = ballot(bit);
            peers &= bit ? m : ~m;
        }
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
            uint32_t d = digit_of(key[k], val[k], cl, shift);
            uint32_t lp = s_local[d] + s_wcnt[w][d] + rank[k];
            s_key[lp] = key[k];
            s_val[lp] = val[k];
        }
    }
    __syncthreads();

    for (int p = t; p < tile_n; p += kSortThreads) {
        uint64_t k = s_key[p];
        uint32_t d = digit_of(k, s_val[p], cl, shift);
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

__global__ void __launch_bounds__(256)
scan_partials_kernel(uint32_t *__restrict__ part, int nblk, uint32_t *__restrict__ total)
{
    __shared__ uint32_t s_tmp[4];
    uint32_t run = 0;
    for (int b0 = 0; b0 < nblk; b0 += 256) {
        int b = b0 + threadIdx.x;
        uint32_t v = b < nblk ? part[b] : 0u;
        uint32_t sum;
        uint32_t ex = block_excl_scan_256(v, s_tmp, &sum);
        if (b < nblk) part[b] = run + ex;
        run += sum;
    }
    if (threadIdx.x == 0 && total) *total = run;
}

// Writes the positions of set flags, in order, to idx[0..count).
__global__ void __launch_bounds__(kScanThreads)
compact_down_kernel(const uint8_t *__restrict__ flags, int64_t n, const uint32_t *__restrict__ part,
                    uint32_t *__restrict__ idx)
{
    __shared__ uint32_t s_tmp[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? (uint32_t)(flags[base + k] != 0) : 0u;
        s += v[k];
    }
    uint32_t sum;
    uint32_t run = part[blockIdx.x] + block_excl_scan_256(s, s_tmp, &sum);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (v[k]) idx[run++] = (uint32_t)(base + k);
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
                           c->key[src], c->val[src], cl, n, shift, hist, nblk);
        BH_LAUNCH_CHECK();
        hipLaunchKernelGGL(scan_digit_kernel, dim3(kRadix), dim3(256), 0, c->stream, hist, nblk,
                           tot);
        BH_LAUNCH_CHECK();
        hipLaunchKernelGGL(scatter_kernel, dim3(nblk), dim3(kSortThreads), 0, c->stream,
                           c->key[src], c->val[src], c->key[src ^ 1], c->val[src ^ 1], cl, n, shift,
                           hist, tot, nblk);
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

hipError_t compact_flags(bh_ctx *c, const uint8_t *flags, int64_t n, uint32_t *idx,
                         uint32_t *count)
{
    const int nblk = (int)((n + kScanTile - 1) / kScanTile);
    uint32_t *part = c->scan_tmp;
    hipLaunchKernelGGL(scan_reduce_kernel<uint8_t>, dim3(nblk), dim3(kScanThreads), 0, c->stream,
                       flags, n, part);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(256), 0, c->stream, part, nblk, count);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(compact_down_kernel, dim3(nblk), dim3(kScanThreads), 0, c->stream, flags, n,
                       part, idx);
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
