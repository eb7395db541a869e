// integrate.hip - leapfrog kicks and drifts (Sect. 3.1) and the float64 energy
// and momentum sums used for the energy error of Eq. (3); plus the copies
// between the caller's order and the library's sorted order.
#include "bh_internal.h"

#pragma clang fp contract(off)

namespace bh {
namespace {

constexpr int kBlock = 256;
static_assert(kBlock == kChunkThreads, "per-chunk kernels share box_partial");

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// The kick-drift of a leapfrog step, one workgroup per chunk (each chunk in one
// cluster), with the chunk's bounding-box partials of the drifted positions for
// the rebuild that follows (the partials and error bit of bbox_kernel).
__global__ void __launch_bounds__(kBlock)
kick_drift_box_kernel(const Chunk *__restrict__ chunks, const DevCluster *__restrict__ clus,
                      const float4 *__restrict__ acc4, double4 *__restrict__ v4,
                      double4 *__restrict__ p4, double *__restrict__ part, DevMisc *m)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) reset_build_counts(m);
    const Chunk ch = chunks[blockIdx.x];
    const double dt = clus[ch.cluster].dt;
    const double h = 0.5 * dt;
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    constexpr int kU = 4;       // particles of a thread in flight at once
    for (uint32_t i0 = ch.begin + threadIdx.x; i0 < ch.end; i0 += kU * kBlock) {
        float4 a[kU];
        double4 v[kU], p[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t i = i0 + (uint32_t)u * kBlock;
            if (i < ch.end) {
                a[u] = acc4[i];
                v[u] = v4[i];
                p[u] = p4[i];
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t i = i0 + (uint32_t)u * kBlock;
            if (i >= ch.end) continue;
            v[u].x = v[u].x + (double)a[u].x * h;
            v[u].y = v[u].y + (double)a[u].y * h;
            v[u].z = v[u].z + (double)a[u].z * h;
            v4[i] = v[u];
            p[u].x = p[u].x + v[u].x * dt;
            p[u].y = p[u].y + v[u].y * dt;
            p[u].z = p[u].z + v[u].z * dt;
            p4[i] = p[u];
            const double x[3] = {p[u].x, p[u].y, p[u].z};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                bad |= !isfinite(x[k]);
                lo[k] = fmin(lo[k], x[k]);
                hi[k] = fmax(hi[k], x[k]);
            }
        }
    }
    box_partial(lo, hi, bad, part, m);
}

// x += v dt for every particle (a drift without rebuilding the tree)
__global__ void __launch_bounds__(kBlock)
drift_kernel(int64_t n, const double4 *__restrict__ v4, double4 *__restrict__ p4, double dt)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double4 v = v4[i];
    double4 p = p4[i];
    p.x = p.x + v.x * dt;
    p.y = p.y + v.y * dt;
    p.z = p.z + v.z * dt;
    p4[i] = p;
}

// v += a dt for the particles whose flag (caller order) is set, all if none given
__global__ void __launch_bounds__(kBlock)
kick_masked_kernel(int64_t n, const uint32_t *__restrict__ pid, const uint8_t *__restrict__ active,
                   const float4 *__restrict__ acc4, double4 *__restrict__ v4, double dt)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (active && !active[pid[i]]) return;
    const float4 a = acc4[i];
    double4 v = v4[i];
    v.x = v.x + (double)a.x * dt;
    v.y = v.y + (double)a.y * dt;
    v.z = v.z + (double)a.z * dt;
    v4[i] = v;
}

// Per chunk: the closing kick v += a dt/2 of the chunk's cluster, then the T, W,
// Px, Py, Pz partial sums of the new state (same order as energy_partial_kernel).
__global__ void __launch_bounds__(kBlock)
kick_energy_kernel(const Chunk *__restrict__ chunks, const DevCluster *__restrict__ clus,
                   double4 *__restrict__ v4,
                   const float4 *__restrict__ acc4, double *__restrict__ part)
{
    const Chunk ch = chunks[blockIdx.x];
    const double h = 0.5 * clus[ch.cluster].dt;
    double s[5] = {0, 0, 0, 0, 0};
    constexpr int kU = 4;       // particles of a thread in flight at once (same sum order)
    for (uint32_t i0 = ch.begin + threadIdx.x; i0 < ch.end; i0 += kU * kBlock) {
        float4 a[kU];
        double4 v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t i = i0 + (uint32_t)u * kBlock;
            if (i < ch.end) {
                a[u] = acc4[i];
                v[u] = v4[i];
            }
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const uint32_t i = i0 + (uint32_t)u * kBlock;
            if (i >= ch.end) continue;
            v[u].x = v[u].x + (double)a[u].x * h;
            v[u].y = v[u].y + (double)a[u].y * h;
            v[u].z = v[u].z + (double)a[u].z * h;
            v4[i] = v[u];
            const double m = v[u].w;        // the velocity record carries the mass
            s[0] += 0.5 * m * ((v[u].x * v[u].x + v[u].y * v[u].y) + v[u].z * v[u].z);
            s[1] += 0.5 * m * (double)a[u].w;
            s[2] += m * v[u].x;
            s[3] += m * v[u].y;
            s[4] += m * v[u].z;
        }
    }
    __shared__ double sh[5][kBlock];
#pragma unroll
    for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int d = kBlock / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) part[5 * (int64_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// Per chunk: T, W, Px, Py, Pz partial sums (fixed order: strided per thread,
// then a tree over the block); part[5 chunk + k].
__global__ void __launch_bounds__(kBlock)
energy_partial_kernel(const Chunk *__restrict__ chunks, const double4 *__restrict__ v4,
                      const float4 *__restrict__ acc4, double *__restrict__ part)
{
    const Chunk ch = chunks[blockIdx.x];
    double s[5] = {0, 0, 0, 0, 0};
    for (uint32_t i = ch.begin + threadIdx.x; i < ch.end; i += kBlock) {
        const double4 v = v4[i];
        const double m = v.w;           // the velocity record carries the mass
        s[0] += 0.5 * m * ((v.x * v.x + v.y * v.y) + v.z * v.z);
        s[1] += 0.5 * m * (double)acc4[i].w;
        s[2] += m * v.x;
        s[3] += m * v.y;
        s[4] += m * v.z;
    }
    __shared__ double sh[5][kBlock];
#pragma unroll
    for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int d = kBlock / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) part[5 * (int64_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// One block per cluster: its chunk partials, strided per thread then a tree
// (a fixed order); out[5 cluster + k].
__global__ void __launch_bounds__(kBlock)
energy_final_kernel(const DevCluster *__restrict__ clus, const double *__restrict__ part,
                    double *__restrict__ out)
{
    const DevCluster &cl = clus[blockIdx.x];
    double s[5] = {0, 0, 0, 0, 0};
    for (uint32_t b = cl.chunk0 + threadIdx.x; b < cl.chunk0 + cl.nchunk; b += kBlock) {
#pragma unroll
        for (int k = 0; k < 5; ++k) s[k] += part[5 * (int64_t)b + k];
    }
    __shared__ double sh[5][kBlock];
#pragma unroll
    for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int d = kBlock / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) out[5 * (int64_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(kBlock)
gather_vel_kernel(int64_t n, const double *__restrict__ vel, const uint32_t *__restrict__ pid,
                  const double4 *__restrict__ p4, double4 *__restrict__ v4)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t o = pid[i];
    v4[i] = make_double4(vel[3 * o], vel[3 * o + 1], vel[3 * o + 2], p4[i].w);   // w: the mass
}

__global__ void __launch_bounds__(kBlock)
gather_pos_kernel(int64_t n, const double *__restrict__ pos, const uint32_t *__restrict__ pid,
                  double4 *__restrict__ p4)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t o = pid[i];
    double4 p = p4[i];
    p.x = pos[3 * o];
    p.y = pos[3 * o + 1];
    p.z = pos[3 * o + 2];
    p4[i] = p;
}

__global__ void __launch_bounds__(kBlock)
state_out_kernel(int64_t n, const double4 *__restrict__ p4, const double4 *__restrict__ v4,
                 const uint32_t *__restrict__ pid, double *__restrict__ pos, double *__restrict__ vel)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t o = pid[i];
    if (pos) {
        const double4 p = p4[i];
        pos[3 * o] = p.x;
        pos[3 * o + 1] = p.y;
        pos[3 * o + 2] = p.z;
    }
    if (vel) {
        const double4 v = v4[i];
        vel[3 * o] = v.x;
        vel[3 * o + 1] = v.y;
        vel[3 * o + 2] = v.z;
    }
}

}  // namespace

hipError_t launch_kick_drift(bh_ctx *c)
{
    hipLaunchKernelGGL(kick_drift_box_kernel, dim3((unsigned)c->nchunks), dim3(kBlock), 0,
                       c->stream, c->chunks, c->clus, c->acc4, c->v4[c->cur], c->p4[c->cur],
                       c->bb_part, c->misc);
    BH_LAUNCH_CHECK();
    c->box_ready = true;        // the rebuild that follows skips its bbox pass
    return hipSuccess;
}

hipError_t launch_drift(bh_ctx *c, double dt)
{
    hipLaunchKernelGGL(drift_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n,
                       c->v4[c->cur], c->p4[c->cur], dt);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_kick_masked(bh_ctx *c, double dt, const uint8_t *active)
{
    hipLaunchKernelGGL(kick_masked_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n,
                       c->pid[c->cur], active, c->acc4, c->v4[c->cur], dt);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_kick_energy(bh_ctx *c)
{
    hipLaunchKernelGGL(kick_energy_kernel, dim3((unsigned)c->nchunks), dim3(kBlock), 0, c->stream,
                       c->chunks, c->clus, c->v4[c->cur], c->acc4, c->e_part);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(energy_final_kernel, dim3((unsigned)c->K), dim3(kBlock), 0, c->stream,
                       c->clus, c->e_part, c->e_out);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_energy(bh_ctx *c)
{
    hipLaunchKernelGGL(energy_partial_kernel, dim3((unsigned)c->nchunks), dim3(kBlock), 0, c->stream,
                       c->chunks, c->v4[c->cur], c->acc4, c->e_part);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(energy_final_kernel, dim3((unsigned)c->K), dim3(kBlock), 0, c->stream,
                       c->clus, c->e_part, c->e_out);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_set_velocities(bh_ctx *c, const double *vel)
{
    hipLaunchKernelGGL(gather_vel_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n, vel,
                       c->pid[c->cur], c->p4[c->cur], c->v4[c->cur]);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_set_positions(bh_ctx *c, const double *pos, const double *vel)
{
    if (pos)
        hipLaunchKernelGGL(gather_pos_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n,
                           pos, c->pid[c->cur], c->p4[c->cur]);
    BH_LAUNCH_CHECK();
    if (vel) return launch_set_velocities(c, vel);
    return hipSuccess;
}

hipError_t launch_get_state(bh_ctx *c, double *pos, double *vel, float *acc, float *pot)
{
    if (pos || vel) {
        hipLaunchKernelGGL(state_out_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n,
                           c->p4[c->cur], c->v4[c->cur], c->pid[c->cur], pos, vel);
        BH_LAUNCH_CHECK();
    }
    return launch_scatter(c, acc, pot);
}

}  // namespace bh
