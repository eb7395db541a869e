// integrate.hip - leapfrog kicks and drifts (Sect. 3.1) and the float64 energy
// and momentum sums used for the energy error of Eq. (3); plus the copies
// between the caller's order and the library's sorted order.
#include "bh_internal.h"

#pragma clang fp contract(off)

namespace bh {
namespace {

constexpr int kBlock = 256;
constexpr int kRedBlocks = 1024;

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__global__ void __launch_bounds__(kBlock)
kick_kernel(int64_t n, const float4 *__restrict__ acc4, double4 *__restrict__ v4, double h)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float4 a = acc4[i];
    double4 v = v4[i];
    v.x = v.x + (double)a.x * h;
    v.y = v.y + (double)a.y * h;
    v.z = v.z + (double)a.z * h;
    v4[i] = v;
}

// v += a h; x += v dt in one pass (the first half of a kick-drift-kick step)
__global__ void __launch_bounds__(kBlock)
kick_drift_kernel(int64_t n, const float4 *__restrict__ acc4, double4 *__restrict__ v4,
                  double4 *__restrict__ p4, double h, double dt)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float4 a = acc4[i];
    double4 v = v4[i];
    v.x = v.x + (double)a.x * h;
    v.y = v.y + (double)a.y * h;
    v.z = v.z + (double)a.z * h;
    v4[i] = v;
    double4 p = p4[i];
    p.x = p.x + v.x * dt;
    p.y = p.y + v.y * dt;
    p.z = p.z + v.z * dt;
    p4[i] = p;
}

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

// Block partial sums of T, W, Px, Py, Pz over a grid-stride range (fixed order),
// then one block adds the partials in block order.
__global__ void __launch_bounds__(kBlock)
energy_partial_kernel(int64_t n, const double4 *__restrict__ p4, const double4 *__restrict__ v4,
                      const float4 *__restrict__ acc4, double *__restrict__ part)
{
    double s[5] = {0, 0, 0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double m = p4[i].w;
        const double4 v = v4[i];
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
    if (threadIdx.x < 5) part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = sh[threadIdx.x][0];
}

// Fixed-order sum of the block partials: strided per thread, then a tree.
__global__ void __launch_bounds__(kBlock)
energy_final_kernel(const double *__restrict__ part, int nblk, double *__restrict__ out)
{
    __shared__ double sh[5][kBlock];
    for (int k = 0; k < 5; ++k) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kBlock) s += part[(int64_t)k * nblk + b];
        sh[k][threadIdx.x] = s;
    }
    __syncthreads();
    for (int d = kBlock / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x < 5) out[threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(kBlock)
gather_vel_kernel(int64_t n, const double *__restrict__ vel, const uint32_t *__restrict__ pid,
                  double4 *__restrict__ v4)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t o = pid[i];
    v4[i] = make_double4(vel[3 * o], vel[3 * o + 1], vel[3 * o + 2], 0.0);
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

hipError_t launch_kick(bh_ctx *c, double h)
{
    hipLaunchKernelGGL(kick_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n, c->acc4,
                       c->v4[c->cur], h);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_kick_drift(bh_ctx *c, double h, double dt)
{
    hipLaunchKernelGGL(kick_drift_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n,
                       c->acc4, c->v4[c->cur], c->p4[c->cur], h, dt);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_drift(bh_ctx *c, double dt)
{
    hipLaunchKernelGGL(drift_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n,
                       c->v4[c->cur], c->p4[c->cur], dt);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_energy(bh_ctx *c)
{
    int nblk = (int)grid_for(c->n);
    if (nblk > kRedBlocks) nblk = kRedBlocks;
    hipLaunchKernelGGL(energy_partial_kernel, dim3(nblk), dim3(kBlock), 0, c->stream, c->n,
                       c->p4[c->cur], c->v4[c->cur], c->acc4, c->red);
    BH_LAUNCH_CHECK();
    hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kBlock), 0, c->stream, c->red, nblk,
                       c->red + 5 * kRedBlocks);
    BH_LAUNCH_CHECK();
    return hipSuccess;
}

int64_t energy_words() { return 5 * (int64_t)kRedBlocks + 8; }

hipError_t launch_set_velocities(bh_ctx *c, const double *vel)
{
    hipLaunchKernelGGL(gather_vel_kernel, dim3(grid_for(c->n)), dim3(kBlock), 0, c->stream, c->n, vel,
                       c->pid[c->cur], c->v4[c->cur]);
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
