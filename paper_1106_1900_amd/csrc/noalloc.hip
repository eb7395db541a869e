// noalloc.hip - bh_forces_static: the build of bh_build_tree followed by the walk
// of bh_compute_forces for one small particle set, with every intermediate
// buffer (keys, cells, groups, walk stacks, counters) carved from one
// file-scope device array instead of memory the library allocates.  For callers
// that cannot allocate device memory (code under graph capture that must not
// call hipMalloc, tight serving loops, harnesses that forbid allocation).
//
// The array exists once per GPU the library runs on and is held until the
// process ends.  Host code never passes the array's name to a kernel (in host
// code it names a host-side stand-in); it takes the device address once per
// device from hipGetSymbolAddress and carves the context's buffers from that.
// Every call on a device shares that device's array and the host-side record
// that describes it, so calls that overlap on one GPU (two host threads, or two
// streams in flight at once) race.
#include <cstring>

#include "bh_internal.h"

using namespace bh;

namespace {

// Largest particle count of one call, and the fixed leaf and group sizes.
constexpr int64_t kStaticMaxN = BH_STATIC_MAX_N;
constexpr int kStaticNleaf = 16;
constexpr int kStaticNcrit = 64;
// Wavefronts of the walk grid: one workgroup of four per CU of a 256-CU device
// (each wavefront owns a stack spill region of the array).
constexpr int64_t kStaticWaves = 1024;
// Size of the array: the carved layout for kStaticMaxN particles needs about
// 35 MB; the first call checks the layout against it.
constexpr size_t kScratchBytes = (size_t)40 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Host-side record of one device's array.
struct StaticSlot {
    bool ready = false;
    char *base = nullptr;          // device address of this device's scratch
    bh_ctx ctx;                    // its buffers point into [base, base + kScratchBytes)
    DevMisc misc_h;                // host copy of the counts and error bits
};
StaticSlot g_slot[kMaxDevices];

// message of the calling thread's last failed call (string literals only)
thread_local const char *g_msg = "no error";

int fail(int code, const char *msg)
{
    g_msg = msg;
    return code;
}

// The one-cluster table, the chunk table and a cleared misc block, written on the
// device so that no host staging memory is needed.
__global__ void __launch_bounds__(64)
static_table_kernel(uint32_t n, float theta, float eps, DevCluster *__restrict__ clus,
                    Chunk *__restrict__ chunks, DevMisc *__restrict__ m)
{
    const int t = threadIdx.x;
    const uint32_t nch = (n + kChunk - 1) / kChunk;
    if (t == 0) {
        DevCluster d;
        d.dt = 0.0;
        d.theta = theta;
        d.eps2 = eps * eps;     // the float32 square, as for every other cluster
        d.first = 0;
        d.n = n;
        d.nleaf = kStaticNleaf;
        d.ncrit = kStaticNcrit;
        d.chunk0 = 0;
        d.nchunk = nch;
        d.mac = 0;
        d.pad = 0;
        clus[0] = d;
    }
    for (uint32_t b = t; b < nch; b += 64) {
        Chunk ch;
        ch.cluster = 0;
        ch.begin = b * kChunk;
        ch.end = (b + 1) * kChunk < n ? (b + 1) * kChunk : n;
        ch.pad = 0;
        chunks[b] = ch;
    }
    // every field of the misc block starts at zero (error bits, counts, the
    // walk's work counter and totals): the array keeps the last call's values
    uint32_t *w = reinterpret_cast<uint32_t *>(m);
    for (size_t i = t; i < sizeof(DevMisc) / sizeof(uint32_t); i += 64) w[i] = 0u;
}

int init_slot(StaticSlot &s, int device)
{
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return BH_EDEVICE;
    }
    bh_ctx &c = s.ctx;
    c.device = device;
    bh_default_params(&c.p);
    c.p.nleaf = kStaticNleaf;
    c.p.ncrit = kStaticNcrit;
    const int64_t need = ctx_carve(&c, kStaticMaxN, kStaticNleaf, kStaticWaves,
                                   static_cast<char *>(ptr), (int64_t)kScratchBytes);
    if (need > (int64_t)kScratchBytes) return BH_ENOMEM;
    c.misc_h = &s.misc_h;
    memset(&s.misc_h, 0, sizeof(DevMisc));
    s.base = static_cast<char *>(ptr);
    s.ready = true;
    return BH_OK;
}

// Waits for the stream and reports the error bits the device raised.
int wait_check(StaticSlot &s, bool walked)
{
    bh_ctx &c = s.ctx;
    if (hipMemcpyAsync(&s.misc_h, c.misc, sizeof(DevMisc), hipMemcpyDeviceToHost, c.stream) !=
            hipSuccess ||
        hipStreamSynchronize(c.stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BH_EDEVICE, "device error during the build or walk");
    }
    const DevMisc &m = s.misc_h;
    if (m.nonfinite & 1u) return fail(BH_EINVAL, "non-finite particle coordinate");
    if (m.nonfinite & 2u) return fail(BH_EINVAL, "particle mass must be finite and > 0");
    if (m.nonfinite) return fail(BH_EDEVICE, "internal error in the tree construction");
    if (walked && m.walk_overflow) return fail(BH_EDEVICE, "walk list overflow");
    if (m.ncells < 1 || m.ncells > (uint64_t)c.cap_c || m.ngroups < 1 ||
        m.ngroups > (uint64_t)c.n)
        return fail(BH_EDEVICE, "tree construction produced inconsistent counts");
    return BH_OK;
}

#define TRY_ST(expr)           \
    do {                       \
        int st__ = (expr);     \
        if (st__) return st__; \
    } while (0)

}  // namespace

extern "C" {

int bh_forces_static(const double *pos, const double *mass, int64_t n, float theta, float eps,
                     float *acc, float *pot, void *hip_stream)
{
    if (!pos || !mass) return fail(BH_EINVAL, "null pos or mass");
    if (!acc && !pot) return fail(BH_EINVAL, "acc and pot are both null");
    if (n < 1 || n > kStaticMaxN) return fail(BH_EINVAL, "n must be in [1, BH_STATIC_MAX_N]");
    if (!(theta > 0.0f && theta <= 1.0f)) return fail(BH_EINVAL, "theta must be in (0, 1]");
    if (!(eps >= 0.0f) || !(eps <= 3.4e38f)) return fail(BH_EINVAL, "eps must be finite and >= 0");
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BH_EDEVICE, "hipGetDevice failed");
    }
    if (device < 0 || device >= kMaxDevices) return fail(BH_EDEVICE, "device index beyond 63");
    StaticSlot &s = g_slot[device];
    if (!s.ready) {
        const int st = init_slot(s, device);
        if (st == BH_ENOMEM) return fail(st, "scratch array smaller than the carved layout");
        if (st) return fail(st, "hipGetSymbolAddress of the scratch array failed");
    }
    bh_ctx &c = s.ctx;
    c.stream = (hipStream_t)hip_stream;
    const int64_t nch = (n + kChunk - 1) / kChunk;
    hipLaunchKernelGGL(static_table_kernel, dim3(1), dim3(64), 0, c.stream, (uint32_t)n, theta,
                       eps, c.clus, c.chunks, c.misc);
    if (hipGetLastError() != hipSuccess) return fail(BH_EDEVICE, "launch of the table kernel failed");
    c.n = n;
    c.K = 1;
    c.nchunks = nch;
    c.max_nleaf = kStaticNleaf;
    c.any_eps0 = !(eps > 0.0f) || !(eps * eps > 0.0f);
    c.layout += 1;
    if (ctx_enqueue_load(&c, pos, mass) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BH_EDEVICE, "launch of the build failed");
    }
    // the build's error bits are checked before the walk runs on its tree, as
    // bh_build_tree does; the counts also refresh the launch hints
    TRY_ST(wait_check(s, false));
    if (ctx_enqueue_forces_out(&c, acc, pot) != hipSuccess) {
        (void)hipGetLastError();
        return fail(BH_EDEVICE, "launch of the walk failed");
    }
    TRY_ST(wait_check(s, true));
    g_msg = "no error";
    return BH_OK;
}

const char *bh_forces_static_error(void) { return g_msg; }

}  // extern "C"
