/*
 * bh.h - C ABI of libbh, an MI355X (gfx950) implementation of the sparse-octree
 * gravitational tree-code of Bedorf, Gaburov & Portegies Zwart, "A sparse octree
 * gravitational N-body code that runs entirely on the GPU processor" (J. Comput.
 * Phys. 231 (2012); arXiv:1106.1900).
 *
 * The library keeps one particle system per context on the device: it builds the
 * octree from Morton keys level by level (Sect. 2.1, App. A, App. B), computes
 * float64 monopole and quadrupole moments bottom-up (Sect. 3.2), walks the tree
 * breadth-first per group of particles with the opening test of Eq. (1) (Sect.
 * 2.2, 3.3), and advances the system with a leapfrog (Sect. 3.1).  G = 1.
 *
 * Conventions for every call:
 *  - Every pointer argument named as "device" is HIP device memory (for example
 *    the data pointer of a torch CUDA tensor).  Host pointers are marked "host".
 *  - Work is enqueued on the context's stream; device outputs are valid once the
 *    caller has synchronised that stream.  Calls marked "synchronous" return
 *    after the stream has drained.
 *  - Arrays indexed by particle are in the caller's original order unless a
 *    comment says "sorted order" (the Morton order the library uses inside).
 *  - Return value: BH_OK or a negative status; bh_last_error() then holds a
 *    message.  Nothing aborts, throws or exits across this interface.
 *  - One context must not be used from two host threads at the same time.
 */
#ifndef BH_H
#define BH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BH_OK       0
#define BH_EINVAL  (-1)   /* bad argument: null pointer, n < 1, theta outside (0,1], eps < 0, non-finite input */
#define BH_ENOMEM  (-2)   /* device allocation failed or over the context's memory budget */
#define BH_EDEVICE (-3)   /* a HIP call failed (the message names it) */
#define BH_ESTATE  (-4)   /* call out of order, e.g. forces before a tree exists */

typedef struct bh_ctx bh_ctx;

/* Tunables.  nleaf: most particles a leaf may hold (Sect. 2.1, 16 in the paper);
 * ncrit: most particles in a walk group (Sect. 2.2, 64 in the paper; at most 64
 * here, one wavefront per group); max_n: particles to reserve room for up front
 * (0: grow on demand); hbm_budget_bytes: cap on the device memory the context
 * may hold (0: no cap); max_clusters: clusters of a batch to reserve room for
 * (0: grow on demand). */
typedef struct {
    int32_t nleaf;
    int32_t ncrit;
    int64_t max_n;
    int64_t hbm_budget_bytes;
    int64_t max_clusters;
} bh_params;

/* Per-build and per-walk figures.  Times are device time between events on the
 * context stream, in milliseconds, for the most recent build / force call. */
typedef struct {
    int64_t n;
    int64_t ncells;
    int64_t nleaves;
    int64_t ngroups;
    int32_t depth;          /* deepest level holding a cell (root = 0) */
    int32_t lanes_per_group_max;
    int64_t sum_npp;        /* sum over groups of size(g) * npp(g): particle-particle interactions */
    int64_t sum_npc;        /* sum over groups of size(g) * npc(g): particle-cell interactions */
    double ms_keys;         /* bounding box + keys */
    double ms_sort;         /* radix sort */
    double ms_move;         /* reorder of particle data */
    double ms_tree;         /* cells, links, groups */
    double ms_moments;      /* multipole moments */
    double ms_walk;         /* opening radii + walk + scatter */
    int64_t device_bytes;   /* device memory held by the context */
    /* The walk kernel alone, timed with events on the context stream around each
     * launch: last launch, and totals since the context was created. */
    double ms_walk_kernel;
    double walk_kernel_ms_total;
    int64_t walk_kernel_launches;
    int64_t total_npp;      /* sum_npp accumulated over all walks */
    int64_t total_npc;      /* sum_npc accumulated over all walks */
    int64_t nclusters;      /* clusters loaded (1 after bh_build_tree) */
    int64_t graph_launches; /* captured steps replayed by bh_batch_run */
} bh_stats;

/* Host copies of the tree for checking it element by element.  Every pointer is
 * optional (NULL: skipped) and caller-owned host memory sized from bh_stats:
 * [n] arrays for particles, [ncells] for cells, [ngroups] for groups.  Cells are
 * in (level, key prefix) order; particles in sorted order. */
typedef struct {
    uint64_t *key;      /* [n] Morton keys, sorted order */
    int64_t *perm;      /* [n] caller index of each sorted particle */
    uint8_t *level;     /* [ncells] */
    uint64_t *prefix;   /* [ncells] key >> 3 (20 - level) of the cell's particles */
    int64_t *first;     /* [ncells] first sorted particle */
    int64_t *count;     /* [ncells] particles in the cell */
    uint8_t *is_leaf;   /* [ncells] */
    int64_t *parent;    /* [ncells] -1 at the root */
    int64_t *child;     /* [ncells] first child (nodes) or -1 (leaves) */
    int32_t *nchild;    /* [ncells] children of a node, 0 for leaves */
    double *mass;       /* [ncells] float64 cell mass */
    double *com;        /* [ncells][3] float64 centre of mass */
    double *S;          /* [ncells][6] float64 second moment about the centre of
                           mass: xx, yy, zz, xy, xz, yz */
    float *rcrit2;      /* [ncells] squared opening radius of the last force call */
    int64_t *gfirst;    /* [ngroups] first sorted particle of each group */
    int64_t *gcount;    /* [ngroups] */
    double *gcentre;    /* [ngroups][3] float64 centre of the group's tight box */
    float *ghalf;       /* [ngroups][3] float32 half-size of that box */
    int64_t *npp;       /* [ngroups] particles in opened leaves (own included), last force call */
    int64_t *npc;       /* [ngroups] accepted cells, last force call */
} bh_tree_host;

/* Fill *p with the defaults: nleaf 16, ncrit 64, max_n 0, budget 0,
 * max_clusters 0. */
int bh_default_params(bh_params *p);

/* Create a context.  p may be NULL (defaults).  hip_stream is a hipStream_t the
 * caller owns and keeps alive for the context's lifetime (NULL: the null
 * stream).  The current HIP device at this call is the context's device. */
int bh_create(bh_ctx **out, const bh_params *p, void *hip_stream);

/* Free all device memory the context holds.  NULL is accepted. */
int bh_destroy(bh_ctx *ctx);

/* Load n particles and build their tree (Sect. 2.1, 3.2).  pos: device [n][3]
 * float64 row-major; mass: device [n] float64, each > 0.  Both are copied in;
 * the caller may reuse them once the stream has synchronised.  Velocities are
 * set to zero.  Synchronous (it reads back the cell and group counts).
 * BH_EINVAL for n < 1, null pointers or a non-finite coordinate. */
int bh_build_tree(bh_ctx *ctx, const double *pos, const double *mass, int64_t n);

/* vel: device [n][3] float64, caller order, for the particles of the last build. */
int bh_set_velocities(bh_ctx *ctx, const double *vel);

/* Accelerations and potentials of every particle by the group walk (Sect. 2.2)
 * with the opening test d > l/theta + delta (Eq. (1)) and Plummer softening
 * eps: phi_i = -sum m_j (r_ij^2 + eps^2)^(-1/2) over particles and the
 * monopole + quadrupole expansion over accepted cells.  The self pair is left
 * out.  theta in (0, 1], eps >= 0.  acc: device [n][3] float32, pot: device [n]
 * float32, caller order, caller-owned (either may be NULL to keep results only
 * inside the context).  Needs a prior build.  Interactions are float32 on
 * offsets from each group's box centre; sums are compensated per particle. */
int bh_compute_forces(bh_ctx *ctx, float theta, float eps, float *acc, float *pot);

/* One leapfrog step (Sect. 3.1) as kick-drift-kick: v += a dt/2; x += v dt
 * (float64); rebuild the tree; forces with the last theta and eps; v += a dt/2.
 * Needs a prior bh_compute_forces.  Enqueued without waiting for the device;
 * device-side errors are reported by the next synchronous call (see
 * bh_batch_run). */
int bh_leapfrog_step(bh_ctx *ctx, double dt);

/* Copy the state out in caller order; any pointer may be NULL.  pos, vel:
 * device [n][3] float64; acc: device [n][3] float32; pot: device [n] float32
 * (acc and pot from the last force evaluation). */
int bh_get_state(bh_ctx *ctx, double *pos, double *vel, float *acc, float *pot);

/* Replace positions and velocities (device [n][3] float64, caller order) of
 * the current n particles and rebuild; forces must be recomputed afterwards. */
int bh_set_state(bh_ctx *ctx, const double *pos, const double *vel);

/* Energy and momentum in float64 from the current velocities and the last
 * potentials (Eq. (3) ingredients): out[0..6] = T, W, E = T + W, Px, Py, Pz,
 * and (E0 - E) / E0 with E0 the energy at the first bh_energy call after a
 * build or set_state (host array).  On a batch: sums over all clusters.
 * Synchronous. */
int bh_energy(bh_ctx *ctx, double out[7]);

/* Host copy of the latest figures.  Synchronous. */
int bh_stats_get(bh_ctx *ctx, bh_stats *out);

/* Host copies of the tree (see bh_tree_host).  Synchronous. */
int bh_export_tree(bh_ctx *ctx, const bh_tree_host *out);

/* ---------------------------------------------------------------------------
 * Batches: K independent particle systems ("clusters") in one context.  Each
 * cluster gets its own domain and tree (the trees of the batch form one forest:
 * cluster k's root is cell k), its own opening angle, softening, leaf and group
 * sizes and time step, while every phase runs as one launch over the whole batch
 * and the walk takes its groups from one queue.  The single-system calls above
 * are the K = 1 case; on a batch, bh_compute_forces and bh_leapfrog_step set theta,
 * eps and dt of every cluster, and bh_get_state / bh_set_state / bh_set_velocities
 * use the concatenated caller order (cluster 0's particles, then cluster 1's, ...).
 */

/* One cluster of a batch. */
typedef struct {
    int64_t n;          /* particles, >= 1 */
    float theta;        /* opening angle of Eq. (1), in (0, 1] */
    float eps;          /* Plummer softening, >= 0 */
    double dt;          /* leapfrog step used by bh_batch_run (finite; 0 leaves the
                           cluster's positions and velocities as they are while its
                           forces are evaluated) */
    int32_t nleaf;      /* 1..64; 0: the context's nleaf */
    int32_t ncrit;      /* 1..64; 0: the context's ncrit */
} bh_cluster;

/* Load k clusters and build their forest.  clusters: host [k].  pos: device
 * [sum n][3] float64, mass: device [sum n] float64 (> 0), vel: device [sum n][3]
 * float64 or NULL (zero), all in concatenated order.  Copied in.  Synchronous
 * (validates the inputs).  BH_EINVAL for k < 1, a bad cluster entry, a total of
 * 2^31 particles or more, or non-finite data. */
int bh_batch_build(bh_ctx *ctx, const bh_cluster *clusters, int64_t k, const double *pos,
                   const double *mass, const double *vel);

/* Change theta, eps and dt of the loaded clusters (host [k], k and each n, nleaf
 * and ncrit as loaded; nleaf / ncrit 0 match the context's values).  Takes effect
 * for work enqueued afterwards. */
int bh_batch_set_params(bh_ctx *ctx, const bh_cluster *clusters, int64_t k);

/* Forces of every cluster with its own theta and eps, from its current tree
 * (see bh_compute_forces for acc and pot; concatenated caller order). */
int bh_batch_forces(bh_ctx *ctx, float *acc, float *pot);

/* nsteps kick-drift-kick steps of every cluster with its own dt (Sect. 3.1):
 * each step rebuilds every tree and recomputes every force.  The step is
 * captured once into a HIP graph per buffer layout and replayed, so it costs
 * one graph launch on the context stream; nothing is read back and the call
 * does not wait for the device.  Needs a prior force evaluation.  Errors found
 * on the device (non-finite coordinates after a step) are reported by the next
 * synchronous call (bh_energy, bh_batch_energy, bh_stats_get, bh_export_tree). */
int bh_batch_run(bh_ctx *ctx, int32_t nsteps);

/* Per-cluster energy and momentum: out host [k][7] as in bh_energy, each
 * cluster's E0 taken at its first call after a build or state change.
 * Synchronous. */
int bh_batch_energy(bh_ctx *ctx, double *out);

/* Message for the last non-zero status of this context (never NULL). */
const char *bh_last_error(bh_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
