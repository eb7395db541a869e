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
 * ncrit: most particles in a walk group (Sect. 2.2, 64 in the paper; 1..128
 * here: one wavefront per group, a lane carrying up to two of its particles);
 * nleaf is 1..64; max_n: particles to reserve room for up front
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
    int64_t graph_captures; /* leapfrog steps captured into a graph (one per buffer parity
                               and cluster layout) */
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
 * with the cluster's opening test (Eq. (1) unless bh_set_mac chose the
 * minimum-distance test) and Plummer softening
 * eps: phi_i = -sum m_j (r_ij^2 + eps^2)^(-1/2) over particles and the
 * monopole + quadrupole expansion over accepted cells.  The self pair is left
 * out.  theta in (0, 1], eps >= 0.  acc: device [n][3] float32, pot: device [n]
 * float32, caller order, caller-owned (either may be NULL to keep results only
 * inside the context).  Needs a prior build.  Interactions are float32 on
 * offsets from each group's box centre; sums are compensated per particle. */
int bh_compute_forces(bh_ctx *ctx, float theta, float eps, float *acc, float *pot);

/* Opening tests.  BH_MAC_EQ1: Eq. (1) of Sect. 3.3, d > l/theta + delta with d the
 * distance from the cell's centre of mass to the group's box.  BH_MAC_MIN_DIST:
 * the minimum-distance test that Sect. 3.3 names as the alternative (Salmon &
 * Warren 1994): the smallest distance between the group's box and the cell's
 * cube (side l about its geometric centre) must exceed l/theta; the paper reports
 * a 10-50% smaller acceleration error for the same theta at a higher cost.  Both
 * are taken in float32 on offsets from the group's box centre. */
#define BH_MAC_EQ1      0
#define BH_MAC_MIN_DIST 1

/* Set the opening test of every loaded cluster and the one bh_build_tree gives
 * the clusters it loads (the context starts with BH_MAC_EQ1).  Takes effect for
 * work enqueued afterwards.  BH_EINVAL for any other value. */
int bh_set_mac(bh_ctx *ctx, int32_t mac);

/* One leapfrog step (Sect. 3.1) as kick-drift-kick: v += a dt/2; x += v dt
 * (float64); rebuild the tree; forces with the last theta and eps; v += a dt/2.
 * Needs a prior bh_compute_forces.  Enqueued without waiting for the device;
 * device-side errors are reported by the next synchronous call (see
 * bh_batch_run). */
int bh_leapfrog_step(bh_ctx *ctx, double dt);

/* Copy the state out in caller order; any pointer may be NULL.  pos, vel:
 * device [n][3] float64; acc: device [n][3] float32; pot: device [n] float32
 * (acc and pot from the last force evaluation).  On a batch the arrays hold
 * every cluster in concatenated order, so one cluster's state is the slice
 * [first, first + n) of them: there is no separate per-cluster getter. */
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

/* Host copy of the latest figures (counts, interaction totals, per-phase
 * times) in one struct.  Synchronous. */
int bh_stats_get(bh_ctx *ctx, bh_stats *out);

/* Host copies of the tree (see bh_tree_host), including the per-group
 * interaction counts of the last force call (npp, npc), so counts and tree come
 * from one call.  Synchronous. */
int bh_export_tree(bh_ctx *ctx, const bh_tree_host *out);

/* ---------------------------------------------------------------------------
 * Between rebuilds (block time-steps, Sect. 5): only some particles need new
 * forces at a given time, and instead of rebuilding the tree it suffices to
 * recompute the multipole moments of the existing cells.  With these calls a
 * caller drives such a scheme: drift all particles, refit, evaluate the forces
 * of the groups that hold active particles, kick the active particles.  The
 * tree must be rebuilt (bh_set_state, bh_leapfrog_step) when the walk's cost
 * grows, since drifted particles leave their geometric cells.
 */

/* x += v dt (float64) for every particle, without touching the tree.  Force
 * calls are refused (BH_ESTATE) until bh_refit or a rebuild. */
int bh_drift(bh_ctx *ctx, double dt);

/* v += a dt (float64, a from the last force evaluation) for the particles
 * whose active[i] != 0 (device [n] uint8, caller order); NULL: all. */
int bh_kick(bh_ctx *ctx, double dt, const uint8_t *active);

/* Multipole-only update (Sect. 5): keep the cells, keys, domain and groups of
 * the last build; recompute every cell's moments and every group's tight box
 * from the current positions, and take as each cell's side in the opening test
 * the larger of its build side and the largest side of its particles' tight box
 * (a refitted tree's cells grow, which is what slows its walk).  Opening radii
 * follow at the next force call. */
int bh_refit(bh_ctx *ctx);

/* Forces of the groups that hold at least one particle with active[i] != 0
 * (device [n] uint8, caller order): the walk visits those groups only (Sect.
 * 2.2, 5); their particles' accelerations and potentials are recomputed, all
 * others keep the values of the previous evaluation.  acc, pot as in
 * bh_compute_forces (whole arrays, caller order; either may be NULL).  Needs a
 * prior full evaluation.  Per-group interaction counts in bh_export_tree are
 * updated for the visited groups only. */
int bh_compute_forces_active(bh_ctx *ctx, float theta, float eps, const uint8_t *active,
                             float *acc, float *pot);

/* ---------------------------------------------------------------------------
 * Block time-steps (Sect. 5): particles advance with power-of-two fractions of a
 * block step; between synchronisation points only the groups holding particles
 * due for an update are walked, on the tree whose moments are refitted to the
 * current positions, and the tree is rebuilt when its walk has grown too
 * expensive.  The paper gives neither the criterion nor the schedule; the
 * readings (criterion dt_i = sqrt(2 eta length / |a_i|), bins held for a block
 * step, kick-drift-kick per bin) are described in block.hip.  Work runs on the
 * context stream with each cluster's theta and eps (from the last force call);
 * the block parameters apply to every cluster.
 */
typedef struct {
    double dt_max;      /* block step: bin b steps with dt_max 2^-b (> 0) */
    double eta;         /* accuracy parameter of the criterion (> 0) */
    double length;      /* length of the criterion, e.g. the softening (> 0) */
    int32_t max_level;  /* B: bins 0..B, 2^B substeps per block step (0..15) */
    float growth;       /* each particle's base is its group's interaction count in
                           the last walk that covered it on a freshly built tree; when
                           a walk of the refitted tree has more than (1 + growth) times
                           the summed base of the particles it covered, the next force
                           evaluation rebuilds the tree instead of refitting it.  <= 0:
                           every force evaluation rebuilds (with B = 0: the leapfrog
                           step).  On a batch the sums run over the whole forest. */
} bh_block_params;

typedef struct {
    int64_t substeps;           /* 2^B */
    int64_t rebuilt;            /* force evaluations of the step on a rebuilt tree */
    int64_t updates;            /* particle steps completed: sum over particles of 2^bin */
    int64_t walked_groups;      /* groups walked over the step (partial and full walks) */
    double sync_interactions;   /* interactions per particle of the final walk (every
                                   group, every particle due) */
    double base_interactions;   /* mean base over the particles after the step */
    int64_t bin_count[16];      /* particles per bin during the step */
} bh_block_stats;

/* Bins of the particles from their current accelerations, as the next block
 * step would assign them.  bins: device [n] uint8, caller order (may be NULL);
 * count: host [16] particles per bin (may be NULL).  Synchronous. */
int bh_block_bins(bh_ctx *ctx, const bh_block_params *p, uint8_t *bins, int64_t *count);

/* One block step of dt_max: bins from the current accelerations, 2^B substeps,
 * each force evaluation on a refitted or a rebuilt tree by the growth rule.
 * Needs current forces of every particle (a force call, leapfrog step or earlier
 * block step, and no drift since); if the tree has not been refitted since it
 * was built, the counts of its last walk become every particle's base.  Whether
 * the next evaluation rebuilds is kept in the context across block steps (and
 * dropped when the tree has been rebuilt since: loads, bh_set_state, leapfrog
 * steps).  out: host, may be NULL.  Synchronous: after the
 * bins, after each walk of a refitted tree (for the rule) and at the end. */
int bh_block_step(bh_ctx *ctx, const bh_block_params *p, bh_block_stats *out);

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
    int32_t ncrit;      /* 1..128; 0: the context's ncrit */
    int32_t mac;        /* opening test: BH_MAC_EQ1 or BH_MAC_MIN_DIST */
    int32_t pad;        /* zero */
} bh_cluster;

/* Load k clusters and build their forest.  clusters: host [k].  pos: device
 * [sum n][3] float64, mass: device [sum n] float64 (> 0), vel: device [sum n][3]
 * float64 or NULL (zero), all in concatenated order.  Copied in.  The whole
 * table is loaded at once (no per-cluster add), so the forest is built in one
 * pass over all clusters.  Synchronous (validates the inputs).  BH_EINVAL for k < 1, a bad cluster entry, a total of
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

/* ---------------------------------------------------------------------------
 * Autotuning of the leaf size (Sect. 2.1) and group size (Sect. 2.2) per class of
 * cluster.  A class is (floor(log2 n), theta).  Clusters given nleaf = 0 or
 * ncrit = 0 take the tuned value of their class when the context holds one, else
 * the context's default.
 */
typedef struct {
    int32_t log2n;      /* class: floor(log2 n) */
    float theta;        /* class: opening angle */
    int32_t nleaf;      /* chosen leaf size */
    int32_t ncrit;      /* chosen group size */
    double ms;          /* device time of one step of the class's clusters with the choice */
    double ms_default;  /* the same with the context's defaults */
} bh_tune_entry;

/* Times one leapfrog step of dt = 0 (rebuild and forces, no motion) of the loaded
 * batch's clusters, class by class in a private context, for every nleaf in
 * {8, 16, 32} and ncrit in {32, 64, 128}, reps steps each, and keeps the fastest
 * pair per class in the context (replacing an earlier table).  out: host
 * [cap] entries (may be NULL); *count: classes found.  Synchronous.  The loaded
 * batch is not changed. */
int bh_autotune(bh_ctx *ctx, int32_t reps, bh_tune_entry *out, int64_t cap, int64_t *count);

/* Install a tuning table (host [count], copied); count 0 clears it. */
int bh_set_tuning(bh_ctx *ctx, const bh_tune_entry *entries, int64_t count);

/* ---------------------------------------------------------------------------
 * Serving: a loop that keeps many independent requests resident on one device
 * and advances them together.  A request is one system: a force evaluation
 * followed by nsteps leapfrog steps.  Admission is first come, first served,
 * while the resident particles and requests fit the capacity derived from the
 * memory budget and the resident-particle limit; every iteration (bh_server_step) advances each resident request
 * by one unit (its force evaluation, then one step), so requests join and leave
 * the batch between iterations (continuous batching at iteration level).
 */

typedef struct bh_server bh_server;

typedef struct {
    int64_t hbm_budget_bytes;   /* device memory the server's batch may hold (> 0) */
    int64_t max_requests;       /* most resident requests (>= 1) */
    int32_t nleaf;              /* defaults for requests that give 0 */
    int32_t ncrit;
    int32_t min_nleaf;          /* smallest leaf size a request may use (1..nleaf; the
                                   cell storage is sized for it; 0: min(8, nleaf)) */
    int32_t pad;
    int64_t max_resident;       /* most resident particles (0: as many as the budget
                                   holds).  A bounded working set keeps iterations short
                                   under overload, so requests finish closer to arrival
                                   order; a request larger than the limit is admitted
                                   when nothing else is resident. */
} bh_server_params;

typedef struct {
    int64_t n;                  /* particles, >= 1 */
    const double *pos;          /* device [n][3] float64 */
    const double *mass;         /* device [n] float64, > 0 */
    const double *vel;          /* device [n][3] float64, or NULL (zero) */
    float theta;                /* (0, 1] */
    float eps;                  /* >= 0 */
    double dt;                  /* leapfrog step, finite */
    int32_t nsteps;             /* steps after the force evaluation, >= 0 */
    int32_t nleaf;              /* 1..64, or 0: the server's */
    int32_t ncrit;              /* 1..128, or 0: the server's */
    int32_t mac;                /* opening test: BH_MAC_EQ1 or BH_MAC_MIN_DIST */
    double arrival;             /* arrival time on the server clock (seconds, see
                                   bh_server_now); a negative value: the time of
                                   the submit call */
    double *out_pos;            /* device [n][3] float64, final positions, or NULL */
    double *out_vel;            /* device [n][3] float64, final velocities, or NULL */
    float *out_acc;             /* device [n][3] float32, final accelerations, or NULL */
    float *out_pot;             /* device [n] float32, final potentials, or NULL */
} bh_request;

#define BH_REQ_QUEUED  0
#define BH_REQ_RUNNING 1
#define BH_REQ_DONE    2
#define BH_REQ_FAILED  3   /* rejected at admission: non-finite data or a mass <= 0 */

typedef struct {
    int32_t state;              /* BH_REQ_* */
    int32_t units_done;         /* force evaluation + steps completed */
    double arrival;             /* server clock, seconds */
    double admitted;            /* when its data was copied in (-1 while queued) */
    double completed;           /* when its outputs were written (-1 before) */
    double energy[7];           /* T, W, E, Px, Py, Pz, (E0 - E) / E0 of its last unit;
                                   E0 after its force evaluation */
} bh_request_status;

typedef struct {
    int64_t submitted, admitted, completed, rejected;
    int64_t queued, resident_requests, resident_particles;
    int64_t capacity_particles;   /* resident particles the budget allows */
    int64_t iterations;
    int64_t particle_evals;       /* sum over completed requests of n (1 + nsteps) */
    double busy_seconds;          /* wall time spent inside bh_server_step */
    double latency_p50, latency_p99, latency_max;   /* completed - arrival, seconds */
    double queue_wait_p50, queue_wait_p99;          /* admitted - arrival, seconds */
} bh_server_stats;

/* Create a server on the current device, its work enqueued on hip_stream (may be
 * NULL).  BH_ENOMEM if the budget cannot hold one particle. */
int bh_server_create(bh_server **out, const bh_server_params *p, void *hip_stream);

int bh_server_destroy(bh_server *srv);

/* Queue a request (copied: the struct, not the arrays).  The device arrays pos,
 * mass and vel must stay valid until the request is admitted (its state leaves
 * BH_REQ_QUEUED); the out arrays until it is done.  *ticket identifies it.
 * BH_ENOMEM if the request alone exceeds the capacity. */
int bh_server_submit(bh_server *srv, const bh_request *req, int64_t *ticket);

/* One iteration: admit queued requests that fit, repack the resident batch if
 * its membership changed, advance every resident request by one unit, write the
 * outputs of the requests that finish and retire them.  Waits for the device.
 * *resident (may be NULL): requests resident during the iteration. */
int bh_server_step(bh_server *srv, int64_t *resident);

/* State of a request.  The record of a finished request (BH_REQ_DONE or
 * BH_REQ_FAILED) is kept for polling until bh_server_release drops it. */
int bh_server_poll(bh_server *srv, int64_t ticket, bh_request_status *out);

/* Drop the record of a finished request, so that a long-running server keeps
 * no memory per past request beyond its latency samples (16 bytes each, for the
 * percentiles of bh_server_stats_get).  BH_ESTATE if the request is still
 * queued or running (the record stays); BH_EINVAL for an unknown or already
 * released ticket. */
int bh_server_release(bh_server *srv, int64_t ticket);

/* Counters, latency percentiles (p50, p99, max) and the served particle
 * evaluations in one struct (host).  Synchronous. */
int bh_server_stats_get(bh_server *srv, bh_server_stats *out);

/* Install a tuning table (see bh_autotune) for requests given nleaf or ncrit 0. */
int bh_server_set_tuning(bh_server *srv, const bh_tune_entry *entries, int64_t count);

/* Seconds on the server clock (a monotonic clock started at creation). */
int bh_server_now(bh_server *srv, double *t);

/* Message for the last non-zero status of this server (never NULL). */
const char *bh_server_last_error(bh_server *srv);

/* Message for the last non-zero status of this context (never NULL). */
const char *bh_last_error(bh_ctx *ctx);

/* ---- without device allocation ----
 * For callers that cannot allocate device memory: code under HIP graph capture
 * that must not call hipMalloc, tight serving loops, harnesses that forbid
 * allocation.  bh_forces_static does what bh_build_tree followed by
 * bh_compute_forces does on a fresh context (nleaf 16, ncrit 64, opening test
 * of Eq. (1)), with identical results, but every intermediate buffer lives in
 * one file-scope device array of the library (40 MiB per GPU, reserved when the
 * library is loaded and held until the process ends); it calls no allocation
 * routine.  The caller owns the inputs and outputs:
 *   pos: device [n][3] float64, mass: device [n] float64 (> 0), caller order;
 *   acc: device [n][3] float32, pot: device [n] float32, caller order (either
 *   may be NULL, not both); 1 <= n <= BH_STATIC_MAX_N; theta in (0, 1]; eps >= 0;
 *   hip_stream: the stream the work is enqueued on (NULL: the null stream).
 * Synchronous: returns after the stream has drained, so device-side errors
 * (non-finite coordinates, bad masses) are reported by the call itself.
 * BH_EINVAL for bad arguments, including n above BH_STATIC_MAX_N; BH_ENOMEM or
 * BH_EDEVICE on failure; bh_forces_static_error() gives the calling thread's
 * last message.  Every call on one GPU uses that GPU's array and keeps nothing
 * between calls that the next call reads; calls that overlap on one GPU (from
 * two host threads, or on two streams in flight at once) race. */
#define BH_STATIC_MAX_N 32768
int bh_forces_static(const double *pos, const double *mass, int64_t n, float theta, float eps,
                     float *acc, float *pot, void *hip_stream);

/* Message of the calling thread's last bh_forces_static failure (never NULL). */
const char *bh_forces_static_error(void);

#ifdef __cplusplus
}
#endif
#endif
