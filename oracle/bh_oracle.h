/*
 * bh_oracle.h - plain, slow, single-threaded CPU oracle for the sparse-octree
 * gravitational tree-code of Bedorf, Gaburov & Portegies Zwart, "A sparse octree
 * gravitational N-body code that runs entirely on the GPU processor" (J. Comput.
 * Phys. 231 (2012); arXiv:1106.1900).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this code.  The product library shares
 * no source, header, table or helper with it.
 *
 * Everything here is float64 arithmetic in the order the comments state, built
 * with -ffp-contract=off so that no multiply-add is fused.  Decisions that the
 * paper takes in single precision (the opening test of Eq. (1)) are taken in
 * float32 here as well, so that the tree, the groups and the interaction lists
 * have one exact answer that the GPU path must reproduce bit for bit.
 *
 * Conventions: positions are [n][3] row-major float64, masses [n] float64.
 * "Sorted order" is the Morton (Z) order of App. B; "input order" is the
 * caller's.  All index outputs are int64.  Functions that allocate return NULL
 * or a negative status on failure; nothing aborts.
 */
#ifndef BH_ORACLE_H
#define BH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LEVEL 20      /* 60-bit keys: 20 levels of 3 bits (App. B) */

/* Integer coordinates and the 60-bit Morton key of one point (App. B).
 * The domain is the cube with lower corner lo and side L; each coordinate is
 * mapped to floor((x - lo) * 2^20 / L), clamped to [0, 2^20 - 1].  Bit b of the
 * x, y, z integers goes to key bit 3b, 3b+1, 3b+2 respectively. */
uint64_t orc_interleave(uint32_t qx, uint32_t qy, uint32_t qz);

/* Domain of a point set: per-axis minimum lo[3], cube side L (the largest
 * extent, 1 if every extent is zero) and scale = 2^20 / L.  Returns 0, or -1
 * if a coordinate is not finite. */
int orc_domain(const double *pos, int64_t n, double lo[3], double *L, double *scale);

/* Keys of all points in input order; q (optional, [n][3]) receives the integer
 * coordinates. */
void orc_keys(const double *pos, int64_t n, const double lo[3], double scale,
              uint64_t *key, uint32_t *q);

/* Stable ascending argsort of keys: perm[i] is the input index of the i-th
 * smallest key; equal keys keep input order (App. A: the split primitive keeps
 * order, so the radix sort built from it is stable). */
int orc_argsort(const uint64_t *key, int64_t n, int64_t *perm);

typedef struct orc_tree orc_tree;

/* Build keys, sorted order, the level-by-level cell array (Sect. 2.1), links,
 * groups (Sect. 2.2) and float64 multipole moments (Sect. 3.2).
 * nleaf >= 1, ncrit >= 1.  Returns NULL on bad arguments or allocation failure. */
orc_tree *orc_build(const double *pos, const double *mass, int64_t n, int nleaf, int ncrit);
void orc_free(orc_tree *t);

/* Multipole-only update (Sect. 5): keep the tree's cells, groups, keys and
 * domain; take new positions (input order, [n][3]) and recompute every cell's
 * moments and every group's box from them.  A cell whose particles all still lie
 * in its key cell (inside the build's bounding box, with the cell's key prefix
 * under the build's integer map) keeps the build's geometry for the opening
 * tests; any other cell takes the tight box of its particles (centre, and side
 * max(L 2^-level, largest extent)), so that the cube of the tests holds every
 * particle of the cell.  Returns 0, or -1 for a non-finite coordinate (the tree
 * is then unchanged) or a null argument. */
int orc_refit(orc_tree *t, const double *pos);

int64_t orc_n(const orc_tree *t);
int64_t orc_ncells(const orc_tree *t);
int64_t orc_ngroups(const orc_tree *t);
int     orc_depth(const orc_tree *t);   /* deepest level that holds a cell */

void orc_get_domain(const orc_tree *t, double lo[3], double *L, double *scale);
/* perm[i] = input index of sorted particle i; key[i] its key. */
void orc_get_order(const orc_tree *t, int64_t *perm, uint64_t *key);
/* Cell table in (level, key prefix) order.  For a node, child/nchild give its
 * contiguous children; for a leaf child = -1, nchild = 0.  parent = -1 at the
 * root.  first/count give the contiguous range of sorted particles. */
void orc_get_cells(const orc_tree *t, uint8_t *level, uint64_t *prefix,
                   int64_t *first, int64_t *count, uint8_t *is_leaf,
                   int64_t *parent, int64_t *child, int32_t *nchild);
/* Groups ordered by first particle; centre = float64 box centre, half = float32
 * box half-size (tight box of the group's particles). */
void orc_get_groups(const orc_tree *t, int64_t *gfirst, int64_t *gcount,
                    double *centre, float *half);
/* Per-cell mass, centre of mass [c][3] and second moment about the centre of
 * mass S [c][6] = xx, yy, zz, xy, xz, yz. */
void orc_get_moments(const orc_tree *t, double *mass, double *com, double *S);

/* Opening test used by the walk functions below: 0 (the default) Eq. (1), 1 the
 * minimum-distance test named in Sect. 3.3 as the alternative. */
void orc_set_mac(orc_tree *t, int mac);
int orc_get_mac(const orc_tree *t);

/* Opening radius of the tree's test.  Eq. (1): r_crit = l / theta + delta, with
 * l = L 2^-level the cell side and delta the distance between the geometric
 * centre and the centre of mass; minimum distance: r_crit = l / theta.  Outputs
 * (each optional): rcrit2[c] = (float)(r_crit^2), centre [c][3] = the cell's
 * centre (geometric after a build; see orc_refit after a refit). */
void orc_rcrit(const orc_tree *t, float theta, float *rcrit2, double *centre);

/* Opening test of Eq. (1) between group g and cell c, given rcrit2 of the cell.
 * Returns 1 if the cell is accepted (its multipole is used), 0 if it is opened. */
int orc_mac_accept(const orc_tree *t, int64_t g, int64_t c, float rcrit2_c);

/* Minimum-distance test between group g and cell c: the smallest distance from
 * the group's box to the cell's cube must exceed l / theta (rmin2_c =
 * (float)((l / theta)^2)).  Returns 1 if the cell is accepted. */
int orc_mac_accept_min(const orc_tree *t, int64_t g, int64_t c, float rmin2_c);

/* Interaction counts per group for opening angle theta (Sect. 2.2): npp = number
 * of particles in opened leaves (the group's own included), npc = number of
 * accepted cells.  Returns 0 or a negative status. */
int orc_walk_counts(const orc_tree *t, float theta, int64_t *npp, int64_t *npc);

/* Interaction lists of one group: the accepted cells (pc, ascending) and the
 * opened leaves (pp_leaves, ascending).  Capacities are in entries; the
 * function returns the number of accepted cells and stores the number of opened
 * leaves in *npp_leaves; -1 if a capacity is too small. */
int64_t orc_group_lists(const orc_tree *t, float theta, int64_t g,
                        int64_t *pc, int64_t pc_cap,
                        int64_t *pp_leaves, int64_t pp_cap, int64_t *npp_leaves);

/* Barnes-Hut accelerations and potentials in float64 for the groups listed in
 * groups[0..ng) (all groups if groups == NULL).  Outputs are in input order and
 * only written for particles of the selected groups: acc [n][3], pot [n];
 * absacc[i] = sum over interactions of |a_ij|, abspot[i] = sum of |phi_ij|
 * (both optional).  G = 1.  Pairs whose softened distance is zero (a particle
 * with itself, or coincident particles when eps = 0) contribute nothing. */
int orc_forces(const orc_tree *t, float theta, float eps,
               const int64_t *groups, int64_t ng,
               double *acc, double *pot, double *absacc, double *abspot);

/* Direct summation for the targets tgt[0..nt) (input indices); outputs are
 * [nt][3] and [nt] in target order.  Same pair rule as orc_forces. */
void orc_direct(const double *pos, const double *mass, int64_t n, float eps,
                const int64_t *tgt, int64_t nt, double *acc, double *pot);

/* One kick-drift-kick step (Sect. 3.1) of the Barnes-Hut system in input order:
 * v += a dt/2; x += v dt; rebuild; new a, phi; v += a dt/2.  acc/pot hold the
 * forces at the incoming positions and are overwritten with the new ones. */
int orc_kdk_step(double *pos, double *vel, const double *mass, int64_t n,
                 double *acc, double *pot, double dt, float theta, float eps,
                 int nleaf, int ncrit);

/* Block time-steps.  Bin of each particle from its float32 acceleration
 * acc [n][3]: the smallest b in [0, max_level] with dt_max 2^-b <= sqrt(2 eta
 * length / |a|), decided as (dt_max 2^-b)^4 |a|^2 <= (2 eta length)^2 in
 * float64 (max_level if none). */
void orc_block_bins(const float *acc, int64_t n, double dt_max, int max_level, double eta,
                    double length, uint8_t *bins);

/* A system advanced by block steps: the arrays are the caller's (caller order)
 * and are updated in place; creation builds the tree and fills acc, pot. */
typedef struct orc_block orc_block;
orc_block *orc_block_new(double *pos, double *vel, const double *mass, int64_t n, double *acc,
                         double *pot, float theta, float eps, int nleaf, int ncrit, int mac);
void orc_block_free(orc_block *b);
/* mean over the particles of their base: the interaction count of the group
 * that held them in the last walk covering them on a freshly built tree */
double orc_block_base(const orc_block *b);
/* 1 if the next force evaluation will be on a rebuilt tree */
int orc_block_rebuild_next(const orc_block *b);
/* One block step of dt_max with the given bins (caller order): 2^max_level
 * substeps; see bh_oracle.c for the schedule and the rebuild rule.  *rebuilt:
 * the number of rebuilds during the step; *sync_inter: interactions per
 * particle of the final walk (every group); kicks (optional, [n]): steps
 * completed per particle. */
int orc_block_step(orc_block *b, const uint8_t *bins, int max_level, double dt_max,
                   double growth, int *rebuilt, double *sync_inter, int64_t *kicks);

/* out = {T, W, E, Px, Py, Pz}: kinetic energy, potential energy (half the
 * mass-weighted sum of phi), their sum, and the linear momentum. */
void orc_energy(const double *vel, const double *mass, const double *pot, int64_t n,
                double out[6]);

#ifdef __cplusplus
}
#endif
#endif
