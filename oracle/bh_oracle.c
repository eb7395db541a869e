/*
 * bh_oracle.c - CPU oracle for the sparse-octree Barnes-Hut tree-code of Bedorf,
 * Gaburov & Portegies Zwart (arXiv:1106.1900).  TEST INFRASTRUCTURE ONLY; see
 * bh_oracle.h for the contract.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math (no fused multiply-add,
 * no reassociation).  Every loop below runs in the order written.
 */
#include "bh_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define QMAX 1048575u            /* 2^20 - 1 */
#define QSPAN 1048576.0          /* 2^20 */

struct orc_tree {
    int64_t n;
    int nleaf, ncrit;
    double lo[3], L, scale;
    double hi[3];       /* per-axis maximum of the build's positions */
    /* particles in sorted order */
    int64_t *perm;
    uint64_t *key;
    uint32_t *q;        /* [n][3] */
    double *x;          /* [n][3] */
    double *m;          /* [n] */
    /* cells */
    int64_t ncells, cap;
    uint8_t *level;
    uint64_t *prefix;
    int64_t *first, *count, *parent, *child;
    uint8_t *leaf;
    int32_t *nchild;
    double *M, *com, *S; /* [c], [c][3], [c][6] */
    double *side;        /* [c] side l of the opening test: L 2^-level after a build;
                            after a refit see orc_refit */
    double *cen;         /* [c][3] centre of the opening test: the geometric centre
                            after a build; after a refit see orc_refit */
    /* groups */
    int64_t ngroups;
    int64_t *gfirst, *gcount;
    double *gc;         /* [g][3] */
    float *gh;          /* [g][3] */
    int depth;
    int mac;            /* opening test: 0 Eq. (1), 1 minimum distance */
};

/* ------------------------------------------------------------------------- */
/* App. B: integer coordinates and Morton keys.                              */

uint64_t orc_interleave(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint64_t k = 0;
    for (int b = 0; b < ORC_MAX_LEVEL; ++b) {
        k |= (uint64_t)((qx >> b) & 1u) << (3 * b);
        k |= (uint64_t)((qy >> b) & 1u) << (3 * b + 1);
        k |= (uint64_t)((qz >> b) & 1u) << (3 * b + 2);
    }
    return k;
}

int orc_domain(const double *pos, int64_t n, double lo[3], double *L, double *scale)
{
    double hi[3];
    for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            double v = pos[3 * i + k];
            if (!isfinite(v)) return -1;
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    double side = 0.0;
    for (int k = 0; k < 3; ++k) {
        double e = hi[k] - lo[k];
        if (e > side) side = e;
    }
    if (side == 0.0) side = 1.0;
    *L = side;
    *scale = QSPAN / side;
    return 0;
}

static uint32_t coord_to_int(double x, double lo, double scale)
{
    double d = x - lo;
    double f = d * scale;
    if (f >= (double)QMAX) return QMAX;
    return (uint32_t)floor(f);
}

void orc_keys(const double *pos, int64_t n, const double lo[3], double scale,
              uint64_t *key, uint32_t *q)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t c[3];
        for (int k = 0; k < 3; ++k) c[k] = coord_to_int(pos[3 * i + k], lo[k], scale);
        key[i] = orc_interleave(c[0], c[1], c[2]);
        if (q) { q[3 * i] = c[0]; q[3 * i + 1] = c[1]; q[3 * i + 2] = c[2]; }
    }
}

/* Stable merge sort of indices by key. */
int orc_argsort(const uint64_t *key, int64_t n, int64_t *perm)
{
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!tmp) return -2;
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    int64_t *src = perm, *dst = tmp;
    for (int64_t w = 1; w < n; w *= 2) {
        for (int64_t s = 0; s < n; s += 2 * w) {
            int64_t a = s, am = s + w < n ? s + w : n;
            int64_t b = am, bm = s + 2 * w < n ? s + 2 * w : n;
            int64_t o = s;
            while (a < am && b < bm) {
                /* take from the left run on ties: keeps input order */
                if (key[src[b]] < key[src[a]]) dst[o++] = src[b++];
                else dst[o++] = src[a++];
            }
            while (a < am) dst[o++] = src[a++];
            while (b < bm) dst[o++] = src[b++];
        }
        int64_t *t = src; src = dst; dst = t;
    }
    if (src != perm) memcpy(perm, src, sizeof(int64_t) * (size_t)n);
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sect. 2.1: level-by-level cell construction and linking.                  */

static int grow_cells(orc_tree *t)
{
    int64_t cap = t->cap ? 2 * t->cap : 64;
#define GROW(field, type) do {                                        \
        type *p = (type *)realloc(t->field, sizeof(type) * (size_t)cap);  \
        if (!p) return -2;                                                \
        t->field = p;                                                     \
    } while (0)
    GROW(level, uint8_t);
    GROW(prefix, uint64_t);
    GROW(first, int64_t);
    GROW(count, int64_t);
    GROW(parent, int64_t);
    GROW(child, int64_t);
    GROW(leaf, uint8_t);
    GROW(nchild, int32_t);
#undef GROW
    t->cap = cap;
    return 0;
}

static int64_t add_cell(orc_tree *t, int lev, uint64_t prefix, int64_t first,
                        int64_t count, int64_t parent)
{
    if (t->ncells == t->cap && grow_cells(t)) return -1;
    int64_t c = t->ncells++;
    t->level[c] = (uint8_t)lev;
    t->prefix[c] = prefix;
    t->first[c] = first;
    t->count[c] = count;
    t->parent[c] = parent;
    t->leaf[c] = (uint8_t)(count <= t->nleaf || lev == ORC_MAX_LEVEL);
    t->child[c] = -1;
    t->nchild[c] = 0;
    return c;
}

/* Open nodes of level l-1 are split, in array order, into maximal runs of equal
 * level-l key prefix; each run becomes a child cell, leaf if it holds at most
 * nleaf particles or sits at the deepest level (the key has no more bits). */
static int build_cells(orc_tree *t)
{
    int64_t n = t->n;
    int64_t *open = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!open || !next) { free(open); free(next); return -2; }
    int64_t nopen = 0;
    if (add_cell(t, 0, 0, 0, n, -1) < 0) { free(open); free(next); return -2; }
    if (!t->leaf[0]) open[nopen++] = 0;
    t->depth = 0;
    for (int l = 1; l <= ORC_MAX_LEVEL && nopen > 0; ++l) {
        int shift = 3 * (ORC_MAX_LEVEL - l);
        int64_t nnext = 0;
        for (int64_t k = 0; k < nopen; ++k) {
            int64_t node = open[k];
            int64_t s = t->first[node], e = s + t->count[node];
            int64_t c0 = t->ncells;
            int64_t i = s;
            while (i < e) {
                uint64_t p = t->key[i] >> shift;
                int64_t j = i + 1;
                while (j < e && (t->key[j] >> shift) == p) ++j;
                int64_t c = add_cell(t, l, p, i, j - i, node);
                if (c < 0) { free(open); free(next); return -2; }
                if (!t->leaf[c]) next[nnext++] = c;
                i = j;
            }
            t->child[node] = c0;
            t->nchild[node] = (int32_t)(t->ncells - c0);
        }
        t->depth = l;
        int64_t *sw = open; open = next; next = sw;
        nopen = nnext;
    }
    free(open);
    free(next);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Sect. 2.2: groups.  A cell is a group if it holds at most ncrit particles   */
/* and its parent holds more (or it is the root); a leaf that still holds more */
/* than ncrit particles is cut into runs of ncrit consecutive particles.       */

static void group_boxes(orc_tree *t);

static int build_groups(orc_tree *t)
{
    int64_t n = t->n;
    uint8_t *start = (uint8_t *)calloc((size_t)n + 1, 1);
    if (!start) return -2;
    for (int64_t c = 0; c < t->ncells; ++c) {
        int64_t cnt = t->count[c];
        int top = (c == 0) || (t->count[t->parent[c]] > t->ncrit);
        if (cnt <= t->ncrit && top) start[t->first[c]] = 1;
        else if (t->leaf[c] && cnt > t->ncrit) {
            for (int64_t o = 0; o < cnt; o += t->ncrit) start[t->first[c] + o] = 1;
        }
    }
    int64_t ng = 0;
    for (int64_t i = 0; i < n; ++i) ng += start[i];
    t->ngroups = ng;
    t->gfirst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ng + 1));
    t->gcount = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ng + 1));
    t->gc = (double *)malloc(sizeof(double) * 3 * (size_t)(ng + 1));
    t->gh = (float *)malloc(sizeof(float) * 3 * (size_t)(ng + 1));
    if (!t->gfirst || !t->gcount || !t->gc || !t->gh) { free(start); return -2; }
    int64_t g = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (start[i]) { ++g; t->gfirst[g] = i; t->gcount[g] = 0; }
        t->gcount[g] += 1;
    }
    free(start);
    group_boxes(t);
    return 0;
}

/* Tight float64 box of each group's particles: centre, float32 half-size. */
static void group_boxes(orc_tree *t)
{
    for (int64_t g = 0; g < t->ngroups; ++g) {
        double bmin[3], bmax[3];
        for (int k = 0; k < 3; ++k) { bmin[k] = INFINITY; bmax[k] = -INFINITY; }
        for (int64_t i = t->gfirst[g]; i < t->gfirst[g] + t->gcount[g]; ++i)
            for (int k = 0; k < 3; ++k) {
                double v = t->x[3 * i + k];
                if (v < bmin[k]) bmin[k] = v;
                if (v > bmax[k]) bmax[k] = v;
            }
        for (int k = 0; k < 3; ++k) {
            t->gc[3 * g + k] = 0.5 * (bmin[k] + bmax[k]);
            t->gh[3 * g + k] = (float)(0.5 * (bmax[k] - bmin[k]));
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Sect. 3.2: monopole and quadrupole moments in float64, leaves from their    */
/* particles, nodes from their children, deepest cells first.                  */

static void build_moments(orc_tree *t)
{
    for (int64_t c = t->ncells - 1; c >= 0; --c) {
        double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
        double *com = t->com + 3 * c, *S = t->S + 6 * c;
        if (t->leaf[c]) {
            int64_t s = t->first[c], e = s + t->count[c];
            for (int64_t j = s; j < e; ++j) M = M + t->m[j];
            for (int64_t j = s; j < e; ++j) {
                sx = sx + t->m[j] * t->x[3 * j];
                sy = sy + t->m[j] * t->x[3 * j + 1];
                sz = sz + t->m[j] * t->x[3 * j + 2];
            }
            com[0] = sx / M; com[1] = sy / M; com[2] = sz / M;
            for (int a = 0; a < 6; ++a) S[a] = 0.0;
            for (int64_t j = s; j < e; ++j) {
                double dx = t->x[3 * j] - com[0];
                double dy = t->x[3 * j + 1] - com[1];
                double dz = t->x[3 * j + 2] - com[2];
                double mj = t->m[j];
                S[0] += mj * dx * dx; S[1] += mj * dy * dy; S[2] += mj * dz * dz;
                S[3] += mj * dx * dy; S[4] += mj * dx * dz; S[5] += mj * dy * dz;
            }
        } else {
            int64_t s = t->child[c], e = s + t->nchild[c];
            for (int64_t k = s; k < e; ++k) M = M + t->M[k];
            for (int64_t k = s; k < e; ++k) {
                sx = sx + t->M[k] * t->com[3 * k];
                sy = sy + t->M[k] * t->com[3 * k + 1];
                sz = sz + t->M[k] * t->com[3 * k + 2];
            }
            com[0] = sx / M; com[1] = sy / M; com[2] = sz / M;
            for (int a = 0; a < 6; ++a) S[a] = 0.0;
            for (int64_t k = s; k < e; ++k) {
                double ex = t->com[3 * k] - com[0];
                double ey = t->com[3 * k + 1] - com[1];
                double ez = t->com[3 * k + 2] - com[2];
                double Mk = t->M[k];
                const double *Sk = t->S + 6 * k;
                S[0] += Sk[0] + Mk * ex * ex; S[1] += Sk[1] + Mk * ey * ey;
                S[2] += Sk[2] + Mk * ez * ez; S[3] += Sk[3] + Mk * ex * ey;
                S[4] += Sk[4] + Mk * ex * ez; S[5] += Sk[5] + Mk * ey * ez;
            }
        }
        t->M[c] = M;
    }
}

/* ------------------------------------------------------------------------- */

static double cell_geometry(const orc_tree *t, int64_t c, double g[3]);

void orc_free(orc_tree *t)
{
    if (!t) return;
    free(t->perm); free(t->key); free(t->q); free(t->x); free(t->m);
    free(t->level); free(t->prefix); free(t->first); free(t->count);
    free(t->parent); free(t->child); free(t->leaf); free(t->nchild);
    free(t->M); free(t->com); free(t->S); free(t->side); free(t->cen);
    free(t->gfirst); free(t->gcount); free(t->gc); free(t->gh);
    free(t);
}

orc_tree *orc_build(const double *pos, const double *mass, int64_t n, int nleaf, int ncrit)
{
    if (!pos || !mass || n < 1 || nleaf < 1 || ncrit < 1) return NULL;
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    if (!t) return NULL;
    t->n = n; t->nleaf = nleaf; t->ncrit = ncrit;
    if (orc_domain(pos, n, t->lo, &t->L, &t->scale)) { orc_free(t); return NULL; }
    for (int k = 0; k < 3; ++k) {
        t->hi[k] = -INFINITY;
        for (int64_t i = 0; i < n; ++i)
            if (pos[3 * i + k] > t->hi[k]) t->hi[k] = pos[3 * i + k];
    }
    uint64_t *key_in = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    uint32_t *q_in = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)n);
    t->perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    t->key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    t->q = (uint32_t *)malloc(sizeof(uint32_t) * 3 * (size_t)n);
    t->x = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    t->m = (double *)malloc(sizeof(double) * (size_t)n);
    if (!key_in || !q_in || !t->perm || !t->key || !t->q || !t->x || !t->m) goto fail;
    orc_keys(pos, n, t->lo, t->scale, key_in, q_in);
    if (orc_argsort(key_in, n, t->perm)) goto fail;
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = t->perm[i];
        t->key[i] = key_in[p];
        t->m[i] = mass[p];
        for (int k = 0; k < 3; ++k) {
            t->q[3 * i + k] = q_in[3 * p + k];
            t->x[3 * i + k] = pos[3 * p + k];
        }
    }
    free(key_in); key_in = NULL;
    free(q_in); q_in = NULL;
    if (build_cells(t)) goto fail;
    t->M = (double *)malloc(sizeof(double) * (size_t)t->ncells);
    t->com = (double *)malloc(sizeof(double) * 3 * (size_t)t->ncells);
    t->S = (double *)malloc(sizeof(double) * 6 * (size_t)t->ncells);
    t->side = (double *)malloc(sizeof(double) * (size_t)t->ncells);
    t->cen = (double *)malloc(sizeof(double) * 3 * (size_t)t->ncells);
    if (!t->M || !t->com || !t->S || !t->side || !t->cen) goto fail;
    for (int64_t c = 0; c < t->ncells; ++c) t->side[c] = cell_geometry(t, c, t->cen + 3 * c);
    build_moments(t);
    if (build_groups(t)) goto fail;
    return t;
fail:
    free(key_in);
    free(q_in);
    orc_free(t);
    return NULL;
}

/* Sect. 5: between rebuilds it suffices to recompute the multipole moments of
 * the cells whose particles moved.  The cells, groups, keys and domain of the
 * build stay; the particles take the new positions (input order) and every
 * cell's moments and every group's box are recomputed from them.  The paper
 * names the growth of the cell size l as what makes the walk of a refitted
 * tree slower.  Both opening tests rely on the cube of side l about the centre
 * of Eq. (1) holding every particle of the cell, so the refit keeps that true:
 * a cell whose particles all still lie in its key cell (inside the build's
 * bounding box, with the cell's key prefix under the build's integer map)
 * keeps the build's geometry; any other cell takes the tight box of its
 * particles, centre 0.5 (lo + hi) per axis and side the larger of L 2^-level
 * and the box's largest extent. */
int orc_refit(orc_tree *t, const double *pos)
{
    if (!t || !pos) return -1;
    for (int64_t i = 0; i < 3 * t->n; ++i)
        if (!isfinite(pos[i])) return -1;
    for (int64_t i = 0; i < t->n; ++i) {
        int64_t p = t->perm[i];
        for (int k = 0; k < 3; ++k) t->x[3 * i + k] = pos[3 * p + k];
    }
    build_moments(t);
    group_boxes(t);
    for (int64_t c = 0; c < t->ncells; ++c) {
        int lev = t->level[c];
        int shift = ORC_MAX_LEVEL - lev;
        double blo[3], bhi[3];
        int inside = 1;
        for (int k = 0; k < 3; ++k) {
            uint32_t cell_k = t->q[3 * t->first[c] + k] >> shift;
            blo[k] = INFINITY;
            bhi[k] = -INFINITY;
            for (int64_t j = t->first[c]; j < t->first[c] + t->count[c]; ++j) {
                double x = t->x[3 * j + k];
                blo[k] = x < blo[k] ? x : blo[k];
                bhi[k] = x > bhi[k] ? x : bhi[k];
                if (!(x >= t->lo[k] && x <= t->hi[k]) ||
                    (coord_to_int(x, t->lo[k], t->scale) >> shift) != cell_k)
                    inside = 0;
            }
        }
        double l = cell_geometry(t, c, t->cen + 3 * c);
        if (inside) {
            t->side[c] = l;
        } else {
            double ext = 0.0;
            for (int k = 0; k < 3; ++k) {
                ext = bhi[k] - blo[k] > ext ? bhi[k] - blo[k] : ext;
                t->cen[3 * c + k] = 0.5 * (blo[k] + bhi[k]);
            }
            t->side[c] = ext > l ? ext : l;
        }
    }
    return 0;
}

int64_t orc_n(const orc_tree *t) { return t->n; }
int64_t orc_ncells(const orc_tree *t) { return t->ncells; }
int64_t orc_ngroups(const orc_tree *t) { return t->ngroups; }
int orc_depth(const orc_tree *t) { return t->depth; }

void orc_get_domain(const orc_tree *t, double lo[3], double *L, double *scale)
{
    for (int k = 0; k < 3; ++k) lo[k] = t->lo[k];
    *L = t->L;
    *scale = t->scale;
}

void orc_get_order(const orc_tree *t, int64_t *perm, uint64_t *key)
{
    if (perm) memcpy(perm, t->perm, sizeof(int64_t) * (size_t)t->n);
    if (key) memcpy(key, t->key, sizeof(uint64_t) * (size_t)t->n);
}

void orc_get_cells(const orc_tree *t, uint8_t *level, uint64_t *prefix,
                   int64_t *first, int64_t *count, uint8_t *is_leaf,
                   int64_t *parent, int64_t *child, int32_t *nchild)
{
    size_t c = (size_t)t->ncells;
    if (level) memcpy(level, t->level, c);
    if (prefix) memcpy(prefix, t->prefix, 8 * c);
    if (first) memcpy(first, t->first, 8 * c);
    if (count) memcpy(count, t->count, 8 * c);
    if (is_leaf) memcpy(is_leaf, t->leaf, c);
    if (parent) memcpy(parent, t->parent, 8 * c);
    if (child) memcpy(child, t->child, 8 * c);
    if (nchild) memcpy(nchild, t->nchild, 4 * c);
}

void orc_get_groups(const orc_tree *t, int64_t *gfirst, int64_t *gcount,
                    double *centre, float *half)
{
    size_t g = (size_t)t->ngroups;
    if (gfirst) memcpy(gfirst, t->gfirst, 8 * g);
    if (gcount) memcpy(gcount, t->gcount, 8 * g);
    if (centre) memcpy(centre, t->gc, 24 * g);
    if (half) memcpy(half, t->gh, 12 * g);
}

void orc_get_moments(const orc_tree *t, double *mass, double *com, double *S)
{
    size_t c = (size_t)t->ncells;
    if (mass) memcpy(mass, t->M, 8 * c);
    if (com) memcpy(com, t->com, 24 * c);
    if (S) memcpy(S, t->S, 48 * c);
}

/* ------------------------------------------------------------------------- */
/* Sect. 3.3, Eq. (1): d > l/theta + delta.                                    */

void orc_set_mac(orc_tree *t, int mac) { t->mac = mac ? 1 : 0; }

int orc_get_mac(const orc_tree *t) { return t->mac; }

/* Geometric centre of cell c (from the key prefix of any of its particles) and
 * its side l. */
static double cell_geometry(const orc_tree *t, int64_t c, double g[3])
{
    int lev = t->level[c];
    double l = ldexp(t->L, -lev);
    const uint32_t *q = t->q + 3 * t->first[c];
    for (int k = 0; k < 3; ++k) {
        uint32_t p = q[k] >> (ORC_MAX_LEVEL - lev);
        g[k] = t->lo[k] + ((double)p + 0.5) * l;
    }
    return l;
}

void orc_rcrit(const orc_tree *t, float theta, float *rcrit2, double *centre)
{
    for (int64_t c = 0; c < t->ncells; ++c) {
        const double *g = t->cen + 3 * c;
        double l = t->side[c];
        double r;
        if (t->mac) {
            /* minimum-distance test: the cell's cube must lie beyond l / theta */
            r = l / (double)theta;
        } else {
            double dx = t->com[3 * c] - g[0];
            double dy = t->com[3 * c + 1] - g[1];
            double dz = t->com[3 * c + 2] - g[2];
            double delta = sqrt((dx * dx + dy * dy) + dz * dz);
            r = l / (double)theta + delta;
        }
        if (rcrit2) rcrit2[c] = (float)(r * r);
        if (centre) { centre[3 * c] = g[0]; centre[3 * c + 1] = g[1]; centre[3 * c + 2] = g[2]; }
    }
}

/* d is the distance from the cell's centre of mass to the group's box, taken in
 * float32 on offsets from the group centre; accept when d^2 > r_crit^2. */
int orc_mac_accept(const orc_tree *t, int64_t g, int64_t c, float rcrit2_c)
{
    float u[3];
    for (int k = 0; k < 3; ++k) {
        float o = (float)(t->com[3 * c + k] - t->gc[3 * g + k]);
        float d = fabsf(o) - t->gh[3 * g + k];
        u[k] = d > 0.0f ? d : 0.0f;
    }
    float d2 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    return d2 > rcrit2_c;
}

/* Minimum-distance test (Salmon & Warren 1994, named in Sect. 3.3 as the
 * alternative): d is the smallest distance between the group's box and the
 * cell's cube (side l about its centre: the geometric centre of a built cell,
 * see orc_refit for a refitted one), taken in float32 on offsets from the group
 * centre with the cube's half side (float)(l / 2); accept when
 * d^2 > rmin2_c = (float)((l / theta)^2). */
int orc_mac_accept_min(const orc_tree *t, int64_t g, int64_t c, float rmin2_c)
{
    const double *gcen = t->cen + 3 * c;
    float h = (float)(0.5 * t->side[c]);
    float u[3];
    for (int k = 0; k < 3; ++k) {
        float o = (float)(gcen[k] - t->gc[3 * g + k]);
        float d = (fabsf(o) - t->gh[3 * g + k]) - h;
        u[k] = d > 0.0f ? d : 0.0f;
    }
    float d2 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    return d2 > rmin2_c;
}

static int accept(const orc_tree *t, int64_t g, int64_t c, float rc2_c)
{
    return t->mac ? orc_mac_accept_min(t, g, c, rc2_c) : orc_mac_accept(t, g, c, rc2_c);
}

/* ------------------------------------------------------------------------- */
/* Sect. 2.2: breadth-first walk of one group.                                 */

typedef struct { int64_t *v; int64_t n, cap; } ivec;

static int ivec_push(ivec *a, int64_t x)
{
    if (a->n == a->cap) {
        int64_t cap = a->cap ? 2 * a->cap : 256;
        int64_t *p = (int64_t *)realloc(a->v, sizeof(int64_t) * (size_t)cap);
        if (!p) return -1;
        a->v = p; a->cap = cap;
    }
    a->v[a->n++] = x;
    return 0;
}

/* Fills pc (accepted cells) and ppl (opened leaves) for group g. */
static int walk_group(const orc_tree *t, const float *rc2, int64_t g, ivec *pc, ivec *ppl,
                      ivec *cur, ivec *nxt)
{
    pc->n = 0; ppl->n = 0; cur->n = 0; nxt->n = 0;
    if (ivec_push(cur, 0)) return -2;
    while (cur->n > 0) {
        nxt->n = 0;
        for (int64_t k = 0; k < cur->n; ++k) {
            int64_t c = cur->v[k];
            if (accept(t, g, c, rc2[c])) {
                if (ivec_push(pc, c)) return -2;
            } else if (t->leaf[c]) {
                if (ivec_push(ppl, c)) return -2;
            } else {
                for (int64_t ch = t->child[c]; ch < t->child[c] + t->nchild[c]; ++ch)
                    if (ivec_push(nxt, ch)) return -2;
            }
        }
        ivec sw = *cur; *cur = *nxt; *nxt = sw;
    }
    return 0;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

int orc_walk_counts(const orc_tree *t, float theta, int64_t *npp, int64_t *npc)
{
    float *rc2 = (float *)malloc(sizeof(float) * (size_t)t->ncells);
    if (!rc2) return -2;
    orc_rcrit(t, theta, rc2, NULL);
    ivec pc = {0}, ppl = {0}, cur = {0}, nxt = {0};
    int st = 0;
    for (int64_t g = 0; g < t->ngroups && !st; ++g) {
        st = walk_group(t, rc2, g, &pc, &ppl, &cur, &nxt);
        int64_t s = 0;
        for (int64_t k = 0; k < ppl.n; ++k) s += t->count[ppl.v[k]];
        npp[g] = s;
        npc[g] = pc.n;
    }
    free(pc.v); free(ppl.v); free(cur.v); free(nxt.v); free(rc2);
    return st;
}

int64_t orc_group_lists(const orc_tree *t, float theta, int64_t g,
                        int64_t *pc_out, int64_t pc_cap,
                        int64_t *pp_out, int64_t pp_cap, int64_t *npp_leaves)
{
    if (g < 0 || g >= t->ngroups) return -1;
    float *rc2 = (float *)malloc(sizeof(float) * (size_t)t->ncells);
    if (!rc2) return -2;
    orc_rcrit(t, theta, rc2, NULL);
    ivec pc = {0}, ppl = {0}, cur = {0}, nxt = {0};
    int64_t ret = walk_group(t, rc2, g, &pc, &ppl, &cur, &nxt);
    if (ret == 0) {
        if (pc.n > pc_cap || ppl.n > pp_cap) ret = -1;
        else {
            qsort(pc.v, (size_t)pc.n, sizeof(int64_t), cmp_i64);
            qsort(ppl.v, (size_t)ppl.n, sizeof(int64_t), cmp_i64);
            memcpy(pc_out, pc.v, sizeof(int64_t) * (size_t)pc.n);
            memcpy(pp_out, ppl.v, sizeof(int64_t) * (size_t)ppl.n);
            *npp_leaves = ppl.n;
            ret = pc.n;
        }
    }
    free(pc.v); free(ppl.v); free(cur.v); free(nxt.v); free(rc2);
    return ret;
}

/* ------------------------------------------------------------------------- */
/* Force evaluation in float64.                                                */

/* Particle j on particle i: a += m r s^(-3/2), phi -= m s^(-1/2), r = x_j - x_i,
 * s = |r|^2 + eps^2 (Plummer softening). */
static void pp_term(const double *xi, const double *xj, double mj, double eps2,
                    double a[3], double *phi, double *aabs, double *pabs)
{
    double rx = xj[0] - xi[0], ry = xj[1] - xi[1], rz = xj[2] - xi[2];
    double s = ((rx * rx + ry * ry) + rz * rz) + eps2;
    if (s == 0.0) return;
    double rinv = 1.0 / sqrt(s);
    double f = mj * rinv * rinv * rinv;
    a[0] += f * rx; a[1] += f * ry; a[2] += f * rz;
    *phi -= mj * rinv;
    *aabs += f * sqrt((rx * rx + ry * ry) + rz * rz);
    *pabs += mj * rinv;
}

/* Cell (mass M, centre of mass com, second moment S about com) on particle i,
 * monopole plus quadrupole with Plummer-softened inverse distance rho:
 *   phi = -M rho - 3/2 (r.S.r) rho^5 + 1/2 tr(S) rho^3
 *   a   = -M rho^3 r + 3 rho^5 S.r + 3/2 tr(S) rho^5 r - 15/2 (r.S.r) rho^7 r
 * with r = x_i - com; a = -grad phi.  Unsoftened this is the traceless
 * quadrupole Q = 3S - tr(S) I of the textbook expansion. */
static void pc_term(const double *xi, const double *com, double M, const double *S,
                    double eps2, double a[3], double *phi, double *aabs, double *pabs)
{
    double rx = xi[0] - com[0], ry = xi[1] - com[1], rz = xi[2] - com[2];
    double s = ((rx * rx + ry * ry) + rz * rz) + eps2;
    if (s == 0.0) return;
    double rho = 1.0 / sqrt(s);
    double rho2 = rho * rho, rho3 = rho2 * rho, rho5 = rho3 * rho2, rho7 = rho5 * rho2;
    double Srx = S[0] * rx + S[3] * ry + S[4] * rz;
    double Sry = S[3] * rx + S[1] * ry + S[5] * rz;
    double Srz = S[4] * rx + S[5] * ry + S[2] * rz;
    double rSr = rx * Srx + ry * Sry + rz * Srz;
    double tr = S[0] + S[1] + S[2];
    double radial = -M * rho3 + 1.5 * tr * rho5 - 7.5 * rSr * rho7;
    double ax = radial * rx + 3.0 * rho5 * Srx;
    double ay = radial * ry + 3.0 * rho5 * Sry;
    double az = radial * rz + 3.0 * rho5 * Srz;
    a[0] += ax; a[1] += ay; a[2] += az;
    double p = -M * rho - 1.5 * rSr * rho5 + 0.5 * tr * rho3;
    *phi += p;
    *aabs += sqrt((ax * ax + ay * ay) + az * az);
    *pabs += fabs(p);
}

int orc_forces(const orc_tree *t, float theta, float eps,
               const int64_t *groups, int64_t ng,
               double *acc, double *pot, double *absacc, double *abspot)
{
    float *rc2 = (float *)malloc(sizeof(float) * (size_t)t->ncells);
    if (!rc2) return -2;
    orc_rcrit(t, theta, rc2, NULL);
    double eps2 = (double)eps * (double)eps;
    ivec pc = {0}, ppl = {0}, cur = {0}, nxt = {0};
    int st = 0;
    int64_t count = groups ? ng : t->ngroups;
    for (int64_t k = 0; k < count && !st; ++k) {
        int64_t g = groups ? groups[k] : k;
        if (g < 0 || g >= t->ngroups) { st = -1; break; }
        st = walk_group(t, rc2, g, &pc, &ppl, &cur, &nxt);
        if (st) break;
        for (int64_t i = t->gfirst[g]; i < t->gfirst[g] + t->gcount[g]; ++i) {
            const double *xi = t->x + 3 * i;
            double a[3] = {0.0, 0.0, 0.0}, phi = 0.0, aabs = 0.0, pabs = 0.0;
            for (int64_t u = 0; u < ppl.n; ++u) {
                int64_t leaf = ppl.v[u];
                for (int64_t j = t->first[leaf]; j < t->first[leaf] + t->count[leaf]; ++j) {
                    if (j == i) continue;
                    pp_term(xi, t->x + 3 * j, t->m[j], eps2, a, &phi, &aabs, &pabs);
                }
            }
            for (int64_t u = 0; u < pc.n; ++u) {
                int64_t c = pc.v[u];
                pc_term(xi, t->com + 3 * c, t->M[c], t->S + 6 * c, eps2, a, &phi, &aabs, &pabs);
            }
            int64_t o = t->perm[i];
            acc[3 * o] = a[0]; acc[3 * o + 1] = a[1]; acc[3 * o + 2] = a[2];
            pot[o] = phi;
            if (absacc) absacc[o] = aabs;
            if (abspot) abspot[o] = pabs;
        }
    }
    free(pc.v); free(ppl.v); free(cur.v); free(nxt.v); free(rc2);
    return st;
}

void orc_direct(const double *pos, const double *mass, int64_t n, float eps,
                const int64_t *tgt, int64_t nt, double *acc, double *pot)
{
    double eps2 = (double)eps * (double)eps;
    for (int64_t k = 0; k < nt; ++k) {
        int64_t i = tgt[k];
        double a[3] = {0.0, 0.0, 0.0}, phi = 0.0, aabs = 0.0, pabs = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            pp_term(pos + 3 * i, pos + 3 * j, mass[j], eps2, a, &phi, &aabs, &pabs);
        }
        acc[3 * k] = a[0]; acc[3 * k + 1] = a[1]; acc[3 * k + 2] = a[2];
        pot[k] = phi;
    }
}

/* ------------------------------------------------------------------------- */
/* Sect. 3.1: leapfrog.  Predicting x with the old acceleration and correcting  */
/* v with the mean of old and new is the same map as kick-drift-kick.           */

int orc_kdk_step(double *pos, double *vel, const double *mass, int64_t n,
                 double *acc, double *pot, double dt, float theta, float eps,
                 int nleaf, int ncrit)
{
    double h = 0.5 * dt;
    for (int64_t i = 0; i < 3 * n; ++i) vel[i] = vel[i] + acc[i] * h;
    for (int64_t i = 0; i < 3 * n; ++i) pos[i] = pos[i] + vel[i] * dt;
    orc_tree *t = orc_build(pos, mass, n, nleaf, ncrit);
    if (!t) return -2;
    int st = orc_forces(t, theta, eps, NULL, 0, acc, pot, NULL, NULL);
    orc_free(t);
    if (st) return st;
    for (int64_t i = 0; i < 3 * n; ++i) vel[i] = vel[i] + acc[i] * h;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Block time-steps (Sect. 5: only the particles due for an update get forces,  */
/* the moments of the existing cells are recomputed in between, and the tree is */
/* rebuilt once the walk has become considerably more expensive).  The paper   */
/* gives neither the time-step criterion nor the schedule; the readings here:   */
/*  - step of particle i: dt_i = sqrt(2 eta l / |a_i|), l a length (the        */
/*    softening), rounded down to a power-of-two fraction dt_max 2^-b of the    */
/*    block step, b in [0, B];                                                  */
/*  - kick-drift-kick per bin: substeps of dt_max 2^-B; a particle of bin b is  */
/*    kicked (half, then half again) at the end of each of its 2^b steps, with  */
/*    forces recomputed for the groups that hold it; at the end of the block    */
/*    step every particle is due.  Every particle drifts before each force      */
/*    evaluation, over the substeps since the previous one (k dt_max 2^-B in    */
/*    one step: no velocity changes in between);                                */
/*  - the cost of a walk: each particle carries the interaction count of its   */
/*    group in the last walk that covered it on a freshly built tree (its       */
/*    base).  A walk on a refitted tree is compared with the base of the        */
/*    particles it covers: more than (1 + growth) times their summed base and   */
/*    the tree is rebuilt, instead of refitted, before the next force           */
/*    evaluation.  growth <= 0: rebuilt before every force evaluation.          */

void orc_block_bins(const float *acc, int64_t n, double dt_max, int max_level, double eta,
                    double length, uint8_t *bins)
{
    /* dt_max 2^-b <= sqrt(2 eta l / |a|)  <=>  (dt_max 2^-b)^4 |a|^2 <= (2 eta l)^2 */
    double k = 2.0 * eta * length;
    k = k * k;
    for (int64_t i = 0; i < n; ++i) {
        double ax = (double)acc[3 * i], ay = (double)acc[3 * i + 1], az = (double)acc[3 * i + 2];
        double a2 = (ax * ax + ay * ay) + az * az;
        int b = 0;
        for (; b < max_level; ++b) {
            double d = ldexp(dt_max, -b);
            double d2 = d * d;
            if ((d2 * d2) * a2 <= k) break;
        }
        bins[i] = (uint8_t)b;
    }
}

struct orc_block {
    orc_tree *t;
    double *pos, *vel, *acc, *pot;   /* caller's arrays, caller order */
    const double *mass;
    int64_t n;
    float theta, eps;
    int nleaf, ncrit, mac;
    int64_t *pbase;                  /* per particle (caller order): its base */
    int rebuild_next;                /* the last walk of a refitted tree grew too much */
};

static int block_rebuild(orc_block *b)
{
    orc_free(b->t);
    b->t = orc_build(b->pos, b->mass, b->n, b->nleaf, b->ncrit);
    if (!b->t) return -2;
    orc_set_mac(b->t, b->mac);
    return 0;
}

/* Forces of the groups gl[0..ng) (every group if gl is NULL), then: on a fresh
 * tree, each covered particle's base becomes its group's interaction count; on
 * a refitted tree, the interactions of the walk (sum over the covered
 * particles) are compared with the covered particles' summed base.  *inter
 * (optional): interactions of the walk per particle of the system. */
static int block_walk(orc_block *b, const int64_t *gl, int64_t ng, int fresh, double growth,
                      double *inter)
{
    const orc_tree *t = b->t;
    int st = orc_forces(t, b->theta, b->eps, gl, ng, b->acc, b->pot, NULL, NULL);
    if (st) return st;
    int64_t *npp = (int64_t *)malloc(sizeof(int64_t) * (size_t)t->ngroups);
    int64_t *npc = (int64_t *)malloc(sizeof(int64_t) * (size_t)t->ngroups);
    if (!npp || !npc) { free(npp); free(npc); return -2; }
    st = orc_walk_counts(t, b->theta, npp, npc);
    int64_t now = 0, base = 0;
    const int64_t cnt = gl ? ng : t->ngroups;
    for (int64_t k = 0; k < cnt && !st; ++k) {
        const int64_t g = gl ? gl[k] : k;
        const int64_t c = npp[g] + npc[g];
        for (int64_t j = t->gfirst[g]; j < t->gfirst[g] + t->gcount[g]; ++j) {
            if (fresh) b->pbase[t->perm[j]] = c;
            else base += b->pbase[t->perm[j]];
        }
        now += t->gcount[g] * c;
    }
    free(npp);
    free(npc);
    b->rebuild_next = !fresh && (double)now > (1.0 + growth) * (double)base;
    if (inter) *inter = (double)now / (double)b->n;
    return st;
}

orc_block *orc_block_new(double *pos, double *vel, const double *mass, int64_t n, double *acc,
                         double *pot, float theta, float eps, int nleaf, int ncrit, int mac)
{
    orc_block *b = (orc_block *)calloc(1, sizeof(orc_block));
    if (!b) return NULL;
    b->pos = pos; b->vel = vel; b->mass = mass; b->acc = acc; b->pot = pot; b->n = n;
    b->theta = theta; b->eps = eps; b->nleaf = nleaf; b->ncrit = ncrit; b->mac = mac;
    b->pbase = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!b->pbase || block_rebuild(b) || block_walk(b, NULL, 0, 1, 0.0, NULL)) {
        orc_block_free(b);
        return NULL;
    }
    return b;
}

void orc_block_free(orc_block *b)
{
    if (!b) return;
    orc_free(b->t);
    free(b->pbase);
    free(b);
}

double orc_block_base(const orc_block *b)
{
    int64_t s = 0;
    for (int64_t i = 0; i < b->n; ++i) s += b->pbase[i];
    return (double)s / (double)b->n;
}

int orc_block_rebuild_next(const orc_block *b) { return b->rebuild_next; }

int orc_block_step(orc_block *b, const uint8_t *bins, int max_level, double dt_max,
                   double growth, int *rebuilt, double *sync_inter, int64_t *kicks)
{
    const int64_t n = b->n;
    if (max_level < 0 || max_level > 30) return -1;
    const int64_t S = (int64_t)1 << max_level;
    const double dtm = ldexp(dt_max, -max_level);
    for (int64_t i = 0; i < n; ++i)
        if (bins[i] > max_level) return -1;
    if (kicks) memset(kicks, 0, sizeof(int64_t) * (size_t)n);
    /* opening half kick of every particle's first step */
    for (int64_t i = 0; i < n; ++i) {
        double h = 0.5 * ldexp(dt_max, -bins[i]);
        for (int k = 0; k < 3; ++k) b->vel[3 * i + k] = b->vel[3 * i + k] + b->acc[3 * i + k] * h;
    }
    int64_t *gl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    uint8_t *due = (uint8_t *)malloc((size_t)n);
    if (!gl || !due) { free(gl); free(due); return -2; }
    int st = 0;
    *rebuilt = 0;
    int64_t pending = 0;   /* substeps since the last drift */
    for (int64_t s = 1; s <= S && !st; ++s) {
        ++pending;
        /* the particles whose step ends now (all of them at the end) */
        int64_t ndue = 0;
        for (int64_t i = 0; i < n; ++i) {
            due[i] = (s % ((int64_t)1 << (max_level - bins[i]))) == 0;
            ndue += due[i];
        }
        if (ndue == 0) continue;
        /* no velocity changes between force evaluations: one drift over the
           substeps since the last one */
        const double span = (double)pending * dtm;
        pending = 0;
        for (int64_t i = 0; i < 3 * n; ++i) b->pos[i] = b->pos[i] + b->vel[i] * span;
        /* the tree for this force evaluation: rebuilt, or refitted to the
           current positions */
        const int fresh = growth <= 0.0 || b->rebuild_next;
        if (fresh) {
            st = block_rebuild(b);
            *rebuilt += 1;
        } else {
            st = orc_refit(b->t, b->pos);
        }
        if (st) break;
        if (s < S) {
            /* forces for the groups holding a due particle */
            const orc_tree *t = b->t;
            int64_t ng = 0;
            for (int64_t g = 0; g < t->ngroups; ++g) {
                int any = 0;
                for (int64_t j = t->gfirst[g]; j < t->gfirst[g] + t->gcount[g]; ++j)
                    any |= due[t->perm[j]];
                if (any) gl[ng++] = g;
            }
            st = block_walk(b, gl, ng, fresh, growth, NULL);
            if (st) break;
            /* closing half kick of the step that ends, opening half kick of the next */
            for (int64_t i = 0; i < n; ++i) {
                if (!due[i]) continue;
                double h = 0.5 * ldexp(dt_max, -bins[i]);
                for (int k = 0; k < 3; ++k) b->vel[3 * i + k] = b->vel[3 * i + k] + b->acc[3 * i + k] * h;
                for (int k = 0; k < 3; ++k) b->vel[3 * i + k] = b->vel[3 * i + k] + b->acc[3 * i + k] * h;
                if (kicks) kicks[i] += 1;
            }
        } else {
            /* every particle is due: every group, then the closing half kicks */
            st = block_walk(b, NULL, 0, fresh, growth, sync_inter);
            if (st) break;
            for (int64_t i = 0; i < n; ++i) {
                double h = 0.5 * ldexp(dt_max, -bins[i]);
                for (int k = 0; k < 3; ++k) b->vel[3 * i + k] = b->vel[3 * i + k] + b->acc[3 * i + k] * h;
                if (kicks) kicks[i] += 1;
            }
        }
    }
    free(gl);
    free(due);
    return st;
}

void orc_energy(const double *vel, const double *mass, const double *pot, int64_t n,
                double out[6])
{
    double T = 0.0, W = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *v = vel + 3 * i;
        T += 0.5 * mass[i] * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
        W += 0.5 * mass[i] * pot[i];
        px += mass[i] * v[0];
        py += mass[i] * v[1];
        pz += mass[i] * v[2];
    }
    out[0] = T; out[1] = W; out[2] = T + W;
    out[3] = px; out[4] = py; out[5] = pz;
}
