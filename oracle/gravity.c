/* TEST INFRASTRUCTURE: CPU oracle of Barnes-Hut monopole self-gravity
 * (section 3.3, eq. gravitational_force; the tree of section 3.5.1).  Only the
 * test-suite, the quick self-check and the benchmark's CPU baseline use it; it
 * shares no code with the HIP library.
 *
 * Tree (section 3.5.1): the root is the cube of edge
 *   s0 = max over axes of (max_a x_a - min_b x_b)
 * with its lower corner at the per-axis minima; a node of depth d has edge
 * s0 / 2^d.  Particles are inserted one by one in index order: a particle goes
 * down the octants of the nodes it meets; an empty child slot takes it, a slot
 * holding another particle is split into new inner nodes, each half the edge of
 * its parent, until the two particles fall into different octants.  So the
 * inner nodes are exactly the cubes that hold at least two particles and the
 * particles are the leaves.
 *
 * Readings (the paper leaves these open):
 *   - octant membership is decided on integer coordinates
 *     q = floor((x - lo) / s0 * 2^21), clamped to [0, 2^21 - 1] (q = 0 when
 *     s0 = 0): at depth d the octant bit of an axis is bit 20 - d of q.  Nodes go
 *     down to depth 21 at most; the particles that share a depth-21 cube are all
 *     leaves of that node, in index order.
 *   - children are visited in octant order 4 bx + 2 by + bz (b the axis bits).
 *   - pseudo-particle of a node: total mass and centre of mass, accumulated over
 *     its children in octant order (an inner child contributes m_c and m_c x_c).
 *   - force: the printed F_a = G m_a m_p (x_a - x_p) / r^3 would repel; gravity
 *     attracts, so a_a = G m_p (x_p - x_a) / (r + eps)^3, eps >= 0 the smoothing
 *     length added to the distance (the paper's second smoothing scheme); a
 *     partner at distance 0 adds nothing.
 *   - walk: from the root, in octant order; an inner node whose edge s and
 *     distance r from the particle to its centre of mass satisfy s / r < theta
 *     (the criterion as section 3.3 prints it, r = sqrt of the squared distance)
 *     acts as one pseudo-particle, else its children are visited; a leaf other
 *     than the particle itself always acts directly.  theta = 0 is the direct sum.
 *   - the squared form s^2 < theta^2 r^2 is the same criterion in real
 *     arithmetic; rounded, the two can differ when s / r lies within a few ulps of
 *     theta.  Each target's walk also evaluates the squared form at every node it
 *     tests and reports (tie) whether the two ever disagreed, so a checker can set
 *     such walks aside instead of requiring one rounding of the criterion.
 * Arithmetic in FP64 without contraction, each sum in the order stated.  */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define GR_DMAX 21
#define GR_EMPTY (-1)

typedef struct {
    int child[8];   /* >= 0 inner node, GR_EMPTY, or -(2 + particle) */
    int depth;
    int bucket;     /* depth GR_DMAX: first particle of the list, -1 none */
    double m, cx, cy, cz;
} gr_node;

typedef struct {
    int64_t n;
    const double *pos;
    const double *m;
    uint32_t *q;        /* 3 per particle */
    int *next;          /* bucket lists */
    gr_node *node;
    int nnode, cap;
    double lo[3], s0;
} gr_tree;

static int gr_new(gr_tree *t, int depth)
{
    if (t->nnode == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 64;
        t->node = (gr_node *)realloc(t->node, (size_t)t->cap * sizeof(gr_node));
    }
    gr_node *nd = &t->node[t->nnode];
    for (int o = 0; o < 8; ++o) nd->child[o] = GR_EMPTY;
    nd->depth = depth;
    nd->bucket = -1;
    nd->m = nd->cx = nd->cy = nd->cz = 0.0;
    return t->nnode++;
}

static int gr_octant(const gr_tree *t, int64_t p, int depth)
{
    const int b = GR_DMAX - 1 - depth;
    const uint32_t *q = &t->q[3 * p];
    return (int)(((q[0] >> b) & 1u) << 2 | ((q[1] >> b) & 1u) << 1 | ((q[2] >> b) & 1u));
}

static void gr_bucket_append(gr_tree *t, int nd, int p)
{
    t->next[p] = -1;
    if (t->node[nd].bucket < 0) {
        t->node[nd].bucket = p;
        return;
    }
    int k = t->node[nd].bucket;
    while (t->next[k] >= 0) k = t->next[k];
    t->next[k] = p;
}

/* place particle p in node nd (which is known to contain its cube position) */
static void gr_insert(gr_tree *t, int nd, int p)
{
    for (;;) {
        if (t->node[nd].depth == GR_DMAX) {
            gr_bucket_append(t, nd, p);
            return;
        }
        const int o = gr_octant(t, p, t->node[nd].depth);
        const int c = t->node[nd].child[o];
        if (c == GR_EMPTY) {
            t->node[nd].child[o] = -(2 + p);
            return;
        }
        if (c >= 0) {
            nd = c;
            continue;
        }
        /* slot holds particle p2: a new inner node half the edge takes it */
        const int p2 = -(2 + c);
        const int nn = gr_new(t, t->node[nd].depth + 1);
        t->node[nd].child[o] = nn;
        if (t->node[nn].depth == GR_DMAX)
            gr_bucket_append(t, nn, p2);
        else
            t->node[nn].child[gr_octant(t, p2, t->node[nn].depth)] = -(2 + p2);
        nd = nn;
    }
}

static void gr_monopole(gr_tree *t, int nd)
{
    double m = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    const int64_t n = t->n;
    for (int o = 0; o < 8; ++o) {
        const int c = t->node[nd].child[o];
        if (c == GR_EMPTY) continue;
        if (c >= 0) {
            gr_monopole(t, c);
            const gr_node *k = &t->node[c];
            m = m + k->m;
            mx = mx + k->m * k->cx;
            my = my + k->m * k->cy;
            mz = mz + k->m * k->cz;
        } else {
            const int p = -(2 + c);
            m = m + t->m[p];
            mx = mx + t->m[p] * t->pos[p];
            my = my + t->m[p] * t->pos[n + p];
            mz = mz + t->m[p] * t->pos[2 * n + p];
        }
    }
    for (int p = t->node[nd].bucket; p >= 0; p = t->next[p]) {
        m = m + t->m[p];
        mx = mx + t->m[p] * t->pos[p];
        my = my + t->m[p] * t->pos[n + p];
        mz = mz + t->m[p] * t->pos[2 * n + p];
    }
    gr_node *k = &t->node[nd];
    k->m = m;
    k->cx = mx / m;
    k->cy = my / m;
    k->cz = mz / m;
}

static void gr_build(gr_tree *t, int64_t n, const double *pos, const double *m)
{
    t->n = n;
    t->pos = pos;
    t->m = m;
    t->node = NULL;
    t->nnode = t->cap = 0;
    t->q = (uint32_t *)malloc((size_t)(3 * (n > 0 ? n : 1)) * sizeof(uint32_t));
    t->next = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    double hi[3];
    for (int a = 0; a < 3; ++a) {
        t->lo[a] = pos[a * n];
        hi[a] = pos[a * n];
        for (int64_t i = 1; i < n; ++i) {
            const double v = pos[a * n + i];
            if (v < t->lo[a]) t->lo[a] = v;
            if (v > hi[a]) hi[a] = v;
        }
    }
    t->s0 = 0.0;
    for (int a = 0; a < 3; ++a)
        if (hi[a] - t->lo[a] > t->s0) t->s0 = hi[a] - t->lo[a];
    const double scale = 2097152.0; /* 2^21 */
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            uint32_t v = 0;
            if (t->s0 > 0.0) {
                const double u = floor((pos[a * n + i] - t->lo[a]) / t->s0 * scale);
                v = u >= scale ? 2097151u : (uint32_t)u;
            }
            t->q[3 * i + a] = v;
        }
    const int root = gr_new(t, 0);
    for (int64_t i = 0; i < n; ++i) gr_insert(t, root, (int)i);
    if (n > 0) gr_monopole(t, root);
}

static void gr_free(gr_tree *t)
{
    free(t->node);
    free(t->q);
    free(t->next);
}

typedef struct {
    double ax, ay, az;
    int64_t count;
    int tie;  /* the printed and the squared opening test disagreed at some node */
} gr_acc;

static void gr_term(gr_acc *A, double G, double eps, double mp, double dx, double dy, double dz)
{
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    A->count += 1;
    if (r == 0.0) return;
    const double d = r + eps;
    const double f = G * mp / (d * d * d);
    A->ax = A->ax + f * dx;
    A->ay = A->ay + f * dy;
    A->az = A->az + f * dz;
}

static void gr_walk(const gr_tree *t, int nd, int64_t a, double G, double theta, double eps,
                    gr_acc *A)
{
    const int64_t n = t->n;
    const double xa = t->pos[a], ya = t->pos[n + a], za = t->pos[2 * n + a];
    const gr_node *k = &t->node[nd];
    const double dx = k->cx - xa, dy = k->cy - ya, dz = k->cz - za;
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double s = ldexp(t->s0, -k->depth);
    const int open_far = s / sqrt(r2) < theta;  /* section 3.3: s / r < theta */
    if (open_far != (s * s < theta * theta * r2)) A->tie = 1;
    if (open_far) {
        gr_term(A, G, eps, k->m, dx, dy, dz);
        return;
    }
    for (int o = 0; o < 8; ++o) {
        const int c = k->child[o];
        if (c == GR_EMPTY) continue;
        if (c >= 0) {
            gr_walk(t, c, a, G, theta, eps, A);
        } else {
            const int p = -(2 + c);
            if (p != a)
                gr_term(A, G, eps, t->m[p], t->pos[p] - xa, t->pos[n + p] - ya,
                        t->pos[2 * n + p] - za);
        }
    }
    for (int p = k->bucket; p >= 0; p = t->next[p])
        if (p != a)
            gr_term(A, G, eps, t->m[p], t->pos[p] - xa, t->pos[n + p] - ya, t->pos[2 * n + p] - za);
}

/* Gravitational acceleration of the targets (targets[0..nt) or, when targets is
 * NULL, every particle, nt = n): pos (3, n), m (n) > 0; acc (3, nt); count (nt,
 * nullable): pseudo-particles and leaves each target took a term from; tie (nt,
 * nullable): 1 where the target's walk met a node at which s / r < theta and
 * s^2 < theta^2 r^2 decide differently.  Returns the number of inner nodes. */
int64_t orc_gravity(int64_t n, const double *pos, const double *m, double G, double theta,
                    double eps, const int64_t *targets, int64_t nt, double *acc, int64_t *count,
                    int32_t *tie)
{
    gr_tree t;
    gr_build(&t, n, pos, m);
    if (!targets) nt = n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < nt; ++j) {
        const int64_t a = targets ? targets[j] : j;
        gr_acc A = {0.0, 0.0, 0.0, 0, 0};
        gr_walk(&t, 0, a, G, theta, eps, &A);
        acc[j] = A.ax;
        acc[nt + j] = A.ay;
        acc[2 * nt + j] = A.az;
        if (count) count[j] = A.count;
        if (tie) tie[j] = A.tie;
    }
    const int64_t nn = n > 0 ? t.nnode : 0;
    gr_free(&t);
    return nn;
}

/* The inner nodes, for checks: depth, the integer corner of the node's cube
 * (q >> (21 - depth) per axis), mass and centre of mass; arrays of length
 * cap (>= the node count, which is returned; nothing is written if it is larger). */
int64_t orc_gravity_tree(int64_t n, const double *pos, const double *m, int64_t cap,
                         int32_t *depth, int64_t *corner, double *mass, double *com)
{
    gr_tree t;
    gr_build(&t, n, pos, m);
    const int64_t nn = n > 0 ? t.nnode : 0;
    if (nn <= cap) {
        /* each node's corner: follow the first particle found below it */
        for (int64_t i = 0; i < nn; ++i) {
            const gr_node *k = &t.node[i];
            int nd = (int)i, p = -1;
            while (p < 0) {
                const gr_node *c = &t.node[nd];
                if (c->bucket >= 0) {
                    p = c->bucket;
                    break;
                }
                for (int o = 0; o < 8; ++o) {
                    if (c->child[o] == GR_EMPTY) continue;
                    if (c->child[o] >= 0)
                        nd = c->child[o];
                    else
                        p = -(2 + c->child[o]);
                    break;
                }
            }
            depth[i] = k->depth;
            for (int a = 0; a < 3; ++a)
                corner[3 * i + a] = (int64_t)(t.q[3 * p + a] >> (GR_DMAX - k->depth));
            mass[i] = k->m;
            com[3 * i] = k->cx;
            com[3 * i + 1] = k->cy;
            com[3 * i + 2] = k->cz;
        }
    }
    gr_free(&t);
    return nn;
}
