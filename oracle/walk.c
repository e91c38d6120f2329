/* The paper's own point location on the host: the barycentric walk of
 * Section 2.2 (Algorithm 1) in plain FP64, from strategy (a)'s start (an
 * incident triangle of the node whose foot is sought, Section 3 (a)).
 *
 * TEST AND BENCHMARK INFRASTRUCTURE ONLY: it gives the walk lengths of the
 * method as the paper states it and the method's speed on the host cores
 * (one thread, as the paper's timings, and all cores).  The GPU library never
 * links or calls it; it shares no code with the library.
 *
 * The walk: compute the barycentric coordinates of q in the current
 * triangle by eq. (barycoords) (ratios of signed areas, so either vertex
 * orientation works); stop when none is negative; otherwise move to the
 * neighbour across the edge opposite the vertex with the most negative
 * coordinate (the lowest local index among equal values).  A boundary edge
 * there means q is outside (the domain is convex).  The result is the
 * first closed container the walk reaches; on an edge or a vertex it
 * depends on the path (the library and the oracle take the smallest id of
 * all containers instead).
 */
#include <math.h>
#include <stdint.h>

#include <omp.h>

/* neighbour of triangle t across the edge opposite its vertex k */
#define NB(t, k) nbr[3 * (int64_t)(t) + (k)]

static double area2(const double *a, const double *b, const double *c)
{
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

/* walk from triangle j towards q; returns the triangle (or -1 outside, -2
 * when cap moves did not end the walk) and the number of element changes */
static int32_t walk_one(const double *xy, const int32_t *tri, const int32_t *nbr, const double *q, int32_t j,
                        int64_t cap, int32_t *moves)
{
    int64_t m = 0;
    for (;;) {
        const double *p0 = xy + 2 * (int64_t)tri[3 * (int64_t)j];
        const double *p1 = xy + 2 * (int64_t)tri[3 * (int64_t)j + 1];
        const double *p2 = xy + 2 * (int64_t)tri[3 * (int64_t)j + 2];
        const double d = area2(p0, p1, p2);
        const double lam[3] = {area2(q, p1, p2) / d, area2(p0, q, p2) / d, area2(p0, p1, q) / d};
        int k = -1;
        double best = 0.0;
        for (int i = 0; i < 3; ++i)
            if (lam[i] < best) {
                best = lam[i];
                k = i;
            }
        if (k < 0) {
            *moves = (int32_t)m;
            return j;
        }
        const int32_t n = NB(j, k);
        if (n < 0) {
            *moves = (int32_t)m;
            return -1;
        }
        j = n;
        if (++m >= cap) {
            *moves = (int32_t)m;
            return -2;
        }
    }
}

static uint64_t splitmix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ULL;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
    return x ^ (x >> 31);
}

/* Strategy (a)'s start for node i with foot q:
 *   rule 0: one of its incident triangles drawn at random (the paper's
 *           choice): index splitmix64(seed + i) mod degree in inc;
 *   rule 1: the incident triangle whose angle at the node contains the
 *           direction q - x_i (closed sector, FP64 signs), the first
 *           incident triangle when none does (a foot outside the domain's
 *           angle at a boundary node, or q = x_i). */
static int32_t start_of(const double *xy, const int32_t *tri, const int32_t *inc_ptr, const int32_t *inc, int64_t i,
                        const double *q, int rule, uint64_t seed)
{
    const int32_t b = inc_ptr[i], e = inc_ptr[i + 1];
    if (e <= b)
        return -1;
    if (rule == 0)
        return inc[b + (int32_t)(splitmix64(seed + (uint64_t)i) % (uint64_t)(e - b))];
    const double *x = xy + 2 * i;
    for (int32_t s = b; s < e; ++s) {
        const int32_t t = inc[s];
        int r = 0;
        while (tri[3 * (int64_t)t + r] != (int32_t)i)
            ++r;
        const double *u = xy + 2 * (int64_t)tri[3 * (int64_t)t + (r + 1) % 3];
        const double *w = xy + 2 * (int64_t)tri[3 * (int64_t)t + (r + 2) % 3];
        double su = area2(x, u, q), sw = area2(x, q, w);
        if (area2(x, u, w) < 0.0) {  /* clockwise triangle: the sector runs from w to u */
            su = -su;
            sw = -sw;
        }
        if (su >= 0.0 && sw >= 0.0 && (q[0] != x[0] || q[1] != x[1]))
            return t;
    }
    return inc[b];
}

/* Locate the feet q (n_nodes x 2) of all nodes: start by rule, then walk.
 * elem, steps: n_nodes each.  threads <= 0: every core.  Returns the number
 * of walks that hit the cap (their elem is -2). */
int64_t o3_locate_nodes(const double *xy, int64_t n_nodes, const int32_t *tri, const int32_t *nbr,
                        const int32_t *inc_ptr, const int32_t *inc, const double *q, int rule, uint64_t seed,
                        int64_t cap, int32_t *elem, int32_t *steps, int threads)
{
    int64_t capped = 0;
    const int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4096) num_threads(nt) reduction(+ : capped)
    for (int64_t i = 0; i < n_nodes; ++i) {
        const int32_t j0 = start_of(xy, tri, inc_ptr, inc, i, q + 2 * i, rule, seed);
        int32_t mv = 0;
        elem[i] = j0 < 0 ? -1 : walk_one(xy, tri, nbr, q + 2 * i, j0, cap, &mv);
        steps[i] = mv;
        capped += elem[i] == -2;
    }
    return capped;
}

/* The same walk from given start triangles (start[i] for point q[i]). */
int64_t o3_walk(const double *xy, const int32_t *tri, const int32_t *nbr, int64_t m, const double *q,
                const int32_t *start, int64_t cap, int32_t *elem, int32_t *steps, int threads)
{
    int64_t capped = 0;
    const int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 4096) num_threads(nt) reduction(+ : capped)
    for (int64_t i = 0; i < m; ++i) {
        int32_t mv = 0;
        elem[i] = walk_one(xy, tri, nbr, q + 2 * i, start[i], cap, &mv);
        steps[i] = mv;
        capped += elem[i] == -2;
    }
    return capped;
}

int o3_max_threads(void) { return omp_get_max_threads(); }
