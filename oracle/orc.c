/*
 * CPU oracle: plain, slow, obviously correct.  TEST INFRASTRUCTURE ONLY --
 * only tests, the package smoke check and the benchmark's CPU-baseline leg
 * load it.  See orc.h for the contract of each function.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no contraction,
 * so every floating-point expression rounds exactly as written).
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Exact orientation: sum of the eight products of the expanded determinant
 * as one big integer.  Every finite double is m * 2^e with an integer
 * |m| < 2^53, so each product is an integer < 2^106 times a power of two;
 * all products are shifted to the smallest exponent present and summed in
 * unsigned limbs, positives and negatives apart, then compared. */

#define NLIMB 80 /* 5120 bits: exponents of double products span < 4300 bits */

typedef struct {
    uint64_t w[NLIMB];
} mag_t;

static void mag_add(mag_t *a, unsigned __int128 v, int shift)
{
    uint64_t vl = (uint64_t)v, vh = (uint64_t)(v >> 64);
    int li = shift >> 6, bo = shift & 63;
    uint64_t part[3];
    if (bo == 0) {
        part[0] = vl;
        part[1] = vh;
        part[2] = 0;
    } else {
        part[0] = vl << bo;
        part[1] = (vl >> (64 - bo)) | (vh << bo);
        part[2] = vh >> (64 - bo);
    }
    uint64_t carry = 0;
    for (int i = li; i < NLIMB; ++i) {
        uint64_t add = (i - li < 3) ? part[i - li] : 0;
        if (i - li >= 3 && carry == 0)
            break;
        unsigned __int128 s = (unsigned __int128)a->w[i] + add + carry;
        a->w[i] = (uint64_t)s;
        carry = (uint64_t)(s >> 64);
    }
}

static int mag_cmp(const mag_t *a, const mag_t *b)
{
    for (int i = NLIMB - 1; i >= 0; --i) {
        if (a->w[i] > b->w[i])
            return 1;
        if (a->w[i] < b->w[i])
            return -1;
    }
    return 0;
}

/* d = m * 2^e with m >= 0 integer; returns the sign of d. */
static int split_double(double d, uint64_t *m, int *e)
{
    if (d == 0.0) {
        *m = 0;
        *e = 0;
        return 0;
    }
    int ex;
    double f = frexp(fabs(d), &ex); /* f in [0.5, 1) */
    *m = (uint64_t)ldexp(f, 53);    /* exact: f has at most 53 bits */
    *e = ex - 53;
    return d > 0 ? 1 : -1;
}

int orc_orient_sign_exact(double ax, double ay, double bx, double by, double cx, double cy)
{
    /* (ax-cx)(by-cy) - (ay-cy)(bx-cx), multiplied out:
     * + ax*by - ax*cy - cx*by + cx*cy - ay*bx + ay*cx + cy*bx - cy*cx */
    const double u[8] = {ax, ax, cx, cx, ay, ay, cy, cy};
    const double v[8] = {by, cy, by, cy, bx, cx, bx, cx};
    const int sgn[8] = {+1, -1, -1, +1, -1, +1, +1, -1};
    uint64_t mu[8], mv[8];
    int eu[8], ev[8], s[8];
    int emin = 1 << 30;
    for (int i = 0; i < 8; ++i) {
        int su = split_double(u[i], &mu[i], &eu[i]);
        int sv = split_double(v[i], &mv[i], &ev[i]);
        s[i] = su * sv * sgn[i];
        if (s[i] != 0 && eu[i] + ev[i] < emin)
            emin = eu[i] + ev[i];
    }
    mag_t pos, neg;
    memset(&pos, 0, sizeof pos);
    memset(&neg, 0, sizeof neg);
    for (int i = 0; i < 8; ++i) {
        if (s[i] == 0)
            continue;
        unsigned __int128 p = (unsigned __int128)mu[i] * mv[i];
        int shift = eu[i] + ev[i] - emin;
        mag_add(s[i] > 0 ? &pos : &neg, p, shift);
    }
    return mag_cmp(&pos, &neg);
}

/* Filter: Shewchuk's static bound for the two-product form,
 * |det_computed - det| <= (3 eps + 16 eps^2)(|detleft| + |detright|),
 * eps = 2^-53, valid without overflow or underflow; the filter is used
 * only when both products are zero by an exactly-zero factor or lie in
 * [2^-900, 2^900], otherwise the exact sum decides. */
static int product_in_range(double u, double v, double p)
{
    if (u == 0.0 || v == 0.0)
        return 1;
    double a = fabs(p);
    return a >= 0x1p-900 && a <= 0x1p900;
}

int orc_orient_sign(double ax, double ay, double bx, double by, double cx, double cy)
{
    const double eps = 0x1p-53;
    double u1 = ax - cx, v1 = by - cy, u2 = ay - cy, v2 = bx - cx;
    double detleft = u1 * v1;
    double detright = u2 * v2;
    if (product_in_range(u1, v1, detleft) && product_in_range(u2, v2, detright)) {
        double det = detleft - detright;
        double bound = (3.0 * eps + 16.0 * eps * eps) * (fabs(detleft) + fabs(detright));
        if (det > bound)
            return 1;
        if (-det > bound)
            return -1;
    }
    return orc_orient_sign_exact(ax, ay, bx, by, cx, cy);
}

void orc_orient_sign_batch(const double *pts, int64_t m, int8_t *out, int use_filter)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        const double *p = pts + 6 * i;
        out[i] = (int8_t)(use_filter ? orc_orient_sign(p[0], p[1], p[2], p[3], p[4], p[5])
                                     : orc_orient_sign_exact(p[0], p[1], p[2], p[3], p[4], p[5]));
    }
}

/* ------------------------------------------------------------------------ */
/* Containment in a closed triangle, by exact signs: q is in the closed
 * triangle (a, b, c) iff no edge orientation has the sign opposite to the
 * triangle's own orientation (either vertex order is accepted). */
static int closed_contains(const double *xy, const int32_t *t, double qx, double qy)
{
    const double *a = xy + 2 * (int64_t)t[0], *b = xy + 2 * (int64_t)t[1], *c = xy + 2 * (int64_t)t[2];
    int st = orc_orient_sign(a[0], a[1], b[0], b[1], c[0], c[1]);
    if (st == 0)
        return 0; /* degenerate triangle contains nothing by convention */
    int s0 = orc_orient_sign(b[0], b[1], c[0], c[1], qx, qy);
    int s1 = orc_orient_sign(c[0], c[1], a[0], a[1], qx, qy);
    int s2 = orc_orient_sign(a[0], a[1], b[0], b[1], qx, qy);
    return s0 * st >= 0 && s1 * st >= 0 && s2 * st >= 0;
}

/* Barycentric coordinates exactly as written in eq. (barycoords). */
static void bary_of(const double *xy, const int32_t *t, double xi, double eta, double *th)
{
    double xi1 = xy[2 * (int64_t)t[0]], eta1 = xy[2 * (int64_t)t[0] + 1];
    double xi2 = xy[2 * (int64_t)t[1]], eta2 = xy[2 * (int64_t)t[1] + 1];
    double xi3 = xy[2 * (int64_t)t[2]], eta3 = xy[2 * (int64_t)t[2] + 1];
    double den = (eta2 - eta3) * (xi1 - xi3) + (xi3 - xi2) * (eta1 - eta3);
    th[0] = ((eta2 - eta3) * (xi - xi3) + (xi3 - xi2) * (eta - eta3)) / den;
    th[1] = ((eta3 - eta1) * (xi - xi3) + (xi1 - xi3) * (eta - eta3)) / den;
    th[2] = 1.0 - th[0] - th[1];
}

typedef struct {
    double x0, y0, wx, wy;
    int g;
    int64_t *start; /* g*g + 1 */
    int32_t *items;
} buckets_t;

/* Cell index of a coordinate.  Rounded subtraction and division by a
 * positive width are monotone, so a point inside a triangle's bounding box
 * always lands in a cell within the box's own (equally computed) cell
 * range: the candidate set is conservative. */
static int cell_of(double v, double v0, double w, int g)
{
    double f = floor((v - v0) / w);
    if (f < 0)
        return 0;
    if (f > g - 1)
        return g - 1;
    return (int)f;
}

static void build_buckets(const double *xy, int64_t n, const int32_t *tri, int64_t nt, buckets_t *b)
{
    double x0 = xy[0], x1 = xy[0], y0 = xy[1], y1 = xy[1];
    for (int64_t i = 1; i < n; ++i) {
        x0 = fmin(x0, xy[2 * i]);
        x1 = fmax(x1, xy[2 * i]);
        y0 = fmin(y0, xy[2 * i + 1]);
        y1 = fmax(y1, xy[2 * i + 1]);
    }
    int g = (int)sqrt((double)nt / 2.0);
    if (g < 1)
        g = 1;
    if (g > 4096)
        g = 4096;
    b->g = g;
    b->x0 = x0;
    b->y0 = y0;
    b->wx = (x1 > x0) ? (x1 - x0) / g : 1.0;
    b->wy = (y1 > y0) ? (y1 - y0) / g : 1.0;
    int64_t ncell = (int64_t)g * g;
    int64_t *count = calloc((size_t)ncell + 1, sizeof(int64_t));
    int32_t *rng = malloc((size_t)nt * 4 * sizeof(int32_t));
    for (int64_t t = 0; t < nt; ++t) {
        double tx0 = 1e300, tx1 = -1e300, ty0 = 1e300, ty1 = -1e300;
        for (int k = 0; k < 3; ++k) {
            const double *p = xy + 2 * (int64_t)tri[3 * t + k];
            tx0 = fmin(tx0, p[0]);
            tx1 = fmax(tx1, p[0]);
            ty0 = fmin(ty0, p[1]);
            ty1 = fmax(ty1, p[1]);
        }
        int cx0 = cell_of(tx0, b->x0, b->wx, g), cx1 = cell_of(tx1, b->x0, b->wx, g);
        int cy0 = cell_of(ty0, b->y0, b->wy, g), cy1 = cell_of(ty1, b->y0, b->wy, g);
        rng[4 * t] = cx0;
        rng[4 * t + 1] = cx1;
        rng[4 * t + 2] = cy0;
        rng[4 * t + 3] = cy1;
        for (int cy = cy0; cy <= cy1; ++cy)
            for (int cx = cx0; cx <= cx1; ++cx)
                count[(int64_t)cy * g + cx + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c)
        count[c + 1] += count[c];
    b->items = malloc((size_t)(count[ncell] > 0 ? count[ncell] : 1) * sizeof(int32_t));
    int64_t *fill = malloc((size_t)ncell * sizeof(int64_t));
    memcpy(fill, count, (size_t)ncell * sizeof(int64_t));
    for (int64_t t = 0; t < nt; ++t)
        for (int cy = rng[4 * t + 2]; cy <= rng[4 * t + 3]; ++cy)
            for (int cx = rng[4 * t]; cx <= rng[4 * t + 1]; ++cx)
                b->items[fill[(int64_t)cy * g + cx]++] = (int32_t)t;
    free(fill);
    free(rng);
    b->start = count;
}

int orc_containers(const double *xy, int64_t n, const int32_t *tri, int64_t nt,
                   double qx, double qy, int32_t *out, int cap)
{
    (void)n;
    int c = 0;
    if (!isfinite(qx) || !isfinite(qy))
        return 0;
    for (int64_t t = 0; t < nt; ++t)
        if (closed_contains(xy, tri + 3 * t, qx, qy)) {
            if (c < cap)
                out[c] = (int32_t)t;
            ++c;
        }
    return c;
}

int orc_locate(const double *xy, int64_t n, const int32_t *tri, int64_t nt,
               const double *q, int64_t m, int32_t *elem, double *bary, int brute)
{
    if (n < 0 || nt < 0 || m < 0 || (m > 0 && (!q || !elem)))
        return -1;
    if (nt == 0 || n == 0) {
        for (int64_t i = 0; i < m; ++i) {
            elem[i] = -1;
            if (bary)
                bary[3 * i] = bary[3 * i + 1] = bary[3 * i + 2] = NAN;
        }
        return 0;
    }
    buckets_t b;
    memset(&b, 0, sizeof b);
    double x0 = xy[0], x1 = xy[0], y0 = xy[1], y1 = xy[1];
    for (int64_t i = 1; i < n; ++i) {
        x0 = fmin(x0, xy[2 * i]);
        x1 = fmax(x1, xy[2 * i]);
        y0 = fmin(y0, xy[2 * i + 1]);
        y1 = fmax(y1, xy[2 * i + 1]);
    }
    if (!brute)
        build_buckets(xy, n, tri, nt, &b);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        double qx = q[2 * i], qy = q[2 * i + 1];
        int32_t best = -1;
        /* a closed triangle lies inside the nodes' bounding box */
        int inside_box = isfinite(qx) && isfinite(qy) && qx >= x0 && qx <= x1 && qy >= y0 && qy <= y1;
        if (inside_box) {
            if (brute) {
                for (int64_t t = 0; t < nt; ++t)
                    if (closed_contains(xy, tri + 3 * t, qx, qy)) {
                        best = (int32_t)t; /* scanning upwards: first hit is the smallest id */
                        break;
                    }
            } else {
                int cx = cell_of(qx, b.x0, b.wx, b.g), cy = cell_of(qy, b.y0, b.wy, b.g);
                int64_t cell = (int64_t)cy * b.g + cx;
                for (int64_t it = b.start[cell]; it < b.start[cell + 1]; ++it) {
                    int32_t t = b.items[it];
                    if ((best < 0 || t < best) && closed_contains(xy, tri + 3 * (int64_t)t, qx, qy))
                        best = t;
                }
            }
        }
        elem[i] = best;
        if (bary) {
            if (best >= 0)
                bary_of(xy, tri + 3 * (int64_t)best, qx, qy, bary + 3 * i);
            else
                bary[3 * i] = bary[3 * i + 1] = bary[3 * i + 2] = NAN;
        }
    }
    if (!brute) {
        free(b.start);
        free(b.items);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Advecting fields and feet (eq. eulero; the explicit midpoint rule as the
 * higher-order ODE solver that Section 3 leaves open). */

/* sin(pi x) with x reduced exactly to f = x - n, n the nearest integer
 * (sin(pi (n + f)) = (-1)^n sin(pi f)): zero exactly at the integers, where
 * sin(pi * x) in floating point leaves a residue of about 1e-16 |x|.  The
 * swirl vanishes on the boundary of the unit square, and with this
 * evaluation it does so exactly. */
static double sin_pi(double x)
{
    const double pi = 3.14159265358979323846;
    if (!isfinite(x))
        return NAN;
    const double n = nearbyint(x);
    const double f = x - n; /* exact for |x| < 2^52 */
    const double s = sin(pi * f);
    return fmod(n, 2.0) != 0.0 ? -s : s;
}

void orc_field(int kind, const double *p, double x, double y, double t, double *out)
{
    const double pi = 3.14159265358979323846;
    switch (kind) {
    case 0: /* constant */
        out[0] = p[0];
        out[1] = p[1];
        break;
    case 1: /* solid body rotation with angular velocity p0 about (p1, p2) */
        out[0] = -p[0] * (y - p[2]);
        out[1] = p[0] * (x - p[1]);
        break;
    case 2: { /* swirl with period p0 */
        double g = cos(pi * t / p[0]);
        double sx = sin_pi(x), sy = sin_pi(y);
        out[0] = g * sx * sx * sin_pi(2.0 * y);
        out[1] = -g * sy * sy * sin_pi(2.0 * x);
        break;
    }
    case 3: { /* the rotating field of Section 4 about (p2, p3) */
        double dx = x - p[2], dy = y - p[3];
        double a = p[0] * sqrt(dx * dx + dy * dy) + p[1] * t;
        out[0] = cos(a);
        out[1] = sin(a);
        break;
    }
    case 4: { /* affine: A (x - c) + b */
        double dx = x - p[4], dy = y - p[5];
        out[0] = p[0] * dx + p[1] * dy + p[6];
        out[1] = p[2] * dx + p[3] * dy + p[7];
        break;
    }
    default:
        out[0] = out[1] = NAN;
    }
}

void orc_feet(const double *xy, int64_t n, int kind, const double *p8,
              double t_np1, double dt, int scheme, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x = xy[2 * i], y = xy[2 * i + 1], f[2];
        orc_field(kind, p8, x, y, t_np1, f);
        if (scheme == 1) {
            double xs = x - 0.5 * dt * f[0], ys = y - 0.5 * dt * f[1];
            orc_field(kind, p8, xs, ys, t_np1 - 0.5 * dt, f);
        }
        out[2 * i] = x - dt * f[0];
        out[2 * i + 1] = y - dt * f[1];
    }
}

/* ------------------------------------------------------------------------ */
/* P2 degrees of freedom and interpolation */

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static uint64_t edge_key(int32_t a, int32_t b)
{
    uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
    return ((uint64_t)lo << 32) | hi;
}

int64_t orc_p2_edges(const int32_t *tri, int64_t nt, int32_t *edges, int32_t *tri_edges)
{
    uint64_t *keys = malloc((size_t)(3 * nt > 0 ? 3 * nt : 1) * sizeof(uint64_t));
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k)
            keys[3 * t + k] = edge_key(tri[3 * t + (k + 1) % 3], tri[3 * t + (k + 2) % 3]);
    qsort(keys, (size_t)(3 * nt), sizeof(uint64_t), cmp_u64);
    int64_t ne = 0;
    for (int64_t i = 0; i < 3 * nt; ++i)
        if (i == 0 || keys[i] != keys[i - 1])
            keys[ne++] = keys[i];
    for (int64_t e = 0; e < ne; ++e) {
        edges[2 * e] = (int32_t)(keys[e] >> 32);
        edges[2 * e + 1] = (int32_t)(keys[e] & 0xffffffffu);
    }
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            uint64_t key = edge_key(tri[3 * t + (k + 1) % 3], tri[3 * t + (k + 2) % 3]);
            uint64_t *hit = bsearch(&key, keys, (size_t)ne, sizeof(uint64_t), cmp_u64);
            tri_edges[3 * t + k] = (int32_t)(hit - keys);
        }
    free(keys);
    return ne;
}

void orc_interp(int order, const int32_t *tri, int64_t nt, const int32_t *tri_edges,
                int64_t n_vert, const int32_t *elem, const double *bary, int64_t m,
                const double *v, int k, double outside_value, double *out)
{
    (void)nt;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        int32_t t = elem[i];
        if (t < 0) {
            for (int f = 0; f < k; ++f)
                out[i * k + f] = outside_value;
            continue;
        }
        const double *th = bary + 3 * i;
        const int32_t *tv = tri + 3 * (int64_t)t;
        if (order == 1) {
            for (int f = 0; f < k; ++f)
                out[i * k + f] = th[0] * v[(int64_t)tv[0] * k + f] + th[1] * v[(int64_t)tv[1] * k + f] +
                                 th[2] * v[(int64_t)tv[2] * k + f];
        } else {
            /* vertex functions theta_a (2 theta_a - 1); edge function of the
             * edge opposite vertex a: 4 theta_b theta_c */
            double phi[6];
            int64_t dof[6];
            for (int a = 0; a < 3; ++a) {
                int b = (a + 1) % 3, c = (a + 2) % 3;
                phi[a] = th[a] * (2.0 * th[a] - 1.0);
                phi[3 + a] = 4.0 * th[b] * th[c];
                dof[a] = tv[a];
                dof[3 + a] = n_vert + tri_edges[3 * (int64_t)t + a];
            }
            for (int f = 0; f < k; ++f) {
                double s = 0.0;
                for (int a = 0; a < 6; ++a)
                    s += phi[a] * v[dof[a] * k + f];
                out[i * k + f] = s;
            }
        }
    }
}
