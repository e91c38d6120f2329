/*
 * CPU oracle for the characteristic-foot location and interpolation path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code
 * with the GPU library: its exact predicate is a big-integer sum, its point
 * location is a brute-force scan over a bucket grid (no walk), and it works
 * on the user's node and triangle numbering throughout.
 *
 * Paper: Cacace & Ferretti, "Efficient implementation of characteristic-based
 * schemes on unstructured triangular grids" (arXiv 2104.09189).
 *
 * Conventions: 0-based indices, coordinates and values in double, node-major
 * value arrays v[dof * k + field].  Every function is synchronous and
 * allocates only what it frees before returning.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sign (-1, 0, +1) of orient2d(a, b, c) = (ax-cx)(by-cy) - (ay-cy)(bx-cx),
 * exact for all finite doubles.  A floating-point filter answers when its
 * error bound allows; otherwise an exact big-integer sum decides. */
int orc_orient_sign(double ax, double ay, double bx, double by, double cx, double cy);

/* The exact big-integer sum alone, no filter (used to pin the filter). */
int orc_orient_sign_exact(double ax, double ay, double bx, double by, double cx, double cy);

/* Batch form: pts is m x 6 (ax ay bx by cx cy); out[i] in {-1,0,1}. */
void orc_orient_sign_batch(const double *pts, int64_t m, int8_t *out, int use_filter);

/* Point location by definition (Section 2.2 stop rule, closed triangles):
 * elem[i] = smallest triangle id whose closed triangle contains q[i], or -1
 * when none does (or q[i] is not finite).  bary (nullable, m x 3) receives
 * the barycentric coordinates of q[i] in elem[i] in the triangle's own
 * vertex order (eq. barycoords), NaN when elem[i] = -1.  brute != 0 scans
 * every triangle; otherwise a bucket grid over triangle bounding boxes
 * supplies candidates.  Returns 0, or -1 on bad arguments. */
int orc_locate(const double *xy, int64_t n, const int32_t *tri, int64_t nt,
               const double *q, int64_t m, int32_t *elem, double *bary, int brute);

/* All closed containers of one query point, up to cap; returns the count. */
int orc_containers(const double *xy, int64_t n, const int32_t *tri, int64_t nt,
                   double qx, double qy, int32_t *out, int cap);

/* Advecting field f(x, t) of a given kind and 8 parameters (kinds as in the
 * workload generator). out = 2 doubles. */
void orc_field(int kind, const double *p8, double x, double y, double t, double *out);

/* Feet of the characteristics through the points xy (n x 2) at t_np1:
 * scheme 0 = explicit Euler backward in time (eq. eulero),
 * scheme 1 = explicit midpoint, x* = x - dt/2 f(x, t_np1),
 *            q = x - dt f(x*, t_np1 - dt/2). */
void orc_feet(const double *xy, int64_t n, int kind, const double *p8,
              double t_np1, double dt, int scheme, double *out);

/* P2 degrees of freedom: edges are the distinct unordered vertex pairs of
 * the triangles, numbered in lexicographic order of (min, max).  edges
 * (capacity 3*nt x 2) receives the pairs; tri_edges (nt x 3) the id of the
 * edge opposite local vertex k.  Returns the edge count. */
int64_t orc_p2_edges(const int32_t *tri, int64_t nt, int32_t *edges, int32_t *tri_edges);

/* Interpolation of V (ndof x k) at located points (eq. schema_trasp).
 * order 1: sum_k theta_k V[i_k] (Remark after eq. barycoords);
 * order 2: quadratic Lagrange basis, vertex DOFs are the node ids, edge DOFs
 * are n_vert + edge id.  elem = -1 gives outside_value. */
void orc_interp(int order, const int32_t *tri, int64_t nt, const int32_t *tri_edges,
                int64_t n_vert, const int32_t *elem, const double *bary, int64_t m,
                const double *v, int k, double outside_value, double *out);

#ifdef __cplusplus
}
#endif
#endif
