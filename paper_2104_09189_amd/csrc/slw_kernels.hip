// Device kernels: feet, start selection, barycentric walk, tie rule,
// interpolation, and the fused semi-Lagrangian step.
//
// One lane handles one foot.  A walk step reads one 48-byte triangle record
// (float coordinates, neighbours, vertex ids), computes the three edge
// orientations of the foot, and either stops (all signs >= 0: the barycentric
// coordinates of Section 2.2 are all non-negative) or crosses the edge with
// the most negative coordinate.  Every sign is exact: a float filter with a
// certified error bound decides almost all of them; the rest are decided on
// the exact coordinates (FP64 filter, then exact expansion arithmetic).  The
// triangle found therefore does not depend on where the walk started.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "slw_internal.h"
#include "slw_mlp.h"
#include "slw_predicates.h"

namespace slw {

namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int32_t kUidMask = 0x7fffffff;

template <bool F32>
struct CT;
template <>
struct CT<false> {
    using R = double;
    using R2 = double2;
};
template <>
struct CT<true> {
    using R = float;
    using R2 = float2;
};

// Accesses marked non-temporal: data a step touches once (the new values,
// the previous element of strategy (b)) need not take cache lines from the
// value rows and triangle records that neighbouring feet reuse.  (A DOF's own
// coordinates are reused: the weights of nearby feet read them.)
__device__ inline void store_stream(float4 *p, float4 v)
{
    typedef float nv4 __attribute__((ext_vector_type(4)));
    nv4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, (nv4 *)p);
}
__device__ inline void store_stream(double2 *p, double2 v)
{
    typedef double nv2 __attribute__((ext_vector_type(2)));
    nv2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, (nv2 *)p);
}
__device__ inline void store_stream(float *p, float v) { __builtin_nontemporal_store(v, p); }
__device__ inline void store_stream(double *p, double v) { __builtin_nontemporal_store(v, p); }
__device__ inline void store_stream(int32_t *p, int32_t v) { __builtin_nontemporal_store(v, p); }
__device__ inline int32_t load_stream(const int32_t *p) { return __builtin_nontemporal_load(p); }

// The previous element of a DOF (strategies (b) and the hybrid) is an
// internal triangle id below 2^29; the hybrid keeps in bits 29-30 how many
// more steps the DOF skips the test on it (its foot moved far lately).
constexpr int32_t kPrevElemMask = (1 << 29) - 1;
constexpr int kPrevSkipShift = 29;
constexpr int kPrevSkipSteps = 3;

// ---------------------------------------------------------------------------
// advecting fields (kinds as in slw_field) and feet

__device__ inline void sincospi_r(double x, double &s, double &c) { sincospi(x, &s, &c); }
__device__ inline void sincospi_r(float x, float &s, float &c) { sincospif(x, &s, &c); }

// f at (x, y) and evaluation time `which` (0: t_{n+1}, 1: t_{n+1} - dt/2);
// the time factors were evaluated once on the host
template <typename R>
__device__ inline void field_eval(const FieldDev &f, int which, R x, R y, R &fx, R &fy)
{
    const R p0 = (R)f.p[0], p1 = (R)f.p[1], p2 = (R)f.p[2], p3 = (R)f.p[3];
    switch (f.kind) {
    case 0:
        fx = p0;
        fy = p1;
        break;
    case 1:
        fx = -p0 * (y - p2);
        fy = p0 * (x - p1);
        break;
    case 2: {
        // sin(2 pi y) = 2 sin(pi y) cos(pi y): one sincospi per coordinate
        const R g = (R)f.g[which];
        R sx, cx, sy, cy;
        sincospi_r(x, sx, cx);
        sincospi_r(y, sy, cy);
        fx = g * sx * sx * ((R)2 * sy * cy);
        fy = -g * sy * sy * ((R)2 * sx * cx);
        break;
    }
    case 3: {
        R dx = x - p2, dy = y - p3;
        R a = p0 * sqrt(dx * dx + dy * dy) + (R)f.g[which];
        fx = cos(a);
        fy = sin(a);
        break;
    }
    case 4: {
        R dx = x - (R)f.p[4], dy = y - (R)f.p[5];
        fx = p0 * dx + p1 * dy + (R)f.p[6];
        fy = p2 * dx + p3 * dy + (R)f.p[7];
        break;
    }
    default:
        fx = fy = (R)NAN;
    }
}

// eq. (eulero): q = x - dt f(x, t_{n+1}); midpoint: x* = x - dt/2 f(x, t_{n+1}),
// q = x - dt f(x*, t_{n+1} - dt/2)
template <typename R>
__device__ inline void foot_of(const FieldDev &f, int scheme, R x, R y, R dt, R &qx, R &qy)
{
    R fx, fy;
    field_eval<R>(f, 0, x, y, fx, fy);
    if (scheme == SLW_RK2) {
        R xs = x - (R)0.5 * dt * fx, ys = y - (R)0.5 * dt * fy;
        field_eval<R>(f, 1, xs, ys, fx, fy);
    }
    qx = x - dt * fx;
    qy = y - dt * fy;
}

}  // namespace

MeshView view_of(const DevMesh &m)
{
    MeshView v;
    v.geo = m.geo;
    v.wrec = m.wrec;
    v.tri_v = m.tri_v;
    v.tri_uf = m.tri_uf;
    v.tedge = m.tedge;
    v.dof_xy = m.dof_xy;
    v.qstart = m.qstart;
    v.vmin = m.vmin;
    v.dof_user = m.dof_user;
    v.tri_int = m.tri_int;
    v.prev = m.prev_elem;
    v.jump = m.jump;
    v.jump_g = m.jump_g;
    v.internal_order = m.internal_order;
    v.n_dofs = m.n_dofs;
    v.n_tris = m.n_tris;
    for (int i = 0; i < 4; ++i)
        v.bb[i] = m.bbox[i];
    v.fc = m.fc;
    v.step_cap = m.step_cap;
    v.hard_limit = m.hard_limit;
    // the hybrid's threshold; 0 picks the best measured for the far-foot
    // start the mesh has (one grid read; two binary searches; the steered start)
    v.hybrid_far = m.hybrid_far > 0.0f ? m.hybrid_far : (m.grid ? 1.0f : (m.chart_table ? 16.0f : 64.0f));
    v.xcd_chunk = m.xcd_chunk;
    v.lds_w = m.lds_w;
    v.bnext = m.bnext;
    v.bprev = m.bprev;
    v.n_boundary = m.n_boundary;
    v.bc_kind = m.bc_kind;
    for (int i = 0; i < 4; ++i)
        v.bc_p[i] = m.bc_p[i];
    v.nonconvex = m.nonconvex;
    v.qt_nodes = m.qt_nodes;
    v.qt_lists = m.qt_lists;
    for (int i = 0; i < 3; ++i)
        v.qt_box[i] = m.qt_box[i];
    v.qt_depth = m.qt_depth;
    v.bedge = m.bedge;
    v.bg_ptr = m.bg_ptr;
    v.bg_list = m.bg_list;
    v.bg_g = m.bg_g;
    v.bg_x0 = m.bg_x0;
    v.bg_y0 = m.bg_y0;
    v.bg_cell = m.bg_cell;
    v.chart_node = m.chart_node;
    v.chart_qx = m.chart_qx;
    v.chart_qy = m.chart_qy;
    v.chart_table = m.chart_table;
    v.chart_g = m.chart_g;
    v.grid = m.grid;
    v.grid_g = m.grid_g;
    v.grid_x0 = m.grid_x0;
    v.grid_y0 = m.grid_y0;
    v.grid_inv = m.grid_inv;
    v.mlp_wpack = m.mlp ? m.mlp->wpack : nullptr;
    v.mlp_bias = m.mlp ? m.mlp->bias : nullptr;
    v.mlp_norm = m.mlp ? m.mlp->norm : nullptr;
    return v;
}

namespace {

// ---------------------------------------------------------------------------
// start selection: strategy (a) of Section 3 (the walk starts at the DOF),
// in the incident triangle that faces the diagonal direction of the foot's
// quadrant

__device__ inline int32_t quadrant_start(const int4 qs, float dx, float dy)
{
    return dx >= 0.0f ? (dy >= 0.0f ? qs.x : qs.w) : (dy >= 0.0f ? qs.y : qs.z);
}

// Of two candidate start triangles, the one whose centroid lies nearer the
// foot q (float frame of the records)
template <bool F32>
__device__ inline int32_t nearer_start(const MeshView &mv, int32_t ja, int32_t jb, typename CT<F32>::R qx,
                                       typename CT<F32>::R qy)
{
    const float fx = F32 ? (float)qx : (float)((double)qx - mv.fc.cx);
    const float fy = F32 ? (float)qy : (float)((double)qy - mv.fc.cy);
    const WalkRec ra = mv.wrec[ja], rb = mv.wrec[jb];
    const float ax = (ra.p[0].x + ra.p[1].x + ra.p[2].x) * (1.f / 3.f) - fx;
    const float ay = (ra.p[0].y + ra.p[1].y + ra.p[2].y) * (1.f / 3.f) - fy;
    const float bx = (rb.p[0].x + rb.p[1].x + rb.p[2].x) * (1.f / 3.f) - fx;
    const float by = (rb.p[0].y + rb.p[1].y + rb.p[2].y) * (1.f / 3.f) - fy;
    return ax * ax + ay * ay < bx * bx + by * by ? ja : jb;
}

// The start id a DOF carries (given, previous or proposed), read before the
// foot is computed: the load does not depend on the foot, so its latency
// overlaps the field evaluation.  The quadrant table row of strategy (a) is
// read once the foot is known (holding it across the field evaluation would
// cost registers).
__device__ inline int32_t start_id(const MeshView &mv, int64_t d, int64_t api, int mode,
                                   const int32_t *__restrict__ start)
{
    if (mode == SLW_START_GIVEN || mode == SLW_START_FIXED)
        return start[mode == SLW_START_GIVEN ? api : 0];  // user id
    if (mode == SLW_START_PREV) {
        const int32_t v = load_stream(mv.prev + d);
        return v >= 0 ? (v & kPrevElemMask) : v;  // without the hybrid's skip count
    }
    if (mode == SLW_START_LEARNED || mode == SLW_START_CHART || mode == SLW_START_LEARNED_INDEX)
        return start[d];  // internal id from the chart
    return -1;
}

// Jump-and-walk start (Muecke, Saias and Zhu 1996): the triangle recorded for
// the cell of the uniform start grid that holds the foot (the grid must
// exist; the foot lies in the mesh's bounding box)
template <typename R>
__device__ inline int32_t grid_start(const MeshView &mv, R qx, R qy)
{
    const int g = mv.grid_g;
    int cx = (int)((float)(((double)qx - mv.grid_x0) * mv.grid_inv));
    int cy = (int)((float)(((double)qy - mv.grid_y0) * mv.grid_inv));
    cx = cx < 0 ? 0 : (cx >= g ? g - 1 : cx);
    cy = cy < 0 ? 0 : (cy >= g ? g - 1 : cy);
    return mv.grid[(int64_t)cy * g + cx];
}

// GRID: whether the grid rule is compiled in (the plain step kernel leaves it
// out; SLW_START_GRID has an instantiation of its own)
template <bool GRID, typename R, typename R2>
__device__ inline int32_t start_pick(const MeshView &mv, int64_t d, int32_t id, int mode, R2 x, R qx, R qy)
{
    // caller-given ids outside [0, n_tris) fall back to the steered start
    if (mode == SLW_START_GIVEN || mode == SLW_START_FIXED) {
        if (id >= 0 && id < mv.n_tris)
            return mv.tri_int[id];
    } else if (mode == SLW_START_PREV) {
        if (id >= 0)
            return id;
    } else if (mode == SLW_START_LEARNED || mode == SLW_START_CHART || mode == SLW_START_LEARNED_INDEX) {
        if (id >= 0 && id < mv.n_tris)
            return id;
    } else if (GRID && mode == SLW_START_GRID) {
        return grid_start(mv, qx, qy);
    }
    return quadrant_start(mv.qstart[d], (float)(qx - x.x), (float)(qy - x.y));
}

template <bool F32>
__device__ inline int32_t start_for(const MeshView &mv, int64_t d, int64_t api, int mode,
                                    const int32_t *__restrict__ start, typename CT<F32>::R2 x,
                                    typename CT<F32>::R qx, typename CT<F32>::R qy)
{
    return start_pick<true>(mv, d, start_id(mv, d, api, mode, start), mode, x, qx, qy);
}

// ---------------------------------------------------------------------------
// exact signs

struct Counters {
    uint32_t exact = 0, fp64 = 0;
};

// sign of orient(a, b, q) on the exact coordinates (FP64 filter, then
// exact), for the rare tests the float filter cannot certify; the exact
// coordinates of a double mesh are read through the vertex ids va, vb
template <bool F32>
__device__ __noinline__ int slow_sign(const void *dof_xy, float2 pa, float2 pb, int32_t va, int32_t vb,
                                      typename CT<F32>::R qx, typename CT<F32>::R qy)
{
    double ax, ay, bx, by;
    if constexpr (F32) {
        ax = pa.x;
        ay = pa.y;
        bx = pb.x;
        by = pb.y;
    } else {
        const double2 *X = (const double2 *)dof_xy;
        const double2 A = X[va], B = X[vb];
        ax = A.x;
        ay = A.y;
        bx = B.x;
        by = B.y;
    }
    bool certain;
    const double d = orient_fp64(ax, ay, bx, by, (double)qx, (double)qy, certain);
    if (certain)
        return sign_of(d);
    return 2 * orient_exact_sign(ax, ay, bx, by, (double)qx, (double)qy);  // x2: tells the caller it was exact
}

// Signs of the three edge orientations o_k = orient(x_{k+1}, x_{k+2}, q) of
// triangle j with float vertex coordinates p: the float filter on the
// rounded inputs (filter_sign_f32) decides when its bound allows, the exact
// coordinates otherwise (read through the vertex ids of geo[j]).  o[] keeps
// the float values, used to pick among negative edges (any negative edge is
// a valid move).
template <bool F32>
__device__ inline void edge_signs(const MeshView &mv, int32_t j, const float2 p[3], float qfx, float qfy,
                                  typename CT<F32>::R qx, typename CT<F32>::R qy, float o[3], int s[3], Counters &c)
{
    float dx[3], dy[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dx[k] = p[k].x - qfx;
        dy[k] = p[k].y - qfy;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        s[k] = filter_sign_f32(dx[a], dy[a], dx[b], dy[b], mv.fc.c1, mv.fc.c2, mv.fc.c3, o[k]);
    }
    if ((s[0] == 0) | (s[1] == 0) | (s[2] == 0)) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (s[k] == 0) {
                const int a = (k + 1) % 3, b = (k + 2) % 3;
                // double meshes read the exact coordinates through the vertex
                // ids; float meshes' record coordinates are exact
                int32_t va = -1, vb = -1;
                if constexpr (!F32) {
                    va = mv.geo[j].v[a];
                    vb = mv.geo[j].v[b];
                }
                const int sg = slow_sign<F32>(mv.dof_xy, p[a], p[b], va, vb, qx, qy);
                ++c.fp64;
                c.exact += (sg == 2 || sg == -2 || sg == 0);
                s[k] = sg > 0 ? 1 : (sg < 0 ? -1 : 0);
            }
        }
    }
}

// the three neighbour codes of a walk record (offsets, 0 boundary,
// kCodeEscape: read GeoRec::nb)
__device__ inline void nb_codes(const WalkRec &r, int32_t cd[3])
{
    static_assert(kCodeBits == 21, "decoding assumes 21-bit codes");
    cd[0] = (int32_t)(r.lo << 11) >> 11;
    cd[1] = (int32_t)(__builtin_amdgcn_alignbit(r.hi, r.lo, 21) << 11) >> 11;
    cd[2] = (int32_t)(r.hi << 1) >> 11;
}

// neighbour k of triangle j from its code (-1 on the boundary)
__device__ inline int32_t nb_of(const MeshView &mv, int32_t j, int k, int32_t code)
{
    if (code == kCodeEscape)
        return mv.geo[j].nb[k];
    return code == 0 ? -1 : j + code;
}

// {nb[2], v[0], v[1], v[2]} of triangle j: the vertex ids with one load
// {nb[2], v[0], v[1], v[2]} of triangle j: the vertex ids with one load, from
// the compact 16-byte copy (a walk's end reads eight triangles per cache
// line instead of the 48-byte records' two or three)
__device__ inline int4 tri_verts(const MeshView &mv, int32_t j) { return mv.tri_v[j]; }
// the same four ids inside the 48-byte record, for reads of the whole record
__device__ inline int4 geo_verts(const MeshView &mv, int32_t j) { return ((const int4 *)(mv.geo + j))[2]; }

__device__ inline int32_t sel3(int k, int32_t a, int32_t b, int32_t c) { return k == 0 ? a : (k == 1 ? b : c); }

__device__ inline uint32_t hash32(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

template <typename R>
struct WalkResult {
    int32_t elem;   // internal triangle id, -1 outside
    int32_t steps;  // element changes
    int32_t flags;  // bit0 fallback walk, bit1 hard limit, bit2 edge tie, bit3 vertex tie,
                    // bit4 left the domain through the boundary edge v[0] -> v[1]
    int32_t v[3];   // internal vertex DOF ids of elem
    R th[3];        // barycentric coordinates in the internal (counter-clockwise) vertex order of elem
};

template <typename R>
__device__ inline WalkResult<R> outside_result(int32_t steps, int32_t flags)
{
    WalkResult<R> w;
    w.elem = -1;
    w.steps = steps;
    w.flags = flags;
    w.v[0] = w.v[1] = w.v[2] = -1;
    w.th[0] = w.th[1] = w.th[2] = (R)0;
    return w;
}

// One move of the barycentric walk of Section 2.2 from triangle j towards
// the foot q: 0 = moved (j is the next triangle), 1 = stopped (every
// coordinate >= 0: r is j's record, zmask has bit k set when s_k = 0),
// 2 = outside (a negative coordinate across boundary edge zmask of r; or
// the hard step limit: then zmask = -1 and flags gets bits 0 and 1).
template <bool F32>
__device__ inline int walk_move(const MeshView &mv, int32_t &j, WalkRec &r, int &zmask, float qfx, float qfy,
                                typename CT<F32>::R qx, typename CT<F32>::R qy, uint32_t seed, int32_t &steps,
                                int32_t &flags, Counters &c)
{
    float o[3];
    int s[3];
    r = mv.wrec[j];
    edge_signs<F32>(mv, j, r.p, qfx, qfy, qx, qy, o, s, c);
    const bool n0 = s[0] < 0, n1 = s[1] < 0, n2 = s[2] < 0;
    if (!(n0 | n1 | n2)) {
        zmask = (int)(s[0] == 0) | ((int)(s[1] == 0) << 1) | ((int)(s[2] == 0) << 2);
        return 1;
    }
    int32_t cd[3];
    nb_codes(r, cd);
    // a negative side on the boundary: the foot is outside the (convex) domain;
    // zmask tells through which edge
    const bool x0 = n0 && cd[0] == 0, x1 = n1 && cd[1] == 0, x2 = n2 && cd[2] == 0;
    if (x0 || x1 || x2) {
        zmask = x0 ? 0 : (x1 ? 1 : 2);
        return 2;
    }
    if (steps >= mv.hard_limit) {
        flags |= 3;
        zmask = -1;
        return 2;
    }
    int k;
    if (steps < mv.step_cap) {
        // most negative barycentric coordinate, lowest index on ties
        // (selects rather than indexing, so the record stays in registers)
        const float m0 = n0 ? o[0] : INFINITY, m1 = n1 ? o[1] : INFINITY, m2 = n2 ? o[2] : INFINITY;
        k = (m1 < m0) ? ((m2 < m1) ? 2 : 1) : ((m2 < m0) ? 2 : 0);
    } else {
        // randomised visibility walk: a uniformly chosen separating edge
        // (terminates with probability 1 on any triangulation)
        flags |= 1;
        const int cnt = (int)n0 + (int)n1 + (int)n2;
        const int pick = (int)(hash32(seed ^ hash32((uint32_t)steps)) % (uint32_t)cnt);
        // the pick-th negative edge
        const int first = n0 ? 0 : (n1 ? 1 : 2);
        const int second = (n0 && n1) ? 1 : 2;
        k = pick == 0 ? first : (pick == 1 ? second : 2);
    }
    const int32_t ck = sel3(k, cd[0], cd[1], cd[2]);  // never 0 here: edge k is interior
    j = ck == kCodeEscape ? mv.geo[j].nb[k] : j + ck;
    ++steps;
    return 0;
}

// Barycentric coordinates of q in a triangle (internal counter-clockwise
// vertex order; float coordinates p, vertex ids v) on the exact coordinates:
// theta_k = o_k / (o_0 + o_1 + o_2), o_k = orient(x_{k+1}, x_{k+2}, q)
template <bool F32>
__device__ inline void exact_weights(const MeshView &mv, const float2 p[3], const int32_t v[3],
                                     typename CT<F32>::R qx, typename CT<F32>::R qy, typename CT<F32>::R th[3])
{
    using R = typename CT<F32>::R;
    R ex[3], ey[3];
    if constexpr (F32) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ex[k] = p[k].x - qx;
            ey[k] = p[k].y - qy;
        }
    } else {
        const double2 *X = (const double2 *)mv.dof_xy;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double2 xv = X[v[k]];
            ex[k] = xv.x - qx;
            ey[k] = xv.y - qy;
        }
    }
    R oo[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        oo[k] = ex[a] * ey[b] - ey[a] * ex[b];
    }
    const R sum = oo[0] + oo[1] + oo[2];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        th[k] = oo[k] / sum;
}

// End of a walk that stopped in triangle j (float vertex coordinates p,
// zero-sign mask zmask; nbz = the neighbour across the zero edge when exactly
// one sign is zero): the tie rule (smallest user id among the closed
// containers), then the weights on the exact coordinates.  tv_j holds j's
// vertex ids when have_tv.
template <bool F32>
__device__ inline WalkResult<typename CT<F32>::R> finish_walk(const MeshView &mv, int32_t j, const float2 pj[3],
                                                              int32_t nbz, int zmask, int32_t steps, int32_t flags,
                                                              typename CT<F32>::R qx, typename CT<F32>::R qy,
                                                              bool have_tv = false, int4 tv_j = int4())
{
    using R = typename CT<F32>::R;
    const int z = (zmask & 1) + ((zmask >> 1) & 1) + ((zmask >> 2) & 1);
    int4 tv = have_tv ? tv_j : tri_verts(mv, j);
    int32_t e = j;
    if (z == 1) {
        flags |= 4;
        if (nbz >= 0 && (mv.tri_uf[nbz] & kUidMask) < (mv.tri_uf[j] & kUidMask))
            e = nbz;
    } else if (z == 2) {
        const int cidx = !(zmask & 1) ? 0 : (!(zmask & 2) ? 1 : 2);
        flags |= 8;
        e = mv.vmin[sel3(cidx, tv.y, tv.z, tv.w)];
    }
    float2 p[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        p[k] = pj[k];
    if (e != j) {
        tv = tri_verts(mv, e);
        if constexpr (F32) {
            const WalkRec re = mv.wrec[e];
#pragma unroll
            for (int k = 0; k < 3; ++k)
                p[k] = re.p[k];
        }
    }
    WalkResult<R> w;
    w.elem = e;
    w.steps = steps;
    w.flags = flags;
    w.v[0] = tv.y;
    w.v[1] = tv.z;
    w.v[2] = tv.w;
    exact_weights<F32>(mv, p, w.v, qx, qy, w.th);
    return w;
}

// the neighbour across the zero edge of a stop with one zero sign (-1 otherwise)
__device__ inline int32_t zero_edge_nb(const MeshView &mv, int32_t j, const WalkRec &r, int zmask)
{
    if (zmask != 1 && zmask != 2 && zmask != 4)
        return -1;
    const int k = zmask == 1 ? 0 : (zmask == 2 ? 1 : 2);
    int32_t cd[3];
    nb_codes(r, cd);
    return nb_of(mv, j, k, sel3(k, cd[0], cd[1], cd[2]));
}

template <bool F32>
__device__ inline WalkResult<typename CT<F32>::R> finish_walk_rec(const MeshView &mv, int32_t j, const WalkRec &r,
                                                                  int zmask, int32_t steps, int32_t flags,
                                                                  typename CT<F32>::R qx, typename CT<F32>::R qy)
{
    return finish_walk<F32>(mv, j, r.p, zero_edge_nb(mv, j, r, zmask), zmask, steps, flags, qx, qy);
}

// One move of the deterministic walk from triangle j (walk record r already
// read) towards q: 0 = moved (j is the next triangle, steps counted), 1 =
// stopped (zmask: zero signs), 2 = outside (zmask: the boundary edge).  No
// step limit here (the callers bound the moves).
template <bool F32>
__device__ inline int det_move(const MeshView &mv, int32_t &j, const WalkRec &r, int &zmask, float qfx, float qfy,
                               typename CT<F32>::R qx, typename CT<F32>::R qy, int32_t &steps, Counters &c)
{
    float o[3];
    int s[3];
    edge_signs<F32>(mv, j, r.p, qfx, qfy, qx, qy, o, s, c);
    const bool n0 = s[0] < 0, n1 = s[1] < 0, n2 = s[2] < 0;
    if (!(n0 | n1 | n2)) {
        zmask = (int)(s[0] == 0) | ((int)(s[1] == 0) << 1) | ((int)(s[2] == 0) << 2);
        return 1;
    }
    int32_t cd[3];
    nb_codes(r, cd);
    const bool x0 = n0 && cd[0] == 0, x1 = n1 && cd[1] == 0, x2 = n2 && cd[2] == 0;
    if (x0 || x1 || x2) {
        zmask = x0 ? 0 : (x1 ? 1 : 2);
        return 2;
    }
    const float m0 = n0 ? o[0] : INFINITY, m1 = n1 ? o[1] : INFINITY, m2 = n2 ? o[2] : INFINITY;
    const int k = (m1 < m0) ? ((m2 < m1) ? 2 : 1) : ((m2 < m0) ? 2 : 0);
    const int32_t ck = sel3(k, cd[0], cd[1], cd[2]);  // never 0: edge k is interior
    j = ck == kCodeEscape ? mv.geo[j].nb[k] : j + ck;
    ++steps;
    return 0;
}

// Exact point location without a walk (the quadtree of Section 2.1): descend
// to the leaf that holds q (a point on a split line goes to the upper/right
// child; a triangle is listed in every leaf its closed bounding box touches,
// so every closed container of q is in q's leaf), test every listed triangle
// with the walk's exact signs, keep the smallest user id among the closed
// containers: the walk's answer by definition.  Returns its internal id (rb:
// its walk record), or -1 when no triangle contains q.  Needs mv.qt_nodes.
template <bool F32>
__device__ inline int32_t qt_find(const MeshView &mv, typename CT<F32>::R qx, typename CT<F32>::R qy,
                                        WalkRec &rb, Counters &c)
{
    const float qfx = F32 ? (float)qx : (float)((double)qx - mv.fc.cx);
    const float qfy = F32 ? (float)qy : (float)((double)qy - mv.fc.cy);
    double bx = mv.qt_box[0], by = mv.qt_box[1], s = mv.qt_box[2];
    int4 nd = mv.qt_nodes[0];
    for (int depth = 0; nd.x >= 0 && depth < mv.qt_depth; ++depth) {
        s *= 0.5;
        const int right = (double)qx >= bx + s, top = (double)qy >= by + s;
        bx += right ? s : 0.0;
        by += top ? s : 0.0;
        nd = mv.qt_nodes[nd.x + right + 2 * top];
    }
    int32_t best = -1, best_uid = 0x7fffffff;
    for (int32_t k = 0; k < nd.z; ++k) {
        const int32_t t = mv.qt_lists[nd.y + k];
        const WalkRec r = mv.wrec[t];
        float o[3];
        int sg[3];
        edge_signs<F32>(mv, t, r.p, qfx, qfy, qx, qy, o, sg, c);
        if (sg[0] >= 0 && sg[1] >= 0 && sg[2] >= 0) {
            const int32_t uid = mv.tri_uf[t] & kUidMask;
            if (uid < best_uid) {
                best_uid = uid;
                best = t;
                rb = r;
            }
        }
    }
    return best;
}

// End of a walk whose deterministic moves stopped with status st (0: the step
// cap was reached; the walk goes on with the randomised choice and the hard
// limit), then the outside result or the tie rule and the weights.
template <bool F32>
__device__ inline WalkResult<typename CT<F32>::R> walk_end(const MeshView &mv, int32_t j, WalkRec r, int zmask,
                                                           float qfx, float qfy, typename CT<F32>::R qx,
                                                           typename CT<F32>::R qy, uint32_t seed, int32_t steps,
                                                           int32_t flags, int st, Counters &c)
{
    using R = typename CT<F32>::R;
    while (st == 0)
        st = walk_move<F32>(mv, j, r, zmask, qfx, qfy, qx, qy, seed, steps, flags, c);
    if (st == 2 && zmask >= 0 && mv.nonconvex) {
        // blocked by the boundary of a domain that is not one convex disk:
        // the foot may lie across a notch or a hole, so the exact search
        // decides (flag bit 5)
        WalkRec rb;
        const int32_t e = qt_find<F32>(mv, qx, qy, rb, c);
        flags |= 32;
        if (e < 0) {
            WalkResult<R> w = outside_result<R>(steps, flags | 16);  // crossing: scanned by the caller
            return w;
        }
        const int4 tv = tri_verts(mv, e);
        WalkResult<R> w;
        w.elem = e;
        w.steps = steps;
        w.flags = flags;
        w.v[0] = tv.y;
        w.v[1] = tv.z;
        w.v[2] = tv.w;
        exact_weights<F32>(mv, rb.p, w.v, qx, qy, w.th);
        return w;
    }
    if (st == 2) {
        WalkResult<R> w = outside_result<R>(steps, flags);
        if (zmask >= 0) {  // the boundary edge opposite vertex zmask, counter-clockwise
            const int4 tv = tri_verts(mv, j);
            w.v[0] = sel3(zmask, tv.z, tv.w, tv.y);
            w.v[1] = sel3(zmask, tv.w, tv.y, tv.z);
            w.flags |= 16;
        }
        return w;
    }
    return finish_walk_rec<F32>(mv, j, r, zmask, steps, flags, qx, qy);
}

// The first test of a walk on a likely start j (the previous element):
// 1 = the foot is in j (res holds the located result, tie rule and weights
// done), 0 = it is not; then theta_min is the smallest barycentric
// coordinate of the foot in j (float, from the filter's determinants): the
// foot lies about -theta_min heights of j beyond its nearest side.
template <bool F32>
__device__ inline int first_test(const MeshView &mv, int32_t j, typename CT<F32>::R qx, typename CT<F32>::R qy,
                                 float &theta_min, WalkResult<typename CT<F32>::R> &res, Counters &c)
{
    const float qfx = F32 ? (float)qx : (float)((double)qx - mv.fc.cx);
    const float qfy = F32 ? (float)qy : (float)((double)qy - mv.fc.cy);
    const float4 p01 = ((const float4 *)(mv.geo + j))[0];
    const float2 p2 = ((const float2 *)(mv.geo + j))[2];
    const int4 tv = geo_verts(mv, j);  // {nb[2], v[0], v[1], v[2]}
    const float2 pj[3] = {make_float2(p01.x, p01.y), make_float2(p01.z, p01.w), p2};
    float o[3];
    int s[3];
    Counters c0;
    edge_signs<F32>(mv, j, pj, qfx, qfy, qx, qy, o, s, c0);
    if (s[0] >= 0 && s[1] >= 0 && s[2] >= 0) {
        c.exact += c0.exact;
        c.fp64 += c0.fp64;
        const int zm = (int)(s[0] == 0) | ((int)(s[1] == 0) << 1) | ((int)(s[2] == 0) << 2);
        const int32_t nbz = zm == 4 ? tv.x : ((zm == 1 || zm == 2) ? mv.geo[j].nb[zm >> 1] : -1);
        res = finish_walk<F32>(mv, j, pj, nbz, zm, 0, 0, qx, qy, true, tv);
        return 1;
    }
    const float sum = o[0] + o[1] + o[2];  // twice the area (> 0)
    theta_min = fminf(fminf(o[0], o[1]), o[2]) / sum;
    return 0;
}

// Barycentric walk of Section 2.2 from triangle j to the foot q, then the tie
// rule, then the weights; fetch(t) gives triangle t's walk record.
template <bool F32, typename Fetch>
__device__ __forceinline__ WalkResult<typename CT<F32>::R> walk_with(const MeshView &mv, int32_t j,
                                                                     typename CT<F32>::R qx, typename CT<F32>::R qy,
                                                                     uint32_t seed, Counters &c, bool likely_stop,
                                                                     Fetch fetch)
{
    const float qfx = F32 ? (float)qx : (float)((double)qx - mv.fc.cx);
    const float qfy = F32 ? (float)qy : (float)((double)qy - mv.fc.cy);
    // when the start is likely to contain the foot (strategy (b)), the first
    // test reads its full record (coordinates, neighbours and vertex ids in
    // one place); if the foot lies elsewhere the walk starts there as usual
    if (likely_stop) {
        const float4 p01 = ((const float4 *)(mv.geo + j))[0];
        const float2 p2 = ((const float2 *)(mv.geo + j))[2];
        const int4 tv = geo_verts(mv, j);  // {nb[2], v[0], v[1], v[2]}
        const float2 pj[3] = {make_float2(p01.x, p01.y), make_float2(p01.z, p01.w), p2};
        float o[3];
        int s[3];
        Counters c0;  // counted only if the walk ends here (else the loop repeats the test)
        edge_signs<F32>(mv, j, pj, qfx, qfy, qx, qy, o, s, c0);
        if (s[0] >= 0 && s[1] >= 0 && s[2] >= 0) {
            c.exact += c0.exact;
            c.fp64 += c0.fp64;
            const int zm = (int)(s[0] == 0) | ((int)(s[1] == 0) << 1) | ((int)(s[2] == 0) << 2);
            const int32_t nbz = zm == 4 ? tv.x : ((zm == 1 || zm == 2) ? mv.geo[j].nb[zm >> 1] : -1);
            return finish_walk<F32>(mv, j, pj, nbz, zm, 0, 0, qx, qy, true, tv);
        }
    }
    WalkRec r{};
    int zmask = 0;
    int32_t steps = 0, flags = 0;
    int st = 0;
    // the deterministic walk (most negative coordinate) up to the step cap,
    // in a loop of its own: the cap, the hard limit and the randomised choice
    // stay out of the hot loop
    const int32_t fast_lim = mv.step_cap < mv.hard_limit ? mv.step_cap : mv.hard_limit;
    while (steps < fast_lim) {
        r = fetch(j);
        st = det_move<F32>(mv, j, r, zmask, qfx, qfy, qx, qy, steps, c);
        if (st != 0)
            break;
    }
    return walk_end<F32>(mv, j, r, zmask, qfx, qfy, qx, qy, seed, steps, flags, st, c);
}

template <bool F32>
__device__ WalkResult<typename CT<F32>::R> walk(const MeshView &mv, int32_t j, typename CT<F32>::R qx,
                                                 typename CT<F32>::R qy, uint32_t seed, Counters &c,
                                                 bool likely_stop = false)
{
    return walk_with<F32>(mv, j, qx, qy, seed, c, likely_stop, [&](int32_t t) { return mv.wrec[t]; });
}

// The walk of the staged-window step: the records of triangles
// [lbase, lbase + lcount) come from the workgroup's copy in LDS.
template <bool F32>
__device__ WalkResult<typename CT<F32>::R> walk_win(const MeshView &mv, int32_t j, typename CT<F32>::R qx,
                                                     typename CT<F32>::R qy, uint32_t seed, Counters &c,
                                                     const WalkRec *lw, int32_t lbase, int32_t lcount)
{
    return walk_with<F32>(mv, j, qx, qy, seed, c, false, [&](int32_t t) {
        return (uint32_t)(t - lbase) < (uint32_t)lcount ? lw[t - lbase] : mv.wrec[t];
    });
}

__device__ inline unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}
__device__ inline unsigned long long wave_max(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long w = __shfl_xor(v, off, 64);
        v = w > v ? w : v;
    }
    return v;
}

struct LaneStats {
    uint32_t feet = 0, outside = 0, steps = 0, max_steps = 0, fallback = 0, edge = 0, vertex = 0, hard = 0,
             search = 0;
    Counters c;
    template <typename R>
    __device__ void add(const WalkResult<R> &w)
    {
        ++feet;
        outside += w.elem < 0;
        steps += w.steps;
        max_steps = max_steps > (uint32_t)w.steps ? max_steps : (uint32_t)w.steps;
        fallback += (w.flags & 1) != 0;
        hard += (w.flags & 2) != 0;
        edge += (w.flags & 4) != 0;
        vertex += (w.flags & 8) != 0;
        search += (w.flags & 32) != 0;
    }
    // a walk's end (inside or outside) and, separately, its tie flags
    __device__ void add_walk(bool inside, int32_t st, int32_t flags)
    {
        ++feet;
        outside += !inside;
        steps += st;
        max_steps = max_steps > (uint32_t)st ? max_steps : (uint32_t)st;
        fallback += (flags & 1) != 0;
        hard += (flags & 2) != 0;
    }
    __device__ void add_ties(int32_t flags)
    {
        edge += (flags & 4) != 0;
        vertex += (flags & 8) != 0;
    }
};

// called by every lane of the wavefront
__device__ inline void flush_stats(const LaneStats &ls, DevStats *st)
{
    unsigned long long v[11] = {ls.feet, ls.outside, ls.steps, ls.max_steps, ls.c.exact, ls.c.fp64, ls.fallback,
                                ls.edge, ls.vertex, ls.hard, ls.search};
    unsigned long long *dst[11] = {&st->feet, &st->outside, &st->walk_steps, &st->max_steps, &st->exact_tests,
                                   &st->fp64_tests, &st->fallback_walks, &st->edge_ties, &st->vertex_ties,
                                   &st->hard_fail, &st->boundary_searches};
    const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
    for (int i = 0; i < 11; ++i) {
        unsigned long long r = (i == 3) ? wave_max(v[i]) : wave_sum(v[i]);
        if (lead && r != 0) {
            if (i == 3)
                atomicMax(dst[i], r);
            else
                atomicAdd(dst[i], r);
        }
    }
}

// bin of a walk of `steps` element changes in DevStats::step_hist
__device__ inline int hist_bin(int32_t steps)
{
    if (steps <= 0)
        return 0;
    const int b = 32 - __clz(steps);  // steps in [2^(b-1), 2^b)
    return b < kHistBins - 1 ? b : kHistBins - 1;
}

// one walk per calling lane into the histogram: the calling lanes are
// grouped by bin, one atomic per distinct bin
__device__ inline void hist_add(DevStats *st, int32_t steps)
{
    const int bin = hist_bin(steps);
    unsigned long long todo = __ballot(1);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lb = __shfl(bin, leader, kWave);
        const unsigned long long same = __ballot(bin == lb) & todo;
        if ((int)(threadIdx.x & (kWave - 1)) == leader)
            atomicAdd(&st->step_hist[lb], (unsigned long long)__popcll(same));
        todo &= ~same;
    }
}

// queries outside the mesh's bounding box (or not finite) are outside
// without a walk; written so that NaN compares false
template <typename R>
__device__ inline bool in_box(R qx, R qy, const double bb[4])
{
    return (double)qx >= bb[0] && (double)qx <= bb[2] && (double)qy >= bb[1] && (double)qy <= bb[3];
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b mod 8).  Tiles are consecutive in the Morton order.  chunk = 0 gives each
// XCD one contiguous range of tiles, so the records and value rows its tiles
// share stay in its L2; but the walk lengths of a graded mesh differ between
// regions, and the XCD whose range holds the refined part finishes last.
// chunk = C > 0 deals chunks of C consecutive tiles to the XCDs in turn, so
// every XCD gets the same mix of regions; the last, incomplete round of
// chunks falls back to contiguous ranges.  Both are bijections of
// [0, nb) onto the tiles.
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb, int64_t chunk = 0)
{
    constexpr int64_t kXcd = 8;
    if (chunk > 0) {
        const int64_t full = nb / (kXcd * chunk) * (kXcd * chunk);
        if (b < full) {
            const int64_t x = b % kXcd, local = b / kXcd;
            return ((local / chunk) * kXcd + x) * chunk + local % chunk;
        }
        b -= full;  // a multiple of 8 was taken off: b keeps its XCD
        nb -= full;
        const int64_t q = nb / kXcd, r = nb % kXcd;
        const int64_t x = b % kXcd, local = b / kXcd;
        return full + (x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local);
    }
    const int64_t q = nb / kXcd, r = nb % kXcd;
    const int64_t x = b % kXcd, local = b / kXcd;
    return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

template <typename R>
__device__ inline void user_bary(int32_t uf, const R th[3], R out[3])
{
    out[0] = th[0];
    if (uf < 0) {  // vertices 1 and 2 were swapped at upload
        out[1] = th[2];
        out[2] = th[1];
    } else {
        out[1] = th[1];
        out[2] = th[2];
    }
}

// ---------------------------------------------------------------------------
// kernels

template <bool F32>
__global__ void __launch_bounds__(kBlock) k_locate(MeshView mv, const typename CT<F32>::R2 *__restrict__ q,
                                                   int64_t m, const int32_t *__restrict__ start,
                                                   int32_t *__restrict__ elem, typename CT<F32>::R *__restrict__ bary,
                                                   int32_t *__restrict__ steps, DevStats *st)
{
    using R = typename CT<F32>::R;
    LaneStats ls;
    const int64_t i = xcd_tile(blockIdx.x, gridDim.x, mv.xcd_chunk) * kBlock + threadIdx.x;
    if (i < m) {
        R qx = q[i].x, qy = q[i].y;
        WalkResult<R> w = outside_result<R>(0, 0);
        if (in_box<R>(qx, qy, mv.bb)) {
            int32_t j0;
            const int32_t su = start ? start[i] : -1;
            if (su >= 0 && su < mv.n_tris) {
                j0 = mv.tri_int[su];
            } else {
                const double wx = (mv.bb[2] - mv.bb[0]), wy = (mv.bb[3] - mv.bb[1]);
                const double span = wx > wy ? wx : wy;
                const double cw = span > 0 ? span / mv.jump_g : 1.0;
                int cx = (int)floor(((double)qx - mv.bb[0]) / cw), cy = (int)floor(((double)qy - mv.bb[1]) / cw);
                cx = cx < 0 ? 0 : (cx >= mv.jump_g ? mv.jump_g - 1 : cx);
                cy = cy < 0 ? 0 : (cy >= mv.jump_g ? mv.jump_g - 1 : cy);
                j0 = mv.jump[(int64_t)cy * mv.jump_g + cx];
            }
            w = walk<F32>(mv, j0, qx, qy, (uint32_t)i * 2654435761u, ls.c);
        }
        if (st) {
            ls.add(w);
            hist_add(st, w.steps);
        }
        const int32_t uf = w.elem >= 0 ? mv.tri_uf[w.elem] : -1;
        elem[i] = w.elem >= 0 ? (uf & kUidMask) : -1;
        if (bary) {
            if (w.elem >= 0) {
                R ub[3];
                user_bary<R>(uf, w.th, ub);
                bary[3 * i] = ub[0];
                bary[3 * i + 1] = ub[1];
                bary[3 * i + 2] = ub[2];
            } else {
                bary[3 * i] = bary[3 * i + 1] = bary[3 * i + 2] = (R)NAN;
            }
        }
        if (steps)
            steps[i] = w.steps;
    }
    if (st)
        flush_stats(ls, st);
}

// Non-walking locator for comparison (the quadtree of Section 2.1): every
// query by the exact search qt_find, no walk.
template <bool F32>
__global__ void __launch_bounds__(kBlock)
    k_qt_locate(MeshView mv, const typename CT<F32>::R2 *__restrict__ q, int64_t m, int32_t *__restrict__ elem,
                typename CT<F32>::R *__restrict__ bary, DevStats *st)
{
    using R = typename CT<F32>::R;
    LaneStats ls;
    const int64_t i = xcd_tile(blockIdx.x, gridDim.x, mv.xcd_chunk) * kBlock + threadIdx.x;
    if (i < m) {
        const R qx = q[i].x, qy = q[i].y;
        int32_t best = -1;
        WalkRec rb;
        if (in_box<R>(qx, qy, mv.bb))
            best = qt_find<F32>(mv, qx, qy, rb, ls.c);
        if (st) {
            ++ls.feet;
            ls.outside += best < 0;
        }
        elem[i] = best >= 0 ? (mv.tri_uf[best] & kUidMask) : -1;
        if (bary) {
            if (best >= 0) {
                R th[3], ub[3];
                const int4 tv = tri_verts(mv, best);
                const int32_t v[3] = {tv.y, tv.z, tv.w};
                exact_weights<F32>(mv, rb.p, v, qx, qy, th);
                user_bary<R>(mv.tri_uf[best], th, ub);
                bary[3 * i] = ub[0];
                bary[3 * i + 1] = ub[1];
                bary[3 * i + 2] = ub[2];
            } else {
                bary[3 * i] = bary[3 * i + 1] = bary[3 * i + 2] = (R)NAN;
            }
        }
    }
    if (st)
        flush_stats(ls, st);
}

// The jump-and-walk start grid: cell c of a g x g grid of square cells from
// (x0, y0) records the triangle that holds its centre, located by the walk
// from the upload's coarse bucket grid; a centre outside the mesh keeps the
// coarse grid's triangle (any start gives the same results).
template <bool F32>
__global__ void __launch_bounds__(kBlock) k_grid_build(MeshView mv, int32_t *__restrict__ grid, int g, double x0,
                                                       double y0, double cell)
{
    using R = typename CT<F32>::R;
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= (int64_t)g * g)
        return;
    const int cx = (int)(c % g), cy = (int)(c / g);
    const double px = x0 + ((double)cx + 0.5) * cell, py = y0 + ((double)cy + 0.5) * cell;
    const double wx = mv.bb[2] - mv.bb[0], wy = mv.bb[3] - mv.bb[1];
    const double span = wx > wy ? wx : wy;
    const double cw = span > 0 ? span / mv.jump_g : 1.0;
    int jx = (int)floor((px - mv.bb[0]) / cw), jy = (int)floor((py - mv.bb[1]) / cw);
    jx = jx < 0 ? 0 : (jx >= mv.jump_g ? mv.jump_g - 1 : jx);
    jy = jy < 0 ? 0 : (jy >= mv.jump_g ? mv.jump_g - 1 : jy);
    const int32_t j0 = mv.jump[(int64_t)jy * mv.jump_g + jx];
    int32_t j = j0;
    const R qx = (R)px, qy = (R)py;
    if (in_box<R>(qx, qy, mv.bb)) {
        LaneStats ls;
        const WalkResult<R> w = walk<F32>(mv, j0, qx, qy, (uint32_t)c * 2654435761u, ls.c);
        if (w.elem >= 0)
            j = w.elem;
    }
    grid[c] = j;
}

template <bool F32>
__global__ void __launch_bounds__(kBlock)
    k_locate_feet(MeshView mv, FieldDev f, double dt, int scheme, int mode, const int32_t *__restrict__ start,
                  int feet_in, typename CT<F32>::R2 *__restrict__ feet, int32_t *__restrict__ elem,
                  typename CT<F32>::R *__restrict__ bary, int32_t *__restrict__ steps, DevStats *st)
{
    using R = typename CT<F32>::R;
    using R2 = typename CT<F32>::R2;
    LaneStats ls;
    const int64_t d = xcd_tile(blockIdx.x, gridDim.x, mv.xcd_chunk) * kBlock + threadIdx.x;
    if (d < mv.n_dofs) {
        const int64_t api = mv.internal_order ? d : mv.dof_user[d];
        const R2 x = ((const R2 *)mv.dof_xy)[d];
        R qx, qy;
        if (feet_in) {
            qx = feet[api].x;
            qy = feet[api].y;
        } else {
            foot_of<R>(f, scheme, x.x, x.y, (R)dt, qx, qy);
            if (feet) {
                R2 o;
                o.x = qx;
                o.y = qy;
                feet[api] = o;
            }
        }
        WalkResult<R> w = outside_result<R>(0, 0);
        if (in_box<R>(qx, qy, mv.bb)) {
            const int32_t j0 = start_for<F32>(mv, d, api, mode, start, x, qx, qy);
            w = walk<F32>(mv, j0, qx, qy, (uint32_t)d * 2654435761u, ls.c);
        }
        if (mode == SLW_START_PREV)
            store_stream(mv.prev + d, w.elem);
        if (st) {
            ls.add(w);
            hist_add(st, w.steps);
        }
        const int32_t uf = w.elem >= 0 ? mv.tri_uf[w.elem] : -1;
        if (elem)
            elem[api] = w.elem >= 0 ? (uf & kUidMask) : -1;
        if (bary) {
            if (w.elem >= 0) {
                R ub[3];
                user_bary<R>(uf, w.th, ub);
                bary[3 * api] = ub[0];
                bary[3 * api + 1] = ub[1];
                bary[3 * api + 2] = ub[2];
            } else {
                bary[3 * api] = bary[3 * api + 1] = bary[3 * api + 2] = (R)NAN;
            }
        }
        if (steps)
            steps[api] = w.steps;
    }
    if (st)
        flush_stats(ls, st);
}

// ---------------------------------------------------------------------------
// interpolation helpers

template <typename VV>
__device__ inline VV vv_zero();
template <>
__device__ inline float4 vv_zero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <>
__device__ inline double2 vv_zero<double2>() { return make_double2(0.0, 0.0); }
__device__ inline float4 vv_fill(float v) { return make_float4(v, v, v, v); }
__device__ inline double2 vv_fill(double v) { return make_double2(v, v); }
__device__ inline void vv_fma(float w, const float4 r, float4 &acc)
{
    acc.x = fmaf(w, r.x, acc.x);
    acc.y = fmaf(w, r.y, acc.y);
    acc.z = fmaf(w, r.z, acc.z);
    acc.w = fmaf(w, r.w, acc.w);
}
__device__ inline void vv_fma(double w, const double2 r, double2 &acc)
{
    acc.x = fma(w, r.x, acc.x);
    acc.y = fma(w, r.y, acc.y);
}

// Lagrange weights and value rows of a located point: P1 (NA = 3), the
// barycentric coordinates; P2 (NA = 6), theta_a (2 theta_a - 1) at the
// vertices and 4 theta_b theta_c at the midpoint of the edge opposite a.
template <typename R, typename V, int NA>
__device__ inline void lagrange(const MeshView &mv, int32_t e, const int32_t v[3], const R th[3], int32_t row[NA],
                                V wgt[NA])
{
    if constexpr (NA == 3) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            row[a] = v[a];
            wgt[a] = (V)th[a];
        }
    } else {
        const int4 te = mv.tedge[e];
        const int32_t ev[3] = {te.x, te.y, te.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int b = (a + 1) % 3, c = (a + 2) % 3;
            row[a] = v[a];
            row[3 + a] = ev[a];
            wgt[a] = (V)(th[a] * ((R)2 * th[a] - (R)1));
            wgt[3 + a] = (V)((R)4 * th[b] * th[c]);
        }
    }
}

// wave_interp for rows of K = VW * CH fields (CH 16-byte chunks per row, a
// compile-time count): the same items as below, lane L of pass p handles
// point p * (64 / CH) + L / CH, chunk L % CH.  The passes are unrolled with
// constant index arithmetic, and the gathers of B passes at a time are
// issued before any of them is used (outside points and the lanes past the
// last point read row 0 and discard it), so their latencies overlap.
template <typename V, int NA, int CH>
__device__ inline void wave_interp_ch(const int32_t row[NA], const V wgt[NA], int nf, const V *__restrict__ vin,
                                      V *__restrict__ vout, const int32_t *__restrict__ out_map, int64_t base,
                                      V outside)
{
    constexpr int VW = sizeof(V) == 4 ? 4 : 2;
    constexpr int K = VW * CH;
    constexpr int PER = kWave / CH;  // points per pass
    constexpr int B = (NA == 3 && CH >= 2) ? 2 : 1;  // passes whose gathers are in flight together (four would cost registers)
    using VV = typename std::conditional<sizeof(V) == 4, float4, double2>::type;
    const int lane = threadIdx.x & (kWave - 1);
    const int c = lane % CH;
#pragma unroll
    for (int p0 = 0; p0 < CH; p0 += B) {
        int32_t rr[B][NA];
        V ww[B][NA];
        VV g[B][NA];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int f = (p0 + b) * PER + lane / CH;
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                rr[b][a] = __shfl(row[a], f, kWave);
                ww[b][a] = __shfl(wgt[a], f, kWave);
            }
            const bool live = f < nf && rr[b][0] >= 0;
#pragma unroll
            for (int a = 0; a < NA; ++a)
                g[b][a] = *((const VV *)(vin + (int64_t)(live ? rr[b][a] : 0) * K) + c);
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int f = (p0 + b) * PER + lane / CH;
            VV acc = vv_zero<VV>();
            if (rr[b][0] < 0) {
                acc = vv_fill(rr[b][0] == -2 ? ww[b][0] : outside);  // -2: boundary value in the first weight
            } else {
#pragma unroll
                for (int a = 0; a < NA; ++a)
                    vv_fma(ww[b][a], g[b][a], acc);
            }
            if (f < nf) {
                const int64_t o = out_map ? (int64_t)out_map[base + f] : base + f;
                store_stream((VV *)(vout + o * K) + c, acc);
            }
        }
    }
}

// Values of the 64 points of a wavefront, computed cooperatively: lane L of
// pass p handles item p * 64 + L = (point f, chunk c of VW fields), reading
// point f's rows and weights from lane f with cross-lane shuffles.  The
// chunks of consecutive lanes are contiguous in memory (gathers read whole
// row segments, stores are contiguous).  row[0] < 0 marks an outside point.
// Every lane of the wavefront calls it (the shuffles need all of them).
template <typename V, int NA>
__device__ inline void wave_interp(const int32_t row[NA], const V wgt[NA], int nf, const V *__restrict__ vin, int k,
                                   V *__restrict__ vout, const int32_t *__restrict__ out_map, int64_t base, V outside)
{
    const int lane = threadIdx.x & (kWave - 1);
    constexpr int VW = sizeof(V) == 4 ? 4 : 2;
    using VV = typename std::conditional<sizeof(V) == 4, float4, double2>::type;
    const bool vec = (k % VW == 0) &&
                     (((reinterpret_cast<uintptr_t>(vin) | reinterpret_cast<uintptr_t>(vout)) & 15) == 0);
    // the common field counts with a constant chunk count (uniform branches)
    if (vec && k == VW) {
        wave_interp_ch<V, NA, 1>(row, wgt, nf, vin, vout, out_map, base, outside);
        return;
    }
    if (vec && k == 4 * VW) {
        wave_interp_ch<V, NA, 4>(row, wgt, nf, vin, vout, out_map, base, outside);
        return;
    }
    const int chunks = vec ? k / VW : k;
    const int total = nf * chunks;
    // chunks is uniform; a power of two (the common k = 1, 4, 16 ...) divides by shifting
    const bool pow2 = (chunks & (chunks - 1)) == 0;
    const int sh = __builtin_ctz((unsigned)chunks);
    for (int p0 = 0; p0 < total; p0 += kWave) {
        const int it = p0 + lane;
        const int q = pow2 ? (it >> sh) : it / chunks;
        const int fl = it < total ? q : 0;
        const int c = it - fl * chunks;
        int32_t rr[NA];
        V ww[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            rr[a] = __shfl(row[a], fl, kWave);
            ww[a] = __shfl(wgt[a], fl, kWave);
        }
        if (it < total) {
            const int64_t o = out_map ? (int64_t)out_map[base + fl] : base + fl;
            if (vec) {
                VV acc = vv_zero<VV>();
                if (rr[0] < 0) {
                    acc = vv_fill(rr[0] == -2 ? ww[0] : outside);  // -2: boundary value in the first weight
                } else {
#pragma unroll
                    for (int a = 0; a < NA; ++a)
                        vv_fma(ww[a], *((const VV *)(vin + (int64_t)rr[a] * k) + c), acc);
                }
                store_stream((VV *)(vout + o * (int64_t)k) + c, acc);
            } else {
                V acc = rr[0] == -2 ? ww[0] : outside;
                if (rr[0] >= 0) {
                    acc = (V)0;
#pragma unroll
                    for (int a = 0; a < NA; ++a)
                        acc = fma(ww[a], vin[(int64_t)rr[a] * k + c], acc);
                }
                store_stream(vout + o * (int64_t)k + c, acc);
            }
        }
    }
}

template <bool F32, typename V, int NA>
__global__ void __launch_bounds__(kBlock)
    k_interp(MeshView mv, const int32_t *__restrict__ elem, const typename CT<F32>::R *__restrict__ bary, int64_t m,
             const V *__restrict__ vin, int k, V *__restrict__ vout, double outside, int user_rows)
{
    using R = typename CT<F32>::R;
    const int64_t base = xcd_tile(blockIdx.x, gridDim.x, mv.xcd_chunk) * kBlock + (threadIdx.x & ~(kWave - 1));
    const int64_t i = base + (threadIdx.x & (kWave - 1));
    int32_t row[NA];
    V wgt[NA];
    row[0] = -1;
#pragma unroll
    for (int a = 1; a < NA; ++a)
        row[a] = 0;
#pragma unroll
    for (int a = 0; a < NA; ++a)
        wgt[a] = (V)0;
    if (i < m) {
        const int32_t u = elem[i];
        // ids outside [0, n_tris) are treated as outside
        const int32_t e = (u >= 0 && u < mv.n_tris) ? mv.tri_int[u] : -1;
        if (e >= 0) {
            const int4 tv = tri_verts(mv, e);
            const int32_t v[3] = {tv.y, tv.z, tv.w};
            const bool flip = mv.tri_uf[e] < 0;
            // user vertex order -> internal order
            R th[3];
            th[0] = bary[3 * i];
            th[1] = flip ? bary[3 * i + 2] : bary[3 * i + 1];
            th[2] = flip ? bary[3 * i + 1] : bary[3 * i + 2];
            lagrange<R, V, NA>(mv, e, v, th, row, wgt);
            if (user_rows) {
#pragma unroll
                for (int a = 0; a < NA; ++a)
                    row[a] = mv.dof_user[row[a]];
            }
        }
    }
    if (base >= m)
        return;
    const int nf = (int)min<int64_t>(kWave, m - base);
    wave_interp<V, NA>(row, wgt, nf, vin, k, vout, nullptr, base, (V)outside);
}

// ---------------------------------------------------------------------------
// learned start proposal: the network maps a foot to chart coordinates and
// the chart table to a start triangle; the walk above finishes the search

// raw network inputs of a foot: the node's position (in chart coordinates),
// its displacement to the foot, time
template <typename R>
__device__ inline void raw_features(float2 node_uv, R x, R y, R qx, R qy, double t, float f[5])
{
    f[0] = node_uv.x;
    f[1] = node_uv.y;
    f[2] = (float)(qx - x);
    f[3] = (float)(qy - y);
    f[4] = (float)t;
}

// largest i in [0, n) with tab[i] <= x (0 when there is none; tab sorted);
// the trip count depends on n only
__device__ inline int upper_index(const float *__restrict__ tab, int n, float x)
{
    int lo = 0;
    while (n > 1) {
        const int half = n >> 1;
        lo = tab[lo + half] <= x ? lo + half : lo;
        n -= half;
    }
    return lo;
}

// upper_index searched outwards from a guess i0 (exponential steps, then
// bisection): the same answer, in about 2 log2 |answer - i0| probes
__device__ inline int gallop_index(const float *__restrict__ tab, int n, float x, int i0)
{
    i0 = i0 < 0 ? 0 : (i0 >= n ? n - 1 : i0);
    int lo, hi;  // tab[lo] <= x or lo = 0; hi = n or tab[hi] > x
    if (tab[i0] <= x || i0 == 0) {
        lo = i0;
        int step = 1;
        hi = lo + 1;
        while (hi < n && tab[hi] <= x) {
            lo = hi;
            step <<= 1;
            hi = lo + step;
        }
        hi = hi < n ? hi : n;
    } else {
        hi = i0;
        int step = 1;
        lo = hi - 1;
        while (lo > 0 && tab[lo] > x) {
            hi = lo;
            step <<= 1;
            lo = hi - step;
        }
        lo = lo > 0 ? lo : 0;
    }
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tab[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Chart start of DOF d (internal order; valid: d is a DOF whose foot q lies
// in the bounding box).  KIND 0: the cell that holds the foot (binary
// searches in the quantile tables); 1: the table cell of chart(node) +
// network output; 2 (a learned index): the network's cell as the guess of
// galloping searches that end in the foot's own cell.  Then whichever of that
// proposal and the node's steered start lies nearer the foot.  With KIND > 0
// every lane of the wavefront must call it (the network runs on the whole
// wavefront); the result is meaningful on valid lanes only.
template <bool F32, int KIND>
__device__ inline int32_t chart_start(const MeshView &mv, bool valid, int64_t d, typename CT<F32>::R2 x,
                                      typename CT<F32>::R qx, typename CT<F32>::R qy, double t_np1)
{
    using R = typename CT<F32>::R;
    constexpr bool NET = KIND > 0;
    int32_t j = 0;
    float2 guess = make_float2(0.f, 0.f);
    if (NET) {
        float feat[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        float2 c = make_float2(0.f, 0.f);
        if (valid) {
            c = mv.chart_node[d];
            raw_features<R>(c, x.x, x.y, qx, qy, t_np1, feat);
            mlp_normalise(mv.mlp_norm, feat);
        }
        const float2 duv = mlp_forward_wave(mv.mlp_wpack, mv.mlp_bias, feat);  // every lane
        guess = make_float2(c.x + duv.x, c.y + duv.y);
        if (valid && KIND == 1)
            j = chart_lookup(mv.chart_table, mv.chart_g, guess);
    }
    if (!valid)
        return -1;
    // the foot in the records' float frame, as the chart was built
    const float fx = F32 ? (float)qx : (float)((double)qx - mv.fc.cx);
    const float fy = F32 ? (float)qy : (float)((double)qy - mv.fc.cy);
    if (KIND != 1) {
        const int g = mv.chart_g;
        int bu, bv;
        if (KIND == 0) {
            bu = upper_index(mv.chart_qx, g, fx);
            bv = upper_index(mv.chart_qy + (int64_t)bu * g, g, fy);
        } else {
            const float u = fminf(fmaxf(guess.x, 0.f), 0.99999994f), v = fminf(fmaxf(guess.y, 0.f), 0.99999994f);
            bu = gallop_index(mv.chart_qx, g, fx, (int)(u * (float)g));
            bv = gallop_index(mv.chart_qy + (int64_t)bu * g, g, fy, (int)(v * (float)g));
        }
        j = mv.chart_table[(int64_t)bu * g + bv];
    }
    const int32_t js = quadrant_start(mv.qstart[d], (float)(qx - x.x), (float)(qy - x.y));
    return nearer_start<F32>(mv, j, js, qx, qy);
}

// Variable step at the boundary: a characteristic that leaves the domain is
// stopped where it crosses the boundary (the treatment of Dirichlet
// conditions mentioned after eq. (eulero)).  The segment x -> q from the DOF
// to its foot is intersected with the boundary loop, starting at the edge
// a -> b through which the walk left and moving along the loop until the
// crossing lies on the current edge; the value is the boundary datum at the
// crossing point and at the time the characteristic passes there,
// t_{n+1} - theta dt.  Returns false (no crossing found) only on degenerate
// input; the caller then keeps the outside value.
__device__ inline bool boundary_value(const MeshView &mv, bool f32, double xx, double xy, double qx, double qy,
                                      int32_t a, int32_t b, double t_np1, double dt, double &g)
{
    const double wx = qx - xx, wy = qy - xy;
    for (int64_t it = 0; it <= mv.n_boundary + 1 && a >= 0 && b >= 0; ++it) {
        double ax, ay, bx, by;
        if (f32) {
            const float2 A = ((const float2 *)mv.dof_xy)[a], B = ((const float2 *)mv.dof_xy)[b];
            ax = A.x, ay = A.y, bx = B.x, by = B.y;
        } else {
            const double2 A = ((const double2 *)mv.dof_xy)[a], B = ((const double2 *)mv.dof_xy)[b];
            ax = A.x, ay = A.y, bx = B.x, by = B.y;
        }
        const double ex = bx - ax, ey = by - ay, rx = ax - xx, ry = ay - xy;
        const double den = wx * ey - wy * ex;  // w x e > 0: the segment leaves across this edge's line
        if (den > 0.0) {
            const double la = (rx * wy - ry * wx) / den;
            if (la < 0.0) {
                b = a;
                a = mv.bprev[a];
                continue;
            }
            if (la > 1.0) {
                a = b;
                b = mv.bnext[b];
                continue;
            }
            double th = (rx * ey - ry * ex) / den;
            th = th < 0.0 ? 0.0 : (th > 1.0 ? 1.0 : th);
            const double px = xx + th * wx, py = xy + th * wy, t = t_np1 - th * dt;
            g = mv.bc_kind == 1 ? mv.bc_p[0] : mv.bc_p[0] + mv.bc_p[1] * px + mv.bc_p[2] * py + mv.bc_p[3] * t;
            return true;
        }
        // parallel to (or entering across) this edge's line: move towards q
        if ((qx - ax) * ex + (qy - ay) * ey < 0.0) {
            b = a;
            a = mv.bprev[a];
        } else {
            a = b;
            b = mv.bnext[b];
        }
    }
    return false;
}

// boundary_value for a domain that is not one convex disk: the segment
// x -> q may leave and re-enter, so every boundary edge is scanned for the
// first crossing from inside to outside (smallest theta).  False when the
// segment crosses no boundary edge outwards (degenerate input).
__device__ inline bool boundary_value_scan(const MeshView &mv, bool f32, double xx, double xy, double qx, double qy,
                                           double t_np1, double dt, double &g)
{
    const double wx = qx - xx, wy = qy - xy;
    double best = INFINITY;
    // outward crossing parameter of boundary edge i (the smaller into best)
    auto test_edge = [&](int64_t i) {
        const int32_t a = mv.bedge[i], b = mv.bnext[a];
        double ax, ay, bx, by;
        if (f32) {
            const float2 A = ((const float2 *)mv.dof_xy)[a], B = ((const float2 *)mv.dof_xy)[b];
            ax = A.x, ay = A.y, bx = B.x, by = B.y;
        } else {
            const double2 A = ((const double2 *)mv.dof_xy)[a], B = ((const double2 *)mv.dof_xy)[b];
            ax = A.x, ay = A.y, bx = B.x, by = B.y;
        }
        const double ex = bx - ax, ey = by - ay, rx = ax - xx, ry = ay - xy;
        const double den = wx * ey - wy * ex;  // > 0: the segment crosses this edge's line outwards
        if (!(den > 0.0))
            return;
        const double la = (rx * wy - ry * wx) / den, th = (rx * ey - ry * ex) / den;
        if (la >= 0.0 && la <= 1.0 && th >= -1e-12 && th <= 1.0 + 1e-12)
            best = fmin(best, th < 0.0 ? 0.0 : (th > 1.0 ? 1.0 : th));
    };
    if (!mv.bg_ptr) {
        for (int64_t i = 0; i < mv.n_boundary; ++i)
            test_edge(i);
    } else {
        // the cells of the edge grid in the order the segment meets them
        // (Amanatides and Woo 1987); a crossing at theta lies in a cell the
        // segment enters at or before theta, so once the best crossing
        // precedes the current cell's exit no later cell can improve it
        // (the margins absorb the rounding of the cell parameters; the
        // edges' boxes are padded for the same reason)
        const int G = mv.bg_g;
        // in units of cells from the grid's corner, in float: the order of
        // the cells needs no more (the margins and the padding absorb it)
        const float ux = (float)((xx - mv.bg_x0) / mv.bg_cell), uy = (float)((xy - mv.bg_y0) / mv.bg_cell);
        const float vx = (float)(wx / mv.bg_cell), vy = (float)(wy / mv.bg_cell);
        int cx = (int)floorf(ux), cy = (int)floorf(uy);
        cx = cx < 0 ? 0 : (cx >= G ? G - 1 : cx);
        cy = cy < 0 ? 0 : (cy >= G ? G - 1 : cy);
        const int sx = vx > 0.f ? 1 : (vx < 0.f ? -1 : 0), sy = vy > 0.f ? 1 : (vy < 0.f ? -1 : 0);
        for (int it = 0; it < 4 * G + 4; ++it) {  // a segment meets at most 2 G cells
            const int c = cy * G + cx;
            for (int32_t e = mv.bg_ptr[c]; e < mv.bg_ptr[c + 1]; ++e)
                test_edge(mv.bg_list[e]);
            // where the segment leaves this cell, from the cell's own lines
            // (no accumulated increments: a few ulps of error)
            const float tmx = sx > 0 ? ((float)(cx + 1) - ux) / vx : (sx < 0 ? ((float)cx - ux) / vx : INFINITY);
            const float tmy = sy > 0 ? ((float)(cy + 1) - uy) / vy : (sy < 0 ? ((float)cy - uy) / vy : INFINITY);
            const float texit = fminf(tmx, tmy);
            if (best < (double)texit - 1e-5 || texit >= 1.f)
                break;
            if (tmx < tmy)
                cx += sx;
            else
                cy += sy;
            if (cx < 0 || cy < 0 || cx >= G || cy >= G)
                break;
        }
    }
    if (!(best <= 1.0))
        return false;
    const double px = xx + best * wx, py = xy + best * wy, t = t_np1 - best * dt;
    g = mv.bc_kind == 1 ? mv.bc_p[0] : mv.bc_p[0] + mv.bc_p[1] * px + mv.bc_p[2] * py + mv.bc_p[3] * t;
    return true;
}

// The fused step (Algorithm 2, one pass of its loop) for the 64 DOFs
// [base, base + 64) of one wavefront: one lane per foot for foot -> start ->
// walk -> tie rule -> weights; then the wavefront computes its feet's values
// cooperatively.  Every lane of the wavefront calls it.  KIND: -1 the start
// given by `mode`; -2 strategy (b) (its own instantiation: the first test
// reads the full record of the previous element, which holds registers the
// other starts do not need); 0 / 2 chart starts computed here; -3 / -4 the
// roots / the other DOFs of strategy (c)'s forest: positions index the
// forest's lists (fv), not the DOFs.
template <bool F32, typename V, int NA, int KIND = -1>
__device__ inline void step_wave(const MeshView &mv, const FieldDev &f, double dt, double t_np1, int scheme, int mode,
                                 const int32_t *__restrict__ start, const V *__restrict__ vin, int k,
                                 V *__restrict__ vout, double outside, int write_prev,
                                 const int32_t *__restrict__ out_map, int32_t *__restrict__ elem_out,
                                 int64_t n_iter, int64_t base, DevStats *st, ForestView fv = ForestView(),
                                 const WalkRec *lw = nullptr, int32_t lbase = 0, int32_t lcount = 0)
{
    using R = typename CT<F32>::R;
    using R2 = typename CT<F32>::R2;
    constexpr bool FOREST = KIND == -3 || KIND == -4;
    const int64_t pos = base + (threadIdx.x & (kWave - 1));
    const bool valid = pos < n_iter;
    int64_t d = pos;
    if constexpr (FOREST) {
        d = valid ? (int64_t)fv.list[pos] : 0;
        out_map = fv.out;  // output row of each list position
    }
    // output row of this lane's DOF
    const int64_t orow = FOREST ? (valid ? (int64_t)fv.out[pos] : 0) : (out_map && valid ? (int64_t)out_map[d] : d);
    LaneStats ls;
    int32_t row[NA];
    V wgt[NA];
    row[0] = -1;
#pragma unroll
    for (int a = 1; a < NA; ++a)
        row[a] = 0;
#pragma unroll
    for (int a = 0; a < NA; ++a)
        wgt[a] = (V)0;
    R2 x;
    x.x = x.y = (R)0;
    R qx = (R)0, qy = (R)0;
    int32_t sid = -1;
    if (valid) {
        x = ((const R2 *)mv.dof_xy)[d];
        int32_t p = -1;
        if constexpr (KIND == -4) {
            // strategy (c): the element found for this DOF's parent (a root
            // within three hops of it in the mesh) by the roots' launch
            p = fv.parent[pos];
            sid = p >= 0 ? fv.elem[p] : -1;
        } else if constexpr (KIND == -5) {
            sid = load_stream(mv.prev + d);  // the previous step's element (strategy (b)), with its skip count
        } else if constexpr (KIND < 0 && KIND != -3) {
            const int64_t api = (mode == SLW_START_GIVEN && !mv.internal_order) ? mv.dof_user[d] : d;
            sid = start_id(mv, d, api, mode, start);
        }
        foot_of<R>(f, scheme, x.x, x.y, (R)dt, qx, qy);
        if constexpr (KIND == -4) {
            if (sid >= 0) {
                // the parent's foot lies about as far from this foot as the
                // parent node from this node: start from the parent's element
                // unless this node is nearer its own foot (then its own
                // steered start, strategy (a))
                const R2 xp = ((const R2 *)mv.dof_xy)[p];
                const float ex = (float)(xp.x - x.x), ey = (float)(xp.y - x.y);
                const float ux = (float)(qx - x.x), uy = (float)(qy - x.y);
                if (ex * ex + ey * ey >= ux * ux + uy * uy)
                    sid = -1;
            }
        }
    }
    // with boundary data every finite foot is walked (to learn where it leaves)
    const bool run = valid && (mv.bc_kind ? (isfinite((double)qx) && isfinite((double)qy))
                                          : in_box<R>(qx, qy, mv.bb));
    int32_t jc = 0;
    if constexpr (KIND >= 0)  // chart starts computed here, for the whole wavefront
        jc = chart_start<F32, KIND>(mv, run, d, x, qx, qy, t_np1);
    if (valid) {
        WalkResult<R> w = outside_result<R>(0, 0);
        if constexpr (KIND == -5) {
            // Hybrid start, chosen per foot from how far it moved: the
            // previous element first (strategy (b)); a foot inside it is
            // located at once.  A foot less than hybrid_far heights of that
            // element beyond it walks on from there; a farther one, or one
            // without a previous element, starts from its cell of the start
            // grid when the mesh has one, else from its chart cell when the
            // mesh has a chart (the nearer of that cell's triangle and the
            // steered start), else from the steered start (strategy (a)).
            // A foot found far from its previous element skips that test for
            // the next kPrevSkipSteps steps (feet of a fast flow stay fast).
            // (Only with a grid or a chart: without them a far foot starts
            // from the steered start, slower than walking on.)
            const bool far_start = mv.grid || mv.chart_table;
            const int skip = (sid >= 0 && far_start) ? (sid >> kPrevSkipShift) : 0;
            const int32_t pe = sid >= 0 ? (sid & kPrevElemMask) : -1;
            int next_skip = skip > 0 ? skip - 1 : 0;
            if (run) {
                bool done = false;
                int32_t j0 = -1;
                // (the grid cell is read only for feet that need it: read
                // beside the previous element's record for every foot, it
                // measured slower at low Courant numbers)
                if (pe >= 0 && skip == 0) {
                    float tmin = 0.f;
                    done = first_test<F32>(mv, pe, qx, qy, tmin, w, ls.c) != 0;
                    if (!done && tmin > -mv.hybrid_far)
                        j0 = pe;
                    else if (!done && far_start)
                        next_skip = kPrevSkipSteps;
                }
                if (!done) {
                    if (j0 < 0)
                        j0 = mv.grid ? grid_start(mv, qx, qy)
                                     : (mv.chart_table ? chart_start<F32, 0>(mv, true, d, x, qx, qy, t_np1)
                                                       : quadrant_start(mv.qstart[d], (float)(qx - x.x),
                                                                        (float)(qy - x.y)));
                    w = walk<F32>(mv, j0, qx, qy, (uint32_t)d * 2654435761u, ls.c);
                }
            }
            store_stream(mv.prev + d, w.elem >= 0 ? (w.elem | (next_skip << kPrevSkipShift)) : w.elem);
        } else if (run) {
            int32_t j0 = jc;
            if constexpr (KIND == -3)
                // a root of the forest: from its cell of the start grid when
                // the mesh has one, else strategy (a)
                j0 = mv.grid ? grid_start(mv, qx, qy)
                             : quadrant_start(mv.qstart[d], (float)(qx - x.x), (float)(qy - x.y));
            else if constexpr (KIND == -4)
                j0 = sid >= 0 ? sid : quadrant_start(mv.qstart[d], (float)(qx - x.x), (float)(qy - x.y));
            else if constexpr (KIND < 0)
                j0 = start_pick<KIND == -6>(mv, d, sid, mode, x, qx, qy);
            if constexpr (KIND == -7)
                w = walk_win<F32>(mv, j0, qx, qy, (uint32_t)d * 2654435761u, ls.c, lw, lbase, lcount);
            else
                w = walk<F32>(mv, j0, qx, qy, (uint32_t)d * 2654435761u, ls.c, KIND == -2);
        }
        if constexpr (KIND == -3)
            fv.elem[d] = w.elem;
        if (write_prev)
            store_stream(mv.prev + d, w.elem);
        if (elem_out)
            elem_out[orow] = w.elem >= 0 ? (mv.tri_uf[w.elem] & kUidMask) : -1;
        if (st) {
            ls.add(w);
            hist_add(st, w.steps);
        }
        if (w.elem >= 0) {
            lagrange<R, V, NA>(mv, w.elem, w.v, w.th, row, wgt);
        } else if (mv.bc_kind && (w.flags & 16)) {
            double gv;
            const bool hit = mv.nonconvex ? boundary_value_scan(mv, F32, (double)x.x, (double)x.y, (double)qx,
                                                                (double)qy, t_np1, dt, gv)
                                          : boundary_value(mv, F32, (double)x.x, (double)x.y, (double)qx, (double)qy,
                                                           w.v[0], w.v[1], t_np1, dt, gv);
            if (hit) {
                row[0] = -2;  // value given in wgt[0]
                wgt[0] = (V)gv;
            }
        }
    }
    if (st)
        flush_stats(ls, st);
    if (base >= n_iter)
        return;
    const int nf = (int)min<int64_t>(kWave, n_iter - base);
    wave_interp<V, NA>(row, wgt, nf, vin, k, vout, out_map, base, (V)outside);
}

// Occupancy floor per instantiation: seven wavefronts per SIMD for strategy
// (b) (its first test holds a full record; without the floor it takes 74
// registers and six wavefronts); four for the learned index (the network's
// accumulators would take 140 registers and three wavefronts; at four the
// compiler spills 32 bytes, measured 5% faster; five spills more and is
// slower).  The others keep the compiler's choice (the plain step takes 66
// registers, seven wavefronts; forcing eight spills one value and measured
// slower).
constexpr int step_waves_per_eu(int kind) { return kind == -2 || kind == -7 ? 7 : (kind == 2 ? 4 : 1); }

template <bool F32, typename V, int NA, int KIND = -1>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(step_waves_per_eu(KIND))))
    k_step(MeshView mv, FieldDev f, double dt, double t_np1, int scheme, int mode, const int32_t *__restrict__ start,
           const V *__restrict__ vin, int k, V *__restrict__ vout, double outside, int write_prev,
           const int32_t *__restrict__ out_map, int32_t *__restrict__ elem_out, int64_t n_iter, DevStats *st,
           ForestView fv)
{
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x, mv.xcd_chunk);
    const int64_t base = tile * kBlock + (threadIdx.x & ~(kWave - 1));
    if constexpr (KIND == -7) {
        // The staged-window step: the workgroup first copies the lds_w walk
        // records around its tile (centred on an incident triangle of the
        // tile's middle DOF; triangles and DOFs share the Morton order) into
        // LDS, and its walks read the records of that window from there.
        extern __shared__ WalkRec win[];
        int64_t mid = tile * kBlock + kBlock / 2;
        mid = mid < n_iter ? mid : n_iter - 1;
        const int32_t lc = mv.n_tris < (int64_t)mv.lds_w ? (int32_t)mv.n_tris : mv.lds_w;
        int32_t lb = mv.qstart[mid].x - lc / 2;
        lb = lb < 0 ? 0 : lb;
        lb = lb > (int32_t)mv.n_tris - lc ? (int32_t)mv.n_tris - lc : lb;
        for (int i = threadIdx.x; i < lc; i += kBlock)
            win[i] = mv.wrec[lb + i];
        __syncthreads();
        step_wave<F32, V, NA, KIND>(mv, f, dt, t_np1, scheme, mode, start, vin, k, vout, outside, write_prev,
                                    out_map, elem_out, n_iter, base, st, fv, win, lb, lc);
    } else {
        step_wave<F32, V, NA, KIND>(mv, f, dt, t_np1, scheme, mode, start, vin, k, vout, outside, write_prev,
                                    out_map, elem_out, n_iter, base, st, fv);
    }
}

// ---------------------------------------------------------------------------
// strategy (c): the start is the element found for a neighbouring node

// orders the LDS accesses of the lanes of one wavefront around it (the
// wavefront's LDS operations complete in issue order)
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Strategy (c) of Section 3 starts node i's walk from the element that
// contains the foot of an adjacent node (its parent in a spanning tree), so
// that the walk covers about the distance between two neighbouring feet.  A
// breadth-first tree has about sqrt(N) sequential levels, each a global
// round trip on a GPU; here the spanning forest is made of chains of L
// consecutive Morton-ordered nodes (neighbours or near neighbours): lane t of
// a wavefront walks the chain [base + L t, base + L t + L) in order, the
// first foot from its steered start (strategy (a)), every later foot from
// the element found for the previous one, unless its own steered start lies
// nearer (the Z curve jumps between blocks now and then: a jump would cost a
// walk across the mesh).  Rows and weights are staged in
// LDS, then the wavefront interpolates 64 consecutive DOFs at a time
// (contiguous stores).  One wavefront per workgroup.
template <bool F32, typename V, int NA, int L>
__global__ void __launch_bounds__(kWave)
    k_step_chain(MeshView mv, FieldDev f, double dt, int scheme, const V *__restrict__ vin, int k,
                 V *__restrict__ vout, double outside, const int32_t *__restrict__ out_map,
                 int32_t *__restrict__ elem_out, int64_t n_iter, DevStats *st)
{
    using R = typename CT<F32>::R;
    using R2 = typename CT<F32>::R2;
    constexpr int C = kWave * L;
    __shared__ int32_t srow[C * NA];
    __shared__ V swgt[C * NA];
    const int lane = threadIdx.x;
    const int64_t base = xcd_tile(blockIdx.x, gridDim.x, mv.xcd_chunk) * (int64_t)C;
    LaneStats ls;
    int32_t prev = -1;  // element of the previous foot of this lane's chain
#pragma unroll 1
    for (int r = 0; r < L; ++r) {
        const int o = lane * L + r;
        const int64_t d = base + o;
        int32_t row[NA];
        V wgt[NA];
        row[0] = -1;
#pragma unroll
        for (int a = 1; a < NA; ++a)
            row[a] = 0;
#pragma unroll
        for (int a = 0; a < NA; ++a)
            wgt[a] = (V)0;
        if (d < n_iter) {
            const R2 x = ((const R2 *)mv.dof_xy)[d];
            R qx, qy;
            foot_of<R>(f, scheme, x.x, x.y, (R)dt, qx, qy);
            WalkResult<R> w = outside_result<R>(0, 0);
            if (in_box<R>(qx, qy, mv.bb)) {
                int32_t j0 = quadrant_start(mv.qstart[d], (float)(qx - x.x), (float)(qy - x.y));
                if (prev >= 0)
                    j0 = nearer_start<F32>(mv, prev, j0, qx, qy);
                w = walk<F32>(mv, j0, qx, qy, (uint32_t)d * 2654435761u, ls.c);
            }
            if (st) {
                ls.add(w);
                hist_add(st, w.steps);
            }
            if (elem_out)
                elem_out[out_map ? (int64_t)out_map[d] : d] = w.elem >= 0 ? (mv.tri_uf[w.elem] & kUidMask) : -1;
            prev = w.elem;
            if (w.elem >= 0)
                lagrange<R, V, NA>(mv, w.elem, w.v, w.th, row, wgt);
        }
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            srow[o * NA + a] = row[a];
            swgt[o * NA + a] = wgt[a];
        }
    }
    wave_lds_sync();
#pragma unroll 1
    for (int b = 0; b < L; ++b) {
        const int64_t gb = base + (int64_t)b * kWave;
        if (gb >= n_iter)
            break;
        const int o = b * kWave + lane;
        int32_t row[NA];
        V wgt[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            row[a] = srow[o * NA + a];
            wgt[a] = swgt[o * NA + a];
        }
        const int nf = (int)min<int64_t>(kWave, n_iter - gb);
        wave_interp<V, NA>(row, wgt, nf, vin, k, vout, out_map, gb, (V)outside);
    }
    if (st)
        flush_stats(ls, st);
}

// ---------------------------------------------------------------------------
// batches: every mesh of a batch advanced by one step in one launch

// time factors of a field on the device (per workgroup; uniform values)
__device__ inline void field_time_factors_dev(FieldDev &f, double t_np1, double dt)
{
    const double pi = 3.14159265358979323846;
    const double t[2] = {t_np1, t_np1 - 0.5 * dt};
#pragma unroll
    for (int i = 0; i < 2; ++i)
        f.g[i] = f.kind == 2 ? cos(pi * t[i] / f.p[0]) : (f.kind == 3 ? f.p[1] * t[i] : 0.0);
}

// Items of the concatenated tile space [0, total) of a batch: mesh m owns
// tiles [items[m].tile0, items[m + 1].tile0).
template <bool F32, typename V, int BS>
__device__ __forceinline__ void batch_tile(const BatchItem *__restrict__ items, int n_items, int64_t tile, int64_t step,
                                  int scheme, int k, double outside, DevStats *st)
{
    int lo = 0, hi = n_items - 1;  // last item with tile0 <= tile (uniform binary search)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile0 <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BatchItem &it = items[lo];
    FieldDev f = it.f;
    field_time_factors_dev(f, it.t0 + (double)(step + 1) * it.dt, it.dt);
    const bool even = (step & 1) == 0;
    const V *vin = (const V *)(even ? it.va : it.vb);
    V *vout = (V *)(even ? it.vb : it.va);
    const int64_t base = (tile - it.tile0) * BS + (threadIdx.x & ~(kWave - 1));
    step_wave<F32, V, 3>(it.mv, f, it.dt, it.t0 + (double)(step + 1) * it.dt, scheme, it.start_mode, nullptr, vin,
                         k, vout, outside, it.start_mode == SLW_START_PREV, nullptr, it.elem, it.n_iter, base, st);
}

// schedule 0: one workgroup per tile, XCD-contiguous ranges of the
// concatenated tile space; schedule 1: persistent workgroups pulling tiles
// from 8 per-XCD queues (each queue covers one XCD's contiguous range) and
// stealing from the other queues when their own is empty; schedule 2: one
// workgroup per tile, chunks of 16,384 nodes' tiles dealt to the XCDs in
// turn (even work per XCD when the meshes' walks differ).
template <bool F32, typename V, int BS>
__device__ inline void batch_persistent(const BatchItem *__restrict__ items, int n_items, int64_t total,
                                        int64_t step, int scheme, int k, double outside, unsigned *queues,
                                        DevStats *st);

// (The schedule is a template parameter: the persistent loop's state would
// otherwise raise the register count, and lower the occupancy, of both.)
template <bool F32, typename V, int BS, int SCHEDULE>
__global__ void __launch_bounds__(BS)
    k_batch_step(const BatchItem *__restrict__ items, int n_items, int64_t total, const int64_t *__restrict__ counter,
                 int scheme, int k, double outside, unsigned *queues, DevStats *st)
{
    const int64_t step = *counter;
    if constexpr (SCHEDULE == 0)
        batch_tile<F32, V, BS>(items, n_items, xcd_tile(blockIdx.x, gridDim.x), step, scheme, k, outside, st);
    else if constexpr (SCHEDULE == 2)
        batch_tile<F32, V, BS>(items, n_items, xcd_tile(blockIdx.x, gridDim.x, 16384 / BS), step, scheme, k, outside,
                               st);
    else
        batch_persistent<F32, V, BS>(items, n_items, total, step, scheme, k, outside, queues, st);
}

template <bool F32, typename V, int BS>
__device__ inline void batch_persistent(const BatchItem *__restrict__ items, int n_items, int64_t total,
                                        int64_t step, int scheme, int k, double outside, unsigned *queues,
                                        DevStats *st)
{
    __shared__ int64_t s_tile;
    constexpr int64_t kXcd = 8;
    const int64_t q = total / kXcd, r = total % kXcd;
    int x = (int)(blockIdx.x % kXcd);
    int tried = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t got = -1;
            while (tried < kXcd) {
                const int64_t size = q + (x < r ? 1 : 0);
                const int64_t first = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
                const unsigned i = atomicAdd(&queues[x], 1u);
                if ((int64_t)i < size) {
                    got = first + i;
                    break;
                }
                x = (x + 1) % (int)kXcd;
                ++tried;
            }
            s_tile = got;
        }
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile < 0)
            return;  // every queue is empty: all waves of the workgroup exit together
        batch_tile<F32, V, BS>(items, n_items, tile, step, scheme, k, outside, st);
    }
}

__global__ void k_zero_u32(unsigned *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0u;
}

__global__ void k_advance(int64_t *counter, int64_t by)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *counter += by;
}

__global__ void k_permute_rows(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, int64_t rows,
                               int64_t words, const int32_t *__restrict__ map, int scatter)
{
    const int64_t total = rows * words;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / words, w = i - r * words;
        if (scatter)
            dst[(int64_t)map[r] * words + w] = src[i];
        else
            dst[i] = src[(int64_t)map[r] * words + w];
    }
}

// start[d] for the DOFs [0, n_iter) (internal order) by chart_start; feet
// computed from the field or read from feet_in (indexed like
// slw_locate_feet's feet)
template <bool F32, int KIND>
__global__ void __launch_bounds__(kBlock)
    k_chart_start(MeshView mv, FieldDev f, double dt, double t_np1, int scheme,
                  const typename CT<F32>::R2 *__restrict__ feet_in, int64_t n_iter, int32_t *__restrict__ start)
{
    using R = typename CT<F32>::R;
    using R2 = typename CT<F32>::R2;
    const int64_t d = xcd_tile(blockIdx.x, gridDim.x, mv.xcd_chunk) * kBlock + threadIdx.x;
    R2 x;
    x.x = (R)0;
    x.y = (R)0;
    R qx = 0, qy = 0;
    if (d < n_iter) {
        x = ((const R2 *)mv.dof_xy)[d];
        if (feet_in) {
            const int64_t api = mv.internal_order ? d : mv.dof_user[d];
            qx = feet_in[api].x;
            qy = feet_in[api].y;
        } else {
            foot_of<R>(f, scheme, x.x, x.y, (R)dt, qx, qy);
        }
    }
    // outside the box the walk does not run; the steered start is written
    const bool valid = d < n_iter && in_box<R>(qx, qy, mv.bb);
    const int32_t j = chart_start<F32, KIND>(mv, valid, d, x, qx, qy, t_np1);
    if (d < n_iter)
        start[d] = valid ? j : mv.qstart[d].x;
}

// ---------------------------------------------------------------------------
// the step with lane repacking


// The fused step for a chunk of 64 RP consecutive DOFs [base, base + 64 RP)
// owned by one wavefront.  Walk lengths differ from foot to foot; instead of
// holding every lane until the longest walk of its 64 ends, a lane whose walk
// ends takes the next unstarted foot of the chunk (ballot + prefix count),
// so the wavefront's time follows the chunk's total walk length.  Feet and
// start triangles are computed first and staged in LDS (sq, sj); a finished
// walk leaves its triangle and zero-sign mask there (sj, sz); the tie rule,
// the weights and the cooperative interpolation then run 64 feet at a time.
// Every lane of the wavefront calls it.
template <bool F32, typename V, int NA, int RP, bool NET>
__device__ inline void step_chunk(const MeshView &mv, const FieldDev &f, double dt, double t_np1, int scheme, int mode,
                                  const int32_t *__restrict__ start, const V *__restrict__ vin, int k,
                                  V *__restrict__ vout, double outside, int write_prev,
                                  const int32_t *__restrict__ out_map, int32_t *__restrict__ elem_out,
                                  int64_t n_iter, int64_t base, typename CT<F32>::R2 *sq, int32_t *sj, int8_t *sz,
                                  DevStats *st)
{
    using R = typename CT<F32>::R;
    using R2 = typename CT<F32>::R2;
    constexpr int C = kWave * RP;
    const int lane = threadIdx.x & (kWave - 1);
    LaneStats ls;
    // 1. feet and start triangles (-1: outside the bounding box; -2: no DOF);
    // chart starts (learned or exact) are computed here, for the whole
    // wavefront at once
#pragma unroll
    for (int rr = 0; rr < RP; ++rr) {
        const int slot = rr * kWave + lane;
        const int64_t d = base + slot;
        int32_t j0 = -2;
        R2 q, x;
        q.x = q.y = x.x = x.y = (R)0;
        if (d < n_iter) {
            x = ((const R2 *)mv.dof_xy)[d];
            foot_of<R>(f, scheme, x.x, x.y, (R)dt, q.x, q.y);
            j0 = -1;
        }
        const bool valid = d < n_iter && in_box<R>(q.x, q.y, mv.bb);
        if constexpr (NET) {  // the learned start (kernels instantiated for it alone)
            const int32_t jc = chart_start<F32, 1>(mv, valid, d, x, q.x, q.y, t_np1);
            j0 = valid ? jc : j0;
        } else if (mode == SLW_START_CHART) {
            const int32_t jc = chart_start<F32, 0>(mv, valid, d, x, q.x, q.y, t_np1);
            j0 = valid ? jc : j0;
        } else if (valid) {
            const int64_t api = (mode == SLW_START_GIVEN && !mv.internal_order) ? mv.dof_user[d] : d;
            j0 = start_for<F32>(mv, d, api, mode, start, x, q.x, q.y);
        }
        sq[slot] = q;
        sj[slot] = j0;
    }
    wave_lds_sync();
    // 2. walks, one move per iteration for every busy lane; idle lanes refill
    int slot = -1;
    int32_t j = 0, steps = 0, flags = 0;
    R qx = (R)0, qy = (R)0;
    float qfx = 0.f, qfy = 0.f;
    uint32_t seed = 0;
    int next = 0;  // first unstarted foot of the chunk (uniform)
    const unsigned long long below = (1ull << lane) - 1ull;
    for (;;) {
        const bool idle = slot < 0;
        const unsigned long long need = __ballot(idle);
        if (need != 0ull && next < C) {
            if (idle) {
                const int cand = next + __popcll(need & below);
                if (cand < C) {
                    const int32_t j0 = sj[cand];
                    if (j0 >= 0) {
                        const R2 q = sq[cand];
                        slot = cand;
                        j = j0;
                        qx = q.x;
                        qy = q.y;
                        qfx = F32 ? (float)qx : (float)((double)qx - mv.fc.cx);
                        qfy = F32 ? (float)qy : (float)((double)qy - mv.fc.cy);
                        steps = 0;
                        flags = 0;
                        seed = (uint32_t)(base + cand) * 2654435761u;
                    } else if (j0 == -1) {
                        ls.add_walk(false, 0, 0);
                        if (st)
                            hist_add(st, 0);
                    }
                }
            }
            next += __popcll(need);
        }
        if (__ballot(slot >= 0) == 0ull) {
            if (next >= C)
                break;
            continue;
        }
        if (slot >= 0) {
            WalkRec r;
            int zmask = 0;
            const int res = walk_move<F32>(mv, j, r, zmask, qfx, qfy, qx, qy, seed, steps, flags, ls.c);
            if (res != 0) {
                sj[slot] = res == 1 ? j : -1;
                sz[slot] = (int8_t)zmask;
                ls.add_walk(res == 1, steps, flags);
                if (st)
                    hist_add(st, steps);
                slot = -1;
            }
        }
    }
    wave_lds_sync();
    // 3. tie rule, weights, values
#pragma unroll
    for (int rr = 0; rr < RP; ++rr) {
        const int64_t gbase = base + rr * kWave;
        if (gbase >= n_iter)
            break;
        const int sl = rr * kWave + lane;
        const int64_t d = gbase + lane;
        int32_t row[NA];
        V wgt[NA];
        row[0] = -1;
#pragma unroll
        for (int a = 1; a < NA; ++a)
            row[a] = 0;
#pragma unroll
        for (int a = 0; a < NA; ++a)
            wgt[a] = (V)0;
        if (d < n_iter) {
            const int32_t e0 = sj[sl];
            int32_t elem = -1;
            if (e0 >= 0) {
                const R2 q = sq[sl];
                const WalkResult<R> w = finish_walk_rec<F32>(mv, e0, mv.wrec[e0], (int)sz[sl], 0, 0, q.x, q.y);
                ls.add_ties(w.flags);
                elem = w.elem;
                lagrange<R, V, NA>(mv, w.elem, w.v, w.th, row, wgt);
            }
            if (write_prev)
                store_stream(mv.prev + d, elem);
            if (elem_out)
                elem_out[out_map ? (int64_t)out_map[d] : d] = elem >= 0 ? (mv.tri_uf[elem] & kUidMask) : -1;
        }
        const int nf = (int)min<int64_t>(kWave, n_iter - gbase);
        wave_interp<V, NA>(row, wgt, nf, vin, k, vout, out_map, gbase, (V)outside);
    }
    if (st)
        flush_stats(ls, st);
}

template <bool F32, typename V, int NA, int RP, bool NET>
__global__ void __launch_bounds__(kBlock)
    k_step_rp(MeshView mv, FieldDev f, double dt, double t_np1, int scheme, int mode, const int32_t *__restrict__ start,
              const V *__restrict__ vin, int k, V *__restrict__ vout, double outside, int write_prev,
              const int32_t *__restrict__ out_map, int32_t *__restrict__ elem_out, int64_t n_iter, DevStats *st)
{
    constexpr int W = kBlock / kWave, C = kWave * RP;
    __shared__ typename CT<F32>::R2 sq[W][C];
    __shared__ int32_t sj[W][C];
    __shared__ int8_t sz[W][C];
    const int w = threadIdx.x / kWave;
    const int64_t base = xcd_tile(blockIdx.x, gridDim.x, mv.xcd_chunk) * (int64_t)(kBlock * RP) + (int64_t)w * C;
    step_chunk<F32, V, NA, RP, NET>(mv, f, dt, t_np1, scheme, mode, start, vin, k, vout, outside, write_prev, out_map,
                                    elem_out, n_iter, base, sq[w], sj[w], sz[w], st);
}

// Training pairs: for the DOFs dofs[i] (internal positions) the plain walk
// (strategy (a) start) locates the foot; X[i] = raw features, Y[i] = chart
// coordinates of the element found minus those of the DOF, NaN when the foot
// is outside.
template <bool F32>
__global__ void __launch_bounds__(kBlock)
    k_gather(MeshView mv, FieldDev f, double dt, double t_np1, int scheme, const int32_t *__restrict__ dofs,
             int64_t m, const float2 *__restrict__ chart_uv, const float2 *__restrict__ node, float *__restrict__ X,
             float2 *__restrict__ Y)
{
    using R = typename CT<F32>::R;
    using R2 = typename CT<F32>::R2;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m)
        return;
    const int64_t d = dofs[i];
    if (d < 0 || d >= mv.n_dofs) {
        for (int c = 0; c < 5; ++c)
            X[5 * i + c] = 0.f;
        Y[i] = make_float2(NAN, NAN);
        return;
    }
    const R2 x = ((const R2 *)mv.dof_xy)[d];
    R qx, qy;
    foot_of<R>(f, scheme, x.x, x.y, (R)dt, qx, qy);
    int32_t e = -1;
    if (in_box<R>(qx, qy, mv.bb)) {
        Counters c;
        const int32_t j0 = quadrant_start(mv.qstart[d], (float)(qx - x.x), (float)(qy - x.y));
        e = walk<F32>(mv, j0, qx, qy, (uint32_t)d * 2654435761u, c).elem;
    }
    float feat[5];
    raw_features<R>(node[d], x.x, x.y, qx, qy, t_np1, feat);
    for (int c = 0; c < 5; ++c)
        X[5 * i + c] = feat[c];
    if (e >= 0) {
        const float2 c = chart_uv[e], o = node[d];
        Y[i] = make_float2(c.x - o.x, c.y - o.y);
    } else {
        Y[i] = make_float2(NAN, NAN);
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0ull;
}

// number of kBlock tiles covering n items (one workgroup per tile)
inline bool tiles_for(int64_t n, unsigned &g)
{
    const int64_t t = (n + kBlock - 1) / kBlock;
    if (t > (int64_t)INT32_MAX)
        return false;
    g = (unsigned)(t < 1 ? 1 : t);
    return true;
}

}  // namespace

void field_time_factors(FieldDev &f, double t_np1, double dt)
{
    const double pi = 3.14159265358979323846;
    const double t[2] = {t_np1, t_np1 - 0.5 * dt};
    for (int i = 0; i < 2; ++i) {
        if (f.kind == 2)
            f.g[i] = cos(pi * t[i] / f.p[0]);
        else if (f.kind == 3)
            f.g[i] = f.p[1] * t[i];
        else
            f.g[i] = 0.0;
    }
}

hipError_t launch_locate(const DevMesh &m, hipStream_t st, const void *q, int64_t mp, const int32_t *start,
                         int32_t *elem, void *bary, int32_t *steps, DevStats *stats)
{
    if (mp == 0)
        return hipSuccess;
    unsigned g;
    if (!tiles_for(mp, g))
        return hipErrorInvalidValue;
    MeshView mv = view_of(m);
    if (m.coords_f32)
        hipLaunchKernelGGL(k_locate<true>, dim3(g), dim3(kBlock), 0, st, mv, (const float2 *)q, mp, start, elem,
                           (float *)bary, steps, stats);
    else
        hipLaunchKernelGGL(k_locate<false>, dim3(g), dim3(kBlock), 0, st, mv, (const double2 *)q, mp, start, elem,
                           (double *)bary, steps, stats);
    return hipGetLastError();
}

hipError_t launch_qt_locate(const DevMesh &m, hipStream_t st, const void *q, int64_t mp, int32_t *elem, void *bary,
                            DevStats *stats)
{
    if (mp == 0)
        return hipSuccess;
    if (!m.qt_nodes)
        return hipErrorInvalidValue;
    unsigned g;
    if (!tiles_for(mp, g))
        return hipErrorInvalidValue;
    MeshView mv = view_of(m);
    if (m.coords_f32)
        hipLaunchKernelGGL(k_qt_locate<true>, dim3(g), dim3(kBlock), 0, st, mv, (const float2 *)q, mp, elem,
                           (float *)bary, stats);
    else
        hipLaunchKernelGGL(k_qt_locate<false>, dim3(g), dim3(kBlock), 0, st, mv, (const double2 *)q, mp, elem,
                           (double *)bary, stats);
    return hipGetLastError();
}

// previous elements without the hybrid's skip counts
__global__ void k_prev_clear_skip(int32_t *__restrict__ prev, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const int32_t v = prev[i];
        if (v >= 0)
            prev[i] = v & kPrevElemMask;
    }
}

hipError_t launch_prev_clear_skip(hipStream_t st, int32_t *prev, int64_t n)
{
    if (n <= 0)
        return hipSuccess;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > (int64_t)INT32_MAX)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_prev_clear_skip, dim3((unsigned)blocks), dim3(kBlock), 0, st, prev, n);
    return hipGetLastError();
}

hipError_t launch_grid_build(const DevMesh &m, hipStream_t st, int32_t *grid, int g, double x0, double y0,
                             double cell)
{
    const int64_t cells = (int64_t)g * g;
    if (cells <= 0 || !m.jump)
        return hipErrorInvalidValue;
    const int64_t blocks = (cells + kBlock - 1) / kBlock;
    if (blocks > (int64_t)INT32_MAX)
        return hipErrorInvalidValue;
    MeshView mv = view_of(m);
    if (m.coords_f32)
        hipLaunchKernelGGL(k_grid_build<true>, dim3((unsigned)blocks), dim3(kBlock), 0, st, mv, grid, g, x0, y0, cell);
    else
        hipLaunchKernelGGL(k_grid_build<false>, dim3((unsigned)blocks), dim3(kBlock), 0, st, mv, grid, g, x0, y0,
                           cell);
    return hipGetLastError();
}

hipError_t launch_locate_feet(const DevMesh &m, hipStream_t st, const FieldDev *f, double t_np1, double dt,
                              int scheme, int mode, const int32_t *start, bool feet_in, void *feet, int32_t *elem,
                              void *bary, int32_t *steps, DevStats *stats)
{
    unsigned g;
    if (!tiles_for(m.n_dofs, g))
        return hipErrorInvalidValue;
    MeshView mv = view_of(m);
    FieldDev fd = f ? *f : FieldDev{0, {0, 0, 0, 0, 0, 0, 0, 0}, {0, 0}};
    field_time_factors(fd, t_np1, dt);
    if (m.coords_f32)
        hipLaunchKernelGGL(k_locate_feet<true>, dim3(g), dim3(kBlock), 0, st, mv, fd, dt, scheme, mode, start,
                           (int)feet_in, (float2 *)feet, elem, (float *)bary, steps, stats);
    else
        hipLaunchKernelGGL(k_locate_feet<false>, dim3(g), dim3(kBlock), 0, st, mv, fd, dt, scheme, mode, start,
                           (int)feet_in, (double2 *)feet, elem, (double *)bary, steps, stats);
    return hipGetLastError();
}

hipError_t launch_interp(const DevMesh &m, hipStream_t st, int order, const int32_t *elem, const void *bary,
                         int64_t mp, const void *v_in, int vdtype, int k, void *v_out, double outside,
                         bool user_order)
{
    if (mp == 0)
        return hipSuccess;
    unsigned g;
    if (!tiles_for(mp, g))
        return hipErrorInvalidValue;
    MeshView mv = view_of(m);
#define SLW_INTERP(F32, V, NA)                                                                                     \
    hipLaunchKernelGGL((k_interp<F32, V, NA>), dim3(g), dim3(kBlock), 0, st, mv, elem,                            \
                       (const typename CT<F32>::R *)bary, mp, (const V *)v_in, k, (V *)v_out, outside, (int)user_order)
    if (m.coords_f32) {
        if (vdtype == SLW_F32) {
            if (order == 1) SLW_INTERP(true, float, 3); else SLW_INTERP(true, float, 6);
        } else {
            if (order == 1) SLW_INTERP(true, double, 3); else SLW_INTERP(true, double, 6);
        }
    } else {
        if (vdtype == SLW_F32) {
            if (order == 1) SLW_INTERP(false, float, 3); else SLW_INTERP(false, float, 6);
        } else {
            if (order == 1) SLW_INTERP(false, double, 3); else SLW_INTERP(false, double, 6);
        }
    }
#undef SLW_INTERP
    return hipGetLastError();
}

hipError_t launch_step(const DevMesh &m, hipStream_t st, const FieldDev &f0, double t_n, double dt, int scheme,
                       int order, int mode, const int32_t *start, const void *v_in, int vdtype, int k, void *v_out,
                       double outside, bool write_prev, const int32_t *out_map, int32_t *elem_out, DevStats *stats)
{
    MeshView mv = view_of(m);
    FieldDev f = f0;
    field_time_factors(f, t_n + dt, dt);
    const int64_t n_iter = order == 1 ? m.n_nodes : m.n_dofs;
    unsigned g;
    if (!tiles_for(n_iter, g))
        return hipErrorInvalidValue;
    // boundary data and the exact search of non-convex domains are applied
    // by the one-foot-per-lane kernels only
    const int rp = (m.bc_kind || m.nonconvex) ? 0 : m.repack;
    if (m.bc_kind && mode == SLW_START_NEIGHBOR && m.chain != 0)
        return hipErrorNotSupported;
    const bool chart_mode = mode == SLW_START_LEARNED || mode == SLW_START_CHART || mode == SLW_START_LEARNED_INDEX;
    const int kind = mode == SLW_START_CHART ? 0 : (mode == SLW_START_LEARNED ? 1 : 2);
    if (chart_mode && rp == 0 && order == 1 && kind != 1) {
        // one foot per lane, P1: the chart start is computed inside the step
        // kernel (not the plain learned start: the network's registers would
        // lower the occupancy of its long walks; its own kernel runs first)
#define SLW_STEP_CHART(F32, V, KD)                                                                                \
    hipLaunchKernelGGL((k_step<F32, V, 3, KD>), dim3(g), dim3(kBlock), 0, st, mv, f, dt, t_n + dt, scheme, mode,    \
                       start, (const V *)v_in, k, (V *)v_out, outside, (int)write_prev, out_map, elem_out, n_iter, stats, \
                       ForestView())
#define SLW_STEP_CHART_K(F32, V)                                                                                  \
    do {                                                                                                          \
        if (kind == 0) SLW_STEP_CHART(F32, V, 0); else SLW_STEP_CHART(F32, V, 2);                                 \
    } while (0)
        if (m.coords_f32) {
            if (vdtype == SLW_F32) SLW_STEP_CHART_K(true, float); else SLW_STEP_CHART_K(true, double);
        } else {
            if (vdtype == SLW_F32) SLW_STEP_CHART_K(false, float); else SLW_STEP_CHART_K(false, double);
        }
#undef SLW_STEP_CHART_K
#undef SLW_STEP_CHART
        return hipGetLastError();
    }
    if ((chart_mode && rp == 0) || mode == SLW_START_LEARNED_INDEX) {
        // the proposals come from their own kernel (the repacking kernel
        // computes chart and learned starts itself)
        hipError_t e = launch_chart_start(m, st, f0, t_n + dt, dt, scheme, nullptr, n_iter, kind, m.learned_start);
        if (e != hipSuccess)
            return e;
        start = m.learned_start;
    }
    if (mode == SLW_START_HYBRID) {
#define SLW_STEP_HYB(F32, V, NA)                                                                                  \
    hipLaunchKernelGGL((k_step<F32, V, NA, -5>), dim3(g), dim3(kBlock), 0, st, mv, f, dt, t_n + dt, scheme, mode, \
                       start, (const V *)v_in, k, (V *)v_out, outside, 0, out_map, elem_out, n_iter, stats,        \
                       ForestView())
        if (m.coords_f32) {
            if (vdtype == SLW_F32) {
                if (order == 1) SLW_STEP_HYB(true, float, 3); else SLW_STEP_HYB(true, float, 6);
            } else {
                if (order == 1) SLW_STEP_HYB(true, double, 3); else SLW_STEP_HYB(true, double, 6);
            }
        } else {
            if (vdtype == SLW_F32) {
                if (order == 1) SLW_STEP_HYB(false, float, 3); else SLW_STEP_HYB(false, float, 6);
            } else {
                if (order == 1) SLW_STEP_HYB(false, double, 3); else SLW_STEP_HYB(false, double, 6);
            }
        }
#undef SLW_STEP_HYB
        return hipGetLastError();
    }
    if (mode == SLW_START_NEIGHBOR && m.chain == 0) {
        // strategy (c) on the mesh's forest: the roots first, then every
        // other DOF from its parent's element (two launches, stream order)
        const int64_t nr = order == 1 ? m.forest_nr1 : m.forest_nr2;
        const int64_t nl = n_iter - nr;
        const int32_t *roots = order == 1 ? m.forest_list1 : m.forest_list2;
        const int32_t *routs = order == 1 ? m.forest_out1 : m.forest_out2;
        if (!roots)
            return hipErrorInvalidValue;
        ForestView fr{roots, routs, nullptr, m.forest_elem};
        ForestView fl{roots + nr, routs + nr, (order == 1 ? m.forest_parent1 : m.forest_parent2), m.forest_elem};
        unsigned gr, gl;
        if (!tiles_for(nr, gr) || !tiles_for(nl, gl))
            return hipErrorInvalidValue;
#define SLW_STEP_FOREST(F32, V, NA)                                                                               \
    do {                                                                                                          \
        if (nr > 0)                                                                                               \
            hipLaunchKernelGGL((k_step<F32, V, NA, -3>), dim3(gr), dim3(kBlock), 0, st, mv, f, dt, t_n + dt, scheme, \
                               mode, start, (const V *)v_in, k, (V *)v_out, outside, 0, out_map, elem_out, nr, stats, \
                               fr);                                                                               \
        if (nl > 0)                                                                                               \
            hipLaunchKernelGGL((k_step<F32, V, NA, -4>), dim3(gl), dim3(kBlock), 0, st, mv, f, dt, t_n + dt, scheme, \
                               mode, start, (const V *)v_in, k, (V *)v_out, outside, 0, out_map, elem_out, nl, stats, \
                               fl);                                                                               \
    } while (0)
        if (m.coords_f32) {
            if (vdtype == SLW_F32) {
                if (order == 1) SLW_STEP_FOREST(true, float, 3); else SLW_STEP_FOREST(true, float, 6);
            } else {
                if (order == 1) SLW_STEP_FOREST(true, double, 3); else SLW_STEP_FOREST(true, double, 6);
            }
        } else {
            if (vdtype == SLW_F32) {
                if (order == 1) SLW_STEP_FOREST(false, float, 3); else SLW_STEP_FOREST(false, float, 6);
            } else {
                if (order == 1) SLW_STEP_FOREST(false, double, 3); else SLW_STEP_FOREST(false, double, 6);
            }
        }
#undef SLW_STEP_FOREST
        return hipGetLastError();
    }
    if (mode == SLW_START_NEIGHBOR) {
        const int L = m.chain;
        const int64_t t = (n_iter + (int64_t)kWave * L - 1) / ((int64_t)kWave * L);
        if (t > (int64_t)INT32_MAX)
            return hipErrorInvalidValue;
        const unsigned gc = (unsigned)(t < 1 ? 1 : t);
#define SLW_CHAIN_L(F32, V, NA, LL)                                                                               \
    hipLaunchKernelGGL((k_step_chain<F32, V, NA, LL>), dim3(gc), dim3(kWave), 0, st, mv, f, dt, scheme,           \
                       (const V *)v_in, k, (V *)v_out, outside, out_map, elem_out, n_iter, stats)
#define SLW_CHAIN(F32, V, NA)                                \
    do {                                                     \
        switch (L) {                                         \
        case 2: SLW_CHAIN_L(F32, V, NA, 2); break;           \
        case 8: SLW_CHAIN_L(F32, V, NA, 8); break;           \
        case 16: SLW_CHAIN_L(F32, V, NA, 16); break;         \
        default: SLW_CHAIN_L(F32, V, NA, 4); break;          \
        }                                                    \
    } while (0)
        if (m.coords_f32) {
            if (vdtype == SLW_F32) {
                if (order == 1) SLW_CHAIN(true, float, 3); else SLW_CHAIN(true, float, 6);
            } else {
                if (order == 1) SLW_CHAIN(true, double, 3); else SLW_CHAIN(true, double, 6);
            }
        } else {
            if (vdtype == SLW_F32) {
                if (order == 1) SLW_CHAIN(false, float, 3); else SLW_CHAIN(false, float, 6);
            } else {
                if (order == 1) SLW_CHAIN(false, double, 3); else SLW_CHAIN(false, double, 6);
            }
        }
#undef SLW_CHAIN
#undef SLW_CHAIN_L
        return hipGetLastError();
    }
    // the learned start's fused kernel has one chunk size: 4 feet per lane
    const int64_t t4 = (n_iter + (int64_t)kBlock * 4 - 1) / ((int64_t)kBlock * 4);
    const unsigned g4 = (unsigned)(t4 < 1 ? 1 : t4);
    if (rp > 0) {
        const int64_t t = (n_iter + (int64_t)kBlock * rp - 1) / ((int64_t)kBlock * rp);
        if (t > (int64_t)INT32_MAX)
            return hipErrorInvalidValue;
        g = (unsigned)(t < 1 ? 1 : t);
    }
#define SLW_STEP_RP(F32, V, NA, RP)                                                                             \
    hipLaunchKernelGGL((k_step_rp<F32, V, NA, RP, false>), dim3(g), dim3(kBlock), 0, st, mv, f, dt, t_n + dt, scheme,   \
                       mode, start,                                                                             \
                       (const V *)v_in, k, (V *)v_out, outside, (int)write_prev, out_map, elem_out, n_iter, stats)
#define SLW_STEP(F32, V, NA)                                                                                   \
    do {                                                                                                       \
    if (rp > 0 && mode == SLW_START_LEARNED) {                                                                 \
        hipLaunchKernelGGL((k_step_rp<F32, V, NA, 4, true>), dim3(g4), dim3(kBlock), 0, st, mv, f, dt, t_n + dt, \
                           scheme, mode, start, (const V *)v_in, k, (V *)v_out, outside, (int)write_prev,      \
                           out_map, elem_out, n_iter, stats);                                                  \
        break;                                                                                                 \
    }                                                                                                          \
    switch (rp) {                                                                                              \
    case 2: SLW_STEP_RP(F32, V, NA, 2); break;                                                                 \
    case 4: SLW_STEP_RP(F32, V, NA, 4); break;                                                                 \
    case 8: SLW_STEP_RP(F32, V, NA, 8); break;                                                                 \
    default:                                                                                                   \
        if (mode == SLW_START_PREV)                                                                            \
            hipLaunchKernelGGL((k_step<F32, V, NA, -2>), dim3(g), dim3(kBlock), 0, st, mv, f, dt, t_n + dt, scheme, \
                               mode, start, (const V *)v_in, k, (V *)v_out, outside, (int)write_prev, out_map,   \
                               elem_out, n_iter, stats, ForestView());                                         \
        else if (mode == SLW_START_GRID)                                                                       \
            hipLaunchKernelGGL((k_step<F32, V, NA, -6>), dim3(g), dim3(kBlock), 0, st, mv, f, dt, t_n + dt, scheme, \
                               mode, start, (const V *)v_in, k, (V *)v_out, outside, (int)write_prev, out_map,   \
                               elem_out, n_iter, stats, ForestView());                                         \
        else if (NA == 3 && m.lds_w > 0)                                                                       \
            hipLaunchKernelGGL((k_step<F32, V, NA, -7>), dim3(g), dim3(kBlock), (size_t)m.lds_w * sizeof(WalkRec),  \
                               st, mv, f, dt, t_n + dt, scheme, mode, start, (const V *)v_in, k, (V *)v_out,    \
                               outside, (int)write_prev, out_map, elem_out, n_iter, stats, ForestView());       \
        else                                                                                                   \
            hipLaunchKernelGGL((k_step<F32, V, NA>), dim3(g), dim3(kBlock), 0, st, mv, f, dt, t_n + dt, scheme, mode, \
                               start, (const V *)v_in, k, (V *)v_out, outside, (int)write_prev, out_map, elem_out, \
                               n_iter, stats, ForestView());                                                   \
    }                                                                                                          \
    } while (0)
    if (m.coords_f32) {
        if (vdtype == SLW_F32) {
            if (order == 1) SLW_STEP(true, float, 3); else SLW_STEP(true, float, 6);
        } else {
            if (order == 1) SLW_STEP(true, double, 3); else SLW_STEP(true, double, 6);
        }
    } else {
        if (vdtype == SLW_F32) {
            if (order == 1) SLW_STEP(false, float, 3); else SLW_STEP(false, float, 6);
        } else {
            if (order == 1) SLW_STEP(false, double, 3); else SLW_STEP(false, double, 6);
        }
    }
#undef SLW_STEP
#undef SLW_STEP_RP
    return hipGetLastError();
}

hipError_t launch_batch_step(hipStream_t st, int coords_f32, int vdtype, int block, int schedule,
                             const BatchItem *items, int n_items, int64_t total_tiles, int64_t *counter, int scheme,
                             int k, double outside, unsigned *queues, int persistent_blocks, DevStats *stats)
{
    if (total_tiles <= 0)
        return hipSuccess;
    if (total_tiles > (int64_t)INT32_MAX)
        return hipErrorInvalidValue;
    if (schedule == 1) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, queues, 8);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    const unsigned g = schedule == 1 ? (unsigned)persistent_blocks : (unsigned)total_tiles;
#define SLW_BSTEP(F32, V, BS)                                                                                      \
    do {                                                                                                           \
        if (schedule == 1)                                                                                         \
            hipLaunchKernelGGL((k_batch_step<F32, V, BS, 1>), dim3(g), dim3(BS), 0, st, items, n_items, total_tiles, \
                               counter, scheme, k, outside, queues, stats);                                        \
        else if (schedule == 2)                                                                                    \
            hipLaunchKernelGGL((k_batch_step<F32, V, BS, 2>), dim3(g), dim3(BS), 0, st, items, n_items, total_tiles, \
                               counter, scheme, k, outside, queues, stats);                                        \
        else                                                                                                       \
            hipLaunchKernelGGL((k_batch_step<F32, V, BS, 0>), dim3(g), dim3(BS), 0, st, items, n_items, total_tiles, \
                               counter, scheme, k, outside, queues, stats);                                        \
    } while (0)
#define SLW_BSTEP_BS(F32, V)            \
    switch (block) {                    \
    case 64: SLW_BSTEP(F32, V, 64); break;   \
    case 128: SLW_BSTEP(F32, V, 128); break; \
    case 512: SLW_BSTEP(F32, V, 512); break; \
    default: SLW_BSTEP(F32, V, 256); break;  \
    }
    if (coords_f32) {
        if (vdtype == SLW_F32) { SLW_BSTEP_BS(true, float); } else { SLW_BSTEP_BS(true, double); }
    } else {
        if (vdtype == SLW_F32) { SLW_BSTEP_BS(false, float); } else { SLW_BSTEP_BS(false, double); }
    }
#undef SLW_BSTEP_BS
#undef SLW_BSTEP
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, counter, (int64_t)1);
    return hipGetLastError();
}

hipError_t launch_zero_stats(hipStream_t st, DevStats *p)
{
    const int n = (int)(sizeof(DevStats) / sizeof(unsigned long long));
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, (unsigned long long *)p, n);
    return hipGetLastError();
}

hipError_t launch_permute_rows(hipStream_t st, const void *src, void *dst, int64_t rows, int64_t row_bytes,
                               const int32_t *map, int scatter)
{
    if (rows == 0)
        return hipSuccess;
    const int64_t words = row_bytes / 4;
    int64_t g = (rows * words + kBlock - 1) / kBlock;
    g = g < 1 ? 1 : (g > ((int64_t)1 << 20) ? ((int64_t)1 << 20) : g);
    hipLaunchKernelGGL(k_permute_rows, dim3((unsigned)g), dim3(kBlock), 0, st, (const uint32_t *)src,
                       (uint32_t *)dst, rows, words, map, scatter);
    return hipGetLastError();
}

hipError_t launch_chart_start(const DevMesh &m, hipStream_t st, const FieldDev &f0, double t_np1, double dt,
                              int scheme, const void *feet_in, int64_t n_iter, int kind, int32_t *start)
{
    if (n_iter <= 0)
        return hipSuccess;
    if (!m.chart_table || (kind > 0 && !m.mlp) || kind < 0 || kind > 2)
        return hipErrorInvalidValue;
    unsigned g;
    if (!tiles_for(n_iter, g))
        return hipErrorInvalidValue;
    MeshView mv = view_of(m);
    FieldDev f = f0;
    field_time_factors(f, t_np1, dt);
#define SLW_CSTART(F32, KIND, R2)                                                                                 \
    hipLaunchKernelGGL((k_chart_start<F32, KIND>), dim3(g), dim3(kBlock), 0, st, mv, f, dt, t_np1, scheme,       \
                       (const R2 *)feet_in, n_iter, start)
    if (m.coords_f32) {
        if (kind == 2) SLW_CSTART(true, 2, float2); else if (kind == 1) SLW_CSTART(true, 1, float2); else SLW_CSTART(true, 0, float2);
    } else {
        if (kind == 2) SLW_CSTART(false, 2, double2); else if (kind == 1) SLW_CSTART(false, 1, double2); else SLW_CSTART(false, 0, double2);
    }
#undef SLW_CSTART
    return hipGetLastError();
}

hipError_t launch_learned_gather(const DevMesh &m, hipStream_t st, const FieldDev &f0, double t_np1, double dt,
                                 int scheme, const int32_t *dofs, int64_t cnt, float *X, float *Y)
{
    if (cnt <= 0)
        return hipSuccess;
    unsigned g;
    if (!tiles_for(cnt, g))
        return hipErrorInvalidValue;
    MeshView mv = view_of(m);
    FieldDev f = f0;
    field_time_factors(f, t_np1, dt);
    if (m.coords_f32)
        hipLaunchKernelGGL(k_gather<true>, dim3(g), dim3(kBlock), 0, st, mv, f, dt, t_np1, scheme, dofs, cnt,
                           m.chart_uv, m.chart_node, X, (float2 *)Y);
    else
        hipLaunchKernelGGL(k_gather<false>, dim3(g), dim3(kBlock), 0, st, mv, f, dt, t_np1, scheme, dofs, cnt,
                           m.chart_uv, m.chart_node, X, (float2 *)Y);
    return hipGetLastError();
}

}  // namespace slw
