// Device kernels: feet, start selection, barycentric walk, tie rule,
// interpolation, and the fused semi-Lagrangian step.
//
// One lane handles one foot.  A walk step reads one triangle record (vertex
// coordinates + neighbours, 64 B in double, 48 B in float), computes the three
// edge orientations of the foot, and either stops (all signs >= 0: the
// barycentric coordinates of Section 2.2 are all non-negative) or crosses the
// edge with the most negative coordinate.  Signs are exact (filtered FP32 /
// FP64, then exact expansion arithmetic), so the triangle found does not
// depend on where the walk started.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "slw_internal.h"
#include "slw_predicates.h"

namespace slw {

namespace {

constexpr int kBlock = 256;

template <bool F32>
struct CT;
template <>
struct CT<false> {
    using R = double;
    using R2 = double2;
    using Geo = GeoRec64;
};
template <>
struct CT<true> {
    using R = float;
    using R2 = float2;
    using Geo = GeoRec32;
};

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

// ---------------------------------------------------------------------------
// start selection

__device__ inline float pseudo_angle_f(float dx, float dy)
{
    float s = fabsf(dx) + fabsf(dy);
    if (s == 0.0f)
        return 0.0f;
    float r = dx / s;
    return dy >= 0.0f ? 1.0f - r : 3.0f + r;
}

// The incident triangle of DOF d whose angular sector contains the direction
// of the foot (strategy (a) of Section 3 with the element facing the foot).
__device__ inline int32_t steer(const int32_t *__restrict__ sptr, const StarEnt *__restrict__ star, int64_t d,
                                float dx, float dy)
{
    int32_t s0 = sptr[d], s1 = sptr[d + 1];
    float th = pseudo_angle_f(dx, dy);
    int32_t sel = s1 - 1;
    for (int32_t s = s0; s < s1; ++s)
        if (star[s].ang <= th)
            sel = s;
    return star[sel].tri;
}

// ---------------------------------------------------------------------------
// exact edge signs of a triangle record for a point

struct Counters {
    uint32_t exact = 0, fp64 = 0;
};

__device__ inline void edge_signs64(const double2 p[3], double qx, double qy, double o[3], int s[3], Counters &c)
{
    double dx[3], dy[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dx[k] = p[k].x - qx;
        dy[k] = p[k].y - qy;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        bool certain;
        const double det = filter64(dx[a] * dy[b], dy[a] * dx[b], certain);
        o[k] = det;
        if (certain)
            s[k] = sign_of(det);
        else {
            s[k] = orient_exact_sign(p[a].x, p[a].y, p[b].x, p[b].y, qx, qy);
            ++c.exact;
        }
    }
}

__device__ inline void edge_signs32(const float2 p[3], float qx, float qy, float o[3], int s[3], Counters &c)
{
    float dx[3], dy[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dx[k] = p[k].x - qx;
        dy[k] = p[k].y - qy;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int a = (k + 1) % 3, b = (k + 2) % 3;
        bool certain;
        const float det = filter32(dx[a] * dy[b], dy[a] * dx[b], certain);
        o[k] = det;
        if (certain)
            s[k] = (det > 0.0f) - (det < 0.0f);
        else {
            double d64 = orient_fp64((double)p[a].x, (double)p[a].y, (double)p[b].x, (double)p[b].y, (double)qx,
                                     (double)qy, certain);
            ++c.fp64;
            if (certain)
                s[k] = sign_of(d64);
            else {
                s[k] = orient_exact_sign((double)p[a].x, (double)p[a].y, (double)p[b].x, (double)p[b].y,
                                         (double)qx, (double)qy);
                ++c.exact;
            }
        }
    }
}

template <bool F32>
__device__ inline void load_geo(const typename CT<F32>::Geo *__restrict__ geo, int32_t j,
                                typename CT<F32>::R2 p[3], int32_t nb[3], int32_t &uid)
{
    const typename CT<F32>::Geo g = geo[j];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        p[k] = g.p[k];
        nb[k] = g.nb[k];
    }
    uid = g.uid;
}

template <bool F32>
__device__ inline void edge_signs(const typename CT<F32>::R2 p[3], typename CT<F32>::R qx, typename CT<F32>::R qy,
                                  typename CT<F32>::R o[3], int s[3], Counters &c)
{
    if constexpr (F32)
        edge_signs32(p, qx, qy, o, s, c);
    else
        edge_signs64(p, qx, qy, o, s, c);
}

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
    int32_t uid;    // user id of elem
    int32_t steps;  // element changes
    int32_t flags;  // bit0 fallback walk, bit1 hard limit, bit2 edge tie, bit3 vertex tie
    R th[3];        // barycentric coordinates in the internal vertex order of elem
};

struct WalkParams {
    const void *geo;
    const TopRec *top;
    const int32_t *vmin;
    int32_t step_cap;
    int32_t hard_limit;
};

// Barycentric walk of Section 2.2 from triangle j to the foot (qx, qy), then
// the tie rule (smallest user id among the closed containers).
template <bool F32>
__device__ WalkResult<typename CT<F32>::R> walk(const WalkParams &wp, int32_t j, typename CT<F32>::R qx,
                                                 typename CT<F32>::R qy, uint32_t seed, Counters &c)
{
    using R = typename CT<F32>::R;
    using R2 = typename CT<F32>::R2;
    using Geo = typename CT<F32>::Geo;
    const Geo *geo = (const Geo *)wp.geo;
    WalkResult<R> res;
    res.steps = 0;
    res.flags = 0;
    R2 p[3];
    int32_t nb[3], uid;
    R o[3];
    int s[3];
    for (;;) {
        load_geo<F32>(geo, j, p, nb, uid);
        edge_signs<F32>(p, qx, qy, o, s, c);
        const bool n0 = s[0] < 0, n1 = s[1] < 0, n2 = s[2] < 0;
        if (!(n0 | n1 | n2))
            break;
        // a negative side on the boundary: the foot is outside the (convex) domain
        if ((n0 && nb[0] < 0) || (n1 && nb[1] < 0) || (n2 && nb[2] < 0)) {
            res.elem = -1;
            res.uid = -1;
            return res;
        }
        if (res.steps >= wp.hard_limit) {
            res.flags |= 2;
            res.elem = -1;
            res.uid = -1;
            return res;
        }
        int k;
        if (res.steps < wp.step_cap) {
            // most negative barycentric coordinate, lowest index on ties
            k = n0 ? 0 : (n1 ? 1 : 2);
            if (n1 && o[1] < o[k])
                k = 1;
            if (n2 && o[2] < o[k])
                k = 2;
        } else {
            // randomised visibility walk: a uniformly chosen separating edge
            // (terminates with probability 1 on any triangulation)
            res.flags |= 1;
            const int cnt = (int)n0 + (int)n1 + (int)n2;
            int pick = (int)(hash32(seed ^ hash32((uint32_t)res.steps)) % (uint32_t)cnt);
            k = -1;
            for (int q = 0; q < 3; ++q)
                if (s[q] < 0 && pick-- == 0)
                    k = q;
        }
        j = nb[k];
        ++res.steps;
    }
    // tie rule on the closed containers
    const int z = (s[0] == 0) + (s[1] == 0) + (s[2] == 0);
    int32_t e = j;
    if (z == 1) {
        const int k = s[0] == 0 ? 0 : (s[1] == 0 ? 1 : 2);
        res.flags |= 4;
        if (nb[k] >= 0 && geo[nb[k]].uid < uid)
            e = nb[k];
    } else if (z == 2) {
        const int cidx = s[0] != 0 ? 0 : (s[1] != 0 ? 1 : 2);
        res.flags |= 8;
        e = wp.vmin[wp.top[j].v[cidx]];
    }
    if (e != j) {
        load_geo<F32>(geo, e, p, nb, uid);
        edge_signs<F32>(p, qx, qy, o, s, c);
    }
    const R sum = o[0] + o[1] + o[2];
    res.th[0] = o[0] / sum;
    res.th[1] = o[1] / sum;
    res.th[2] = o[2] / sum;
    res.elem = e;
    res.uid = uid;
    return res;
}

// ---------------------------------------------------------------------------
// statistics: one atomic per wavefront

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
    uint32_t feet = 0, outside = 0, steps = 0, max_steps = 0, fallback = 0, edge = 0, vertex = 0, hard = 0;
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
    }
};

__device__ inline void flush_stats(const LaneStats &ls, DevStats *st)
{
    unsigned long long v[10] = {ls.feet, ls.outside, ls.steps, ls.max_steps, ls.c.exact, ls.c.fp64, ls.fallback,
                                ls.edge, ls.vertex, ls.hard};
    unsigned long long *dst[10] = {&st->feet, &st->outside, &st->walk_steps, &st->max_steps, &st->exact_tests,
                                   &st->fp64_tests, &st->fallback_walks, &st->edge_ties, &st->vertex_ties,
                                   &st->hard_fail};
    const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        unsigned long long r = (i == 3) ? wave_max(v[i]) : wave_sum(v[i]);
        if (lead && r != 0) {
            if (i == 3)
                atomicMax(dst[i], r);
            else
                atomicAdd(dst[i], r);
        }
    }
}

// queries outside the mesh's bounding box (or not finite) are outside
// without a walk
template <typename R>
__device__ inline bool in_box(R qx, R qy, const double bb[4])
{
    // written so that NaN compares false and lands outside
    return (double)qx >= bb[0] && (double)qx <= bb[2] && (double)qy >= bb[1] && (double)qy <= bb[3];
}

struct MeshView {
    const void *geo;
    const TopRec *top;
    const int4 *tedge;
    const void *dof_xy;
    const int32_t *sptr;
    const StarEnt *star;
    const int32_t *vmin;
    const int32_t *dof_user;
    const int32_t *tri_int;
    int32_t *prev;
    const int32_t *jump;
    int jump_g;
    int64_t n_dofs;
    int64_t n_tris;
    double bb[4];
    int32_t step_cap, hard_limit;
    int internal_order;
};

MeshView view_of(const DevMesh &m)
{
    MeshView v;
    v.geo = m.geo;
    v.top = m.top;
    v.tedge = m.tedge;
    v.dof_xy = m.dof_xy;
    v.sptr = m.star_ptr;
    v.star = m.star;
    v.vmin = m.vmin;
    v.dof_user = m.dof_user;
    v.tri_int = m.tri_int;
    v.prev = m.prev_elem;
    v.jump = m.jump;
    v.jump_g = m.jump_g;
    v.n_dofs = m.n_dofs;
    v.n_tris = m.n_tris;
    for (int i = 0; i < 4; ++i)
        v.bb[i] = m.bbox[i];
    v.step_cap = m.step_cap;
    v.hard_limit = m.hard_limit;
    v.internal_order = m.internal_order;
    return v;
}

__device__ inline WalkParams walk_params(const MeshView &mv)
{
    WalkParams wp;
    wp.geo = mv.geo;
    wp.top = mv.top;
    wp.vmin = mv.vmin;
    wp.step_cap = mv.step_cap;
    wp.hard_limit = mv.hard_limit;
    return wp;
}

template <typename R>
__device__ inline void user_bary(const TopRec &t, const R th[3], R out[3])
{
    out[0] = th[0];
    if (t.flags & 1) {
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
    const WalkParams wp = walk_params(mv);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        R qx = q[i].x, qy = q[i].y;
        WalkResult<R> w;
        w.elem = -1;
        w.uid = -1;
        w.steps = 0;
        w.flags = 0;
        if (in_box<R>(qx, qy, mv.bb)) {
            int32_t j0;
            const int32_t su = start ? start[i] : -1;
            if (su >= 0 && su < mv.n_tris) {
                j0 = mv.tri_int[su];
            } else {
                const double wx = (mv.bb[2] - mv.bb[0]), wy = (mv.bb[3] - mv.bb[1]);
                const double span = wx > wy ? wx : wy;
                const double w = span > 0 ? span / mv.jump_g : 1.0;
                int cx = (int)floor(((double)qx - mv.bb[0]) / w), cy = (int)floor(((double)qy - mv.bb[1]) / w);
                cx = cx < 0 ? 0 : (cx >= mv.jump_g ? mv.jump_g - 1 : cx);
                cy = cy < 0 ? 0 : (cy >= mv.jump_g ? mv.jump_g - 1 : cy);
                j0 = mv.jump[(int64_t)cy * mv.jump_g + cx];
            }
            w = walk<F32>(wp, j0, qx, qy, (uint32_t)i * 2654435761u, ls.c);
        }
        if (st)
            ls.add(w);
        elem[i] = w.uid;
        if (bary) {
            if (w.elem >= 0) {
                R ub[3];
                user_bary<R>(mv.top[w.elem], w.th, ub);
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

template <bool F32>
__device__ inline int32_t start_for(const MeshView &mv, int64_t d, int64_t api, int mode,
                                    const int32_t *__restrict__ start, float dx, float dy)
{
    // caller-given ids outside [0, n_tris) fall back to the steered start
    if (mode == SLW_START_GIVEN || mode == SLW_START_FIXED) {
        const int32_t u = start[mode == SLW_START_GIVEN ? api : 0];
        if (u >= 0 && u < mv.n_tris)
            return mv.tri_int[u];
    }
    if (mode == SLW_START_PREV) {
        int32_t pe = mv.prev[d];
        if (pe >= 0)
            return pe;
    }
    return steer(mv.sptr, mv.star, d, dx, dy);
}

template <bool F32>
__global__ void __launch_bounds__(kBlock)
    k_locate_feet(MeshView mv, FieldDev f, double t_np1, double dt, int scheme, int mode,
                  const int32_t *__restrict__ start, int feet_in, typename CT<F32>::R2 *__restrict__ feet,
                  int32_t *__restrict__ elem, typename CT<F32>::R *__restrict__ bary, int32_t *__restrict__ steps,
                  DevStats *st)
{
    using R = typename CT<F32>::R;
    using R2 = typename CT<F32>::R2;
    LaneStats ls;
    const WalkParams wp = walk_params(mv);
    const R2 *X = (const R2 *)mv.dof_xy;
    for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < mv.n_dofs;
         d += (int64_t)gridDim.x * blockDim.x) {
        const int64_t api = mv.internal_order ? d : mv.dof_user[d];
        const R2 x = X[d];
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
        WalkResult<R> w;
        w.elem = -1;
        w.uid = -1;
        w.steps = 0;
        w.flags = 0;
        if (in_box<R>(qx, qy, mv.bb)) {
            int32_t j0 = start_for<F32>(mv, d, api, mode, start, (float)(qx - x.x), (float)(qy - x.y));
            w = walk<F32>(wp, j0, qx, qy, (uint32_t)d * 2654435761u, ls.c);
        }
        if (mode == SLW_START_PREV)
            mv.prev[d] = w.elem;
        if (st)
            ls.add(w);
        if (elem)
            elem[api] = w.uid;
        if (bary) {
            if (w.elem >= 0) {
                R ub[3];
                user_bary<R>(mv.top[w.elem], w.th, ub);
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

// weighted sum of rows: out[f] = sum_a w[a] * V[row_a * k + f]
template <typename V, int NA>
__device__ inline void combine_rows(const V *__restrict__ vin, const int64_t rows[NA], const V w[NA], int k,
                                    V *__restrict__ out)
{
    const bool aligned = ((reinterpret_cast<uintptr_t>(vin) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    if constexpr (sizeof(V) == 4) {
        if ((k & 3) == 0 && aligned) {
            for (int f = 0; f < k; f += 4) {
                float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
                for (int a = 0; a < NA; ++a) {
                    const float4 r = *(const float4 *)(vin + rows[a] * k + f);
                    acc.x = fmaf(w[a], r.x, acc.x);
                    acc.y = fmaf(w[a], r.y, acc.y);
                    acc.z = fmaf(w[a], r.z, acc.z);
                    acc.w = fmaf(w[a], r.w, acc.w);
                }
                *(float4 *)(out + f) = acc;
            }
            return;
        }
    } else {
        if ((k & 1) == 0 && aligned) {
            for (int f = 0; f < k; f += 2) {
                double2 acc = make_double2(0.0, 0.0);
#pragma unroll
                for (int a = 0; a < NA; ++a) {
                    const double2 r = *(const double2 *)(vin + rows[a] * k + f);
                    acc.x = fma(w[a], r.x, acc.x);
                    acc.y = fma(w[a], r.y, acc.y);
                }
                *(double2 *)(out + f) = acc;
            }
            return;
        }
    }
    for (int f = 0; f < k; ++f) {
        V acc = (V)0;
#pragma unroll
        for (int a = 0; a < NA; ++a)
            acc = fma(w[a], vin[rows[a] * k + f], acc);
        out[f] = acc;
    }
}

// P1 / P2 values at a located point from internal element e and internal-order
// barycentric coordinates th; rows are internal DOF ids, mapped through
// row_map when the value array is in the user's order.
template <typename R, typename V>
__device__ inline void interp_point(const MeshView &mv, int order, int32_t e, const R th[3],
                                    const V *__restrict__ vin, int k, const int32_t *__restrict__ row_map,
                                    V outside, V *__restrict__ out)
{
    if (e < 0) {
        for (int f = 0; f < k; ++f)
            out[f] = outside;
        return;
    }
    const TopRec t = mv.top[e];
    if (order == 1) {
        int64_t rows[3];
        V w[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            rows[a] = row_map ? row_map[t.v[a]] : t.v[a];
            w[a] = (V)th[a];
        }
        combine_rows<V, 3>(vin, rows, w, k, out);
    } else {
        const int4 te = mv.tedge[e];
        const int32_t ev[3] = {te.x, te.y, te.z};
        int64_t rows[6];
        V w[6];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int b = (a + 1) % 3, c = (a + 2) % 3;
            rows[a] = row_map ? row_map[t.v[a]] : t.v[a];
            rows[3 + a] = row_map ? row_map[ev[a]] : ev[a];
            w[a] = (V)(th[a] * ((R)2 * th[a] - (R)1));
            w[3 + a] = (V)((R)4 * th[b] * th[c]);
        }
        combine_rows<V, 6>(vin, rows, w, k, out);
    }
}

template <bool F32, typename V>
__global__ void __launch_bounds__(kBlock)
    k_interp(MeshView mv, int order, const int32_t *__restrict__ elem, const typename CT<F32>::R *__restrict__ bary,
             int64_t m, const V *__restrict__ vin, int k, V *__restrict__ vout, double outside, int user_rows)
{
    using R = typename CT<F32>::R;
    const int32_t *row_map = user_rows ? mv.dof_user : nullptr;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = elem[i];
        // ids outside [0, n_tris) are treated as outside
        int32_t e = (u >= 0 && u < mv.n_tris) ? mv.tri_int[u] : -1;
        R th[3] = {0, 0, 0};
        if (e >= 0) {
            // user vertex order -> internal order
            const TopRec t = mv.top[e];
            th[0] = bary[3 * i];
            th[1] = (t.flags & 1) ? bary[3 * i + 2] : bary[3 * i + 1];
            th[2] = (t.flags & 1) ? bary[3 * i + 1] : bary[3 * i + 2];
        }
        interp_point<R, V>(mv, order, e, th, vin, k, row_map, (V)outside, vout + i * (int64_t)k);
    }
}

template <typename VV>
__device__ inline VV vv_zero();
template <>
__device__ inline float4 vv_zero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <>
__device__ inline double2 vv_zero<double2>() { return make_double2(0.0, 0.0); }
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

// Workgroups are dispatched to the 8 XCDs round-robin (block b runs on XCD
// b mod 8).  Give each XCD one contiguous range of tiles instead, so that the
// Morton-ordered tiles one XCD processes are spatially compact and the
// triangle records and value rows they share stay in that XCD's L2.
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb)
{
    constexpr int64_t kXcd = 8;
    const int64_t q = nb / kXcd, r = nb % kXcd;
    const int64_t x = b % kXcd, local = b / kXcd;
    return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// The fused step, one workgroup per tile of kBlock consecutive (Morton) DOFs.
// Phase 1, one lane per foot: foot -> start -> walk -> tie rule -> weights;
// the located element's value rows and weights go to LDS.  Phase 2, the
// workgroup interpolates the tile's values cooperatively: work item
// (foot, chunk of VW fields), consecutive lanes on consecutive chunks, so
// the row gathers read whole row segments and the stores are contiguous.
template <bool F32, typename V, int NA>
__global__ void __launch_bounds__(kBlock)
    k_step(MeshView mv, FieldDev f, double dt, int scheme, int mode, const int32_t *__restrict__ start,
           const V *__restrict__ vin, int k, V *__restrict__ vout, double outside, int write_prev,
           const int32_t *__restrict__ out_map, int64_t n_iter, DevStats *st)
{
    using R = typename CT<F32>::R;
    using R2 = typename CT<F32>::R2;
    __shared__ int32_t s_row[NA][kBlock];
    __shared__ V s_w[NA][kBlock];
    const int64_t base = xcd_tile(blockIdx.x, gridDim.x) * kBlock;
    const int tid = threadIdx.x;
    const int64_t d = base + tid;
    LaneStats ls;
    if (d < n_iter) {
        const WalkParams wp = walk_params(mv);
        const R2 x = ((const R2 *)mv.dof_xy)[d];
        R qx, qy;
        foot_of<R>(f, scheme, x.x, x.y, (R)dt, qx, qy);
        WalkResult<R> w;
        w.elem = -1;
        w.uid = -1;
        w.steps = 0;
        w.flags = 0;
        if (in_box<R>(qx, qy, mv.bb)) {
            const int64_t api = (mode == SLW_START_GIVEN && !mv.internal_order) ? mv.dof_user[d] : d;
            const int32_t j0 = start_for<F32>(mv, d, api, mode, start, (float)(qx - x.x), (float)(qy - x.y));
            w = walk<F32>(wp, j0, qx, qy, (uint32_t)d * 2654435761u, ls.c);
        }
        if (write_prev)
            mv.prev[d] = w.elem;
        if (st)
            ls.add(w);
        if (w.elem >= 0) {
            const TopRec t = mv.top[w.elem];
            if constexpr (NA == 3) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    s_row[a][tid] = t.v[a];
                    s_w[a][tid] = (V)w.th[a];
                }
            } else {
                const int4 te = mv.tedge[w.elem];
                const int32_t ev[3] = {te.x, te.y, te.z};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int b = (a + 1) % 3, c = (a + 2) % 3;
                    s_row[a][tid] = t.v[a];
                    s_row[3 + a][tid] = ev[a];
                    s_w[a][tid] = (V)(w.th[a] * ((R)2 * w.th[a] - (R)1));
                    s_w[3 + a][tid] = (V)((R)4 * w.th[b] * w.th[c]);
                }
            }
        } else {
            s_row[0][tid] = -1;
        }
    }
    if (st)
        flush_stats(ls, st);
    __syncthreads();

    const int nf = (int)min<int64_t>(kBlock, n_iter - base);
    constexpr int VW = sizeof(V) == 4 ? 4 : 2;  // fields per 16-byte chunk
    const bool aligned = ((reinterpret_cast<uintptr_t>(vin) | reinterpret_cast<uintptr_t>(vout)) & 15) == 0;
    if (aligned && k % VW == 0) {
        using VV = typename std::conditional<sizeof(V) == 4, float4, double2>::type;
        const int chunks = k / VW;
        for (int it = tid; it < nf * chunks; it += kBlock) {
            const int fl = it / chunks, c = it - fl * chunks;
            const int64_t o = out_map ? out_map[base + fl] : base + fl;
            VV *dst = (VV *)(vout + o * (int64_t)k) + c;
            const int32_t r0 = s_row[0][fl];
            if (r0 < 0) {
                VV z;
                if constexpr (VW == 4)
                    z = make_float4((float)outside, (float)outside, (float)outside, (float)outside);
                else
                    z = make_double2(outside, outside);
                *dst = z;
                continue;
            }
            VV acc = vv_zero<VV>();
#pragma unroll
            for (int a = 0; a < NA; ++a)
                vv_fma(s_w[a][fl], *((const VV *)(vin + (int64_t)s_row[a][fl] * k) + c), acc);
            *dst = acc;
        }
    } else {
        for (int it = tid; it < nf * k; it += kBlock) {
            const int fl = it / k, c = it - fl * k;
            const int64_t o = out_map ? out_map[base + fl] : base + fl;
            const int32_t r0 = s_row[0][fl];
            V acc = (V)outside;
            if (r0 >= 0) {
                acc = (V)0;
#pragma unroll
                for (int a = 0; a < NA; ++a)
                    acc = fma(s_w[a][fl], vin[(int64_t)s_row[a][fl] * k + c], acc);
            }
            vout[o * (int64_t)k + c] = acc;
        }
    }
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

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0ull;
}

inline int grid_for(int64_t n)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g < 1)
        g = 1;
    if (g > (int64_t)1 << 20)
        g = (int64_t)1 << 20;
    return (int)g;
}

}  // namespace

hipError_t launch_locate(const DevMesh &m, hipStream_t st, const void *q, int64_t mp, const int32_t *start,
                         int32_t *elem, void *bary, int32_t *steps, DevStats *stats)
{
    if (mp == 0)
        return hipSuccess;
    MeshView mv = view_of(m);
    if (m.coords_f32)
        hipLaunchKernelGGL(k_locate<true>, dim3(grid_for(mp)), dim3(kBlock), 0, st, mv, (const float2 *)q, mp, start,
                           elem, (float *)bary, steps, stats);
    else
        hipLaunchKernelGGL(k_locate<false>, dim3(grid_for(mp)), dim3(kBlock), 0, st, mv, (const double2 *)q, mp,
                           start, elem, (double *)bary, steps, stats);
    return hipGetLastError();
}

hipError_t launch_locate_feet(const DevMesh &m, hipStream_t st, const FieldDev *f, double t_np1, double dt,
                              int scheme, int mode, const int32_t *start, bool feet_in, void *feet, int32_t *elem,
                              void *bary, int32_t *steps, DevStats *stats)
{
    MeshView mv = view_of(m);
    FieldDev fd = f ? *f : FieldDev{0, {0, 0, 0, 0, 0, 0, 0, 0}, {0, 0}};
    field_time_factors(fd, t_np1, dt);
    if (m.coords_f32)
        hipLaunchKernelGGL(k_locate_feet<true>, dim3(grid_for(m.n_dofs)), dim3(kBlock), 0, st, mv, fd, t_np1, dt,
                           scheme, mode, start, (int)feet_in, (float2 *)feet, elem, (float *)bary, steps, stats);
    else
        hipLaunchKernelGGL(k_locate_feet<false>, dim3(grid_for(m.n_dofs)), dim3(kBlock), 0, st, mv, fd, t_np1, dt,
                           scheme, mode, start, (int)feet_in, (double2 *)feet, elem, (double *)bary, steps, stats);
    return hipGetLastError();
}

hipError_t launch_interp(const DevMesh &m, hipStream_t st, int order, const int32_t *elem, const void *bary,
                         int64_t mp, const void *v_in, int vdtype, int k, void *v_out, double outside,
                         bool user_order)
{
    if (mp == 0)
        return hipSuccess;
    MeshView mv = view_of(m);
    const int g = grid_for(mp);
    if (m.coords_f32) {
        if (vdtype == SLW_F32)
            hipLaunchKernelGGL((k_interp<true, float>), dim3(g), dim3(kBlock), 0, st, mv, order, elem,
                               (const float *)bary, mp, (const float *)v_in, k, (float *)v_out, outside,
                               (int)user_order);
        else
            hipLaunchKernelGGL((k_interp<true, double>), dim3(g), dim3(kBlock), 0, st, mv, order, elem,
                               (const float *)bary, mp, (const double *)v_in, k, (double *)v_out, outside,
                               (int)user_order);
    } else {
        if (vdtype == SLW_F32)
            hipLaunchKernelGGL((k_interp<false, float>), dim3(g), dim3(kBlock), 0, st, mv, order, elem,
                               (const double *)bary, mp, (const float *)v_in, k, (float *)v_out, outside,
                               (int)user_order);
        else
            hipLaunchKernelGGL((k_interp<false, double>), dim3(g), dim3(kBlock), 0, st, mv, order, elem,
                               (const double *)bary, mp, (const double *)v_in, k, (double *)v_out, outside,
                               (int)user_order);
    }
    return hipGetLastError();
}

hipError_t launch_step(const DevMesh &m, hipStream_t st, const FieldDev &f0, double t_n, double dt, int scheme,
                       int order, int mode, const int32_t *start, const void *v_in, int vdtype, int k, void *v_out,
                       double outside, bool write_prev, const int32_t *out_map, DevStats *stats)
{
    MeshView mv = view_of(m);
    FieldDev f = f0;
    field_time_factors(f, t_n + dt, dt);
    const int64_t n_iter = order == 1 ? m.n_nodes : m.n_dofs;
    const int64_t tiles = (n_iter + kBlock - 1) / kBlock;
    if (tiles == 0)
        return hipSuccess;
    if (tiles > (int64_t)INT32_MAX)
        return hipErrorInvalidValue;
    const dim3 g((unsigned)tiles), b(kBlock);
#define SLW_STEP(F32, V, NA)                                                                                   \
    hipLaunchKernelGGL((k_step<F32, V, NA>), g, b, 0, st, mv, f, dt, scheme, mode, start, (const V *)v_in, k, \
                       (V *)v_out, outside, (int)write_prev, out_map, n_iter, stats)
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
    return hipGetLastError();
}

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
    hipLaunchKernelGGL(k_permute_rows, dim3(grid_for(rows * words)), dim3(kBlock), 0, st, (const uint32_t *)src,
                       (uint32_t *)dst, rows, words, map, scatter);
    return hipGetLastError();
}

}  // namespace slw
