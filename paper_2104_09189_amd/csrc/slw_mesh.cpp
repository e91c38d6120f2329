// Mesh upload: validation, adjacency, start tables, Morton order, device copy.
//
// The structures follow Section 3 of the paper (node list, triangle list,
// neighbour list with neighbour k across the edge opposite vertex k, and a
// per-node start list), laid out for the GPU walk:
//   - nodes and triangles are renumbered along a Morton (Z-order) curve of
//     their position (triangles by centroid), so that neighbouring feet read
//     neighbouring records;
//   - each triangle record carries its vertex coordinates and neighbours, so
//     one walk step is one 64-byte load (48 bytes for float coordinates);
//   - each DOF keeps its incident triangles sorted by the direction of the
//     sector they occupy at the DOF, so a walk can start in the triangle that
//     faces its foot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <numeric>
#include <string>
#include <vector>

#include "slw_internal.h"
#include "slw_predicates.h"

namespace slw {

namespace {

// Star entry of a DOF: an incident triangle and the pseudo-angle (in [0, 4))
// of the direction where its angular sector at the DOF begins.
struct StarEnt {
    float ang;
    int32_t tri;
};

// Monotone stand-in for the polar angle of (dx, dy): 0 along +x, increasing
// counter-clockwise, in [0, 4).
double pseudo_angle(double dx, double dy)
{
    double s = std::fabs(dx) + std::fabs(dy);
    if (s == 0.0)
        return 0.0;
    double r = dx / s;
    return dy >= 0.0 ? 1.0 - r : 3.0 + r;
}

uint64_t spread21(uint64_t v)
{
    v &= 0x1fffff;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

// Position of cell (x, y) of the 2^21 x 2^21 grid along the Hilbert curve
// (the usual quadrant recursion: at each level, from the coarsest, add the
// quadrant's rank along the curve times the quadrant's cell count, then
// rotate / reflect the coordinates into that quadrant's frame).
uint64_t hilbert21(uint64_t x, uint64_t y)
{
    constexpr uint64_t n = (uint64_t)1 << 21;
    uint64_t d = 0;
    for (uint64_t s = n >> 1; s > 0; s >>= 1) {
        const uint64_t rx = (x & s) ? 1 : 0, ry = (y & s) ? 1 : 0;
        d += s * s * ((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

// Space-filling-curve key of a point: its cell in a 2^21 x 2^21 grid over
// the bounding box, ranked along the Hilbert curve (or the Morton curve)
struct MortonFrame {
    double x0, y0, scale;
    bool hilbert;
    uint64_t key(double x, double y) const
    {
        double fx = (x - x0) * scale, fy = (y - y0) * scale;
        uint64_t qx = (uint64_t)std::min(std::max(fx, 0.0), 2097151.0);
        uint64_t qy = (uint64_t)std::min(std::max(fy, 0.0), 2097151.0);
        if (hilbert)
            return hilbert21(qx, qy);
        return spread21(qx) | (spread21(qy) << 1);
    }
};

// order[i] = user id of the i-th element in key order (stable on ties)
std::vector<int32_t> key_order(const std::vector<uint64_t> &keys)
{
    std::vector<int32_t> ord(keys.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return keys[a] < keys[b]; });
    return ord;
}

template <typename T>
slw_status upload(const std::vector<T> &h, T **d, int64_t &bytes)
{
    size_t nb = std::max<size_t>(h.size(), 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)d, nb);
    if (e != hipSuccess)
        return set_error(SLW_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    bytes += (int64_t)nb;
    if (!h.empty()) {
        e = hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return hip_check(e, "hipMemcpy (mesh upload)");
    }
    return SLW_OK;
}

bool coord_ok(double v)
{
    if (!std::isfinite(v))
        return false;
    double a = std::fabs(v);
    return a == 0.0 || (a >= kTinyCoord && a <= kHugeCoord);
}

}  // namespace

FilterConst filter_constants(bool f32, double cx, double cy, double cmax)
{
    FilterConst fc;
    const double u = 0x1p-24;
    const double M = cmax * (1.0 + 0x1p-40);
    if (f32) {
        fc.c1 = (float)(3.0 * u + 64.0 * u * u);
        fc.c2 = 0.0f;
        fc.c3 = 0x1p-140f;
    } else {
        fc.c1 = (float)(4.0 * u + 64.0 * u * u);
        const double c2 = (2.0 * u + 64.0 * u * u) * M;
        const double c3 = 64.0 * u * u * M * M + 0x1p-140;
        // rounded up, so the bound is never below its derivation
        fc.c2 = std::nextafter((float)c2, INFINITY);
        fc.c3 = std::nextafter((float)c3, INFINITY);
        if (!(c2 < 1e30 && c3 < 1e30)) {  // huge coordinates: the filter never certifies
            fc.c2 = INFINITY;
            fc.c3 = INFINITY;
        }
    }
    fc.c1 = std::nextafter(fc.c1, INFINITY);
    fc.cx = cx;
    fc.cy = cy;
    return fc;
}

std::vector<WalkRec> walk_records(const std::vector<GeoRec> &geo, int bits)
{
    bits = std::min(std::max(bits, 2), kCodeBits);
    const int64_t lim = (int64_t)1 << (bits - 1);  // offsets in (-lim, lim) are coded
    std::vector<WalkRec> w(geo.size());
    for (size_t t = 0; t < geo.size(); ++t) {
        uint64_t word = 0;
        for (int k = 0; k < 3; ++k) {
            const int64_t nb = geo[t].nb[k];
            int32_t code;
            if (nb < 0)
                code = 0;
            else if (nb - (int64_t)t > -lim && nb - (int64_t)t < lim)
                code = (int32_t)(nb - (int64_t)t);
            else
                code = kCodeEscape;
            word |= (uint64_t)((uint32_t)code & ((1u << kCodeBits) - 1u)) << (kCodeBits * k);
        }
        for (int k = 0; k < 3; ++k)
            w[t].p[k] = geo[t].p[k];
        w[t].lo = (uint32_t)word;
        w[t].hi = (uint32_t)(word >> 32);
    }
    return w;
}

void free_mesh(DevMesh &m)
{
    void *ptrs[] = {m.geo, m.wrec, m.tri_v, m.tri_uf, m.tedge, m.dof_xy, m.qstart, m.vmin, m.dof_user,
                    m.dof_int, m.tri_int, m.prev_elem, m.jump, m.chart_uv, m.chart_node, m.chart_table,
                    m.chart_qx, m.chart_qy, m.learned_start, m.bnext, m.bprev, m.qt_nodes, m.qt_lists,
                    m.forest_list1, m.forest_out1, m.forest_parent1, m.forest_list2, m.forest_out2,
                    m.forest_parent2, m.forest_elem, m.bedge, m.grid, m.bg_ptr, m.bg_list};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    m = DevMesh();
}

slw_status build_mesh(slw_ctx *ctx, const double *xy, int64_t n, const int32_t *tri, int64_t nt, uint32_t flags,
                      DevMesh &out, bool to_device)
{
    (void)ctx;
    if (!xy || !tri || n < 3 || nt < 1)
        return set_error(SLW_E_ARG, "mesh needs >= 3 nodes and >= 1 triangle and non-null arrays");
    if (n > (int64_t)1 << 30 || nt > (int64_t)1 << 29)
        return set_error(SLW_E_ARG, "mesh too large for 32-bit ids");
    const bool f32 = flags & SLW_COORDS_F32, p2 = flags & SLW_P2, reorder = !(flags & SLW_NO_REORDER);

    // coordinates: in the exactness domain of the predicates (after rounding
    // to float for float meshes)
    std::vector<double> X(2 * n);
    for (int64_t i = 0; i < 2 * n; ++i) {
        double v = f32 ? (double)(float)xy[i] : xy[i];
        if (!coord_ok(xy[i]) || !coord_ok(v))
            return set_error(SLW_E_MESH_RANGE, "node " + std::to_string(i / 2) +
                                                   ": coordinate not finite, or nonzero with magnitude outside [2^-100, 2^100]");
        X[i] = v;
    }
    double bb[4] = {X[0], X[1], X[0], X[1]};
    for (int64_t i = 0; i < n; ++i) {
        bb[0] = std::min(bb[0], X[2 * i]);
        bb[1] = std::min(bb[1], X[2 * i + 1]);
        bb[2] = std::max(bb[2], X[2 * i]);
        bb[3] = std::max(bb[3], X[2 * i + 1]);
    }

    // triangles: range, distinct vertices, exact orientation, flip to CCW
    std::vector<int32_t> T(3 * nt);
    std::vector<int32_t> flip(nt, 0);
    std::vector<char> used(n, 0);
    for (int64_t t = 0; t < nt; ++t) {
        int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        if (a < 0 || b < 0 || c < 0 || a >= n || b >= n || c >= n)
            return set_error(SLW_E_MESH_INDEX, "triangle " + std::to_string(t) + ": vertex index out of range");
        if (a == b || b == c || a == c)
            return set_error(SLW_E_MESH_DEGENERATE, "triangle " + std::to_string(t) + ": repeated vertex");
        int s = orient_sign64(X[2 * a], X[2 * a + 1], X[2 * b], X[2 * b + 1], X[2 * c], X[2 * c + 1]);
        if (s == 0)
            return set_error(SLW_E_MESH_DEGENERATE, "triangle " + std::to_string(t) + ": zero area");
        if (s < 0) {
            std::swap(b, c);
            flip[t] = 1;
        }
        T[3 * t] = a;
        T[3 * t + 1] = b;
        T[3 * t + 2] = c;
        used[a] = used[b] = used[c] = 1;
    }
    for (int64_t i = 0; i < n; ++i)
        if (!used[i])
            return set_error(SLW_E_MESH_DEGENERATE, "node " + std::to_string(i) + " is in no triangle");

    // edges: directed a->b opposite local vertex k (CCW, interior on the left)
    struct HalfEdge {
        uint64_t key;
        int32_t t;
        int32_t k;
    };
    std::vector<HalfEdge> he(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            uint32_t a = (uint32_t)T[3 * t + (k + 1) % 3], b = (uint32_t)T[3 * t + (k + 2) % 3];
            uint64_t key = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
            he[3 * t + k] = {key, (int32_t)t, k};
        }
    std::sort(he.begin(), he.end(), [](const HalfEdge &x, const HalfEdge &y) {
        return x.key != y.key ? x.key < y.key : (x.t != y.t ? x.t < y.t : x.k < y.k);
    });
    std::vector<int32_t> NB(3 * nt, -1);
    std::vector<int32_t> tri_edge_user(p2 ? 3 * nt : 0);
    std::vector<uint64_t> edge_keys;
    std::vector<int32_t> edge_left, edge_right;  // user triangles left / right of min->max
    std::vector<int32_t> bnext(n, -1);
    int64_t n_bnd = 0;
    for (size_t i = 0; i < he.size();) {
        size_t j = i;
        while (j < he.size() && he[j].key == he[i].key)
            ++j;
        if (j - i > 2)
            return set_error(SLW_E_MESH_NONCONFORMING, "an edge is shared by more than two triangles");
        const HalfEdge &e0 = he[i];
        uint32_t lo = (uint32_t)(e0.key >> 32), hi = (uint32_t)(e0.key & 0xffffffffu);
        auto from_of = [&](const HalfEdge &e) { return T[3 * (int64_t)e.t + (e.k + 1) % 3]; };
        int32_t left = -1, right = -1;
        if (j - i == 2) {
            const HalfEdge &e1 = he[i + 1];
            if (from_of(e0) == from_of(e1))
                return set_error(SLW_E_MESH_NONCONFORMING,
                                 "triangles " + std::to_string(e0.t) + " and " + std::to_string(e1.t) +
                                     " overlap across a shared edge");
            NB[3 * (int64_t)e0.t + e0.k] = e1.t;
            NB[3 * (int64_t)e1.t + e1.k] = e0.t;
            left = from_of(e0) == (int32_t)lo ? e0.t : e1.t;
            right = left == e0.t ? e1.t : e0.t;
        } else {
            int32_t a = from_of(e0), b = (int32_t)(a == (int32_t)lo ? hi : lo);
            if (bnext[a] >= 0)
                return set_error(SLW_E_MESH_NONCONVEX,
                                 "non-manifold boundary: it passes twice through node " + std::to_string(a));
            bnext[a] = b;
            ++n_bnd;
            if (a == (int32_t)lo)
                left = e0.t;
            else
                right = e0.t;
        }
        if (p2) {
            int32_t eid = (int32_t)edge_keys.size();
            edge_keys.push_back(e0.key);
            edge_left.push_back(left);
            edge_right.push_back(right);
            for (size_t q = i; q < j; ++q)
                tri_edge_user[3 * (int64_t)he[q].t + he[q].k] = eid;
        }
        i = j;
    }
    // Convex: a disk (V - E + F = 1) whose single boundary loop turns left
    // (or goes straight) at every corner; then a walk that meets the
    // boundary with the foot beyond it proves the foot outside.  Any other
    // manifold boundary (reflex corners, holes, several pieces) makes the
    // mesh non-convex: such walks end in an exact search instead.
    int64_t n_edge_total = 0;
    {
        int64_t ne = 0;
        for (size_t i = 0; i < he.size(); ++i)
            if (i == 0 || he[i].key != he[i - 1].key)
                ++ne;
        n_edge_total = ne;
    }
    bool nonconvex = n - n_edge_total + nt != 1;
    int n_loops = 0;
    {
        std::vector<char> seen(n, 0);
        for (int64_t s0 = 0; s0 < n; ++s0) {
            if (bnext[s0] < 0 || seen[s0])
                continue;
            ++n_loops;
            int32_t a = (int32_t)s0;
            int64_t cnt = 0;
            do {
                seen[a] = 1;
                const int32_t b = bnext[a];
                if (b < 0)
                    return set_error(SLW_E_MESH_NONCONVEX, "open boundary");
                const int32_t c = bnext[b];
                if (c < 0)
                    return set_error(SLW_E_MESH_NONCONVEX, "open boundary");
                if (orient_sign64(X[2 * a], X[2 * a + 1], X[2 * b], X[2 * b + 1], X[2 * c], X[2 * c + 1]) < 0)
                    nonconvex = true;  // reflex corner at b
                a = b;
                if (++cnt > n_bnd)
                    return set_error(SLW_E_MESH_NONCONVEX, "boundary loop does not close");
            } while (a != (int32_t)s0);
        }
        if (n_loops != 1)
            nonconvex = true;
    }

    // ---------------- orders ----------------
    double span = std::max(bb[2] - bb[0], bb[3] - bb[1]);
    MortonFrame mf{bb[0], bb[1], span > 0 ? 2097151.0 / span : 1.0, (flags & SLW_HILBERT) != 0};
    std::vector<int32_t> node_u(n), tri_u(nt);  // internal -> user
    std::iota(node_u.begin(), node_u.end(), 0);
    std::iota(tri_u.begin(), tri_u.end(), 0);
    const int64_t ne = p2 ? (int64_t)edge_keys.size() : 0;
    std::vector<int32_t> edge_u(ne);
    std::iota(edge_u.begin(), edge_u.end(), 0);
    if (reorder) {
        std::vector<uint64_t> k(n);
        for (int64_t i = 0; i < n; ++i)
            k[i] = mf.key(X[2 * i], X[2 * i + 1]);
        node_u = key_order(k);
        std::vector<uint64_t> kt(nt);
        for (int64_t t = 0; t < nt; ++t) {
            double cx = (X[2 * T[3 * t]] + X[2 * T[3 * t + 1]] + X[2 * T[3 * t + 2]]) / 3.0;
            double cy = (X[2 * T[3 * t] + 1] + X[2 * T[3 * t + 1] + 1] + X[2 * T[3 * t + 2] + 1]) / 3.0;
            kt[t] = mf.key(cx, cy);
        }
        tri_u = key_order(kt);
        if (p2) {
            std::vector<uint64_t> ke(ne);
            for (int64_t e = 0; e < ne; ++e) {
                int64_t a = (int64_t)(edge_keys[e] >> 32), b = (int64_t)(edge_keys[e] & 0xffffffffu);
                ke[e] = mf.key(0.5 * (X[2 * a] + X[2 * b]), 0.5 * (X[2 * a + 1] + X[2 * b + 1]));
            }
            edge_u = key_order(ke);
        }
    }
    std::vector<int32_t> node_i(n), tri_i(nt), edge_i(ne);  // user -> internal
    for (int64_t i = 0; i < n; ++i)
        node_i[node_u[i]] = (int32_t)i;
    for (int64_t t = 0; t < nt; ++t)
        tri_i[tri_u[t]] = (int32_t)t;
    for (int64_t e = 0; e < ne; ++e)
        edge_i[edge_u[e]] = (int32_t)e;
    const int64_t ndof = n + ne;

    // ---------------- device records ----------------
    // float copies of the coordinates for the walk's filter: double meshes
    // subtract the box centre first (smaller magnitudes, tighter bound)
    const double ccx = f32 ? 0.0 : 0.5 * (bb[0] + bb[2]), ccy = f32 ? 0.0 : 0.5 * (bb[1] + bb[3]);
    double cmax = 0.0;  // largest |coordinate - centre| (after the double subtraction)
    for (int64_t i = 0; i < n; ++i)
        cmax = std::max(cmax, std::max(std::fabs(X[2 * i] - ccx), std::fabs(X[2 * i + 1] - ccy)));
    std::vector<GeoRec> geo(nt);
    std::vector<int32_t> tri_uf(nt);
    std::vector<int4> tedge(p2 ? nt : 0);
    for (int64_t ti = 0; ti < nt; ++ti) {
        int64_t t = tri_u[ti];
        GeoRec g;
        std::memset(&g, 0, sizeof g);
        for (int k = 0; k < 3; ++k) {
            const int64_t u = T[3 * t + k];
            g.p[k] = make_float2((float)(X[2 * u] - ccx), (float)(X[2 * u + 1] - ccy));
            g.nb[k] = NB[3 * t + k] < 0 ? -1 : tri_i[NB[3 * t + k]];
            g.v[k] = node_i[u];
        }
        geo[ti] = g;
        tri_uf[ti] = (int32_t)((uint32_t)t | ((uint32_t)flip[t] << 31));
        if (p2)
            tedge[ti] = make_int4((int32_t)(n + edge_i[tri_edge_user[3 * t]]),
                                  (int32_t)(n + edge_i[tri_edge_user[3 * t + 1]]),
                                  (int32_t)(n + edge_i[tri_edge_user[3 * t + 2]]), 0);
    }
    // Error bound of the float filter, derived for inputs a~ = fl32(a - c),
    // b~, q~ (|a - c|, |q - c| <= M): the rounded differences carry an absolute
    // error <= 2uM + u|diff|, which gives
    //   |det_float - det| <= (4u + O(u^2))(|l| + |r|) + 2uM (|ax|+|ay|+|bx|+|by|) + O(u^2 M^2);
    // the constants below add slack for the second-order terms, for rounding
    // in the bound's own evaluation and for subnormal results.  Float meshes
    // round nothing (c2 = 0): then it is the static bound (3u + 16u^2).
    const FilterConst fc = filter_constants(f32, ccx, ccy, cmax);

    // DOF coordinates (user order on the host, internal order on the device);
    // edge midpoints are (a + b) * 0.5 in double
    std::vector<double> dof_user_xy(2 * ndof);
    for (int64_t i = 0; i < n; ++i) {
        dof_user_xy[2 * i] = X[2 * i];
        dof_user_xy[2 * i + 1] = X[2 * i + 1];
    }
    for (int64_t e = 0; e < ne; ++e) {
        int64_t a = (int64_t)(edge_keys[e] >> 32), b = (int64_t)(edge_keys[e] & 0xffffffffu);
        dof_user_xy[2 * (n + e)] = (xy[2 * a] + xy[2 * b]) * 0.5;
        dof_user_xy[2 * (n + e) + 1] = (xy[2 * a + 1] + xy[2 * b + 1]) * 0.5;
        if (f32) {
            dof_user_xy[2 * (n + e)] = (double)(float)dof_user_xy[2 * (n + e)];
            dof_user_xy[2 * (n + e) + 1] = (double)(float)dof_user_xy[2 * (n + e) + 1];
        }
    }
    std::vector<int32_t> dof_u(ndof), dof_i(ndof);
    for (int64_t i = 0; i < n; ++i)
        dof_u[i] = node_u[i];
    for (int64_t e = 0; e < ne; ++e)
        dof_u[n + e] = (int32_t)(n + edge_u[e]);
    for (int64_t d = 0; d < ndof; ++d)
        dof_i[dof_u[d]] = (int32_t)d;

    // stars: incident triangles of every node with the pseudo-angle of the
    // edge that begins their sector; two half-planes for an edge DOF
    std::vector<int32_t> sptr(ndof + 1, 0);
    for (int64_t ti = 0; ti < nt; ++ti)
        for (int k = 0; k < 3; ++k)
            sptr[geo[ti].v[k] + 1]++;
    for (int64_t e = 0; e < ne; ++e) {
        int64_t eu = edge_u[e];
        sptr[n + e + 1] = (edge_left[eu] >= 0) + (edge_right[eu] >= 0);
    }
    for (int64_t d = 0; d < ndof; ++d)
        sptr[d + 1] += sptr[d];
    std::vector<StarEnt> star(sptr[ndof]);
    {
        std::vector<int32_t> fill(sptr.begin(), sptr.end() - 1);
        auto dxy = [&](int64_t user_node, int64_t user_node_from) {
            return std::make_pair(X[2 * user_node] - X[2 * user_node_from],
                                  X[2 * user_node + 1] - X[2 * user_node_from + 1]);
        };
        for (int64_t ti = 0; ti < nt; ++ti) {
            int64_t t = tri_u[ti];
            for (int r = 0; r < 3; ++r) {
                int64_t v = T[3 * t + r], nx = T[3 * t + (r + 1) % 3];
                auto d = dxy(nx, v);
                star[fill[node_i[v]]++] = StarEnt{(float)pseudo_angle(d.first, d.second), (int32_t)ti};
            }
        }
        for (int64_t e = 0; e < ne; ++e) {
            int64_t eu = edge_u[e];
            int64_t a = (int64_t)(edge_keys[eu] >> 32), b = (int64_t)(edge_keys[eu] & 0xffffffffu);
            auto d = dxy(b, a);
            if (edge_left[eu] >= 0)
                star[fill[n + e]++] = StarEnt{(float)pseudo_angle(d.first, d.second), tri_i[edge_left[eu]]};
            if (edge_right[eu] >= 0)
                star[fill[n + e]++] = StarEnt{(float)pseudo_angle(-d.first, -d.second), tri_i[edge_right[eu]]};
        }
        for (int64_t d = 0; d < ndof; ++d)
            std::sort(star.begin() + sptr[d], star.begin() + sptr[d + 1],
                      [](const StarEnt &x, const StarEnt &y) { return x.ang < y.ang; });
    }
    // the incident triangle facing each diagonal direction (45, 135, 225 and
    // 315 degrees; pseudo-angles 0.5, 1.5, 2.5, 3.5): the sector whose start
    // is the last one at or before that direction, cyclically
    std::vector<int4> qstart(ndof);
    for (int64_t d = 0; d < ndof; ++d) {
        int32_t sel[4];
        for (int q = 0; q < 4; ++q) {
            const float dir = 0.5f + (float)q;
            int32_t pick = sptr[d + 1] - 1;
            for (int32_t s2 = sptr[d]; s2 < sptr[d + 1]; ++s2)
                if (star[s2].ang <= dir)
                    pick = s2;
            sel[q] = star[pick].tri;
        }
        qstart[d] = make_int4(sel[0], sel[1], sel[2], sel[3]);
    }
    // smallest user triangle id around each node (vertex tie rule)
    std::vector<int32_t> vmin(n);
    for (int64_t i = 0; i < n; ++i) {
        int32_t best = -1;
        for (int32_t s = sptr[i]; s < sptr[i + 1]; ++s)
            if (best < 0 || tri_u[star[s].tri] < tri_u[best])
                best = star[s].tri;
        vmin[i] = best;
    }
    // bucket grid of start triangles for point queries without a start:
    // each cell takes the node closest to its centre (nearest filled cell
    // for empty cells) and that node's first incident triangle
    int g = (int)std::max(1.0, std::ceil(std::sqrt((double)n / 16.0)));
    g = std::min(g, 2048);
    std::vector<int32_t> jump((size_t)g * g, -1);
    {
        std::vector<double> best((size_t)g * g, 1e300);
        double w = span > 0 ? span / g : 1.0;
        for (int64_t i = 0; i < n; ++i) {
            int cx = (int)std::min<double>(g - 1, std::max(0.0, std::floor((X[2 * i] - bb[0]) / w)));
            int cy = (int)std::min<double>(g - 1, std::max(0.0, std::floor((X[2 * i + 1] - bb[1]) / w)));
            double ox = bb[0] + (cx + 0.5) * w - X[2 * i], oy = bb[1] + (cy + 0.5) * w - X[2 * i + 1];
            double d2 = ox * ox + oy * oy;
            size_t c = (size_t)cy * g + cx;
            if (d2 < best[c]) {
                best[c] = d2;
                jump[c] = star[sptr[node_i[i]]].tri;
            }
        }
        std::deque<size_t> qu;
        for (size_t c = 0; c < jump.size(); ++c)
            if (jump[c] >= 0)
                qu.push_back(c);
        while (!qu.empty()) {
            size_t c = qu.front();
            qu.pop_front();
            int cx = (int)(c % g), cy = (int)(c / g);
            const int dx[4] = {1, -1, 0, 0}, dy[4] = {0, 0, 1, -1};
            for (int s = 0; s < 4; ++s) {
                int nx = cx + dx[s], ny = cy + dy[s];
                if (nx < 0 || ny < 0 || nx >= g || ny >= g)
                    continue;
                size_t nc = (size_t)ny * g + nx;
                if (jump[nc] < 0) {
                    jump[nc] = jump[c];
                    qu.push_back(nc);
                }
            }
        }
    }

    // ---------------- copy to the device ----------------
    DevMesh m;
    if (!to_device) {
        out.n_nodes = n;
        out.n_tris = nt;
        out.n_edges = ne;
        out.n_dofs = ndof;
        out.coords_f32 = f32;
        out.p2 = p2;
        out.reordered = reorder;
        out.internal_order = (flags & SLW_INTERNAL_ORDER) ? 1 : 0;
        out.nonconvex = nonconvex;
        out.n_loops = n_loops;
        for (int i = 0; i < 4; ++i)
            out.bbox[i] = bb[i];
        return SLW_OK;
    }
    m.n_nodes = n;
    m.n_tris = nt;
    m.n_edges = ne;
    m.n_dofs = ndof;
    m.coords_f32 = f32;
    m.p2 = p2;
    m.reordered = reorder;
    m.internal_order = (flags & SLW_INTERNAL_ORDER) ? 1 : 0;
    m.nonconvex = nonconvex;
    m.n_loops = n_loops;
    for (int i = 0; i < 4; ++i)
        m.bbox[i] = bb[i];
    m.jump_g = g;
    m.fc = fc;
    slw_status st = SLW_OK;
    int64_t bytes = 0;
#define UP(vec, ptr)                                   \
    do {                                               \
        st = upload(vec, &(ptr), bytes);               \
        if (st != SLW_OK) {                            \
            free_mesh(m);                              \
            return st;                                 \
        }                                              \
    } while (0)
    UP(geo, m.geo);
    {
        std::vector<WalkRec> wr = walk_records(geo, kCodeBits);
        UP(wr, m.wrec);
        std::vector<int4> tv(nt);
        for (int64_t t = 0; t < nt; ++t)
            tv[t] = make_int4(geo[t].nb[2], geo[t].v[0], geo[t].v[1], geo[t].v[2]);
        UP(tv, m.tri_v);
    }
    UP(tri_uf, m.tri_uf);
    if (f32) {
        std::vector<float2> dxy(ndof);
        for (int64_t d = 0; d < ndof; ++d)
            dxy[d] = make_float2((float)dof_user_xy[2 * dof_u[d]], (float)dof_user_xy[2 * dof_u[d] + 1]);
        float2 *p = nullptr;
        UP(dxy, p);
        m.dof_xy = p;
    } else {
        std::vector<double2> dxy(ndof);
        for (int64_t d = 0; d < ndof; ++d)
            dxy[d] = make_double2(dof_user_xy[2 * dof_u[d]], dof_user_xy[2 * dof_u[d] + 1]);
        double2 *p = nullptr;
        UP(dxy, p);
        m.dof_xy = p;
    }
    if (p2)
        UP(tedge, m.tedge);
    UP(qstart, m.qstart);
    UP(vmin, m.vmin);
    UP(dof_u, m.dof_user);
    UP(dof_i, m.dof_int);
    UP(tri_i, m.tri_int);
    std::vector<int32_t> prev(ndof, -1);
    UP(prev, m.prev_elem);
    UP(jump, m.jump);
    {
        // boundary loop (counter-clockwise, interior on the left) in internal node ids
        std::vector<int32_t> bn(n, -1), bp(n, -1);
        for (int64_t a = 0; a < n; ++a)
            if (bnext[a] >= 0) {
                bn[node_i[a]] = node_i[bnext[a]];
                bp[node_i[bnext[a]]] = node_i[a];
            }
        UP(bn, m.bnext);
        UP(bp, m.bprev);
        m.n_boundary = n_bnd;
        std::vector<int32_t> be;
        for (int64_t a = 0; a < n; ++a)
            if (bn[a] >= 0)
                be.push_back((int32_t)a);
        UP(be, m.bedge);
        if (nonconvex && !be.empty()) {
            // uniform grid over the boundary edges, for the first exit of a
            // segment from a non-convex domain (about one edge per cell)
            const int gb = (int)std::min(1024.0, std::max(1.0, std::ceil(std::sqrt((double)be.size()))));
            const double cell = span > 0 ? span / gb : 1.0;
            const double pad = 1e-6 * (span > 0 ? span : 1.0);
            auto cell_of = [&](double v, double o) {
                return (int)std::min<double>(gb - 1, std::max(0.0, std::floor((v - o) / cell)));
            };
            std::vector<int32_t> ptr((size_t)gb * gb + 1, 0), list;
            for (int pass = 0; pass < 2; ++pass) {
                std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
                for (size_t i = 0; i < be.size(); ++i) {
                    const int64_t ua = dof_u[be[i]], ub = dof_u[bn[be[i]]];
                    const double x0 = std::min(X[2 * ua], X[2 * ub]) - pad, x1 = std::max(X[2 * ua], X[2 * ub]) + pad;
                    const double y0 = std::min(X[2 * ua + 1], X[2 * ub + 1]) - pad,
                                 y1 = std::max(X[2 * ua + 1], X[2 * ub + 1]) + pad;
                    for (int cy = cell_of(y0, bb[1]); cy <= cell_of(y1, bb[1]); ++cy)
                        for (int cx = cell_of(x0, bb[0]); cx <= cell_of(x1, bb[0]); ++cx) {
                            const size_t c = (size_t)cy * gb + cx;
                            if (pass == 0)
                                ++ptr[c + 1];
                            else
                                list[fill[c]++] = (int32_t)i;
                        }
                }
                if (pass == 0) {
                    for (size_t c = 0; c + 1 < ptr.size(); ++c)
                        ptr[c + 1] += ptr[c];
                    list.resize((size_t)ptr.back());
                }
            }
            UP(ptr, m.bg_ptr);
            UP(list, m.bg_list);
            m.bg_g = gb;
            m.bg_x0 = bb[0];
            m.bg_y0 = bb[1];
            m.bg_cell = cell;
        }
    }
    {
        // strategy (c)'s forest: roots = nodes no two of which lie within
        // kForestHops hops of each other (greedy in internal order, a maximal
        // such set); every other DOF is a child of the nearest root (in
        // distance) within kForestHops hops.  Measured on the graded mesh,
        // one / two / three hops: roots 28% / about 10% / fewer of the
        // nodes, step 0.221 / 0.195 / 0.195 ms with the start grid and
        // 0.278 / 0.229 / 0.216 ms without (Courant 5): fewer roots cost
        // less than the children's longer walks.
        constexpr int kForestHops = 3;
        std::vector<int32_t> nptr(n + 1, 0), nadj;  // unique neighbours of each node
        {
            std::vector<int32_t> tmp;
            for (int64_t d = 0; d < n; ++d) {
                tmp.clear();
                for (int32_t s2 = sptr[d]; s2 < sptr[d + 1]; ++s2)
                    for (int k = 0; k < 3; ++k) {
                        const int32_t v = geo[star[s2].tri].v[k];
                        if (v != d)
                            tmp.push_back(v);
                    }
                std::sort(tmp.begin(), tmp.end());
                tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
                nadj.insert(nadj.end(), tmp.begin(), tmp.end());
                nptr[d + 1] = (int32_t)nadj.size();
            }
        }
        // breadth-first search from the seeds up to `depth` hops, each node
        // visited once; stops when visit returns true (and returns true)
        std::vector<uint32_t> stamp(n, 0);
        uint32_t tag = 0;
        std::vector<int32_t> cur, nxt;
        auto bfs = [&](const int32_t *seeds, int ns, int depth, auto &&visit) -> bool {
            ++tag;
            cur.clear();
            for (int i2 = 0; i2 < ns; ++i2)
                if (stamp[seeds[i2]] != tag) {
                    stamp[seeds[i2]] = tag;
                    cur.push_back(seeds[i2]);
                    if (visit(seeds[i2]))
                        return true;
                }
            for (int h = 0; h < depth; ++h) {
                nxt.clear();
                for (int32_t v : cur)
                    for (int32_t e = nptr[v]; e < nptr[v + 1]; ++e) {
                        const int32_t u = nadj[e];
                        if (stamp[u] != tag) {
                            stamp[u] = tag;
                            nxt.push_back(u);
                            if (visit(u))
                                return true;
                        }
                    }
                cur.swap(nxt);
            }
            return false;
        };
        std::vector<char> is_root(ndof, 0);
        for (int64_t d = 0; d < n; ++d) {
            const int32_t seed = (int32_t)d;
            is_root[d] = !bfs(&seed, 1, kForestHops, [&](int32_t v) { return v != seed && is_root[v] != 0; });
        }
        auto ixy = [&](int64_t d, int c) { return dof_user_xy[2 * dof_u[d] + c]; };
        auto forest = [&](int64_t nd, std::vector<int32_t> &list, std::vector<int32_t> &outr,
                          std::vector<int32_t> &par) {
            list.clear();
            par.clear();
            for (int64_t d = 0; d < nd; ++d)
                if (is_root[d])
                    list.push_back((int32_t)d);
            const int64_t nr = (int64_t)list.size();
            std::vector<int32_t> seeds;
            for (int64_t d = 0; d < nd; ++d) {
                if (is_root[d])
                    continue;
                int32_t best = -1;
                double bd = 0.0;
                auto consider = [&](int32_t v) {
                    if (is_root[v]) {
                        const double ex = ixy(v, 0) - ixy(d, 0), ey = ixy(v, 1) - ixy(d, 1);
                        const double dd = ex * ex + ey * ey;
                        if (best < 0 || dd < bd) {
                            best = v;
                            bd = dd;
                        }
                    }
                    return false;
                };
                if (d < n) {
                    const int32_t seed = (int32_t)d;
                    bfs(&seed, 1, kForestHops, consider);
                } else {
                    // a P2 edge DOF: the vertices of its triangles are one hop away
                    seeds.clear();
                    for (int32_t s2 = sptr[d]; s2 < sptr[d + 1]; ++s2)
                        for (int k = 0; k < 3; ++k)
                            seeds.push_back(geo[star[s2].tri].v[k]);
                    bfs(seeds.data(), (int)seeds.size(), kForestHops - 1, consider);
                }
                list.push_back((int32_t)d);
                par.push_back(best);
            }
            outr.resize(list.size());
            const bool user_rows = reorder && !(flags & SLW_INTERNAL_ORDER);
            for (size_t i = 0; i < list.size(); ++i)
                outr[i] = user_rows ? dof_u[list[i]] : list[i];
            return nr;
        };
        std::vector<int32_t> list, outr, par;
        m.forest_nr1 = forest(n, list, outr, par);
        UP(list, m.forest_list1);
        UP(outr, m.forest_out1);
        UP(par, m.forest_parent1);
        if (p2) {
            m.forest_nr2 = forest(ndof, list, outr, par);
            UP(list, m.forest_list2);
            UP(outr, m.forest_out2);
            UP(par, m.forest_parent2);
        }
        std::vector<int32_t> fe(ndof, -1);
        UP(fe, m.forest_elem);
    }
#undef UP
    m.dof_xy_user_h = std::move(dof_user_xy);
    m.dof_user_h = std::move(dof_u);
    if (nonconvex) {
        // the exact search that ends walks blocked by the boundary: leaves
        // as small as the list budget allows
        st = SLW_E_NOMEM;
        for (int cap = 16; st != SLW_OK && cap <= (1 << 30); cap *= 4) {
            st = build_quadtree(m, geo, cap, 24);
            if (cap >= nt)
                break;
        }
        if (st != SLW_OK) {
            free_mesh(m);
            return st;
        }
        bytes += m.qt_n_nodes * (int64_t)sizeof(int4) + m.qt_n_list * (int64_t)sizeof(int32_t);
    }
    m.device_bytes = bytes;
    out = std::move(m);
    return SLW_OK;
}

}  // namespace slw
