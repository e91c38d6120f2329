// Quadtree over the triangles of a mesh: the non-walking point location of
// Section 2.1, kept as a comparator for the walks.  Built on the host from
// the device records; queried by k_qt_locate (slw_kernels.hip).
//
// The root is the square [x0, x0 + side] x [y0, y0 + side] that covers the
// mesh's bounding box.  A node splits at its centre while it lists more than
// leaf_cap triangles, is shallower than max_depth, and the split separates
// something (no child keeps every triangle); a triangle is listed
// in every child that its closed bounding box touches, so a point's closed
// containers are all listed in the leaf the point descends to.  The split
// coordinates are computed here exactly as the query computes them
// (x0 + side/2 + side/4 ..., halving in double), so host and device agree on
// which child a point on a split line belongs to (the upper / right one).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <vector>

#include "slw_internal.h"

using namespace slw;

namespace {

struct Pending {
    int32_t node;
    int depth;
    double bx, by, s;
    std::vector<int32_t> tris;
};

}  // namespace

namespace slw {

slw_status build_quadtree(DevMesh &m, const std::vector<GeoRec> &geo, int leaf_cap, int max_depth)
{
    const int64_t nt = m.n_tris;
    // closed bounding boxes on the exact coordinates (float meshes: the floats)
    std::vector<double> box(4 * (size_t)nt);
    for (int64_t t = 0; t < nt; ++t) {
        double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
        for (int k = 0; k < 3; ++k) {
            const int64_t u = m.dof_user_h[geo[t].v[k]];
            double x = m.dof_xy_user_h[2 * u], y = m.dof_xy_user_h[2 * u + 1];
            if (m.coords_f32) {
                x = (double)(float)x;
                y = (double)(float)y;
            }
            x0 = std::min(x0, x);
            x1 = std::max(x1, x);
            y0 = std::min(y0, y);
            y1 = std::max(y1, y);
        }
        box[4 * t] = x0;
        box[4 * t + 1] = y0;
        box[4 * t + 2] = x1;
        box[4 * t + 3] = y1;
    }
    const double ox = m.bbox[0], oy = m.bbox[1];
    const double side = std::max(m.bbox[2] - m.bbox[0], m.bbox[3] - m.bbox[1]);
    std::vector<int4> nodes(1);
    std::vector<int32_t> lists;
    lists.reserve((size_t)nt * 2);
    std::deque<Pending> work;
    {
        Pending root{0, 0, ox, oy, side, std::vector<int32_t>(nt)};
        for (int64_t t = 0; t < nt; ++t)
            root.tris[t] = (int32_t)t;
        work.push_back(std::move(root));
    }
    int depth_max = 0;
    // list entries allowed in all (a triangle appears in every leaf its box
    // touches): beyond this the build fails rather than exhaust memory
    const int64_t budget = 16 * nt + (1 << 20);
    int64_t listed = nt;
    while (!work.empty()) {
        Pending p = std::move(work.front());
        work.pop_front();
        bool leaf = (int64_t)p.tris.size() <= leaf_cap || p.depth >= max_depth;
        Pending ch[4];
        const double h = p.s * 0.5;
        if (!leaf) {
            const double sx = p.bx + h, sy = p.by + h;  // as the query computes them
            for (int q = 0; q < 4; ++q) {
                const int right = q & 1, top = q >> 1;
                ch[q] = Pending{0, p.depth + 1, right ? p.bx + h : p.bx, top ? p.by + h : p.by, h, {}};
            }
            for (int32_t t : p.tris) {
                const double *b = &box[4 * (size_t)t];
                const bool l = b[0] <= sx, r = b[2] >= sx, lo = b[1] <= sy, hi = b[3] >= sy;
                if (l && lo)
                    ch[0].tris.push_back(t);
                if (r && lo)
                    ch[1].tris.push_back(t);
                if (l && hi)
                    ch[2].tris.push_back(t);
                if (r && hi)
                    ch[3].tris.push_back(t);
            }
            // a split in which some child keeps every triangle makes no
            // progress there (overlapping boxes): stop at this node
            size_t most = 0, added = 0;
            for (int q = 0; q < 4; ++q) {
                most = std::max(most, ch[q].tris.size());
                added += ch[q].tris.size();
            }
            if (most == p.tris.size())
                leaf = true;
            else if ((listed += (int64_t)added - (int64_t)p.tris.size()) > budget)
                return set_error(SLW_E_NOMEM, "quadtree: more than 16 list entries per triangle "
                                              "(raise leaf_cap or lower max_depth)");
        }
        if (leaf) {
            if (lists.size() + p.tris.size() > (size_t)INT32_MAX)
                return set_error(SLW_E_NOMEM, "quadtree: lists exceed 2^31 entries");
            nodes[p.node] = make_int4(-1, (int32_t)lists.size(), (int32_t)p.tris.size(), 0);
            lists.insert(lists.end(), p.tris.begin(), p.tris.end());
            depth_max = std::max(depth_max, p.depth);
            continue;
        }
        const int32_t c0 = (int32_t)nodes.size();
        nodes.resize(nodes.size() + 4);
        nodes[p.node] = make_int4(c0, 0, 0, 0);
        std::vector<int32_t>().swap(p.tris);
        for (int q = 0; q < 4; ++q) {
            ch[q].node = c0 + q;
            work.push_back(std::move(ch[q]));
        }
    }
    if (lists.empty())
        lists.push_back(0);
    int4 *nd = nullptr;
    int32_t *ls = nullptr;
    if (hipMalloc((void **)&nd, nodes.size() * sizeof(int4)) != hipSuccess ||
        hipMalloc((void **)&ls, lists.size() * sizeof(int32_t)) != hipSuccess) {
        if (nd)
            (void)hipFree(nd);
        return set_error(SLW_E_NOMEM, "quadtree: device arrays");
    }
    if (hipMemcpy(nd, nodes.data(), nodes.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ls, lists.data(), lists.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(nd);
        (void)hipFree(ls);
        return set_error(SLW_E_HIP, "quadtree: copy to the device");
    }
    if (m.qt_nodes)
        (void)hipFree(m.qt_nodes);
    if (m.qt_lists)
        (void)hipFree(m.qt_lists);
    m.qt_nodes = nd;
    m.qt_lists = ls;
    m.qt_box[0] = ox;
    m.qt_box[1] = oy;
    m.qt_box[2] = side;
    m.qt_depth = depth_max;
    m.qt_n_nodes = (int64_t)nodes.size();
    m.qt_n_list = (int64_t)lists.size();
    return SLW_OK;
}

}  // namespace slw

extern "C" {

slw_status slw_quadtree_build(slw_mesh *mesh, int leaf_cap, int max_depth)
{
    if (!mesh || leaf_cap < 1 || max_depth < 0 || max_depth > 30)
        return set_error(SLW_E_ARG, "slw_quadtree_build: leaf_cap >= 1 and max_depth in [0, 30]");
    DevMesh &m = mesh->m;
    DeviceGuard gd(mesh->ctx->device);
    const int64_t nt = m.n_tris;
    std::vector<GeoRec> geo(nt);
    slw_status st = hip_check(hipStreamSynchronize(mesh->ctx->stream), "hipStreamSynchronize");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(geo.data(), m.geo, nt * sizeof(GeoRec), hipMemcpyDeviceToHost), "copy records");
    if (st != SLW_OK)
        return st;
    return build_quadtree(m, geo, leaf_cap, max_depth);
}

slw_status slw_quadtree_info(const slw_mesh *mesh, int64_t *n_nodes_h, int64_t *n_list_h, int *depth_h)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    if (n_nodes_h)
        *n_nodes_h = mesh->m.qt_n_nodes;
    if (n_list_h)
        *n_list_h = mesh->m.qt_n_list;
    if (depth_h)
        *depth_h = mesh->m.qt_depth;
    return SLW_OK;
}

}  // extern "C"
