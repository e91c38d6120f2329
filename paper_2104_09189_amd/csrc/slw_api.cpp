// C-ABI entry points: argument checks, context/stream handling, statistics.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>

#include "slw_internal.h"
#include "slw_predicates.h"

namespace {
thread_local std::string g_last_error;
}

namespace slw {

slw_status set_error(slw_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

slw_status hip_check(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return SLW_OK;
    return set_error(SLW_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

slw_status ensure_work(slw_ctx *ctx, size_t bytes)
{
    if (ctx->work_bytes >= bytes)
        return SLW_OK;
    if (ctx->work) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess)
            return hip_check(e, "hipStreamSynchronize");
        (void)hipFree(ctx->work);
        ctx->work = nullptr;
        ctx->work_bytes = 0;
    }
    hipError_t e = hipMalloc(&ctx->work, bytes);
    if (e != hipSuccess)
        return set_error(SLW_E_NOMEM, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
    ctx->work_bytes = bytes;
    return SLW_OK;
}

}  // namespace slw

using namespace slw;

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0)
            (void)hipSetDevice(prev);
    }
};

slw_status begin_stats(slw_ctx *ctx, slw_stats *stats_h)
{
    if (!stats_h)
        return SLW_OK;
    // a fill kernel rather than a memset node keeps the call graph-capturable
    return hip_check(launch_zero_stats(ctx->stream, ctx->stats), "zero stats");
}

slw_status end_stats(slw_ctx *ctx, slw_stats *stats_h)
{
    if (!stats_h)
        return SLW_OK;
    DevStats h;
    slw_status st = hip_check(hipMemcpyAsync(&h, ctx->stats, sizeof h, hipMemcpyDeviceToHost, ctx->stream),
                              "hipMemcpyAsync(stats)");
    if (st != SLW_OK)
        return st;
    st = hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (st != SLW_OK)
        return st;
    std::memset(stats_h, 0, sizeof *stats_h);
    stats_h->feet = (int64_t)h.feet;
    stats_h->outside = (int64_t)h.outside;
    stats_h->walk_steps = (int64_t)h.walk_steps;
    stats_h->max_steps = (int64_t)h.max_steps;
    stats_h->exact_tests = (int64_t)h.exact_tests;
    stats_h->fp64_tests = (int64_t)h.fp64_tests;
    stats_h->fallback_walks = (int64_t)h.fallback_walks;
    stats_h->edge_ties = (int64_t)h.edge_ties;
    stats_h->vertex_ties = (int64_t)h.vertex_ties;
    if (h.hard_fail)
        return set_error(SLW_E_WALK, std::to_string(h.hard_fail) + " walks exceeded the hard step limit");
    return SLW_OK;
}

bool field_ok(const slw_field *f) { return f && f->kind >= 0 && f->kind <= 4; }

FieldDev to_dev(const slw_field *f)
{
    FieldDev d{};
    if (f) {
        d.kind = f->kind;
        for (int i = 0; i < 8; ++i)
            d.p[i] = f->p[i];
    }
    return d;
}

}  // namespace

extern "C" {

const char *slw_status_string(slw_status s)
{
    switch (s) {
    case SLW_OK: return "ok";
    case SLW_E_ARG: return "invalid argument";
    case SLW_E_MESH_INDEX: return "mesh: vertex index out of range";
    case SLW_E_MESH_DEGENERATE: return "mesh: degenerate triangle or unused node";
    case SLW_E_MESH_NONCONFORMING: return "mesh: non-conforming";
    case SLW_E_MESH_NONCONVEX: return "mesh: domain not a convex disk";
    case SLW_E_MESH_RANGE: return "mesh: coordinate outside the exactness domain";
    case SLW_E_HIP: return "HIP runtime error";
    case SLW_E_NOMEM: return "out of memory";
    case SLW_E_UNSUPPORTED: return "unsupported";
    case SLW_E_WALK: return "walk exceeded the hard step limit";
    }
    return "unknown status";
}

const char *slw_last_error(void) { return g_last_error.c_str(); }

slw_status slw_ctx_create(int device, void *hip_stream, slw_ctx **out)
{
    if (!out)
        return set_error(SLW_E_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess)
        return hip_check(e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return set_error(SLW_E_ARG, "device index out of range");
    DeviceGuard g(device);
    slw_ctx *c = new (std::nothrow) slw_ctx();
    if (!c)
        return set_error(SLW_E_NOMEM, "context");
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    e = hipMalloc((void **)&c->stats, sizeof(DevStats));
    if (e != hipSuccess) {
        delete c;
        return set_error(SLW_E_NOMEM, std::string("hipMalloc(stats): ") + hipGetErrorString(e));
    }
    *out = c;
    return SLW_OK;
}

slw_status slw_ctx_set_stream(slw_ctx *ctx, void *hip_stream)
{
    if (!ctx)
        return set_error(SLW_E_ARG, "ctx is NULL");
    ctx->stream = (hipStream_t)hip_stream;
    return SLW_OK;
}

void slw_ctx_destroy(slw_ctx *ctx)
{
    if (!ctx)
        return;
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->stats)
        (void)hipFree(ctx->stats);
    if (ctx->work)
        (void)hipFree(ctx->work);
    delete ctx;
}

slw_status slw_mesh_upload(slw_ctx *ctx, const double *xy_h, int64_t n_nodes, const int32_t *tri_h, int64_t n_tris,
                           uint32_t flags, slw_mesh **out)
{
    if (!ctx || !out)
        return set_error(SLW_E_ARG, "ctx or out is NULL");
    *out = nullptr;
    if (flags & ~(uint32_t)(SLW_COORDS_F32 | SLW_P2 | SLW_NO_REORDER | SLW_INTERNAL_ORDER))
        return set_error(SLW_E_ARG, "unknown mesh flag");
    DeviceGuard g(ctx->device);
    slw_mesh *m = new (std::nothrow) slw_mesh();
    if (!m)
        return set_error(SLW_E_NOMEM, "mesh handle");
    m->ctx = ctx;
    slw_status st = build_mesh(ctx, xy_h, n_nodes, tri_h, n_tris, flags, m->m, true);
    if (st != SLW_OK) {
        delete m;
        return st;
    }
    *out = m;
    return SLW_OK;
}

slw_status slw_mesh_check(const double *xy_h, int64_t n_nodes, const int32_t *tri_h, int64_t n_tris,
                          uint32_t flags, slw_mesh_info *info_h)
{
    if (flags & ~(uint32_t)(SLW_COORDS_F32 | SLW_P2 | SLW_NO_REORDER | SLW_INTERNAL_ORDER))
        return set_error(SLW_E_ARG, "unknown mesh flag");
    DevMesh m;
    slw_status st = build_mesh(nullptr, xy_h, n_nodes, tri_h, n_tris, flags, m, false);
    if (st != SLW_OK)
        return st;
    if (info_h) {
        std::memset(info_h, 0, sizeof *info_h);
        info_h->n_nodes = m.n_nodes;
        info_h->n_tris = m.n_tris;
        info_h->n_edges = m.n_edges;
        info_h->n_dofs = m.n_dofs;
        info_h->coords_f32 = m.coords_f32;
        info_h->p2 = m.p2;
        info_h->reordered = m.reordered;
        info_h->internal_order = m.internal_order;
        for (int i = 0; i < 4; ++i)
            info_h->bbox[i] = m.bbox[i];
    }
    return SLW_OK;
}

slw_status slw_mesh_free(slw_mesh *mesh)
{
    if (!mesh)
        return SLW_OK;
    DeviceGuard g(mesh->ctx->device);
    (void)hipStreamSynchronize(mesh->ctx->stream);
    free_mesh(mesh->m);
    delete mesh;
    return SLW_OK;
}

slw_status slw_mesh_get_info(const slw_mesh *mesh, slw_mesh_info *out_h)
{
    if (!mesh || !out_h)
        return set_error(SLW_E_ARG, "mesh or out is NULL");
    const DevMesh &m = mesh->m;
    std::memset(out_h, 0, sizeof *out_h);
    out_h->n_nodes = m.n_nodes;
    out_h->n_tris = m.n_tris;
    out_h->n_edges = m.n_edges;
    out_h->n_dofs = m.n_dofs;
    out_h->device_bytes = m.device_bytes;
    out_h->coords_f32 = m.coords_f32;
    out_h->p2 = m.p2;
    out_h->reordered = m.reordered;
    out_h->internal_order = m.internal_order;
    for (int i = 0; i < 4; ++i)
        out_h->bbox[i] = m.bbox[i];
    return SLW_OK;
}

slw_status slw_mesh_dof_coords(const slw_mesh *mesh, double *xy_h)
{
    if (!mesh || !xy_h)
        return set_error(SLW_E_ARG, "mesh or xy_h is NULL");
    const DevMesh &m = mesh->m;
    for (int64_t d = 0; d < m.n_dofs; ++d) {
        const int64_t src = m.internal_order ? m.dof_user_h[d] : d;
        xy_h[2 * d] = m.dof_xy_user_h[2 * src];
        xy_h[2 * d + 1] = m.dof_xy_user_h[2 * src + 1];
    }
    return SLW_OK;
}

slw_status slw_mesh_dof_order(const slw_mesh *mesh, int32_t *user_of_internal_h)
{
    if (!mesh || !user_of_internal_h)
        return set_error(SLW_E_ARG, "mesh or output is NULL");
    std::memcpy(user_of_internal_h, mesh->m.dof_user_h.data(), mesh->m.n_dofs * sizeof(int32_t));
    return SLW_OK;
}

slw_status slw_mesh_set_walk_limits(slw_mesh *mesh, int32_t step_cap, int32_t hard_limit)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    if (step_cap > 0)
        mesh->m.step_cap = step_cap;
    if (hard_limit > 0)
        mesh->m.hard_limit = hard_limit;
    return SLW_OK;
}

slw_status slw_locate(slw_mesh *mesh, const void *q, int64_t m, const int32_t *start, int32_t *elem, void *bary,
                      int32_t *steps)
{
    if (!mesh || m < 0 || (m > 0 && (!q || !elem)))
        return set_error(SLW_E_ARG, "slw_locate: null pointer or negative size");
    if (m > ((int64_t)1 << 31) - 1)
        return set_error(SLW_E_ARG, "slw_locate: at most 2^31-1 points per call");
    slw_ctx *ctx = mesh->ctx;
    DeviceGuard g(ctx->device);
    return hip_check(launch_locate(mesh->m, ctx->stream, q, m, start, elem, bary, steps, nullptr), "slw_locate");
}

slw_status slw_locate_feet(slw_mesh *mesh, const slw_field *field, double t_np1, double dt, int scheme,
                           int start_mode, const int32_t *start, uint32_t flags, void *feet, int32_t *elem,
                           void *bary, int32_t *steps, slw_stats *stats_h)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    const bool feet_in = flags & SLW_FEET_IN;
    if (flags & ~(uint32_t)SLW_FEET_IN)
        return set_error(SLW_E_ARG, "unknown flag");
    if (feet_in ? !feet : !field_ok(field))
        return set_error(SLW_E_ARG, "feet (SLW_FEET_IN) or a valid field is required");
    if (scheme != SLW_EULER && scheme != SLW_RK2)
        return set_error(SLW_E_ARG, "unknown scheme");
    if (start_mode < SLW_START_STEERED || start_mode > SLW_START_FIXED)
        return set_error(SLW_E_ARG, "unknown start mode");
    if ((start_mode == SLW_START_GIVEN || start_mode == SLW_START_FIXED) && !start)
        return set_error(SLW_E_ARG, "start array required for this start mode");
    slw_ctx *ctx = mesh->ctx;
    DeviceGuard g(ctx->device);
    slw_status st = begin_stats(ctx, stats_h);
    if (st != SLW_OK)
        return st;
    FieldDev fd = to_dev(field);
    st = hip_check(launch_locate_feet(mesh->m, ctx->stream, feet_in ? nullptr : &fd, t_np1, dt, scheme, start_mode,
                                      start, feet_in, feet, elem, bary, steps, stats_h ? ctx->stats : nullptr),
                   "slw_locate_feet");
    if (st != SLW_OK)
        return st;
    return end_stats(ctx, stats_h);
}

slw_status slw_interpolate(slw_mesh *mesh, int order, const int32_t *elem, const void *bary, int64_t m,
                           const void *v_in, int vdtype, int k, void *v_out, double outside_value)
{
    if (!mesh || m < 0 || k < 1 || (m > 0 && (!elem || !bary || !v_in || !v_out)))
        return set_error(SLW_E_ARG, "slw_interpolate: null pointer or bad size");
    if (order != 1 && order != 2)
        return set_error(SLW_E_ARG, "order must be 1 or 2");
    if (order == 2 && !mesh->m.p2)
        return set_error(SLW_E_UNSUPPORTED, "P2 needs a mesh uploaded with SLW_P2");
    if (vdtype != SLW_F64 && vdtype != SLW_F32)
        return set_error(SLW_E_ARG, "unknown vdtype");
    slw_ctx *ctx = mesh->ctx;
    DeviceGuard g(ctx->device);
    return hip_check(launch_interp(mesh->m, ctx->stream, order, elem, bary, m, v_in, vdtype, k, v_out,
                                   outside_value, !mesh->m.internal_order),
                     "slw_interpolate");
}

slw_status slw_step(slw_mesh *mesh, const slw_field *field, double t_n, double dt, int scheme, int order,
                    int start_mode, const int32_t *start, const void *v_in, int vdtype, int k, void *v_out,
                    double outside_value, slw_stats *stats_h)
{
    if (!mesh || !field_ok(field) || !v_in || !v_out || k < 1)
        return set_error(SLW_E_ARG, "slw_step: null pointer, bad field or k < 1");
    if (order != 1 && order != 2)
        return set_error(SLW_E_ARG, "order must be 1 or 2");
    if (order == 2 && !mesh->m.p2)
        return set_error(SLW_E_UNSUPPORTED, "P2 needs a mesh uploaded with SLW_P2");
    if (scheme != SLW_EULER && scheme != SLW_RK2)
        return set_error(SLW_E_ARG, "unknown scheme");
    if (vdtype != SLW_F64 && vdtype != SLW_F32)
        return set_error(SLW_E_ARG, "unknown vdtype");
    if (start_mode < SLW_START_STEERED || start_mode > SLW_START_FIXED)
        return set_error(SLW_E_ARG, "unknown start mode");
    if ((start_mode == SLW_START_GIVEN || start_mode == SLW_START_FIXED) && !start)
        return set_error(SLW_E_ARG, "start array required for this start mode");
    const DevMesh &m = mesh->m;
    // P1 uses the vertex DOFs only (the first n_nodes of either order)
    const int64_t rows = order == 1 ? m.n_nodes : m.n_dofs;
    const size_t vsz = vdtype == SLW_F64 ? 8 : 4;
    const size_t bytes = (size_t)rows * (size_t)k * vsz;
    const char *vi = (const char *)v_in, *vo = (const char *)v_out;
    if (vi < vo + bytes && vo < vi + bytes)
        return set_error(SLW_E_ARG, "v_in and v_out overlap");
    slw_ctx *ctx = mesh->ctx;
    DeviceGuard g(ctx->device);
    slw_status st = begin_stats(ctx, stats_h);
    if (st != SLW_OK)
        return st;
    const void *vin_int = v_in;
    const int32_t *out_map = nullptr;
    if (!m.internal_order && m.reordered) {
        st = ensure_work(ctx, bytes);
        if (st != SLW_OK)
            return st;
        st = hip_check(launch_permute_rows(ctx->stream, v_in, ctx->work, rows, (int64_t)(k * vsz), m.dof_user, 0),
                       "permute v_in");
        if (st != SLW_OK)
            return st;
        vin_int = ctx->work;
        out_map = m.dof_user;
    }
    const bool write_prev = start_mode == SLW_START_PREV;
    FieldDev fd = to_dev(field);
    st = hip_check(launch_step(m, ctx->stream, fd, t_n, dt, scheme, order, start_mode, start, vin_int, vdtype, k,
                               v_out, outside_value, write_prev, out_map, stats_h ? ctx->stats : nullptr),
                   "slw_step");
    if (st != SLW_OK)
        return st;
    return end_stats(ctx, stats_h);
}

slw_status slw_orient_sign_host(const double *pts_h, int64_t m, int8_t *out_h, int mode)
{
    if (m < 0 || (m > 0 && (!pts_h || !out_h)) || mode < 0 || mode > 2)
        return set_error(SLW_E_ARG, "slw_orient_sign_host: bad arguments");
    for (int64_t i = 0; i < m; ++i) {
        const double *p = pts_h + 6 * i;
        int s;
        if (mode == 0)
            s = orient_sign64(p[0], p[1], p[2], p[3], p[4], p[5]);
        else if (mode == 1)
            s = orient_exact_sign(p[0], p[1], p[2], p[3], p[4], p[5]);
        else
            s = orient_sign32((float)p[0], (float)p[1], (float)p[2], (float)p[3], (float)p[4], (float)p[5]);
        out_h[i] = (int8_t)s;
    }
    return SLW_OK;
}

slw_status slw_float_filter_host(const double *pts_h, int64_t m, double cx, double cy, double cmax, int f32,
                                 int8_t *out_h)
{
    if (m < 0 || (m > 0 && (!pts_h || !out_h)) || !(cmax >= 0.0))
        return set_error(SLW_E_ARG, "slw_float_filter_host: bad arguments");
    const FilterConst fc = filter_constants(f32 != 0, f32 ? 0.0 : cx, f32 ? 0.0 : cy, cmax);
    for (int64_t i = 0; i < m; ++i) {
        const double *p = pts_h + 6 * i;
        float r[6];
        for (int j = 0; j < 6; ++j)
            r[j] = f32 ? (float)p[j] : (float)(p[j] - ((j & 1) ? fc.cy : fc.cx));
        float det;
        const int s = filter_sign_f32(r[0] - r[4], r[1] - r[5], r[2] - r[4], r[3] - r[5], fc.c1, fc.c2, fc.c3, det);
        out_h[i] = (int8_t)(s != 0 ? s : 2);
    }
    return SLW_OK;
}

slw_status slw_permute_rows(slw_mesh *mesh, const void *src, void *dst, int64_t row_bytes, int to_internal)
{
    if (!mesh || !src || !dst || row_bytes <= 0 || (row_bytes & 3))
        return set_error(SLW_E_ARG, "slw_permute_rows: null pointer or row_bytes not a positive multiple of 4");
    if (src == dst)
        return set_error(SLW_E_ARG, "slw_permute_rows: src and dst must differ");
    slw_ctx *ctx = mesh->ctx;
    DeviceGuard g(ctx->device);
    // user -> internal: dst[d] = src[user(d)] (gather); internal -> user: scatter
    return hip_check(launch_permute_rows(ctx->stream, src, dst, mesh->m.n_dofs, row_bytes, mesh->m.dof_user,
                                         to_internal ? 0 : 1),
                     "slw_permute_rows");
}

}  // extern "C"
