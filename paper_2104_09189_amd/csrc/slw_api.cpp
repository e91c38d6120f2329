// C-ABI entry points: argument checks, context/stream handling, statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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

slw_status copy_stats(slw_ctx *ctx, const DevStats *counters, slw_stats *stats_h)
{
    if (!stats_h)
        return SLW_OK;
    DevStats h;
    slw_status st = hip_check(hipMemcpyAsync(&h, counters, sizeof h, hipMemcpyDeviceToHost, ctx->stream),
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
    stats_h->boundary_searches = (int64_t)h.boundary_searches;
    for (int b = 0; b < kHistBins; ++b)
        stats_h->step_hist[b] = (int64_t)h.step_hist[b];
    if (h.hard_fail)
        return set_error(SLW_E_WALK, std::to_string(h.hard_fail) + " walks exceeded the hard step limit");
    return SLW_OK;
}

}  // namespace slw

using namespace slw;

namespace {

slw_status begin_stats(slw_ctx *ctx, slw_stats *stats_h)
{
    if (!stats_h)
        return SLW_OK;
    // a fill kernel rather than a memset node keeps the call graph-capturable
    return hip_check(launch_zero_stats(ctx->stream, ctx->stats), "zero stats");
}

slw_status end_stats(slw_ctx *ctx, slw_stats *stats_h) { return copy_stats(ctx, ctx->stats, stats_h); }

}  // namespace

namespace slw {

// slw_step and slw_step_noalloc: checks, the permutation of v_in into the
// internal order (user-order meshes), the step launch and the statistics.
// With sc.stats == nullptr the context's counters and grow-only workspace are
// used; otherwise sc.stats and sc.work (sc.work_bytes at most, never grown).
slw_status step_impl(slw_mesh *mesh, const slw_field *field, double t_n, double dt, int scheme, int order,
                     int start_mode, const int32_t *start, const void *v_in, int vdtype, int k, void *v_out,
                     double outside_value, int32_t *elem, slw_stats *stats_h, const StepScratch &sc,
                     const char *who)
{
    const std::string w(who);
    if (!mesh || !field_ok(field) || !v_in || !v_out || k < 1)
        return set_error(SLW_E_ARG, w + ": null pointer, bad field or k < 1");
    if (order != 1 && order != 2)
        return set_error(SLW_E_ARG, w + ": order must be 1 or 2");
    if (order == 2 && !mesh->m.p2)
        return set_error(SLW_E_UNSUPPORTED, w + ": P2 needs a mesh uploaded with SLW_P2");
    if (scheme != SLW_EULER && scheme != SLW_RK2)
        return set_error(SLW_E_ARG, w + ": unknown scheme");
    if (vdtype != SLW_F64 && vdtype != SLW_F32)
        return set_error(SLW_E_ARG, w + ": unknown vdtype");
    if (start_mode < SLW_START_STEERED || start_mode > SLW_START_GRID)
        return set_error(SLW_E_ARG, w + ": unknown start mode");
    if (start_mode == SLW_START_GRID && !mesh->m.grid)
        return set_error(SLW_E_ARG, w + ": SLW_START_GRID needs a start grid (slw_mesh_build_grid)");
    if ((start_mode == SLW_START_PREV || start_mode == SLW_START_HYBRID) && mesh->m.n_tris >= ((int64_t)1 << 29))
        return set_error(SLW_E_UNSUPPORTED, w + ": previous elements need fewer than 2^29 triangles");
    if ((start_mode == SLW_START_GIVEN || start_mode == SLW_START_FIXED) && !start)
        return set_error(SLW_E_ARG, w + ": start array required for this start mode");
    if ((start_mode == SLW_START_LEARNED || start_mode == SLW_START_LEARNED_INDEX) && !mesh->m.mlp)
        return set_error(SLW_E_ARG, w + ": learned starts need a network attached (slw_mesh_attach_mlp)");
    if (start_mode == SLW_START_CHART && !mesh->m.chart_table)
        return set_error(SLW_E_ARG, w + ": SLW_START_CHART needs a chart (slw_chart_build)");
    const DevMesh &m = mesh->m;
    if (m.bc_kind && start_mode == SLW_START_NEIGHBOR && m.chain != 0)
        return set_error(SLW_E_UNSUPPORTED, w + ": boundary data with SLW_START_NEIGHBOR on chains");
    // P1 uses the vertex DOFs only (the first n_nodes of either order)
    const int64_t rows = order == 1 ? m.n_nodes : m.n_dofs;
    const size_t vsz = vdtype == SLW_F64 ? 8 : 4;
    const size_t bytes = (size_t)rows * (size_t)k * vsz;
    const char *vi = (const char *)v_in, *vo = (const char *)v_out;
    if (vi < vo + bytes && vo < vi + bytes)
        return set_error(SLW_E_ARG, w + ": v_in and v_out overlap");
    const bool permute = !m.internal_order && m.reordered;
    if (sc.stats && permute && bytes > sc.work_bytes)
        return set_error(SLW_E_ARG, w + ": v_in needs " + std::to_string(bytes) +
                                        " bytes of scratch for the permutation into the internal order, at most " +
                                        std::to_string(sc.work_bytes) + " are available (use SLW_INTERNAL_ORDER)");
    slw_ctx *ctx = mesh->ctx;
    DeviceGuard g(ctx->device);
    DevStats *counters = sc.stats ? sc.stats : ctx->stats;
    slw_status st = SLW_OK;
    if (stats_h)
        st = hip_check(launch_zero_stats(ctx->stream, counters), "zero stats");
    if (st != SLW_OK)
        return st;
    const void *vin_int = v_in;
    const int32_t *out_map = nullptr;
    if (permute) {
        void *work = sc.work;
        if (!sc.stats) {
            st = ensure_work(ctx, bytes);
            if (st != SLW_OK)
                return st;
            work = ctx->work;
        }
        st = hip_check(launch_permute_rows(ctx->stream, v_in, work, rows, (int64_t)(k * vsz), m.dof_user, 0),
                       "permute v_in");
        if (st != SLW_OK)
            return st;
        vin_int = work;
        out_map = m.dof_user;
    }
    const bool write_prev = start_mode == SLW_START_PREV;
    FieldDev fd = to_dev(field);
    st = hip_check(launch_step(m, ctx->stream, fd, t_n, dt, scheme, order, start_mode, start, vin_int, vdtype, k,
                               v_out, outside_value, write_prev, out_map, elem, stats_h ? counters : nullptr),
                   who);
    if (st != SLW_OK)
        return st;
    return copy_stats(ctx, counters, stats_h);
}

}  // namespace slw

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
    slw_status sn = noalloc_init(device);
    if (sn != SLW_OK) {
        delete c;
        return sn;
    }
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
    if (flags & ~(uint32_t)(SLW_COORDS_F32 | SLW_P2 | SLW_NO_REORDER | SLW_INTERNAL_ORDER | SLW_HILBERT))
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
    if (flags & ~(uint32_t)(SLW_COORDS_F32 | SLW_P2 | SLW_NO_REORDER | SLW_INTERNAL_ORDER | SLW_HILBERT))
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
        info_h->nonconvex = m.nonconvex;
        info_h->boundary_loops = m.n_loops;
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
    out_h->nonconvex = m.nonconvex;
    out_h->boundary_loops = m.n_loops;
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

slw_status slw_mesh_set_repack(slw_mesh *mesh, int feet_per_lane)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    if (feet_per_lane != 0 && feet_per_lane != 1 && feet_per_lane != 2 && feet_per_lane != 4 && feet_per_lane != 8)
        return set_error(SLW_E_ARG, "slw_mesh_set_repack: feet per lane must be 1, 2, 4 or 8");
    mesh->m.repack = feet_per_lane <= 1 ? 0 : feet_per_lane;
    return SLW_OK;
}

slw_status slw_mesh_set_neighbour_codes(slw_mesh *mesh, int bits)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    if (bits == 0)
        bits = kCodeBits;
    if (bits < 2 || bits > kCodeBits)
        return set_error(SLW_E_ARG, "slw_mesh_set_neighbour_codes: bits must be in [2, 21] (0: default)");
    DevMesh &m = mesh->m;
    DeviceGuard g(mesh->ctx->device);
    std::vector<GeoRec> geo(m.n_tris);
    slw_status st = hip_check(hipStreamSynchronize(mesh->ctx->stream), "synchronize before recoding");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(geo.data(), m.geo, m.n_tris * sizeof(GeoRec), hipMemcpyDeviceToHost), "copy records");
    if (st != SLW_OK)
        return st;
    const std::vector<WalkRec> w = walk_records(geo, bits);
    st = hip_check(hipMemcpy(m.wrec, w.data(), m.n_tris * sizeof(WalkRec), hipMemcpyHostToDevice), "copy walk records");
    if (st == SLW_OK)
        m.code_bits = bits;
    return st;
}

slw_status slw_walk_codes_host(const int32_t *nb_h, int64_t n_tris, int bits, uint32_t *words_h)
{
    if (!nb_h || !words_h || n_tris < 0)
        return set_error(SLW_E_ARG, "slw_walk_codes_host: null array or negative size");
    if (bits < 2 || bits > kCodeBits)
        return set_error(SLW_E_ARG, "slw_walk_codes_host: bits must be in [2, 21]");
    std::vector<GeoRec> geo(n_tris);
    for (int64_t t = 0; t < n_tris; ++t) {
        std::memset(&geo[t], 0, sizeof(GeoRec));
        for (int k = 0; k < 3; ++k)
            geo[t].nb[k] = nb_h[3 * t + k];
    }
    const std::vector<WalkRec> w = walk_records(geo, bits);
    for (int64_t t = 0; t < n_tris; ++t) {
        words_h[2 * t] = w[t].lo;
        words_h[2 * t + 1] = w[t].hi;
    }
    return SLW_OK;
}

slw_status slw_mesh_set_boundary(slw_mesh *mesh, int kind, const double *p_h)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    if (kind < SLW_BC_NONE || kind > SLW_BC_AFFINE || (kind != SLW_BC_NONE && !p_h))
        return set_error(SLW_E_ARG, "slw_mesh_set_boundary: unknown kind or missing parameters");
    mesh->m.bc_kind = kind;
    for (int i = 0; i < 4; ++i)
        mesh->m.bc_p[i] = kind == SLW_BC_NONE ? 0.0 : p_h[i];
    return SLW_OK;
}

slw_status slw_mesh_set_hybrid(slw_mesh *mesh, float far)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    if (!(far >= 0.0f) || !std::isfinite(far))
        return set_error(SLW_E_ARG, "slw_mesh_set_hybrid: far must be 0 (automatic) or a positive finite number");
    mesh->m.hybrid_far = far;
    return SLW_OK;
}

slw_status slw_mesh_set_lds_window(slw_mesh *mesh, int records)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    if (records != 0 && (records < 64 || records > 2048))
        return set_error(SLW_E_ARG, "slw_mesh_set_lds_window: records must be 0 or 64 ... 2048");
    mesh->m.lds_w = records;
    return SLW_OK;
}

slw_status slw_mesh_build_grid(slw_mesh *mesh, int g)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    DevMesh &m = mesh->m;
    if (g == 0) {
        if (m.grid) {
            DeviceGuard dg(mesh->ctx->device);
            (void)hipStreamSynchronize(mesh->ctx->stream);
            (void)hipFree(m.grid);
            m.device_bytes -= (int64_t)m.grid_g * m.grid_g * 4;
        }
        m.grid = nullptr;
        m.grid_g = 0;
        return SLW_OK;
    }
    if (g < 16 || g > 16384)
        return set_error(SLW_E_ARG, "slw_mesh_build_grid: g must be 0 (remove) or 16 ... 16384");
    DeviceGuard dg(mesh->ctx->device);
    const double wx = m.bbox[2] - m.bbox[0], wy = m.bbox[3] - m.bbox[1];
    const double span = wx > wy ? wx : wy;
    const double cell = span > 0 ? span / g : 1.0;
    int32_t *grid = nullptr;
    const size_t bytes = (size_t)g * (size_t)g * sizeof(int32_t);
    if (hipMalloc((void **)&grid, bytes) != hipSuccess)
        return set_error(SLW_E_NOMEM, "slw_mesh_build_grid: device memory");
    slw_status st = hip_check(launch_grid_build(m, mesh->ctx->stream, grid, g, m.bbox[0], m.bbox[1], cell),
                              "grid build");
    if (st == SLW_OK)
        st = hip_check(hipStreamSynchronize(mesh->ctx->stream), "hipStreamSynchronize");
    if (st != SLW_OK) {
        (void)hipFree(grid);
        return st;
    }
    if (m.grid) {
        (void)hipFree(m.grid);
        m.device_bytes -= (int64_t)m.grid_g * m.grid_g * 4;
    }
    m.grid = grid;
    m.grid_g = g;
    m.grid_x0 = m.bbox[0];
    m.grid_y0 = m.bbox[1];
    m.grid_inv = 1.0 / cell;
    m.device_bytes += (int64_t)bytes;
    return SLW_OK;
}

slw_status slw_mesh_set_xcd_chunk(slw_mesh *mesh, int chunk)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    if (chunk < 0 || chunk > 4096)
        return set_error(SLW_E_ARG, "slw_mesh_set_xcd_chunk: chunk must be 0 ... 4096");
    mesh->m.xcd_chunk = chunk;
    return SLW_OK;
}

slw_status slw_mesh_set_chain(slw_mesh *mesh, int length)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "mesh is NULL");
    if (length != 0 && length != 2 && length != 4 && length != 8 && length != 16)
        return set_error(SLW_E_ARG, "slw_mesh_set_chain: length must be 0 (the mesh forest), 2, 4, 8 or 16");
    mesh->m.chain = length;
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

slw_status slw_locate_quadtree(slw_mesh *mesh, const void *q, int64_t m, int32_t *elem, void *bary,
                               slw_stats *stats_h)
{
    if (!mesh || m < 0 || (m > 0 && (!q || !elem)))
        return set_error(SLW_E_ARG, "slw_locate_quadtree: null pointer or negative size");
    if (m > ((int64_t)1 << 31) - 1)
        return set_error(SLW_E_ARG, "slw_locate_quadtree: at most 2^31-1 points per call");
    if (!mesh->m.qt_nodes)
        return set_error(SLW_E_ARG, "slw_locate_quadtree: no quadtree (slw_quadtree_build)");
    slw_ctx *ctx = mesh->ctx;
    DeviceGuard g(ctx->device);
    slw_status st = begin_stats(ctx, stats_h);
    if (st != SLW_OK)
        return st;
    st = hip_check(launch_qt_locate(mesh->m, ctx->stream, q, m, elem, bary, stats_h ? ctx->stats : nullptr),
                   "slw_locate_quadtree");
    if (st != SLW_OK)
        return st;
    return end_stats(ctx, stats_h);
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
    if (start_mode < SLW_START_STEERED || start_mode == SLW_START_NEIGHBOR || start_mode == SLW_START_HYBRID ||
        start_mode > SLW_START_GRID)
        return set_error(SLW_E_ARG, "unknown start mode (SLW_START_NEIGHBOR and SLW_START_HYBRID are for slw_step)");
    if (start_mode == SLW_START_GRID && !mesh->m.grid)
        return set_error(SLW_E_ARG, "SLW_START_GRID needs a start grid (slw_mesh_build_grid)");
    if (start_mode == SLW_START_PREV && mesh->m.n_tris >= ((int64_t)1 << 29))
        return set_error(SLW_E_UNSUPPORTED, "previous elements need fewer than 2^29 triangles");
    if ((start_mode == SLW_START_GIVEN || start_mode == SLW_START_FIXED) && !start)
        return set_error(SLW_E_ARG, "start array required for this start mode");
    if ((start_mode == SLW_START_LEARNED || start_mode == SLW_START_LEARNED_INDEX) && !mesh->m.mlp)
        return set_error(SLW_E_ARG, "learned starts need a network attached (slw_mesh_attach_mlp)");
    if (start_mode == SLW_START_CHART && !mesh->m.chart_table)
        return set_error(SLW_E_ARG, "SLW_START_CHART needs a chart (slw_chart_build)");
    slw_ctx *ctx = mesh->ctx;
    DeviceGuard g(ctx->device);
    slw_status st = begin_stats(ctx, stats_h);
    if (st != SLW_OK)
        return st;
    FieldDev fd = to_dev(field);
    if (start_mode == SLW_START_LEARNED || start_mode == SLW_START_CHART || start_mode == SLW_START_LEARNED_INDEX) {
        const int kind = start_mode == SLW_START_CHART ? 0 : (start_mode == SLW_START_LEARNED ? 1 : 2);
        st = hip_check(launch_chart_start(mesh->m, ctx->stream, fd, t_np1, dt, scheme, feet_in ? feet : nullptr,
                                          mesh->m.n_dofs, kind, mesh->m.learned_start),
                       "chart start");
        if (st != SLW_OK)
            return st;
        start = mesh->m.learned_start;
    }
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
                    double outside_value, int32_t *elem, slw_stats *stats_h)
{
    StepScratch sc;  // the context's counters and grow-only workspace
    return step_impl(mesh, field, t_n, dt, scheme, order, start_mode, start, v_in, vdtype, k, v_out, outside_value,
                     elem, stats_h, sc, "slw_step");
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

// ===========================================================================
// batches of meshes, graphs, autotuning

#include <chrono>
#include <cstdio>
#include <fstream>
#include <sstream>

struct slw_batch {
    slw_ctx *ctx = nullptr;
    std::vector<slw_mesh *> meshes;
    std::vector<slw::BatchItem> items_h;  // tile0 filled for `block`
    slw::BatchItem *items = nullptr;      // device copy
    int64_t *counter = nullptr;           // device step counter
    unsigned *queues = nullptr;           // 8 per-XCD queues
    int coords_f32 = 0;
    int vdtype = SLW_F32;
    int k = 0;
    int block = 256;
    int schedule = 0;
    int have_fields = 0, have_values = 0;
    int64_t total_tiles = 0;
    int persistent_blocks = 0;
};

struct slw_graph {
    slw_ctx *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

slw_status batch_upload_items(slw_batch *b)
{
    int64_t tile = 0;
    for (auto &it : b->items_h) {
        it.tile0 = tile;
        tile += (it.n_iter + b->block - 1) / b->block;
    }
    b->total_tiles = tile;
    return hip_check(hipMemcpy(b->items, b->items_h.data(), b->items_h.size() * sizeof(slw::BatchItem),
                               hipMemcpyHostToDevice),
                     "hipMemcpy(batch items)");
}

int device_cu_count(int dev)
{
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
        cu = 256;
    return cu;
}

slw_status batch_launch(slw_batch *b, int scheme, double outside, slw::DevStats *st, hipStream_t stream)
{
    return hip_check(launch_batch_step(stream, b->coords_f32, b->vdtype, b->block, b->schedule, b->items,
                                       (int)b->items_h.size(), b->total_tiles, b->counter, scheme, b->k, outside,
                                       b->queues, b->persistent_blocks, st),
                     "batch step");
}

}  // namespace

extern "C" {

slw_status slw_batch_create(slw_ctx *ctx, slw_mesh *const *meshes_h, int n, slw_batch **out)
{
    if (!ctx || !meshes_h || n < 1 || !out)
        return set_error(SLW_E_ARG, "slw_batch_create: null pointer or n < 1");
    *out = nullptr;
    int f32 = -1;
    for (int i = 0; i < n; ++i) {
        if (!meshes_h[i] || meshes_h[i]->ctx != ctx)
            return set_error(SLW_E_ARG, "slw_batch_create: mesh missing or from another context");
        if (!meshes_h[i]->m.internal_order)
            return set_error(SLW_E_UNSUPPORTED, "slw_batch_create: meshes must use SLW_INTERNAL_ORDER");
        if (f32 >= 0 && f32 != meshes_h[i]->m.coords_f32)
            return set_error(SLW_E_UNSUPPORTED, "slw_batch_create: all meshes need the same coordinate type");
        f32 = meshes_h[i]->m.coords_f32;
    }
    DeviceGuard g(ctx->device);
    slw_batch *b = new (std::nothrow) slw_batch();
    if (!b)
        return set_error(SLW_E_NOMEM, "batch");
    b->ctx = ctx;
    b->coords_f32 = f32;
    b->meshes.assign(meshes_h, meshes_h + n);
    b->items_h.resize(n);
    for (int i = 0; i < n; ++i) {
        slw::BatchItem &it = b->items_h[i];
        std::memset(&it, 0, sizeof it);
        it.mv = view_of(meshes_h[i]->m);
        it.n_iter = meshes_h[i]->m.n_nodes;
    }
    b->persistent_blocks = device_cu_count(ctx->device) * 8;
    if (hipMalloc((void **)&b->items, n * sizeof(slw::BatchItem)) != hipSuccess ||
        hipMalloc((void **)&b->counter, sizeof(int64_t)) != hipSuccess ||
        hipMalloc((void **)&b->queues, 8 * sizeof(unsigned)) != hipSuccess) {
        slw_batch_free(b);
        return set_error(SLW_E_NOMEM, "batch device tables");
    }
    int64_t zero = 0;
    slw_status st = hip_check(hipMemcpy(b->counter, &zero, sizeof zero, hipMemcpyHostToDevice), "hipMemcpy(counter)");
    if (st == SLW_OK)
        st = batch_upload_items(b);
    if (st != SLW_OK) {
        slw_batch_free(b);
        return st;
    }
    *out = b;
    return SLW_OK;
}

slw_status slw_batch_free(slw_batch *b)
{
    if (!b)
        return SLW_OK;
    DeviceGuard g(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    if (b->items)
        (void)hipFree(b->items);
    if (b->counter)
        (void)hipFree(b->counter);
    if (b->queues)
        (void)hipFree(b->queues);
    delete b;
    return SLW_OK;
}

slw_status slw_batch_set_fields(slw_batch *b, const slw_field *fields_h, const double *dt_h, const double *t0_h)
{
    if (!b || !fields_h || !dt_h)
        return set_error(SLW_E_ARG, "slw_batch_set_fields: null pointer");
    for (size_t i = 0; i < b->items_h.size(); ++i) {
        if (!field_ok(&fields_h[i]) || !(dt_h[i] == dt_h[i]))
            return set_error(SLW_E_ARG, "slw_batch_set_fields: bad field or dt at mesh " + std::to_string(i));
        b->items_h[i].f = to_dev(&fields_h[i]);
        b->items_h[i].dt = dt_h[i];
        b->items_h[i].t0 = t0_h ? t0_h[i] : 0.0;
    }
    b->have_fields = 1;
    DeviceGuard g(b->ctx->device);
    return batch_upload_items(b);
}

slw_status slw_batch_set_values(slw_batch *b, void *const *va_h, void *const *vb_h, int vdtype, int k)
{
    if (!b || !va_h || !vb_h || k < 1 || (vdtype != SLW_F32 && vdtype != SLW_F64))
        return set_error(SLW_E_ARG, "slw_batch_set_values: bad arguments");
    for (size_t i = 0; i < b->items_h.size(); ++i) {
        if (!va_h[i] || !vb_h[i] || va_h[i] == vb_h[i])
            return set_error(SLW_E_ARG, "slw_batch_set_values: value buffers missing or equal at mesh " +
                                            std::to_string(i));
        b->items_h[i].va = va_h[i];
        b->items_h[i].vb = vb_h[i];
    }
    b->vdtype = vdtype;
    b->k = k;
    b->have_values = 1;
    DeviceGuard g(b->ctx->device);
    return batch_upload_items(b);
}

slw_status slw_batch_set_elem_out(slw_batch *b, int32_t *const *elem_h)
{
    if (!b)
        return set_error(SLW_E_ARG, "slw_batch_set_elem_out: batch is NULL");
    for (size_t i = 0; i < b->items_h.size(); ++i)
        b->items_h[i].elem = elem_h ? elem_h[i] : nullptr;
    DeviceGuard g(b->ctx->device);
    return batch_upload_items(b);
}

slw_status slw_batch_set_start(slw_batch *b, int start_mode)
{
    if (!b || (start_mode != SLW_START_STEERED && start_mode != SLW_START_PREV))
        return set_error(SLW_E_ARG, "slw_batch_set_start: SLW_START_STEERED or SLW_START_PREV");
    for (slw_mesh *m : b->meshes)
        if (start_mode == SLW_START_PREV && m->m.n_tris >= ((int64_t)1 << 29))
            return set_error(SLW_E_UNSUPPORTED, "slw_batch_set_start: previous elements need fewer than 2^29 triangles");
    for (auto &it : b->items_h)
        it.start_mode = start_mode;
    DeviceGuard g(b->ctx->device);
    return batch_upload_items(b);
}

slw_status slw_batch_set_step(slw_batch *b, int64_t n)
{
    if (!b || n < 0)
        return set_error(SLW_E_ARG, "slw_batch_set_step: bad arguments");
    DeviceGuard g(b->ctx->device);
    slw_status st = hip_check(hipStreamSynchronize(b->ctx->stream), "hipStreamSynchronize");
    if (st != SLW_OK)
        return st;
    return hip_check(hipMemcpy(b->counter, &n, sizeof n, hipMemcpyHostToDevice), "hipMemcpy(counter)");
}

slw_status slw_batch_get_step(slw_batch *b, int64_t *n_h)
{
    if (!b || !n_h)
        return set_error(SLW_E_ARG, "slw_batch_get_step: bad arguments");
    DeviceGuard g(b->ctx->device);
    slw_status st = hip_check(hipStreamSynchronize(b->ctx->stream), "hipStreamSynchronize");
    if (st != SLW_OK)
        return st;
    return hip_check(hipMemcpy(n_h, b->counter, sizeof *n_h, hipMemcpyDeviceToHost), "hipMemcpy(counter)");
}

slw_status slw_batch_set_schedule(slw_batch *b, int schedule, int block)
{
    if (!b || (schedule < 0 || schedule > 2) || (block != 64 && block != 128 && block != 256 && block != 512))
        return set_error(SLW_E_ARG, "slw_batch_set_schedule: schedule 0/1/2, block 64/128/256/512");
    b->schedule = schedule;
    b->block = block;
    DeviceGuard g(b->ctx->device);
    return batch_upload_items(b);
}

slw_status slw_batch_step(slw_batch *b, int scheme, double outside_value, slw_stats *stats_h)
{
    if (!b || (scheme != SLW_EULER && scheme != SLW_RK2))
        return set_error(SLW_E_ARG, "slw_batch_step: bad arguments");
    if (!b->have_fields || !b->have_values)
        return set_error(SLW_E_ARG, "slw_batch_step: set fields and values first");
    DeviceGuard g(b->ctx->device);
    slw_status st = begin_stats(b->ctx, stats_h);
    if (st != SLW_OK)
        return st;
    st = batch_launch(b, scheme, outside_value, stats_h ? b->ctx->stats : nullptr, b->ctx->stream);
    if (st != SLW_OK)
        return st;
    return end_stats(b->ctx, stats_h);
}

slw_status slw_batch_graph_capture(slw_batch *b, int n_steps, int scheme, double outside_value, slw_graph **out)
{
    if (!b || n_steps < 1 || !out || (scheme != SLW_EULER && scheme != SLW_RK2))
        return set_error(SLW_E_ARG, "slw_batch_graph_capture: bad arguments");
    if (!b->have_fields || !b->have_values)
        return set_error(SLW_E_ARG, "slw_batch_graph_capture: set fields and values first");
    *out = nullptr;
    DeviceGuard g(b->ctx->device);
    slw_status st = hip_check(hipStreamSynchronize(b->ctx->stream), "hipStreamSynchronize");
    if (st != SLW_OK)
        return st;
    // capture on a private stream (the caller's may be the null stream); default priority
    hipStream_t cs = nullptr;
    st = hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
    if (st != SLW_OK)
        return st;
    hipGraph_t graph = nullptr;
    st = hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (st == SLW_OK) {
        for (int i = 0; i < n_steps && st == SLW_OK; ++i)
            st = batch_launch(b, scheme, outside_value, nullptr, cs);
        hipError_t e = hipStreamEndCapture(cs, &graph);
        if (st == SLW_OK)
            st = hip_check(e, "hipStreamEndCapture");
    }
    (void)hipStreamDestroy(cs);
    if (st != SLW_OK) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return st;
    }
    slw_graph *gr = new (std::nothrow) slw_graph();
    if (!gr) {
        (void)hipGraphDestroy(graph);
        return set_error(SLW_E_NOMEM, "graph");
    }
    gr->ctx = b->ctx;
    gr->graph = graph;
    st = hip_check(hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (st != SLW_OK) {
        slw_graph_free(gr);
        return st;
    }
    *out = gr;
    return SLW_OK;
}

slw_status slw_graph_launch(slw_graph *gr)
{
    if (!gr || !gr->exec)
        return set_error(SLW_E_ARG, "slw_graph_launch: null graph");
    DeviceGuard g(gr->ctx->device);
    return hip_check(hipGraphLaunch(gr->exec, gr->ctx->stream), "hipGraphLaunch");
}

slw_status slw_graph_free(slw_graph *gr)
{
    if (!gr)
        return SLW_OK;
    DeviceGuard g(gr->ctx->device);
    (void)hipStreamSynchronize(gr->ctx->stream);
    if (gr->exec)
        (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph)
        (void)hipGraphDestroy(gr->graph);
    delete gr;
    return SLW_OK;
}

}  // extern "C"

namespace {

std::string batch_signature(const slw_batch *b)
{
    int64_t dofs = 0;
    for (const auto &it : b->items_h)
        dofs += it.n_iter;
    int bucket = 0;
    while ((int64_t)1 << (bucket + 1) <= dofs)
        ++bucket;
    std::ostringstream os;
    os << "meshes" << b->items_h.size() << "_dofs2^" << bucket << "_c" << (b->coords_f32 ? "f32" : "f64") << "_v"
       << (b->vdtype == SLW_F32 ? "f32" : "f64") << "_k" << b->k
       << (b->items_h.empty() || b->items_h[0].start_mode == SLW_START_STEERED ? "" : "_prev");
    return os.str();
}

// tiny JSON cache: {"signature": {"schedule": s, "block": b, "ms": t}, ...}
bool cache_lookup(const char *path, const std::string &sig, int &schedule, int &block)
{
    std::ifstream f(path);
    if (!f)
        return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string txt = ss.str();
    const size_t at = txt.find("\"" + sig + "\"");
    if (at == std::string::npos)
        return false;
    const size_t s1 = txt.find("\"schedule\":", at), b1 = txt.find("\"block\":", at);
    if (s1 == std::string::npos || b1 == std::string::npos)
        return false;
    schedule = std::atoi(txt.c_str() + s1 + 11);
    block = std::atoi(txt.c_str() + b1 + 8);
    return (schedule >= 0 && schedule <= 2) && (block == 64 || block == 128 || block == 256 || block == 512);
}

void cache_store(const char *path, const std::string &sig, int schedule, int block, double ms)
{
    std::string txt;
    {
        std::ifstream f(path);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            txt = ss.str();
        }
    }
    std::ostringstream entry;
    entry << "\"" << sig << "\": {\"schedule\": " << schedule << ", \"block\": " << block << ", \"ms\": " << ms << "}";
    const size_t at = txt.find("\"" + sig + "\"");
    if (at != std::string::npos) {
        const size_t end = txt.find('}', at);
        txt.replace(at, end + 1 - at, entry.str());
    } else {
        const size_t close = txt.rfind('}');
        if (txt.empty() || close == std::string::npos)
            txt = "{\n  " + entry.str() + "\n}\n";
        else {
            const bool empty = txt.find('"') == std::string::npos;
            txt.insert(close, (empty ? "  " : ",\n  ") + entry.str() + "\n");
        }
    }
    std::ofstream f(path);
    f << txt;
}

}  // namespace

extern "C" slw_status slw_batch_autotune(slw_batch *b, int scheme, const char *cache_path, int *schedule_out,
                                         int *block_out)
{
    if (!b || (scheme != SLW_EULER && scheme != SLW_RK2))
        return set_error(SLW_E_ARG, "slw_batch_autotune: bad arguments");
    if (!b->have_fields || !b->have_values)
        return set_error(SLW_E_ARG, "slw_batch_autotune: set fields and values first");
    DeviceGuard g(b->ctx->device);
    const std::string sig = batch_signature(b);
    int schedule = 0, block = 256;
    if (cache_path && cache_lookup(cache_path, sig, schedule, block)) {
        slw_status st = slw_batch_set_schedule(b, schedule, block);
        if (st == SLW_OK) {
            if (schedule_out)
                *schedule_out = schedule;
            if (block_out)
                *block_out = block;
        }
        return st;
    }
    // Tune on private copies of the value buffers (the caller's stay untouched):
    // every candidate runs the same first step from the same input and must
    // reproduce the reference candidate's output bit for bit (parity guard),
    // then is timed over a few steps.
    const size_t vsz = b->vdtype == SLW_F64 ? 8 : 4;
    std::vector<size_t> bytes(b->items_h.size());
    size_t total = 0;
    for (size_t i = 0; i < b->items_h.size(); ++i) {
        bytes[i] = (size_t)b->items_h[i].n_iter * b->k * vsz;
        total += bytes[i];
    }
    char *work = nullptr;
    if (hipMalloc((void **)&work, 3 * total) != hipSuccess)
        return set_error(SLW_E_NOMEM, "autotune workspace");
    std::vector<slw::BatchItem> saved = b->items_h;
    int64_t saved_step = 0;
    slw_status st = hip_check(hipStreamSynchronize(b->ctx->stream), "hipStreamSynchronize");
    // with the previous-element start every candidate starts from the
    // meshes' previous elements as they are now, and they are left so
    const bool keeps_prev = !b->items_h.empty() && b->items_h[0].start_mode == SLW_START_PREV;
    size_t prev_total = 0;
    if (keeps_prev)
        for (slw_mesh *m : b->meshes)
            prev_total += (size_t)m->m.n_dofs;
    int32_t *prev_saved = nullptr;
    if (st == SLW_OK && keeps_prev && hipMalloc((void **)&prev_saved, prev_total * sizeof(int32_t)) != hipSuccess)
        st = set_error(SLW_E_NOMEM, "autotune workspace (previous elements)");
    auto copy_prev = [&](bool save) -> slw_status {
        size_t o = 0;
        for (slw_mesh *m : b->meshes) {
            const size_t nb = (size_t)m->m.n_dofs * sizeof(int32_t);
            slw_status s2 = hip_check(hipMemcpy(save ? (void *)(prev_saved + o) : (void *)m->m.prev_elem,
                                                save ? (const void *)m->m.prev_elem : (const void *)(prev_saved + o),
                                                nb, hipMemcpyDeviceToDevice),
                                      "copy previous elements");
            if (s2 != SLW_OK)
                return s2;
            o += (size_t)m->m.n_dofs;
        }
        return SLW_OK;
    };
    if (st == SLW_OK && keeps_prev)
        st = copy_prev(true);
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(&saved_step, b->counter, sizeof saved_step, hipMemcpyDeviceToHost), "counter");
    const int saved_schedule = b->schedule, saved_block = b->block;
    // layout of work: [A copies | B copies | reference output]
    size_t off = 0;
    for (size_t i = 0; i < b->items_h.size() && st == SLW_OK; ++i) {
        st = hip_check(hipMemcpy(work + off, saved[i].va, bytes[i], hipMemcpyDeviceToDevice), "copy values");
        b->items_h[i].va = work + off;
        b->items_h[i].vb = work + total + off;
        off += bytes[i];
    }
    const int64_t even_step = saved_step & ~(int64_t)1;
    double best_ms = 1e300;
    int best_s = saved_schedule, best_b = saved_block;
    bool have_ref = false;
    std::vector<char> ref_h, out_h;
    const int schedules[3] = {0, 1, 2};
    const int blocks[4] = {64, 128, 256, 512};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == SLW_OK)
        st = hip_check(hipEventCreate(&e0), "hipEventCreate");
    if (st == SLW_OK)
        st = hip_check(hipEventCreate(&e1), "hipEventCreate");
    for (int si = 0; si < 3 && st == SLW_OK; ++si)
        for (int bi = 0; bi < 4 && st == SLW_OK; ++bi) {
            b->schedule = schedules[si];
            b->block = blocks[bi];
            st = batch_upload_items(b);
            if (st != SLW_OK)
                break;
            // parity guard: one step from the copy of the input (even step: A -> B)
            if (keeps_prev)
                st = copy_prev(false);
            if (st == SLW_OK)
                st = slw_batch_set_step(b, even_step);
            if (st == SLW_OK)
                st = batch_launch(b, scheme, 0.0, nullptr, b->ctx->stream);
            if (st == SLW_OK)
                st = hip_check(hipStreamSynchronize(b->ctx->stream), "sync");
            if (st != SLW_OK)
                break;
            out_h.resize(total);
            st = hip_check(hipMemcpy(out_h.data(), work + total, total, hipMemcpyDeviceToHost), "copy output");
            if (st != SLW_OK)
                break;
            if (!have_ref) {
                ref_h = out_h;
                have_ref = true;
            } else if (std::memcmp(ref_h.data(), out_h.data(), total) != 0) {
                continue;  // not bit-identical: never chosen
            }
            // timing: 5 steps (values evolve in the private buffers)
            const int reps = 5;
            st = hip_check(hipEventRecord(e0, b->ctx->stream), "event");
            for (int r = 0; r < reps && st == SLW_OK; ++r)
                st = batch_launch(b, scheme, 0.0, nullptr, b->ctx->stream);
            if (st == SLW_OK)
                st = hip_check(hipEventRecord(e1, b->ctx->stream), "event");
            if (st == SLW_OK)
                st = hip_check(hipEventSynchronize(e1), "event sync");
            float ms = 0.f;
            if (st == SLW_OK)
                st = hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
            if (st == SLW_OK && ms / reps < best_ms) {
                best_ms = ms / reps;
                best_s = b->schedule;
                best_b = b->block;
            }
            // restore the private input for the next candidate
            off = 0;
            for (size_t i = 0; i < b->items_h.size() && st == SLW_OK; ++i) {
                st = hip_check(hipMemcpy(work + off, saved[i].va, bytes[i], hipMemcpyDeviceToDevice), "copy values");
                off += bytes[i];
            }
        }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    // restore the caller's buffers and step; keep the winner
    for (size_t i = 0; i < b->items_h.size(); ++i) {
        b->items_h[i].va = saved[i].va;
        b->items_h[i].vb = saved[i].vb;
    }
    b->schedule = st == SLW_OK ? best_s : saved_schedule;
    b->block = st == SLW_OK ? best_b : saved_block;
    slw_status st2 = batch_upload_items(b);
    slw_status st3 = slw_batch_set_step(b, saved_step);
    if (prev_saved) {
        const slw_status st4 = copy_prev(false);
        if (st2 == SLW_OK)
            st2 = st4;
        (void)hipFree(prev_saved);
    }
    (void)hipFree(work);
    if (st != SLW_OK)
        return st;
    if (st2 != SLW_OK)
        return st2;
    if (st3 != SLW_OK)
        return st3;
    if (cache_path)
        cache_store(cache_path, sig, b->schedule, b->block, best_ms);
    if (schedule_out)
        *schedule_out = b->schedule;
    if (block_out)
        *block_out = b->block;
    return SLW_OK;
}

// ===========================================================================
// autotuning of slw_step's schedule knobs

namespace {

// value of "key" in the cache entry of signature sig (false if absent)
bool cache_lookup_num(const char *path, const std::string &sig, const char *key, double &val)
{
    std::ifstream f(path);
    if (!f)
        return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string txt = ss.str();
    const size_t at = txt.find("\"" + sig + "\"");
    if (at == std::string::npos)
        return false;
    const size_t end = txt.find('}', at);
    const size_t k = txt.find(std::string("\"") + key + "\":", at);
    if (k == std::string::npos || k > end)
        return false;
    val = std::atof(txt.c_str() + k + std::strlen(key) + 3);
    return true;
}

// replaces or adds the entry "sig": {body} (body without braces)
void cache_store_entry(const char *path, const std::string &sig, const std::string &body)
{
    std::string txt;
    {
        std::ifstream f(path);
        if (f) {
            std::stringstream ss;
            ss << f.rdbuf();
            txt = ss.str();
        }
    }
    const std::string entry = "\"" + sig + "\": {" + body + "}";
    const size_t at = txt.find("\"" + sig + "\"");
    if (at != std::string::npos) {
        const size_t end = txt.find('}', at);
        txt.replace(at, end + 1 - at, entry);
    } else {
        const size_t close = txt.rfind('}');
        if (txt.empty() || close == std::string::npos)
            txt = "{\n  " + entry + "\n}\n";
        else {
            const bool empty = txt.find('"') == std::string::npos;
            txt.insert(close, (empty ? "  " : ",\n  ") + entry + "\n");
        }
    }
    std::ofstream f(path);
    f << txt;
}

// the knob a start mode is tuned on, and its candidate values
const char *knob_name(int mode)
{
    if (mode == SLW_START_HYBRID)
        return "hybrid_far";
    if (mode == SLW_START_NEIGHBOR)
        return "chain";
    return "feet_per_lane";
}

// XCD chunks the step autotuner tries (slw_mesh_set_xcd_chunk)
constexpr int kXcdChunks[] = {0, 16, 32, 64, 128};
// LDS windows it tries (slw_mesh_set_lds_window) for the plain step's modes
constexpr int kLdsWindows[] = {0, 256, 512, 768};
bool plain_step_mode(int mode)
{
    return mode == SLW_START_STEERED || mode == SLW_START_GIVEN || mode == SLW_START_FIXED;
}

std::vector<double> knob_values(int mode, bool bc)
{
    if (mode == SLW_START_HYBRID)
        return {0.5, 1, 2, 4, 8, 16, 32, 64};
    if (mode == SLW_START_NEIGHBOR)
        return bc ? std::vector<double>{0} : std::vector<double>{0, 2, 4, 8, 16};
    if (mode == SLW_START_LEARNED_INDEX || bc)
        return {1};  // one-foot-per-lane kernels only
    return {1, 2, 4, 8};
}  // bc: boundary data or a non-convex domain (one-foot-per-lane kernels only)

double knob_get(const DevMesh &m, int mode)
{
    if (mode == SLW_START_HYBRID)
        return m.hybrid_far;
    if (mode == SLW_START_NEIGHBOR)
        return m.chain;
    return m.repack ? m.repack : 1;
}

void knob_set(DevMesh &m, int mode, double v)
{
    if (mode == SLW_START_HYBRID)
        m.hybrid_far = (float)v;
    else if (mode == SLW_START_NEIGHBOR)
        m.chain = (int)v;
    else
        m.repack = (int)v <= 1 ? 0 : (int)v;
}

}  // namespace

extern "C" slw_status slw_step_autotune(slw_mesh *mesh, const slw_field *field, double t_n, double dt, int scheme,
                                        int order, int start_mode, const int32_t *start, const void *v_in,
                                        int vdtype, int k, const char *cache_path, double *value_out,
                                        int32_t *xcd_chunk_out, double *ms_out)
{
    if (!mesh || !v_in)
        return set_error(SLW_E_ARG, "slw_step_autotune: mesh or v_in is NULL");
    DevMesh &m = mesh->m;
    slw_ctx *ctx = mesh->ctx;
    DeviceGuard g(ctx->device);
    const int64_t rows = order == 1 ? m.n_nodes : m.n_dofs;
    const size_t vsz = vdtype == SLW_F64 ? 8 : 4;
    const size_t bytes = (size_t)rows * (size_t)(k > 0 ? k : 1) * vsz;
    const double saved = knob_get(m, start_mode);
    const int saved_chunk = m.xcd_chunk;
    const int saved_lds = m.lds_w;
    const bool keeps_prev = start_mode == SLW_START_PREV || start_mode == SLW_START_HYBRID;
    void *vout = nullptr;
    int32_t *prev0 = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    std::vector<char> ref_h, out_h;
    slw_stats st0;
    slw_status st = SLW_OK;
    auto release = [&]() {
        if (vout)
            (void)hipFree(vout);
        if (prev0)
            (void)hipFree(prev0);
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
    };
    if (hipMalloc(&vout, bytes) != hipSuccess ||
        (keeps_prev && hipMalloc((void **)&prev0, (size_t)m.n_dofs * sizeof(int32_t)) != hipSuccess)) {
        release();
        return set_error(SLW_E_NOMEM, "slw_step_autotune: workspace");
    }
    st = hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (st == SLW_OK && keeps_prev)  // the caller's previous elements: every candidate starts from them
        st = hip_check(hipMemcpy(prev0, m.prev_elem, (size_t)m.n_dofs * sizeof(int32_t), hipMemcpyDeviceToDevice),
                       "save previous elements");
    if (st == SLW_OK)
        st = hip_check(hipEventCreate(&e0), "hipEventCreate");
    if (st == SLW_OK)
        st = hip_check(hipEventCreate(&e1), "hipEventCreate");
    auto restore_prev = [&]() -> slw_status {
        if (!keeps_prev)
            return SLW_OK;
        return hip_check(hipMemcpyAsync(m.prev_elem, prev0, (size_t)m.n_dofs * sizeof(int32_t),
                                        hipMemcpyDeviceToDevice, ctx->stream),
                         "restore previous elements");
    };
    // the regime of the step for the cache signature: the walk lengths of
    // strategy (a) (the feet's displacement in cells), whatever the knobs
    if (st == SLW_OK)
        st = step_impl(mesh, field, t_n, dt, scheme, order, SLW_START_STEERED, nullptr, v_in, vdtype, k, vout, 0.0,
                       nullptr, &st0, StepScratch(), "slw_step_autotune");
    // the reference: the mesh's current setting
    if (st == SLW_OK)
        st = restore_prev();
    if (st == SLW_OK)
        st = step_impl(mesh, field, t_n, dt, scheme, order, start_mode, start, v_in, vdtype, k, vout, 0.0, nullptr,
                       nullptr, StepScratch(), "slw_step_autotune");
    if (st == SLW_OK) {
        ref_h.resize(bytes);
        st = hip_check(hipMemcpy(ref_h.data(), vout, bytes, hipMemcpyDeviceToHost), "copy reference");
    }
    std::string sig;
    if (st == SLW_OK) {
        int nb = 0, wb = 0;
        while (((int64_t)1 << (nb + 1)) <= rows)
            ++nb;
        const double mean = st0.feet ? (double)st0.walk_steps / (double)st0.feet : 0.0;
        while ((double)((int64_t)1 << (wb + 1)) <= 1.0 + mean)
            ++wb;
        std::ostringstream os;
        os << "step_dofs2^" << nb << "_c" << (m.coords_f32 ? "f32" : "f64") << "_v" << (vdtype == SLW_F32 ? "f32" : "f64")
           << "_k" << k << "_o" << order << "_mode" << start_mode << "_s" << scheme << "_walk2^" << wb
           << (m.bc_kind ? "_bc" : "");
        sig = os.str();
        double cached = 0.0, cms = 0.0;
        if (cache_path && cache_lookup_num(cache_path, sig, knob_name(start_mode), cached)) {
            (void)cache_lookup_num(cache_path, sig, "ms", cms);
            const std::vector<double> ok = knob_values(start_mode, m.bc_kind != 0 || m.nonconvex != 0);
            bool valid = false;
            for (double v : ok)
                valid = valid || v == cached;
            if (valid) {
                st = restore_prev();
                if (st == SLW_OK)
                    st = hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
                release();
                if (st != SLW_OK)
                    return st;
                knob_set(m, start_mode, cached);
                double cc = 0.0;
                if (cache_lookup_num(cache_path, sig, "xcd_chunk", cc) && cc >= 0.0 && cc <= 4096.0)
                    m.xcd_chunk = (int)cc;
                if (cache_lookup_num(cache_path, sig, "lds_window", cc) && (cc == 0.0 || (cc >= 64.0 && cc <= 2048.0)))
                    m.lds_w = (int)cc;
                if (value_out)
                    *value_out = cached;
                if (xcd_chunk_out)
                    *xcd_chunk_out = m.xcd_chunk;
                if (ms_out)
                    *ms_out = cms;
                return SLW_OK;
            }
        }
    }
    // one candidate (the knobs as set on the mesh): its step from the same
    // state must give the reference's bits (else it is never chosen); then,
    // from the caller's previous elements (the hybrid's skip counts
    // cleared, so that each candidate sets its own), one untimed step from
    // t_n - dt and five timed consecutive steps from t_n; the median
    auto time_candidate = [&](float &median) -> bool {
        st = restore_prev();
        if (st == SLW_OK)
            st = step_impl(mesh, field, t_n, dt, scheme, order, start_mode, start, v_in, vdtype, k, vout, 0.0,
                           nullptr, nullptr, StepScratch(), "slw_step_autotune");
        if (st == SLW_OK) {
            out_h.resize(bytes);
            st = hip_check(hipMemcpy(out_h.data(), vout, bytes, hipMemcpyDeviceToHost), "copy candidate");
        }
        if (st != SLW_OK || std::memcmp(out_h.data(), ref_h.data(), bytes) != 0)
            return false;
        std::vector<float> ts;
        st = restore_prev();
        if (st == SLW_OK && keeps_prev)
            st = hip_check(launch_prev_clear_skip(ctx->stream, m.prev_elem, m.n_dofs), "clear skip counts");
        if (st == SLW_OK)
            st = step_impl(mesh, field, t_n - dt, dt, scheme, order, start_mode, start, v_in, vdtype, k, vout, 0.0,
                           nullptr, nullptr, StepScratch(), "slw_step_autotune");
        for (int r = 0; r < 5 && st == SLW_OK; ++r) {
            st = hip_check(hipEventRecord(e0, ctx->stream), "event");
            if (st == SLW_OK)
                st = step_impl(mesh, field, t_n + r * dt, dt, scheme, order, start_mode, start, v_in, vdtype, k, vout,
                               0.0, nullptr, nullptr, StepScratch(), "slw_step_autotune");
            if (st == SLW_OK)
                st = hip_check(hipEventRecord(e1, ctx->stream), "event");
            if (st == SLW_OK)
                st = hip_check(hipEventSynchronize(e1), "event sync");
            float ms = 0.f;
            if (st == SLW_OK)
                st = hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
            ts.push_back(ms);
        }
        if (st != SLW_OK)
            return false;
        std::sort(ts.begin(), ts.end());
        median = ts[2];
        return true;
    };
    // first the mode's own knob (at the mesh's XCD chunk), then the XCD chunk
    // for the chosen value
    double best_v = saved, best_ms = 1e300;
    int best_c = saved_chunk, best_l = saved_lds;
    for (double v : knob_values(start_mode, m.bc_kind != 0 || m.nonconvex != 0)) {
        if (st != SLW_OK)
            break;
        knob_set(m, start_mode, v);
        float ms = 0.f;
        if (time_candidate(ms) && ms < best_ms) {
            best_ms = ms;
            best_v = v;
        }
    }
    if (st == SLW_OK && best_ms < 1e300) {
        knob_set(m, start_mode, best_v);
        for (int c : kXcdChunks) {
            if (st != SLW_OK)
                break;
            if (c == saved_chunk)
                continue;  // timed above
            m.xcd_chunk = c;
            float ms = 0.f;
            if (time_candidate(ms) && ms < best_ms) {
                best_ms = ms;
                best_c = c;
            }
        }
        // then the LDS window of the plain step (one foot per lane)
        m.xcd_chunk = best_c;
        if (plain_step_mode(start_mode) && best_v <= 1.0 && order == 1)
            for (int lw : kLdsWindows) {
                if (st != SLW_OK)
                    break;
                if (lw == saved_lds)
                    continue;  // timed above
                m.lds_w = lw;
                float ms = 0.f;
                if (time_candidate(ms) && ms < best_ms) {
                    best_ms = ms;
                    best_l = lw;
                }
            }
    }
    // the caller's previous elements are left as they were
    slw_status st2 = restore_prev();
    if (st2 == SLW_OK)
        st2 = hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    release();
    knob_set(m, start_mode, st == SLW_OK ? best_v : saved);
    m.xcd_chunk = st == SLW_OK ? best_c : saved_chunk;
    m.lds_w = st == SLW_OK ? best_l : saved_lds;
    if (st != SLW_OK)
        return st;
    if (st2 != SLW_OK)
        return st2;
    if (cache_path) {
        std::ostringstream body;
        body << "\"" << knob_name(start_mode) << "\": " << best_v << ", \"xcd_chunk\": " << best_c
             << ", \"lds_window\": " << best_l << ", \"ms\": " << best_ms;
        cache_store_entry(cache_path, sig, body.str());
    }
    if (value_out)
        *value_out = best_v;
    if (xcd_chunk_out)
        *xcd_chunk_out = best_c;
    if (ms_out)
        *ms_out = best_ms;
    return SLW_OK;
}
