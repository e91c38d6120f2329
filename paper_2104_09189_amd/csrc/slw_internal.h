// Internal data layout of the library (device side and handles).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/slwalk.h"

namespace slw {

// Triangle record read by every walk step (48 bytes, three 16-byte loads):
// vertex coordinates as float (for double meshes: relative to the centre of
// the bounding box, rounded; for float meshes: the coordinates themselves),
// the neighbours (neighbour k across the edge opposite vertex k, -1 on the
// boundary) and the internal ids of the three vertices.  Walk decisions are
// taken on the float coordinates only when a certified error bound allows
// it; otherwise the exact coordinates are read through the vertex ids.
struct alignas(16) GeoRec {
    float2 p[3];
    int32_t nb[3];
    int32_t v[3];
};
static_assert(sizeof(GeoRec) == 48, "GeoRec layout");

// Walk record (32 bytes: two 16-byte loads that never straddle a cache
// line), the part of GeoRec a walk move needs: the same float coordinates and
// the three neighbours as 21-bit two's-complement offsets from the
// triangle's own internal id, code k in bits [21k, 21k + 21) of the 64-bit
// word (hi:lo).  Code 0 marks a boundary edge (a triangle is never its own
// neighbour); kCodeEscape marks an offset that does not fit, the neighbour is
// then read from GeoRec::nb.  Along a Morton order nearly every neighbour
// lies within 2^20 ids (all of them for meshes of up to 2^20 triangles).
struct alignas(32) WalkRec {
    float2 p[3];
    uint32_t lo, hi;
};
static_assert(sizeof(WalkRec) == 32, "WalkRec layout");
constexpr int kCodeBits = 21;
constexpr int32_t kCodeEscape = -(1 << (kCodeBits - 1));

// Coefficients of the float filter's error bound (see the walk kernel):
// |det_float - det| <= c1 (|l| + |r|) + c2 (|ax|+|ay|+|bx|+|by|) + c3.
struct FilterConst {
    float c1, c2, c3;
    double cx, cy;  // centre subtracted from coordinates before rounding to float
};

struct DevMesh {
    int64_t n_nodes = 0, n_tris = 0, n_edges = 0, n_dofs = 0;
    int coords_f32 = 0, p2 = 0, reordered = 0, internal_order = 0;
    double bbox[4] = {0, 0, 0, 0};
    FilterConst fc = {0, 0, 0, 0, 0};
    // device arrays (internal order)
    GeoRec *geo = nullptr;        // [n_tris]
    WalkRec *wrec = nullptr;      // [n_tris] the walk's copy of geo (packed neighbours)
    int code_bits = kCodeBits;    // widest neighbour offset coded in wrec (narrower: more escapes)
    int4 *tri_v = nullptr;        // [n_tris] {nb[2], v[0], v[1], v[2]} of geo, compact (read where walks end)
    int32_t *tri_uf = nullptr;    // [n_tris] user id | (1 << 31 if vertices 1, 2 were swapped to make it CCW)
    int4 *tedge = nullptr;        // [n_tris] P2: internal DOF ids of the edge opposite vertex k
    void *dof_xy = nullptr;       // double2/float2 [n_dofs], exact coordinates
    int4 *qstart = nullptr;       // [n_dofs] incident triangle facing each diagonal direction
    int32_t *vmin = nullptr;      // [n_nodes] internal tri with the smallest user id around the node
    int32_t *dof_user = nullptr;  // [n_dofs] internal -> user DOF id
    int32_t *dof_int = nullptr;   // [n_dofs] user -> internal DOF id
    int32_t *tri_int = nullptr;   // [n_tris] user -> internal triangle id
    int32_t *prev_elem = nullptr; // [n_dofs] internal tri of the last location (strategy b)
    int32_t *jump = nullptr;      // [jump_g * jump_g] bucket grid of start triangles (internal)
    int jump_g = 1;
    // quadtree (non-walking locator): nodes {first child or -1, list begin,
    // list count, 0}, leaf lists of internal triangle ids, root square
    int4 *qt_nodes = nullptr;
    int32_t *qt_lists = nullptr;
    double qt_box[3] = {0, 0, 0};  // x0, y0, side
    int qt_depth = 0;              // deepest leaf
    int64_t qt_n_nodes = 0, qt_n_list = 0;
    int32_t *bnext = nullptr;     // [n_nodes] next boundary node, counter-clockwise (-1: interior node)
    int32_t *bprev = nullptr;     // [n_nodes] previous boundary node
    int64_t n_boundary = 0;
    // a domain that is not one convex disk (reflex corners, holes, several
    // pieces): a walk blocked by the boundary ends in an exact search (the
    // quadtree below, built at upload); boundary crossings of the variable
    // step scan every boundary edge
    int nonconvex = 0;
    int n_loops = 0;               // boundary loops
    int32_t *bedge = nullptr;      // [n_boundary] internal node a of every boundary edge a -> bnext[a]
    // non-convex domains: uniform grid over the boundary edges (bg_g x bg_g
    // square cells of side bg_cell from (bg_x0, bg_y0)); cell c lists the
    // indices into bedge of the edges whose padded bounding box meets it
    int32_t *bg_ptr = nullptr;   // [bg_g^2 + 1]
    int32_t *bg_list = nullptr;
    int bg_g = 0;
    double bg_x0 = 0.0, bg_y0 = 0.0, bg_cell = 1.0;
    // boundary data for feet outside the domain (variable step); kind 0: none
    int bc_kind = 0;
    double bc_p[4] = {0, 0, 0, 0};
    // chart starts (learned and exact): chart coordinates of triangle
    // centroids and of DOFs, the start table, the quantile tables that give
    // a point's chart cell, the attached network and a start workspace
    float2 *chart_uv = nullptr;       // [n_tris]
    float2 *chart_node = nullptr;     // [n_dofs]
    int32_t *chart_table = nullptr;   // [chart_g * chart_g] internal triangle ids
    float *chart_qx = nullptr;        // [chart_g] smallest centroid x of each u slab
    float *chart_qy = nullptr;        // [chart_g * chart_g] smallest centroid y of each cell of a slab
    int chart_g = 0;
    // jump-and-walk start grid (slw_mesh_build_grid): grid_g x grid_g square
    // cells from (grid_x0, grid_y0), internal id of a triangle holding each
    // cell's centre (or near it)
    int32_t *grid = nullptr;
    int grid_g = 0;
    double grid_x0 = 0.0, grid_y0 = 0.0, grid_inv = 0.0;  // cells per unit length
    int32_t *learned_start = nullptr; // [n_dofs]
    struct slw_mlp *mlp = nullptr;    // borrowed
    // host copies kept for queries about the mesh
    std::vector<double> dof_xy_user_h;  // n_dofs x 2, user order
    std::vector<int32_t> dof_user_h;    // internal -> user
    int64_t device_bytes = 0;
    int32_t step_cap = 4096;
    int32_t hard_limit = 1 << 22;
    float hybrid_far = 0.0f;  // SLW_START_HYBRID: feet farther than this many heights of their previous element start afresh (0: automatic)
    int repack = 0;  // step kernel: 0 one foot per lane; 2, 4, 8: chunks of 64 x repack feet per wavefront
    int chain = 0;   // strategy (c): 0 the mesh forest below; 2, 4, 8, 16 Morton chains of that length per lane
    int xcd_chunk = 64;  // tiles per XCD turn: 0 one contiguous range of tiles per XCD; C > 0 chunks of C tiles dealt round-robin
    int lds_w = 512;     // walk records staged in LDS per workgroup by the plain step (0: none)
    // strategy (c)'s forest (depth one): roots = a maximal independent set of
    // the nodes (greedy in internal order), every other DOF a child of an
    // adjacent root.  List = roots then children, each part in internal
    // order; out = the output row of each list entry (user DOF id for
    // user-order meshes, else the internal id); parent = internal id of the
    // root of each child (-1: none adjacent).  Suffix 1: the nodes (P1);
    // 2: every DOF (P2 meshes).  elem: the element found for each root.
    int32_t *forest_list1 = nullptr, *forest_out1 = nullptr, *forest_parent1 = nullptr;
    int32_t *forest_list2 = nullptr, *forest_out2 = nullptr, *forest_parent2 = nullptr;
    int64_t forest_nr1 = 0, forest_nr2 = 0;
    int32_t *forest_elem = nullptr;  // [n_dofs]
};

// Device counters accumulated by the kernels (all int64, see slw_stats).
// step_hist: walks by element changes, bin 0 = no change, bin b in [1, 14]
// = [2^(b-1), 2^b) changes, bin 15 = 2^14 or more.
constexpr int kHistBins = 16;
struct DevStats {
    unsigned long long feet, outside, walk_steps, max_steps, exact_tests, fp64_tests, fallback_walks,
        edge_ties, vertex_ties, hard_fail, boundary_searches, pad[5];
    unsigned long long step_hist[kHistBins];
};

}  // namespace slw

struct slw_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    slw::DevStats *stats = nullptr;  // device counters
    void *work = nullptr;            // grow-only workspace for permutations
    size_t work_bytes = 0;
};

struct slw_mesh {
    slw_ctx *ctx = nullptr;
    slw::DevMesh m;
};

// The start-proposal network 5 -> 64 -> 64 -> 2 (ReLU hidden layers):
// FP32 master parameters, Adam moments, gradient buffers, input
// normalisation, and the weights repacked as bfloat16 in the per-lane
// operand layout of the matrix-core forward pass.
struct slw_mlp {
    slw_ctx *ctx = nullptr;
    float *params = nullptr;   // [kMlpParams]
    float *adam_m = nullptr, *adam_v = nullptr;
    float *grad = nullptr;     // [kMlpParams]
    float *partial = nullptr;  // [kMlpPartials * (kMlpParams + 2)]
    float *norm = nullptr;     // [10]: shift[5], scale[5]
    uint16_t *wpack = nullptr; // bfloat16 operands, see the forward kernel
    float *bias = nullptr;     // [64 + 64 + 16] biases in accumulator order
    int64_t adam_t = 0;
};

namespace slw {
// where a step keeps its counters and its permutation workspace: stats ==
// nullptr selects the context's (counters from slw_ctx_create, workspace
// grown on demand); otherwise the given memory, work_bytes at most
struct StepScratch {
    DevStats *stats = nullptr;
    void *work = nullptr;
    size_t work_bytes = 0;
};
slw_status step_impl(slw_mesh *mesh, const slw_field *field, double t_n, double dt, int scheme, int order,
                     int start_mode, const int32_t *start, const void *v_in, int vdtype, int k, void *v_out,
                     double outside_value, int32_t *elem, slw_stats *stats_h, const StepScratch &sc,
                     const char *who);
slw_status copy_stats(slw_ctx *ctx, const DevStats *counters, slw_stats *stats_h);
// resolves, once per device, the device address of the no-allocation
// entry point's static scratch array (slw_noalloc.hip); the device must be
// current
slw_status noalloc_init(int device);
slw_status set_error(slw_status s, const std::string &msg);
slw_status hip_check(hipError_t e, const char *what);
slw_status ensure_work(slw_ctx *ctx, size_t bytes);
bool field_ok(const slw_field *f);
struct FieldDev;
FieldDev to_dev(const slw_field *f);

// makes a device current for the lifetime of the guard
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

constexpr int kMlpParams = 5 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2;  // 4674
constexpr int kMlpPartials = 1024;                                   // workgroups per gradient pass

// mesh construction (slw_mesh.cpp)
slw_status build_mesh(slw_ctx *ctx, const double *xy, int64_t n, const int32_t *tri, int64_t nt, uint32_t flags,
                      DevMesh &out, bool to_device);
void free_mesh(DevMesh &m);
// quadtree over the triangles geo (internal order; exact coordinates from the
// mesh's host copies): see slw_quadtree_build
slw_status build_quadtree(DevMesh &m, const std::vector<GeoRec> &geo, int leaf_cap, int max_depth);
// coefficients of the walk's float filter for a mesh whose float coordinates
// are fl32(x - (cx, cy)) with |x - c| <= cmax (f32: coordinates already float)
FilterConst filter_constants(bool f32, double cx, double cy, double cmax);
// walk records of the records geo, neighbour offsets coded when they fit in
// `bits` bits (2 <= bits <= kCodeBits), escaped otherwise
std::vector<WalkRec> walk_records(const std::vector<GeoRec> &geo, int bits);

// launchers (slw_kernels.hip)

// A step over a list of DOFs instead of all of them (strategy (c)'s roots or
// children): list[pos] = internal DOF id, out[pos] = its output row,
// parent[pos] = the root whose element it starts from (children only),
// elem[d] = element found for root d.
struct ForestView {
    const int32_t *list = nullptr;
    const int32_t *out = nullptr;
    const int32_t *parent = nullptr;
    int32_t *elem = nullptr;
};

// Everything a kernel needs to know about a mesh (device pointers, sizes,
// filter constants), passed by value.
struct MeshView {
    const GeoRec *geo;
    const WalkRec *wrec;
    const int4 *tri_v;
    const int32_t *tri_uf;
    const int4 *tedge;
    const void *dof_xy;
    const int4 *qstart;
    const int32_t *vmin;
    const int32_t *dof_user;
    const int32_t *tri_int;
    int32_t *prev;
    const int32_t *jump;
    int jump_g;
    int internal_order;
    int64_t n_dofs;
    int64_t n_tris;
    double bb[4];
    FilterConst fc;
    int32_t step_cap, hard_limit;
    float hybrid_far;
    int xcd_chunk;
    int lds_w;
    // variable step at the boundary (bc_kind 0: off)
    const int32_t *bnext, *bprev;
    int64_t n_boundary;
    // non-convex domains: exact search of a blocked foot (quadtree) and the
    // boundary edges for crossings
    int nonconvex;
    const int4 *qt_nodes;
    const int32_t *qt_lists;
    double qt_box[3];
    int qt_depth;
    const int32_t *bedge;
    const int32_t *bg_ptr, *bg_list;
    int bg_g;
    double bg_x0, bg_y0, bg_cell;
    int bc_kind;
    double bc_p[4];
    // chart starts (null without a chart / network)
    const float2 *chart_node;
    const float *chart_qx, *chart_qy;
    const int32_t *chart_table;
    int chart_g;
    const int32_t *grid;
    int grid_g;
    double grid_x0, grid_y0, grid_inv;
    const uint16_t *mlp_wpack;
    const float *mlp_bias, *mlp_norm;
};
MeshView view_of(const DevMesh &m);

struct FieldDev {
    int kind;
    double p[8];
    // time-dependent factors of the two evaluation times of a step, computed
    // on the host: [0] at t_{n+1}, [1] at t_{n+1} - dt/2 (midpoint stage).
    // swirl: cos(pi t / p0); rotating field: p1 t.
    double g[2];
};
// fill FieldDev::g for evaluation times t_np1 and t_np1 - dt/2
void field_time_factors(FieldDev &f, double t_np1, double dt);

hipError_t launch_locate(const DevMesh &m, hipStream_t st, const void *q, int64_t m_pts, const int32_t *start,
                         int32_t *elem, void *bary, int32_t *steps, DevStats *stats);
hipError_t launch_qt_locate(const DevMesh &m, hipStream_t st, const void *q, int64_t m_pts, int32_t *elem, void *bary,
                            DevStats *stats);
hipError_t launch_grid_build(const DevMesh &m, hipStream_t st, int32_t *grid, int g, double x0, double y0,
                             double cell);
hipError_t launch_prev_clear_skip(hipStream_t st, int32_t *prev, int64_t n);
hipError_t launch_locate_feet(const DevMesh &m, hipStream_t st, const FieldDev *f, double t_np1, double dt,
                              int scheme, int start_mode, const int32_t *start, bool feet_in, void *feet,
                              int32_t *elem, void *bary, int32_t *steps, DevStats *stats);
hipError_t launch_interp(const DevMesh &m, hipStream_t st, int order, const int32_t *elem, const void *bary,
                         int64_t m_pts, const void *v_in, int vdtype, int k, void *v_out, double outside,
                         bool user_order);
hipError_t launch_step(const DevMesh &m, hipStream_t st, const FieldDev &f, double t_n, double dt, int scheme,
                       int order, int start_mode, const int32_t *start, const void *v_in, int vdtype, int k,
                       void *v_out, double outside, bool write_prev, const int32_t *out_map, int32_t *elem_out,
                       DevStats *stats);
hipError_t launch_zero_stats(hipStream_t st, DevStats *p);
// chart starts (the mesh needs a chart; kind 0: the exact chart cell of the
// foot; 1: the attached network's cell; 2: the network's cell corrected by
// galloping searches to the foot's own cell)
hipError_t launch_chart_start(const DevMesh &m, hipStream_t st, const FieldDev &f, double t_np1, double dt,
                              int scheme, const void *feet_in, int64_t n_iter, int kind, int32_t *start);
hipError_t launch_learned_gather(const DevMesh &m, hipStream_t st, const FieldDev &f, double t_np1, double dt,
                                 int scheme, const int32_t *dofs, int64_t cnt, float *X, float *Y);

// one mesh of a batch (device table; see slw_batch_* in slwalk.h)
struct BatchItem {
    MeshView mv;
    FieldDev f;      // g is filled on the device for each step
    double dt, t0;   // step n advances from t0 + n dt to t0 + (n + 1) dt
    const void *va;  // even steps read va and write vb, odd steps the reverse
    void *vb;
    int32_t *elem;   // nullable: user triangle id of each node's foot (-1 outside), internal node order
    int64_t n_iter;  // DOFs stepped (the nodes: P1)
    int64_t tile0;   // first tile of this mesh in the concatenated tile space
    int start_mode;  // SLW_START_STEERED or SLW_START_PREV (the mesh's previous elements)
};
hipError_t launch_batch_step(hipStream_t st, int coords_f32, int vdtype, int block, int schedule,
                             const BatchItem *items, int n_items, int64_t total_tiles, int64_t *counter, int scheme,
                             int k, double outside, unsigned *queues, int persistent_blocks, DevStats *stats);
hipError_t launch_permute_rows(hipStream_t st, const void *src, void *dst, int64_t rows, int64_t row_bytes,
                               const int32_t *map, int scatter);
}  // namespace slw
