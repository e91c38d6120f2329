/*
 * slwalk — characteristic-foot location and interpolation on unstructured
 * triangular meshes, for MI355X (gfx950).
 *
 * Method: Cacace & Ferretti, "Efficient implementation of characteristic-
 * based schemes on unstructured triangular grids", arXiv 2104.09189.
 *   - semi-Lagrangian step v_i^{n+1} = I[V^n](X^Delta(x_i, t_{n+1}; t_n)),
 *     eq. (schema_trasp);
 *   - foot by explicit Euler backward in time, eq. (eulero), or by the
 *     explicit midpoint rule (the higher-order ODE solver that Section 3
 *     leaves open);
 *   - point location by the barycentric walk of Section 2.2 (stop when all
 *     barycentric coordinates are >= 0, else cross the edge opposite the
 *     most negative one), started from the node's own incident triangles as
 *     in strategy (a) of Section 3, with the incident triangle chosen by the
 *     direction of the foot; strategy (b) (start from the previous step's
 *     element) is available as a start mode;
 *   - P1 interpolation with the barycentric weights (Remark after
 *     eq. barycoords) and P2 Lagrange interpolation.
 *
 * Conventions shared by every call
 *   - Indices are 0-based.  Triangle ids at this interface are always the
 *     user's ids (the position in the tri array given to slw_mesh_upload).
 *   - Degrees of freedom (DOFs): for P1 the nodes; for P2 the nodes followed
 *     by the edge midpoints, edges numbered in lexicographic order of their
 *     (min, max) user vertex pair.  DOF-indexed arrays (v_in, v_out, feet,
 *     elem and steps of slw_locate_feet, start) follow the user's DOF order,
 *     unless the mesh was uploaded with SLW_INTERNAL_ORDER; then they follow
 *     the library's internal (Morton) order, obtainable with
 *     slw_mesh_dof_order.  The internal order avoids two permutation passes
 *     per call.
 *   - Pointers without the _h suffix are device pointers (e.g. the
 *     data_ptr() of a torch tensor on the context's device) and stay owned
 *     by the caller; _h pointers are host memory.  The library owns only
 *     what it allocates inside a handle, and frees it in the destroy/free
 *     call.
 *   - Coordinates, feet and barycentric coordinates use the mesh's
 *     coordinate type (double, or float with SLW_COORDS_F32).  Values use
 *     the vdtype given to each call (SLW_F64 or SLW_F32) and are node-major:
 *     v[dof * k + field].
 *   - Every call returns SLW_OK or an error code; slw_last_error() then
 *     describes the failure (thread-local).  Outputs are unspecified after an
 *     error.  Kernel launches are asynchronous on the context's stream: the
 *     caller synchronises before reading outputs on the host.  A call that
 *     returns statistics (stats_h) synchronises the stream itself.
 *   - Location results are exact: every stop/move/outside decision uses the
 *     exact sign of an orientation determinant (filtered floating point,
 *     then exact expansion arithmetic), so the element returned does not
 *     depend on the start element, the walk path, the precision mode or the
 *     launch configuration.  When a point lies on an edge or a vertex (several
 *     closed triangles contain it), the result is the smallest user triangle
 *     id among them.  A point contained in no triangle gets elem = -1
 *     ("outside"), NaN barycentric coordinates and outside_value as value.
 *   - Exactness domain: mesh coordinates must be finite and either 0 or of
 *     magnitude in [2^-100, 2^100] (checked at upload); query coordinates
 *     may be any double (non-finite ones, and points outside the mesh's
 *     bounding box, are outside).
 *   - Teardown order: free every handle (graphs, batches, networks,
 *     meshes, then contexts) while the HIP runtime is still loaded, i.e.
 *     before the process's exit handlers unload it.  A handle released after
 *     that (for instance by a garbage collector running during interpreter
 *     shutdown) calls hipFree on a runtime that is gone, which can crash the
 *     process at exit; the Python binding frees all live handles from an
 *     exit hook registered after the runtime was loaded, which runs first.
 *   - The mesh must be conforming (every edge shared by at most two
 *     triangles, consistently oriented), free of zero-area triangles, and
 *     its boundary a manifold (no node where the boundary passes twice).
 *     When the domain is one convex disk (one boundary loop, no reflex
 *     corner), a walk that meets the boundary with the foot beyond it
 *     proves the foot outside.  Otherwise (reflex corners, holes, several
 *     pieces: slw_mesh_info.nonconvex) the foot may lie across a notch or a
 *     hole: such a walk ends in an exact search (a quadtree over the
 *     triangles, built at upload, whose leaf is scanned with the walk's exact
 *     signs: the smallest user id among the closed containers, or outside
 *     when there is none), so results are the same as on convex meshes.
 */
#ifndef SLWALK_H
#define SLWALK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum slw_status {
    SLW_OK = 0,
    SLW_E_ARG = 1,                /* invalid argument (null, size, enum) */
    SLW_E_MESH_INDEX = 2,         /* triangle vertex index out of range */
    SLW_E_MESH_DEGENERATE = 3,    /* zero-area triangle or repeated vertex */
    SLW_E_MESH_NONCONFORMING = 4, /* edge in >2 triangles, or overlapping pair */
    SLW_E_MESH_NONCONVEX = 5,     /* boundary not one convex loop */
    SLW_E_MESH_RANGE = 6,         /* coordinate not finite or outside the exactness domain */
    SLW_E_HIP = 7,                /* HIP runtime error (message has the HIP error string) */
    SLW_E_NOMEM = 8,              /* device or host allocation failed */
    SLW_E_UNSUPPORTED = 9,        /* valid request that this build does not handle */
    SLW_E_WALK = 10               /* a walk exceeded the hard step limit */
} slw_status;

typedef struct slw_ctx slw_ctx;
typedef struct slw_mesh slw_mesh;
typedef struct slw_mlp slw_mlp;

/* dtype codes */
enum { SLW_F64 = 0, SLW_F32 = 1 };
/* foot schemes: eq. (eulero); explicit midpoint */
enum { SLW_EULER = 0, SLW_RK2 = 1 };
/* start modes of slw_locate_feet / slw_step */
enum {
    SLW_START_STEERED = 0, /* strategy (a): the DOF's incident triangle facing the foot */
    SLW_START_GIVEN = 1,   /* start[dof] = user triangle id */
    SLW_START_PREV = 2,    /* strategy (b): the element found for this DOF by the previous
                              SLW_START_PREV call on this mesh (steered when there is none);
                              meshes of fewer than 2^29 triangles (SLW_E_UNSUPPORTED) */
    SLW_START_FIXED = 3,   /* every walk starts at user triangle start[0] (the paper's
                              fixed-start baseline, Section 2.2 complexity) */
    SLW_START_LEARNED = 4, /* the triangle proposed by the network attached with
                              slw_mesh_attach_mlp (learned start; see below) */
    SLW_START_CHART = 5,   /* the start-table triangle of the foot's own chart cell
                              (exact chart lookup, no network; needs slw_chart_build) */
    SLW_START_NEIGHBOR = 6, /* strategy (c): the element found for a neighbouring node, its
                              parent in a spanning forest of the internal-order nodes
                              (slw_step only; see slw_mesh_set_chain) */
    SLW_START_LEARNED_INDEX = 7, /* a learned index: the network's chart cell as the guess of
                              galloping searches in the chart's quantile tables, which end
                              in the foot's own cell (the start of SLW_START_CHART) */
    SLW_START_HYBRID = 8,  /* chosen per foot from how far it moved (slw_step only; see
                              slw_mesh_set_hybrid): the previous element (as SLW_START_PREV)
                              when the foot is in it or near it, else the foot's cell of the
                              start grid (as SLW_START_GRID) when the mesh has one, else its
                              chart cell (as SLW_START_CHART) when the mesh has a chart, else
                              the steered start; keeps the previous elements as SLW_START_PREV.
                              With a grid or a chart, a foot found far from its previous
                              element goes straight to the grid or chart for the next three
                              steps, then is tested again */
    SLW_START_GRID = 9     /* the triangle recorded for the foot's cell of the uniform start
                              grid (jump-and-walk; needs slw_mesh_build_grid) */
};
/* slw_mesh_upload flags */
#define SLW_COORDS_F32 0x1u     /* store coordinates as float (FP32 walk, FP64/exact fallback) */
#define SLW_P2 0x2u             /* build P2 edge DOFs */
#define SLW_NO_REORDER 0x4u     /* keep the user's node/triangle order internally */
#define SLW_INTERNAL_ORDER 0x8u /* DOF-indexed arrays at this interface use the internal order */
#define SLW_HILBERT 0x10u       /* order along the Hilbert curve instead of the Morton curve (measured:
                                   faster for short walks and one launch per mesh, slower for the long
                                   walks of a graded mesh) */
/* slw_locate_feet flags */
#define SLW_FEET_IN 0x1u        /* feet are an input (not computed from the field) */

/* Advecting field f(x, t).  kind / parameters p[0..7]:
 *   0 constant:     f = (p0, p1)
 *   1 solid body:   f = p0 * (-(y - p2), x - p1)
 *   2 swirl:        f = cos(pi t / p0) (sin^2(pi x) sin(2 pi y), -sin^2(pi y) sin(2 pi x))
 *   3 rotating field of Section 4: f = (cos a, sin a), a = p0 |x - (p2, p3)| + p1 t
 *   4 affine:       f = [[p0, p1], [p2, p3]] (x - (p4, p5)) + (p6, p7)            */
typedef struct slw_field {
    int32_t kind;
    int32_t reserved;
    double p[8];
} slw_field;

/* Per-call statistics (device counters copied back when stats_h != NULL). */
typedef struct slw_stats {
    int64_t feet;           /* feet located */
    int64_t outside;        /* feet with no containing triangle (incl. non-finite) */
    int64_t walk_steps;     /* element changes summed over feet (Section 2.2 walk steps) */
    int64_t max_steps;      /* longest walk */
    int64_t exact_tests;    /* orientation signs decided by exact arithmetic */
    int64_t fp64_tests;     /* FP32 meshes: signs decided by the FP64 stage */
    int64_t fallback_walks; /* walks that reached the step cap and finished randomised */
    int64_t edge_ties;      /* feet on an edge shared by two triangles */
    int64_t vertex_ties;    /* feet on a mesh vertex */
    int64_t boundary_searches; /* non-convex domains: walks blocked by the boundary and ended by
                                  the exact search (located inside, or proven outside) */
    int64_t reserved[6];
    /* Walks by length (Section 2.2 walk steps = element changes): bin 0 counts
     * walks with no change (feet outside the bounding box included), bin b
     * for 1 <= b <= 14 those with [2^(b-1), 2^b) changes, bin 15 those with
     * 2^14 or more.  The bins add up to `feet` (slw_locate_quadtree, which
     * does not walk, leaves them 0). */
    int64_t step_hist[16];
} slw_stats;

typedef struct slw_mesh_info {
    int64_t n_nodes, n_tris, n_edges, n_dofs; /* n_edges, n_dofs: P2 only (else 0, n_nodes) */
    int64_t device_bytes;                     /* device memory held by the handle */
    int32_t coords_f32, p2, reordered, internal_order;
    int32_t nonconvex;                        /* 1: the domain is not one convex disk (see conventions) */
    int32_t boundary_loops;                   /* number of boundary loops (1 + holes, for one piece) */
    double bbox[4];                           /* xmin, ymin, xmax, ymax */
} slw_mesh_info;

const char *slw_status_string(slw_status s);
/* Message for the last failing call on this thread ("" if none). */
const char *slw_last_error(void);

/* Context: one device and one stream (hipStream_t as void*, NULL = the null
 * stream).  The stream is borrowed, never destroyed by the library. */
slw_status slw_ctx_create(int device, void *hip_stream, slw_ctx **out);
slw_status slw_ctx_set_stream(slw_ctx *ctx, void *hip_stream);
void slw_ctx_destroy(slw_ctx *ctx);

/* Mesh upload: validates the triangulation (host arrays xy_h n x 2,
 * tri_h nt x 3), flips clockwise triangles to counter-clockwise (the
 * barycentric coordinates returned still follow the user's vertex order),
 * builds the neighbour lists of Section 3 (neighbour k across the edge
 * opposite vertex k, -1 on the boundary), the incident-triangle lists of
 * every DOF with their edge directions (start selection), the P2 edge DOFs,
 * and a Morton (or, with SLW_HILBERT, Hilbert) order of nodes and triangles
 * (unless SLW_NO_REORDER), and
 * copies the result to the device.  Synchronous. */
slw_status slw_mesh_upload(slw_ctx *ctx, const double *xy_h, int64_t n_nodes, const int32_t *tri_h,
                           int64_t n_tris, uint32_t flags, slw_mesh **out);
/* The host half of slw_mesh_upload alone: the same validation and
 * preprocessing, no device and no allocation that outlives the call.
 * info_h (nullable) receives the sizes the upload would produce. */
slw_status slw_mesh_check(const double *xy_h, int64_t n_nodes, const int32_t *tri_h, int64_t n_tris,
                          uint32_t flags, slw_mesh_info *info_h);
slw_status slw_mesh_free(slw_mesh *mesh);
slw_status slw_mesh_get_info(const slw_mesh *mesh, slw_mesh_info *out_h);
/* DOF coordinates (n_dofs x 2 doubles, host) in the DOF order of this
 * interface (user order, or internal with SLW_INTERNAL_ORDER). */
slw_status slw_mesh_dof_coords(const slw_mesh *mesh, double *xy_h);
/* internal position -> user DOF id (n_dofs ints, host). */
slw_status slw_mesh_dof_order(const slw_mesh *mesh, int32_t *user_of_internal_h);
/* Step cap after which a walk switches to the randomised remembering walk
 * (default 4096), and the hard limit that fails with SLW_E_WALK
 * (default 1 << 22).  Either value <= 0 keeps the current one. */
slw_status slw_mesh_set_walk_limits(slw_mesh *mesh, int32_t step_cap, int32_t hard_limit);
/* Lane schedule of slw_step: with feet_per_lane = 1 every lane of a
 * wavefront walks one foot and the wavefront ends with its longest walk;
 * with 2, 4 or 8 each wavefront owns 64 x feet_per_lane consecutive DOFs and
 * a lane whose walk ends starts the next unstarted one (lane repacking), so
 * the wavefront's time follows the sum of its walks rather than their
 * maximum.  Results are identical for every setting.  0 selects the
 * library's default. */
slw_status slw_mesh_set_repack(slw_mesh *mesh, int feet_per_lane);
/* Width of the neighbour offsets in the walk's 32-byte triangle records.
 * A walk move reads the float vertex coordinates and the three neighbours
 * of one triangle; the neighbours are stored as offsets from the triangle's
 * own (Morton-ordered) id, in `bits`-bit two's complement (2 <= bits <= 21;
 * 0 selects the default 21), and a neighbour whose offset does not fit is
 * read from the full record instead.  Narrower codes only add such escapes:
 * results are identical for every setting.  Rebuilds the records (a device
 * to host to device copy of the mesh's triangle records; synchronous). */
slw_status slw_mesh_set_neighbour_codes(slw_mesh *mesh, int bits);
/* Boundary data for feet that leave the domain (slw_step).  The paper
 * treats Dirichlet conditions by a variable step that stops characteristics
 * on the boundary (remark after eq. eulero).  With kind != SLW_BC_NONE a
 * DOF x whose foot q lies outside the domain gets the value
 * g(p, t_{n+1} - theta dt), where p = x + theta (q - x), theta in [0, 1], is
 * the point where the segment from x to q leaves the domain, and
 * g = p[0] (SLW_BC_CONSTANT) or g = p[0] + p[1] px + p[2] py + p[3] t
 * (SLW_BC_AFFINE), for every field.  SLW_BC_NONE (the default) gives such
 * feet outside_value.  Applied by the one-foot-per-lane step kernel (the
 * lane schedule is ignored while set); not available with the chains of
 * SLW_START_NEIGHBOR (SLW_E_UNSUPPORTED).  p_h: 4 doubles (host), ignored for
 * SLW_BC_NONE. */
enum { SLW_BC_NONE = 0, SLW_BC_CONSTANT = 1, SLW_BC_AFFINE = 2 };
slw_status slw_mesh_set_boundary(slw_mesh *mesh, int kind, const double *p_h);
/* Strategy (c) of Section 3 (SLW_START_NEIGHBOR) starts a walk from the
 * element that contains an adjacent node's foot (its parent in a spanning
 * tree).  The paper's breadth-first tree has about sqrt(N) sequential levels;
 * the spanning forests used here are shallow:
 *   length 0 (the default): a forest of depth one built at upload.  Its
 *     roots are nodes no two of which lie within three hops (mesh edges) of
 *     each other (greedy in internal order, a maximal such set); every other
 *     DOF is a child of the nearest root within three hops.  The
 *     roots are stepped first (from their cell of the start grid when the mesh
 *     has one, slw_mesh_build_grid, else strategy (a)), then the children, each
 *     from its parent's element unless its own node lies nearer its foot than
 *     the parent node (then strategy (a)): two kernel launches per step.
 *     Boundary data (slw_mesh_set_boundary) apply.
 *   length 2, 4, 8 or 16: chains of that many consecutive internal-order
 *     nodes, one chain per lane: the first foot of a chain starts as strategy
 *     (a), each later one from the element found for its predecessor unless
 *     its own steered start lies nearer (no boundary data:
 *     SLW_E_UNSUPPORTED).
 * Results never depend on the forest. */
slw_status slw_mesh_set_chain(slw_mesh *mesh, int length);

/* Schedule knob: how the tiles of 256 consecutive internal-order DOFs are
 * spread over the 8 XCDs (workgroups go to the XCDs in turn).  chunk 0: one
 * contiguous range of tiles per XCD (locality in each XCD's L2); chunk C in
 * 1 ... 4096: chunks of C consecutive tiles dealt to the XCDs in turn (even
 * work per XCD where walk lengths differ between regions of the mesh).
 * Default 64.  Applies to the step, location and interpolation kernels of
 * this mesh, not to batches.  Results never depend on it;
 * SLW_E_ARG outside 0 ... 4096. */
slw_status slw_mesh_set_xcd_chunk(slw_mesh *mesh, int chunk);

/* Schedule knob of the plain step (one foot per lane; starts steered, given
 * or fixed; P1): each workgroup first copies `records` walk records around
 * its tile (triangles and DOFs share the Morton order) into LDS, and its
 * walks read the records of that window from LDS instead of memory.  0
 * turns it off; default 512 (16 KB per workgroup); 64 ... 2048, else
 * SLW_E_ARG.  Results never depend on it. */
slw_status slw_mesh_set_lds_window(slw_mesh *mesh, int records);

/* Jump-and-walk start grid (a bucketing start, Section 2.1's prior art;
 * Muecke, Saias and Zhu 1996): g x g square cells over the mesh's bounding
 * box (side = the box's longer side / g), each recording a triangle that
 * holds its centre, found by the library's own walk at build time (a centre
 * outside the mesh records a nearby triangle).  Starts of SLW_START_GRID and
 * the far feet of SLW_START_HYBRID read one cell.  g in 16 ... 16384 (4 g^2
 * bytes of device memory, replacing an earlier grid); g = 0 removes it.
 * Synchronous.  Results never depend on it. */
slw_status slw_mesh_build_grid(slw_mesh *mesh, int g);
/* The per-foot choice of SLW_START_HYBRID, after the hybrid idea that closes
 * the numerical section (Section 4) of the paper: the start is chosen from
 * the local dynamics, i.e. from how far the foot moved since the previous
 * step.  The foot is first tested against the element found for the DOF at
 * the previous SLW_START_PREV / SLW_START_HYBRID step; if it lies outside,
 * theta_min, its smallest barycentric coordinate there, measures how far
 * (about -theta_min heights of that element beyond its nearest side).  With
 * theta_min > -far the walk continues from the previous element; otherwise
 * (and without a previous element) it starts from the foot's cell of the
 * start grid when slw_mesh_build_grid was called, else from its chart cell
 * when slw_chart_build was called, else from the steered start.  far > 0, or
 * 0 (the default) for the measured best of each case: 1 with a grid, 16 with
 * a chart alone, 64 with neither.  Negative or non-finite: SLW_E_ARG.
 * Results never depend on it. */
slw_status slw_mesh_set_hybrid(slw_mesh *mesh, float far);

/* General point location, the analogue of the paper's [I, B] =
 * pointLocationBW(TBW, Q, s): m query points q (m x 2, mesh coordinate type)
 * -> elem (m ints, user triangle ids, -1 outside), bary (m x 3 in the user's
 * vertex order of elem, nullable), steps (m ints, element changes, nullable).
 * start (nullable, m user triangle ids) gives each walk's first triangle;
 * when NULL the walk starts from a bucket grid of start triangles. */
slw_status slw_locate(slw_mesh *mesh, const void *q, int64_t m, const int32_t *start, int32_t *elem,
                      void *bary, int32_t *steps);

/* Feet of all DOFs at t_np1 with step dt (scheme SLW_EULER / SLW_RK2),
 * located by walks started per start_mode.  feet (n_dofs x 2, nullable)
 * receives the feet; with SLW_FEET_IN in flags it is read instead of
 * computed (field may then be NULL).  elem, bary, steps as in slw_locate
 * (bary and steps nullable; elem nullable too).  start is read for GIVEN
 * (n_dofs ids) and FIXED (one id). */
slw_status slw_locate_feet(slw_mesh *mesh, const slw_field *field, double t_np1, double dt, int scheme,
                           int start_mode, const int32_t *start, uint32_t flags, void *feet,
                           int32_t *elem, void *bary, int32_t *steps, slw_stats *stats_h);

/* Interpolation I[V](x) at m located points (elem, bary from slw_locate or
 * slw_locate_feet): order 1 (P1) or 2 (P2, needs an SLW_P2 mesh).  v_in is
 * n_dofs x k, v_out m x k, both of vdtype.  elem -1 gives outside_value. */
slw_status slw_interpolate(slw_mesh *mesh, int order, const int32_t *elem, const void *bary, int64_t m,
                           const void *v_in, int vdtype, int k, void *v_out, double outside_value);

/* One semi-Lagrangian step (Algorithm 2, one pass of its time loop), fused
 * in one kernel: foot at t_n + dt, start selection, walk, tie rule, weights,
 * and k values per DOF: v_out[i] = I[v_in](foot_i), outside_value for feet
 * outside the domain.  start_mode as in slw_locate_feet (GIVEN/FIXED read
 * start).  v_in and v_out must not overlap.  elem (nullable, device, one int
 * per stepped DOF: the nodes for order 1, every DOF for order 2, in the DOF
 * order of this interface) receives the user id of the triangle the step
 * located each foot in (-1 outside): the same element slw_locate_feet
 * returns for that foot. */
slw_status slw_step(slw_mesh *mesh, const slw_field *field, double t_n, double dt, int scheme, int order,
                    int start_mode, const int32_t *start, const void *v_in, int vdtype, int k,
                    void *v_out, double outside_value, int32_t *elem, slw_stats *stats_h);

/* Autotuner of slw_step's schedule: for the given step (arguments as
 * slw_step) it times every candidate value of the knob that matters for
 * start_mode -- the lane schedule of slw_mesh_set_repack (1, 2, 4, 8 feet
 * per lane) for the steered, given, fixed, previous, chart and learned
 * starts; the threshold of slw_mesh_set_hybrid (0.5 ... 64) for
 * SLW_START_HYBRID; the forest or chain length of slw_mesh_set_chain (0, 2,
 * 4, 8, 16) for SLW_START_NEIGHBOR -- then, for the value chosen, the XCD
 * chunk of slw_mesh_set_xcd_chunk (0, 16, 32, 64, 128), then for the plain
 * step (one foot per lane; steered, given or fixed starts; P1) the LDS
 * window of slw_mesh_set_lds_window (0, 256, 512, 768); each candidate
 * timed over five consecutive steps from t_n (the median), after one untimed
 * step from t_n - dt that starts from the mesh's previous elements (the
 * hybrid's skip counts cleared).  It keeps only candidates whose step is
 * bit-identical to the one of the mesh's current setting, applies the
 * fastest to the mesh and records it in
 * the JSON file cache_path (nullable) under a signature of the step (size,
 * types, k, order, start mode, scheme, and the walk-length regime: the
 * mean walk of strategy (a) on this step, in powers of two); a later call
 * with a cached signature applies the
 * cached value without timing.  Every candidate starts from the mesh's
 * current previous elements (SLW_START_PREV, SLW_START_HYBRID), which are
 * restored afterwards; the caller's v_in is only read.  Allocates a private
 * output buffer; synchronous.  value_out / xcd_chunk_out / ms_out
 * (nullable): the knob value and XCD chunk chosen and their median time per
 * step (ms; the cached time when the cache answered); the LDS window chosen
 * is applied to the mesh (and cached) too. */
slw_status slw_step_autotune(slw_mesh *mesh, const slw_field *field, double t_n, double dt, int scheme, int order,
                             int start_mode, const int32_t *start, const void *v_in, int vdtype, int k,
                             const char *cache_path, double *value_out, int32_t *xcd_chunk_out, double *ms_out);

/* slw_step for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as slw_step, but it calls no hipMalloc,
 * hipFree or allocating library routine: its statistics counters and the
 * workspace that permutes v_in into the internal order (user-order meshes
 * only) live in one static device array of 64 MiB that each GPU the library
 * runs on holds until the process ends (its address is resolved per device
 * by slw_ctx_create).  A user-order mesh needs rows x k x value-size bytes
 * of it (rows = n_nodes for order 1, n_dofs for order 2); more than
 * 64 MiB - 256 B fails with SLW_E_ARG before anything is launched
 * (SLW_INTERNAL_ORDER meshes need none).  Every call on a GPU shares that
 * GPU's array, and the array keeps the last call's contents (counters are
 * cleared by a kernel at the start of each call that returns statistics):
 * calls that overlap on one GPU -- on different streams or host threads --
 * race, and must be serialised by the caller.  With stats_h the call
 * synchronises the context's stream (as slw_step does). */
slw_status slw_step_noalloc(slw_mesh *mesh, const slw_field *field, double t_n, double dt, int scheme, int order,
                            int start_mode, const int32_t *start, const void *v_in, int vdtype, int k,
                            void *v_out, double outside_value, int32_t *elem, slw_stats *stats_h);

/* Permute a DOF-indexed array (n_dofs rows of row_bytes) between the user
 * order and the internal order (to_internal != 0: user -> internal). */
slw_status slw_permute_rows(slw_mesh *mesh, const void *src, void *dst, int64_t row_bytes, int to_internal);

/* ---------------------------------------------------------------------
 * Batches: many meshes advanced by one P1 step each in a single launch
 * (extension of the method to uneven workloads; each mesh is stepped exactly
 * as slw_step with SLW_START_STEERED would).  Work items are the meshes'
 * 256-DOF tiles (block-sized tiles), concatenated; schedule 0 gives each
 * workgroup one tile in an XCD-contiguous order, schedule 1 runs persistent
 * workgroups that pull tiles from per-XCD queues, schedule 2 gives each
 * workgroup one tile with chunks of 16,384 DOFs' tiles dealt to the XCDs in
 * turn.  The step index lives on
 * the device: step n of mesh i advances its values from t0_i + n dt_i to
 * t0_i + (n + 1) dt_i, reading va_i and writing vb_i when n is even and the
 * reverse when n is odd, then the index is incremented -- so a captured
 * graph of steps can be replayed and keeps advancing in time.
 * All meshes must share the coordinate type and use SLW_INTERNAL_ORDER.  The
 * batch references the meshes (they must outlive it).
 * ------------------------------------------------------------------- */
typedef struct slw_batch slw_batch;
typedef struct slw_graph slw_graph;

slw_status slw_batch_create(slw_ctx *ctx, slw_mesh *const *meshes_h, int n, slw_batch **out);
slw_status slw_batch_free(slw_batch *b);
/* fields_h[i], dt_h[i] and (nullable, default 0) t0_h[i] for each mesh */
slw_status slw_batch_set_fields(slw_batch *b, const slw_field *fields_h, const double *dt_h, const double *t0_h);
/* device value buffers va_h[i], vb_h[i] (n_nodes x k of vdtype, internal order) */
slw_status slw_batch_set_values(slw_batch *b, void *const *va_h, void *const *vb_h, int vdtype, int k);
/* Optional element output: elem_h[i] (device, n_nodes ints of mesh i,
 * internal order) receives the user id of the triangle each node's foot was
 * located in (-1 outside) at every later step; elem_h NULL (or an entry
 * NULL) turns it off.  Graphs captured afterwards keep the pointers. */
slw_status slw_batch_set_elem_out(slw_batch *b, int32_t *const *elem_h);
/* set / read the device step index (both synchronise the context's stream) */
slw_status slw_batch_set_step(slw_batch *b, int64_t n);
slw_status slw_batch_get_step(slw_batch *b, int64_t *n_h);
/* schedule 0 (static, XCD-contiguous), 1 (persistent queues) or 2 (static, XCD chunks); workgroup size
 * 64, 128, 256 or 512 */
slw_status slw_batch_set_schedule(slw_batch *b, int schedule, int block);
/* The start of every mesh's walks: SLW_START_STEERED (the default, strategy
 * (a)) or SLW_START_PREV (strategy (b), Section 3 (b): the element found for
 * the node at the mesh's previous SLW_START_PREV step, batched or not; the
 * steered start where there is none).  Graphs read the batch's item table
 * at each replay, so graphs captured earlier follow the new mode (and the
 * element outputs of slw_batch_set_elem_out); after slw_batch_set_schedule
 * or slw_batch_autotune changes the workgroup size, capture again.  Results
 * never depend on the mode.  SLW_E_ARG for other modes; SLW_E_UNSUPPORTED
 * for meshes of 2^29 triangles or more. */
slw_status slw_batch_set_start(slw_batch *b, int start_mode);
/* one step of every mesh (asynchronous unless stats_h is given) */
slw_status slw_batch_step(slw_batch *b, int scheme, double outside_value, slw_stats *stats_h);
/* Capture n_steps batch steps into a HIP graph (on a private stream; no
 * memset nodes: counters are cleared by kernels).  Replays run on the
 * context's stream and advance the device step index by n_steps. */
slw_status slw_batch_graph_capture(slw_batch *b, int n_steps, int scheme, double outside_value, slw_graph **out);
slw_status slw_graph_launch(slw_graph *g);
slw_status slw_graph_free(slw_graph *g);
/* Autotuner: times every (schedule, workgroup size) on private copies of the
 * batch's current values, keeps only candidates whose first step is bit-
 * identical to the reference candidate's, selects the fastest and records it
 * in the JSON file cache_path (nullable) under a signature of the batch
 * (mesh count, DOF count bucket, types, k, start mode); a later call with a
 * cached signature applies the cached choice without timing.  Synchronous;
 * the caller's values, step index and (with SLW_START_PREV) the meshes'
 * previous elements are left as they were. */
slw_status slw_batch_autotune(slw_batch *b, int scheme, const char *cache_path, int *schedule_out, int *block_out);

/* ------------------------------------------------------------------------
 * Learned start proposal.  A network (x, y, dx, dy, t) -> 64 -> 64 -> 2 with
 * ReLU maps a foot (node x, y; displacement dx, dy to the foot; time t =
 * t_{n+1}) to its displacement (du, dv) in a chart of the mesh; the node's
 * own chart coordinates plus (du, dv) give (u, v), a G x G table maps
 * (floor(u G), floor(v G)) to a start triangle, and the exact walk finishes
 * the search.  This follows the hybrid idea that closes the numerical
 * section (Section 4) of the paper: the start comes from local information
 * about the dynamics.  Results never depend on the network: the element
 * found is the walk's exact answer from any start (a bad network only costs
 * steps).  The chart is the Rosenblatt transform of the triangle-centroid
 * distribution: u = rank of the centroid's x among all centroids (in (0,1)),
 * v = rank of its y among the centroids of its u slab (slab = floor(u G)).
 * SLW_START_CHART finds the foot's chart cell exactly instead (binary
 * searches in the slabs' x and y quantiles): the same start without the
 * network, kept as the reference point for the learned one.
 *
 * Parameters: one float vector of 4674 numbers, W1 (5 x 64, input-major:
 * W1[i][j] at i * 64 + j), b1 (64), W2 (64 x 64), b2 (64), W3 (64 x 2), b3
 * (2); a layer computes act(h W + b).  Inputs are normalised as
 * (f - shift) * scale in float, norm = shift[5], scale[5].  Training is FP32
 * (own forward/backward kernels, Adam); inference uses bfloat16 operands
 * (round to nearest even) on the matrix cores with FP32 accumulation.
 * Sample arrays: X (device, m x 5 floats: x, y, dx, dy, t), Y (device, m x 2
 * floats: target du, dv; a NaN du marks a sample without target, which
 * counts in the batch size but not in the loss). */

/* Builds (or rebuilds) the chart of a mesh with a g x g start table
 * (1 <= g <= 8192), on the host from the device records; synchronous.
 * Device memory: 8 B per triangle, 12 B per DOF, 8 g^2 + 4 g B. */
slw_status slw_chart_build(slw_mesh *mesh, int g);
/* Chart coordinates of every triangle's centroid, user triangle order:
 * uv_h[2 t], uv_h[2 t + 1] (host, n_tris x 2); synchronous. */
slw_status slw_chart_coords(slw_mesh *mesh, float *uv_h);
/* New network on the context's device: He-uniform weights (limit
 * sqrt(6 / fan_in), from a splitmix64 stream seeded with seed), zero biases,
 * identity normalisation, zero Adam state.  Free with slw_mlp_free. */
slw_status slw_mlp_create(slw_ctx *ctx, uint64_t seed, slw_mlp **out);
slw_status slw_mlp_free(slw_mlp *n);
/* Host copies of the FP32 parameters (4674 floats) and the normalisation
 * (10 floats); setting parameters also refreshes the bfloat16 operands. */
slw_status slw_mlp_set_params(slw_mlp *n, const float *params_h);
slw_status slw_mlp_get_params(slw_mlp *n, float *params_h);
slw_status slw_mlp_set_normalization(slw_mlp *n, const float *norm_h);
slw_status slw_mlp_get_normalization(slw_mlp *n, float *norm_h);
/* shift = mean, scale = 1 / standard deviation (1 where it is 0) of each
 * input over the m samples X (FP64 sums). */
slw_status slw_mlp_fit_normalization(slw_mlp *n, const float *X, int64_t m);
/* Training samples from the plain walk: for the DOFs dofs[i] (device, m
 * ints, internal positions 0 .. n_dofs-1) the foot of the step ending at
 * t_np1 is computed and located with the strategy (a) start; X[i] gets the
 * foot's inputs, Y[i] the chart coordinates of the element found minus
 * those of the DOF (NaN when outside; out-of-range ids give zeros and NaN).
 * Needs a chart. */
slw_status slw_learned_gather(slw_mesh *mesh, const slw_field *field, double t_np1, double dt, int scheme,
                              const int32_t *dofs, int64_t m, float *X, float *Y);
/* Gradient of the loss = mean over the m samples of |out - Y|^2 (FP32,
 * per-workgroup partial sums added in a fixed order: bit-reproducible).
 * grad_h (host, 4674 floats) and loss_h (mean over samples with a target)
 * are nullable; synchronous. */
slw_status slw_mlp_grad(slw_mlp *n, const float *X, const float *Y, int64_t m, float *grad_h, float *loss_h);
/* Adam (beta 0.9, 0.999, eps 1e-8, step lr) over epochs passes of
 * minibatches of `batch` samples, the samples of each epoch in the order
 * i -> (a i + c) mod m with a, c drawn from seed; loss_h (nullable) gets
 * the loss of the last minibatch before its update; synchronous at the end. */
slw_status slw_mlp_train(slw_mlp *n, const float *X, const float *Y, int64_t m, int epochs, int64_t batch,
                         float lr, uint64_t seed, float *loss_h);
/* Network outputs (bfloat16 matrix-core path) of m samples: out (device,
 * m x 2 floats). */
slw_status slw_mlp_forward(slw_mlp *n, const float *X, int64_t m, float *out);
/* Attaches a network (borrowed: keep it alive while attached; NULL
 * detaches) to a mesh with a chart, for SLW_START_LEARNED. */
slw_status slw_mesh_attach_mlp(slw_mesh *mesh, slw_mlp *n);

/* ------------------------------------------------------------------------
 * Quadtree locator (non-walking, the search of Section 2.1), kept as a
 * comparator for the walks.  slw_quadtree_build splits the square around the
 * mesh's bounding box at its centre while a node lists more than leaf_cap
 * triangles (1 <= leaf_cap), is shallower than max_depth (<= 30) and the
 * split separates something (no child keeps all of the node's triangles); a
 * triangle is listed in every node its closed bounding box touches.  More
 * than 16 list entries per triangle fails with SLW_E_NOMEM.  Synchronous
 * (host build from the device records).  slw_locate_quadtree
 * answers like slw_locate (user triangle ids, smallest id among closed
 * containers, -1 and NaN outside, the same barycentric coordinates) by
 * testing every triangle of the query's leaf with exact signs; stats_h
 * (nullable) counts feet and outside points. */
slw_status slw_quadtree_build(slw_mesh *mesh, int leaf_cap, int max_depth);
slw_status slw_quadtree_info(const slw_mesh *mesh, int64_t *n_nodes_h, int64_t *n_list_h, int *depth_h);
slw_status slw_locate_quadtree(slw_mesh *mesh, const void *q, int64_t m, int32_t *elem, void *bary,
                               slw_stats *stats_h);

/* The library's orientation predicate evaluated on the host, for testing:
 * out_h[i] = sign of orient(a, b, c) for the triple pts_h[6i .. 6i+5] =
 * (ax, ay, bx, by, cx, cy).  mode 0: FP64 filter then exact stage (what a
 * double mesh's walk uses); 1: exact stage alone; 2: the float pipeline on
 * the inputs rounded to float (what a float mesh's walk uses).  Exact on
 * the exactness domain above. */
slw_status slw_orient_sign_host(const double *pts_h, int64_t m, int8_t *out_h, int mode);

/* The walk's float filter evaluated on the host, for testing its error
 * bound: for the triple pts_h[6i .. 6i+5] = (ax, ay, bx, by, qx, qy), the
 * coordinates are rounded to float the way a mesh stores them (minus the
 * centre (cx, cy), for a mesh whose largest |coordinate - centre| is cmax;
 * with f32 != 0 the coordinates themselves, as for a float mesh) and out_h[i]
 * is the filter's certified sign of orient(a, b, q), or 2 when it defers to
 * the exact stages. */
slw_status slw_float_filter_host(const double *pts_h, int64_t m, double cx, double cy, double cmax, int f32,
                                 int8_t *out_h);
/* Host copy of the neighbour coding of the walk records (for tests): for
 * triangles t = 0 .. n_tris-1 with neighbours nb_h[3t .. 3t+2] (-1 on the
 * boundary, ids in the same numbering as t), writes the two 32-bit words
 * (lo, hi) of each record's codes to words_h[2t], words_h[2t+1]: code k in
 * bits [21k, 21k + 21) of hi:lo, 0 for a boundary edge, -2^20 when the
 * offset nb - t does not fit in `bits` bits, else the offset. */
slw_status slw_walk_codes_host(const int32_t *nb_h, int64_t n_tris, int bits, uint32_t *words_h);

#ifdef __cplusplus
}
#endif
#endif
