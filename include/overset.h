/*
 * overset.h — C ABI of the MI355X (gfx950) overset grid-assembly library.
 *
 * The library computes, once per time step, the grid assembly and boundary
 * interpolation between a stationary curvilinear background grid and rigidly
 * moving curvilinear overset grids, after Hedayat & Borazjani, "A parallel
 * dynamic overset grid framework for immersed boundary methods"
 * (arXiv:1910.09315), Sec. 2.2 and Sec. 2.4. A step is five calls, each
 * asynchronous on the caller's HIP stream:
 *
 *   overset_holecut         blank nodes inside other grids' blank regions    (Sec. 2.2.2)
 *   overset_fringe_compact  mark query (fringe) points, compact them in order (Sec. 2.2.3, Alg. 1)
 *   overset_transform       query coordinates into the inertial frame        (Sec. 2.1, Sec. 2.2.3 item 6)
 *   overset_donor_search    donor cell + natural coordinates per query        (Sec. 2.2.5, Alg. 3; Sec. 2.4 item 1)
 *   overset_interp          trilinear gather of u, v, w, p                    (Sec. 2.2.6)
 *
 * Conventions
 *  - Pointers are DEVICE pointers unless marked [host]. The caller owns every
 *    buffer passed to a step call and the grid coordinate arrays given to
 *    ov_grid_add (which must stay alive and unchanged until ov_ctx_destroy).
 *    The library owns only what it allocates in ov_ctx_create / ov_grid_add /
 *    ov_finalize: control cells, FP32 coordinate shadows, warm-start history,
 *    device tables and scan scratch. Step calls allocate nothing and never
 *    synchronise the host, so a step can be captured in a HIP graph.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *  - A grid is (ni, nj, nk) nodes; node (i, j, k) has linear index
 *    i + ni*(j + nj*k) (the paper's local index, Sec. 2.2.6). Grid g's nodes
 *    occupy [node_off[g], node_off[g+1]) of every per-node array (flags,
 *    fields), grids in id order: the paper's packed per-process vector.
 *    A periodic direction of n nodes has n cells (the last wraps to node 0),
 *    otherwise n-1. Cell (ci, cj, ck) has linear index ci + nci*(cj + ncj*ck);
 *    its corner c = c0 + 2 c1 + 4 c2 is node (ci+c0, cj+c1, ck+c2).
 *  - Grid 0 is the background (identity pose); grids 1.. are overset grids.
 *  - A pose is 12 doubles: R (3x3 row-major) then c; a body-frame point X is
 *    at x = R X + c in the inertial frame (R is the transpose of the paper's
 *    rotation tensor Q, Sec. 2.1). `poses` arrays hold ngrids poses.
 *  - Flag byte per node: state in bits 0-1 (0 field, 1 hole, 2 fringe), cause
 *    grid in bits 2-7 (63 = outer boundary of an overset grid).
 *  - Errors: a negative ov_status is returned BEFORE any launch for bad
 *    arguments (message in ov_last_error). Conditions only the device can see
 *    set bits of a device status word read by ov_status_fetch. ORPHAN is a
 *    per-query result, not an error.
 *  - Precision is fixed per context: OV_FP64 keeps query coordinates, s,
 *    fields and outputs in double; OV_MIXED keeps them in float and runs the
 *    transform, walk, Newton and weights in FP32, followed by an FP64 Newton
 *    correction for points near a cell face or in ill-conditioned cells.
 *  - A context is not thread-safe; calls on one context are stream-ordered.
 */
#ifndef OVERSET_H
#define OVERSET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ov_ctx ov_ctx;

enum ov_status {
    OV_OK = 0,
    OV_EINVAL = -1,     /* bad pointer, id, option or size */
    OV_EDIMS = -2,      /* grid dimensions unusable (< 2 nodes along an axis, too many nodes) */
    OV_ECAPACITY = -3,  /* capacity below what the call needs (host-visible) */
    OV_EHIP = -4,       /* a HIP runtime call failed */
    OV_ESTATE = -5      /* call out of order (e.g. step before ov_finalize) */
};

enum ov_precision { OV_FP64 = 0, OV_MIXED = 1 };

enum ov_blank_kind {
    OV_BLANK_NONE = 0,
    OV_BLANK_CYL = 1,       /* prm: r, z0, z1 — x^2 + y^2 < r^2 and z0 <= z <= z1 (body frame) */
    OV_BLANK_SPHERE = 2,    /* prm: r         — x^2 + y^2 + z^2 < r^2 */
    OV_BLANK_ELLIPSOID = 3, /* prm: a, b, c   — (x/a)^2 + (y/b)^2 + (z/c)^2 < 1 */
    OV_BLANK_MESH = 4       /* a closed surface triangulation, set with ov_grid_set_blank_mesh */
};

/* Flag byte fields. */
#define OV_STATE_FIELD 0
#define OV_STATE_HOLE 1
#define OV_STATE_FRINGE 2
#define OV_CAUSE_BOUNDARY 63
#define OV_MAX_GRIDS 63

/* Per-query status written by overset_donor_search: a code in bits 0-1, the
 * FP64-correction flag in bit 2, and in bits 8-15 the number of cells the
 * walk visited (saturating at 255; a diagnostic). */
#define OV_Q_ORPHAN 0         /* no valid donor in any candidate grid */
#define OV_Q_FOUND 1          /* found by the stencil walk */
#define OV_Q_FALLBACK 2       /* found by the brute-force scan of the control cell */
#define OV_Q_FP64_FIXED 4     /* bit: the FP64 correction decided the donor (mixed precision) */

/* Device status word bits (ov_status_fetch). */
#define OV_DEV_CAPACITY 1     /* fringe count exceeded capacity; entries past capacity not written */
#define OV_DEV_WALK_LIMIT 2   /* at least one walk hit max_walk (the fallback still ran) */
#define OV_DEV_NONFINITE 4    /* a non-finite query coordinate was met (the query became an orphan) */

/* Options (ov_set_option). */
enum ov_option {
    OV_OPT_WARM = 1,        /* 1 (default): seed the walk from the previous step's donor; 0: cold */
    OV_OPT_MAX_WALK = 2,    /* walk steps before the brute-force fallback (default 16, >= 1) */
    OV_OPT_SEARCH_BLOCK = 3,/* threads per block of the donor search walk (64..256, multiple of 64) */
    OV_OPT_INTERP_BLOCK = 4,/* threads per block of the interpolation (64..1024, multiple of 64) */
    OV_OPT_HOLECUT_BLOCK = 5,/* threads per block of the hole cut (64..1024, multiple of 64) */
    OV_OPT_HOLECUT_NPT = 6, /* 16-byte coordinate vectors per lane per chunk of the hole cut (1, 2 or 4) */
    OV_OPT_PERSIST = 7,     /* workgroups per CU of persistent launches (1..32; 0 = one item per thread) */
    OV_OPT_HOLECUT_CULL = 8,/* 1 (default): the hole cut reads the coordinates only of 16x8x8 sub-tiles that
                               some blank region may reach (bounding sphere vs. the region's enclosing sphere and
                               body-frame box; same flags); 0: stream every node */
    OV_OPT_HOLECUT_NPL = 9, /* culled hole cut, candidate nodes per lane: 16 (default, one wavefront per
                               sub-tile) or 4 (one block per sub-tile: shorter latency when candidates are few) */
    OV_OPT_BACK_FUSED = 10, /* step executors (ov_pipe_*): 1 (default) runs transform, donor search and
                               interpolation of a step as one kernel; 2 as two kernels, the second taking the
                               queries the first could not decide (FP64 corrections, brute-force scans) from a
                               queue the executor owns, so that the first holds only the walk's registers;
                               0 as the separate kernels of the three calls. Same results. */
    OV_OPT_BACK_BLOCKS = 11,/* workgroups per CU of that one kernel (1..32, default 8) */
    OV_OPT_BACK_BLOCK = 12, /* its threads per workgroup: 64, 128 or 256 (default; also the width of the
                               cooperative fallback scan) */
    OV_OPT_FIELD_LAYOUT = 13,/* layout of the fields given to overset_interp and the executors: 0 (default)
                               four blocks of total_nodes values (u block, v, w, p); 1 interleaved per node
                               (u, v, w, p of node 0, then node 1, ...): one load per donor corner */
    OV_OPT_FRAME_VELOCITY = 14,/* step executors: 1 gives the interpolated u, v, w in the receiver's frame
                               (as overset_frame_velocity does after overset_interp); 0 (default) leaves them
                               in the donor's frame */
    OV_OPT_BACK_QUEUE = 15, /* step executors: 1 lets the back half's workgroups take their chunks of queries
                               from an atomic work queue (each its own first chunk, then the next free one)
                               instead of a fixed stride; 0 (default) the fixed stride. Same results. */
    OV_OPT_BACK_XCD = 16,   /* step executors: k in 1..64 puts runs of k consecutive chunks of queries on the
                               workgroups of one XCD (the runs going to the XCDs in turn) where the back half's
                               workgroups take their chunks by index (every round of the fixed stride, the
                               first chunk with the work queue), so that neighbouring queries, whose donor
                               cells share lines, run under one L2; 0 (default), or a grid that 8 k does not
                               divide: launch order. Same results. */
    OV_OPT_HOLECUT_LIST = 17/* culled hole cut: 1 computes which blank regions may reach each sub-tile in the
                               kernel that starts the step (flag fill or reset) and hands the candidate
                               sub-tiles out in rank order, one per workgroup of the hole cut (no workgroup
                               waits on a second candidate while others idle); 0 (default) each workgroup culls
                               and tests its own share of the sub-tiles. Same flags. */
};

/* Create a context on HIP device `device` with precision `precision`.
 * *out receives the context [host]. Returns OV_EINVAL / OV_EHIP on failure. */
int ov_ctx_create(ov_ctx **out, int device, int precision);

/* Free everything the library allocated for `ctx`. Synchronises the device. */
int ov_ctx_destroy(ov_ctx *ctx);

/* Last error message of `ctx` (static string owned by the context). */
const char *ov_last_error(const ov_ctx *ctx);

/* The blank region of grid `grid` as a closed surface triangulation (the
 * body's surface triangles of Sec. 2.2.2), replacing its implicit shape: a
 * node of another grid is a hole when the ray from it along +x (in this
 * grid's body frame) crosses the surface an odd number of times. Counting
 * rule, exactly that of the FP64 decision on every node:
 *  - a triangle is crossed when the node's (y, z) lies in the triangle's
 *    (y, z) projection, oriented counter-clockwise (edge-on triangles never
 *    count), and the crossing lies beyond the node in x;
 *  - on a projected edge u->v the node counts when v_z > u_z, or v_z = u_z
 *    and v_y > u_y, with the edge function evaluated from the endpoint of
 *    smaller (y, z), so that a crossing through a shared edge or vertex
 *    counts once;
 *  - outside the surface's axis-aligned box a node is outside.
 * The surface must be closed (every edge shared by two triangles, shared
 * vertices bit-identical); the test is decided in FP64 in both precisions.
 *  tri   ntri x 9 doubles (vertices a, b, c) in the grid's body frame [host, copied]
 *  ntri  >= 4
 * Must follow ov_grid_add of that grid and precede ov_finalize. OV_EINVAL
 * for a bad grid id, fewer than 4 triangles or a non-finite coordinate. */
int ov_grid_set_blank_mesh(ov_ctx *ctx, int32_t grid, const double *tri, int64_t ntri);

/* Register a structured grid (Sec. 2.2: a block of the overset system).
 *  ni, nj, nk     nodes per direction, each >= 2; total nodes of all grids < 2^31
 *  periodic       bit mask: 1 = i, 2 = j, 4 = k wraps (the last node joins node 0)
 *  X, Y, Z        body-frame node coordinates, FP64, i fastest [device, caller-owned]
 *  blank_kind     ov_blank_kind of the region this grid cuts from the others
 *                 (the user-defined blank surface of Sec. 2.2.2), body frame
 *  blank_prm      8 doubles of shape parameters [host]
 *  outer          6 ints [host]: query-point layers on faces i-, i+, j-, j+,
 *                 k-, k+ (the overset boundary faces of Sec. 2.2.3 item 1)
 *  grid_id        receives the id [host]; the first grid (id 0) is the background.
 * Must precede ov_finalize. */
int ov_grid_add(ov_ctx *ctx, int32_t ni, int32_t nj, int32_t nk, uint32_t periodic,
                const double *X, const double *Y, const double *Z,
                int32_t blank_kind, const double *blank_prm, const int32_t *outer,
                int32_t *grid_id);

/* Build the per-grid control cells (Sec. 2.2.5: an axis-aligned auxiliary grid
 * over each donor grid whose control cells list the donor cells reaching
 * them), FP32 shadows (mixed precision) and warm-start history, and find
 * each grid's polar ends: in a grid with one periodic axis, an end face of
 * another axis whose nodes coincide along the periodic axis (to 1e-12 of the
 * grid's extent) lies on an axis of revolution, and the FP64 walk goes on
 * across it (a result changes nothing but the walk's path). Synchronises
 * `stream`. After this, no grid can be added. */
int ov_finalize(ov_ctx *ctx, void *stream);

/* Number of grids / total nodes; node offsets (ngrids+1 int64) [host]. */
int32_t ov_num_grids(const ov_ctx *ctx);
int64_t ov_total_nodes(const ov_ctx *ctx);
int ov_node_offsets(const ov_ctx *ctx, int64_t *out);

/* Work counters accumulated by the step calls since the last fetch. */
#define OV_STAT_HOLECUT_NODES_READ 0  /* nodes whose coordinates the hole cut read */
#define OV_STAT_HOLECUT_CALLS 1       /* overset_holecut calls */
/* Donor-search work of the executors' one-kernel back half (counted there only): */
#define OV_STAT_SEARCH_CELLS 2         /* cells the stencil walks visited */
#define OV_STAT_NEWTON_ITERS 3         /* Newton iterations, walks and fallback scans */
#define OV_STAT_SCAN_CANDIDATES 4      /* control-cell list entries the fallback scans tested */
#define OV_STAT_BACK_CALLS 5           /* launches of that kernel */
/* Flag bytes a step's start wrote: every node (the full fill) or only the
 * previous step's near tiles (the executors' incremental reset), and the
 * base-flag bytes it read for grids with outer layers: */
#define OV_STAT_FLAG_BYTES_WRITTEN 6
#define OV_STAT_BASE_BYTES_READ 7
#define OV_STAT_FLAG_STARTS 8          /* fills + resets */
#define OV_STAT_COUNT 9

/* Copy the OV_STAT_COUNT counters into host_out [host] and zero them.
 * Synchronises `stream`. */
int ov_stats_fetch(ov_ctx *ctx, int64_t *host_out, void *stream);

/* Set an option (ov_option); returns OV_EINVAL for an unknown key or a value
 * out of range. Takes effect at the next step call. */
int ov_set_option(ov_ctx *ctx, int32_t key, int64_t value);

/* Forget the warm-start history (next search is cold). Stream-ordered. */
int ov_reset_history(ov_ctx *ctx, void *stream);

/* Copy the device status word into *host_status [host] and clear it.
 * Synchronises `stream`. */
int ov_status_fetch(ov_ctx *ctx, int32_t *host_status, void *stream);

/* The same two calls under the names of the step calls' family:
 * overset_status_fetch is ov_status_fetch (the device conditions of the step
 * calls: capacity overflow, walk limit, non-finite input), and
 * overset_last_error is ov_last_error (the message of the last negative
 * status a call on `ctx` returned). */
int overset_status_fetch(ov_ctx *ctx, int32_t *host_status, void *stream);
const char *overset_last_error(const ov_ctx *ctx);

/* ---------------------------------------------------------------- step */

/* Hole cutting (Sec. 2.2.2, Sec. 2.4 item 2). For every node of every grid A,
 * in A's pose, and every other grid B with a blank region: the node is a HOLE
 * iff it lies strictly inside B's blank region placed at B's pose; the cause
 * is the lowest such B. Every node's flag byte is overwritten: HOLE (cause B);
 * else FRINGE with cause 63 if the node lies in one of its grid's `outer`
 * layers (a fixed set per grid, marked here so that the fringe pass only
 * visits tiles near holes); else FIELD. The call also records, for the
 * fringe pass of the same context, which node tiles hold a hole.
 *  poses   ngrids poses (12 doubles each)
 *  flags   total_nodes bytes, fully overwritten */
int overset_holecut(ov_ctx *ctx, const double *poses, uint8_t *flags, void *stream);

/* Query-point identification and compaction (Sec. 2.2.3 item 1, Alg. 1).
 * FRINGE nodes are (a) the `outer` face layers of each grid, cause 63 (marked
 * by overset_holecut) and (b) the buffer layer: every non-hole node within
 * Chebyshev index distance `nf` of a hole of its own grid (periodic
 * directions wrap), cause = the lowest cause of those holes. Hole > fringe >
 * field. Then writes the fringe nodes in ascending (grid, node) order to
 * q_grid / q_node (local node index) and their number to *d_count (device
 * int64). Entries beyond `capacity` are not written; the device status bit
 * OV_DEV_CAPACITY is set instead.
 *  nf         buffer width, 0..3
 *  flags      hole-cut flags: holes (any cause) and outer-layer FRINGE
 *             nodes as overset_holecut writes them, FIELD elsewhere; updated
 *             in place; 16-byte aligned. The call finds the tiles that hold
 *             a hole from these flags themselves (one read of every flag
 *             byte), so any such buffer may be passed, whichever hole cut
 *             wrote it. */
int overset_fringe_compact(ov_ctx *ctx, int32_t nf, uint8_t *flags, int32_t *q_grid, int32_t *q_node,
                           int64_t capacity, int64_t *d_count, void *stream);

/* overset_fringe_compact for callers that cannot allocate device memory
 * (work under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation). Same arguments, results and errors as overset_fringe_compact;
 * the call's scratch (near-tile list, chunk list, per-chunk and
 * per-superchunk counts) lives in a static device array of the library
 * (6 MiB per device, held until the process ends) instead of the context's
 * memory, and the call allocates nothing. A context whose grids need more
 * scratch than the array holds (about 20 bytes per 64x8x8 node tile plus
 * 17 bytes per 4096 nodes) is refused with OV_ECAPACITY before any launch.
 * All calls on one device share its array, and each starts by clearing it:
 * calls on one device must be ordered (one stream, or streams ordered
 * against each other), or they race. */
int overset_fringe_compact_noalloc(ov_ctx *ctx, int32_t nf, uint8_t *flags, int32_t *q_grid, int32_t *q_node,
                                   int64_t capacity, int64_t *d_count, void *stream);

/* Inertial-frame positions of the compacted queries (the coordinate packets
 * of Sec. 2.2.3 item 6), stored as the offset from the query grid's frame
 * centre: qx = x - c_g = R_g X_g[node], for i < *d_count. The consumer adds
 * c_g in FP64, so an FP32 qx (OV_MIXED) only carries the body-scale offset.
 *  qx   3*capacity values (x block, y block, z block), double (OV_FP64) or
 *       float (OV_MIXED) */
int overset_transform(ov_ctx *ctx, const double *poses, const int32_t *q_grid, const int32_t *q_node,
                      const int64_t *d_count, int64_t capacity, void *qx, void *stream);

/* Donor search (Sec. 2.2.5, Alg. 3) with donor selection (Sec. 2.4 item 1).
 * For query i < *d_count of grid A whose flag carries cause k, candidate donor
 * grids are: k (unless 63 or A), then the background 0, then the other grids
 * in ascending id. In each candidate grid B the query is taken into B's body
 * frame, a stencil walk seeded from the previous step's donor (or from B's
 * control cell) moves cell to cell by the signs of the natural coordinates,
 * and Newton's method solves the trilinear map for s. A cell contains the
 * point iff s lies in [0,1]^3 (up to 1e-12); it is a valid donor iff none of
 * its 8 corners is a HOLE. A walk that leaves the grid, repeats or exceeds
 * max_walk falls back to a brute-force scan of the control cell's candidates,
 * keeping the lowest valid containing cell index. Outputs per query:
 *  donor_grid, donor_cell   int32 (-1 for orphans)
 *  s                        3*capacity natural coordinates (s0 block, s1, s2),
 *                           double or float by context precision; NaN for orphans
 *  status                   OV_Q_* code
 *  flags                    the flags after overset_fringe_compact (read only)
 *  qx                       output of overset_transform */
int overset_donor_search(ov_ctx *ctx, const double *poses, const uint8_t *flags, const int32_t *q_grid,
                         const int32_t *q_node, const void *qx, const int64_t *d_count, int64_t capacity,
                         int32_t *donor_grid, int32_t *donor_cell, void *s, int32_t *status, void *stream);

/* Trilinear interpolation (Sec. 2.2.6): out[f][i] = sum_{c=0..7} w_c F_f[corner c]
 * with w_c = prod_d (c_d ? s_d : 1 - s_d), for the 4 fields u, v, w, p and every
 * query i < *d_count with a donor; orphans are not written.
 *  fields   4*total_nodes values, grids packed by node offset: four blocks (u block, v, w,
 *           p) or, with OV_OPT_FIELD_LAYOUT = 1, interleaved (u, v, w, p per node)
 *  out      4*capacity values
 * Both double (OV_FP64) or float (OV_MIXED). */
int overset_interp(ov_ctx *ctx, const int32_t *donor_grid, const int32_t *donor_cell, const void *s,
                   const int64_t *d_count, int64_t capacity, const void *fields, void *out, void *stream);

/* Velocities in the receiver's frame (Sec. 2.3): each grid's flow is solved
 * in its own non-inertial frame, so the u, v, w that overset_interp gathers
 * from donor grid B are components in B's frame. For every query i <
 * *d_count with a donor this rewrites fields 0, 1, 2 of out in place as the
 * components in the frame of the query's grid A: u_A = R_A^T R_B u_B, with R
 * the rotation of each pose (x = R X + c; R is the transpose of the paper's
 * Q). The pressure (field 3) is a scalar and stays as it is.
 *  poses      ngrids*12 doubles of this step (device)
 *  q_grid, donor_grid, d_count, capacity: as from the compaction and search
 *  out        4*capacity values, context precision (in/out)
 * In the step executors, OV_OPT_FRAME_VELOCITY = 1 does the same inside the
 * back half. */
int overset_frame_velocity(ov_ctx *ctx, const double *poses, const int32_t *q_grid, const int32_t *donor_grid,
                           const int64_t *d_count, int64_t capacity, void *out, void *stream);

/* The interpolation matrix (Sec. 2.2.6, second option; Alg. 4), one row per
 * query i < *d_count in ELL form of 8 entries, row-major: cols[8 i + c] is
 * the global index (node offset of the donor grid + node: the paper's
 * global index on one GPU) of corner c (= c0 + 2 c1 + 4 c2, periodic wrap)
 * of the donor cell, vals[8 i + c] its trilinear weight; a query without a
 * donor has cols -1 and vals 0. Rows from *d_count on are not written.
 *  cols   8*capacity int32 (device); needs total_nodes < 2^31 (OV_EDIMS otherwise)
 *  vals   8*capacity values, context precision */
int overset_interp_matrix(ov_ctx *ctx, const int32_t *donor_grid, const int32_t *donor_cell, const void *s,
                          const int64_t *d_count, int64_t capacity, int32_t *cols, void *vals, void *stream);

/* The matrix applied to nrhs field vectors (the product Alg. 4 repeats at
 * every Newton-Krylov iteration): for every row i < *d_count and vector
 * r < nrhs, y_r[i] = sum over the row's entries with cols >= 0, in corner
 * order, of vals[8 i + c] * x_r[cols[8 i + c]].
 *  layout 0: vectors as blocks, x[r*total_nodes + node], y[r*capacity + i];
 *  layout 1: interleaved per node, x[node*nrhs + r], y[i*nrhs + r] (with
 *            nrhs = 4, one load per corner and one store per row).
 *  x   nrhs*total_nodes values, context precision
 *  y   nrhs*capacity values, context precision; rows from *d_count on are not written
 * cols and vals must be 16-byte aligned; x and y aligned to one value, or to
 * 4 values with layout 1 and nrhs = 4 (OV_EINVAL otherwise). */
int overset_interp_apply(ov_ctx *ctx, const int32_t *cols, const void *vals, const int64_t *d_count,
                         int64_t capacity, const void *x, int32_t nrhs, int32_t layout, void *y, void *stream);

/* ---------------------------------------------------------------- pipelined steps */

/* Every device buffer one step writes (the arguments of the five calls). */
typedef struct ov_step_buffers {
    uint8_t *flags;        /* total_nodes bytes, 16-byte aligned */
    int32_t *q_grid;       /* capacity */
    int32_t *q_node;       /* capacity */
    int64_t *d_count;      /* 1 */
    void *qx;              /* 3*capacity, context precision */
    int32_t *donor_grid;   /* capacity */
    int32_t *donor_cell;   /* capacity */
    void *s;               /* 3*capacity, context precision */
    int32_t *status;       /* capacity */
    void *out;             /* 4*capacity, context precision (unused without fields) */
    int64_t capacity;
} ov_step_buffers;

typedef struct ov_pipe ov_pipe;

/* A one-stream executor of consecutive steps (a scheduling layer over the
 * five calls; not a step of the paper's method): each submitted step's
 * stages run in stream order on `stream`, all steps in the one buffer set
 * *set. No events: the cheapest form for the host. The results of a step
 * are in the set until the next step overwrites them. Other rules as
 * ov_pipe_create. */
int ov_pipe_create1(ov_ctx *ctx, int32_t nf, const ov_step_buffers *set, const void *fields, void *stream,
                    int32_t max_timed, ov_pipe **out);

/* A two-stream executor of consecutive steps (a scheduling layer over the
 * five calls; not a step of the paper's method). Step t uses buffer set
 * sets[t % 2]; its front half (overset_holecut, overset_fringe_compact) runs
 * on stream_front and overlaps the back half (overset_transform,
 * overset_donor_search, overset_interp) of step t-1 on stream_back.
 * front(t) runs after back(t-2) and back(t) after front(t), ordered with
 * stream memory operations (hipStreamWriteValue64 / hipStreamWaitValue64)
 * on sequence counters the executor allocates (16-24 bytes of device
 * memory); back halves follow one another on their stream, which keeps the
 * warm start exact. The back half runs as one kernel unless
 * OV_OPT_BACK_FUSED is 0 (same results). Returns OV_EHIP if the device
 * cannot wait on memory values.
 *  sets        2 buffer sets [host array; the device buffers stay caller-owned]
 *  fields      4*total_nodes field values, or NULL for no interpolation
 *  max_timed   number of steps whose stage may be timed (events, see below)
 * The context must not be used by other calls while the pipeline has work
 * in flight. Streams must differ and stay alive until ov_pipe_destroy. */
int ov_pipe_create(ov_ctx *ctx, int32_t nf, const ov_step_buffers *sets, const void *fields,
                   void *stream_front, void *stream_back, int32_t max_timed, ov_pipe **out);

/* The three-stage variant: the hole cut (stage A, on stream_a), fringe
 * marking + compaction (stage B, stream_b) and the back half (stage C,
 * stream_c) of consecutive steps, with three buffer sets (step t uses
 * sets[t % 3]): A(t+1), B(t) and C(t-1) run at the same time. A and B of a
 * step share front-half scratch slot t % 3 of the context. B(t) runs after
 * A(t), C(t) after B(t) and A(t) after C(t-3). Same rules as ov_pipe_create
 * otherwise; the three streams must differ. */
int ov_pipe_create3(ov_ctx *ctx, int32_t nf, const ov_step_buffers *sets, const void *fields,
                    void *stream_a, void *stream_b, void *stream_c, int32_t max_timed, ov_pipe **out);

/* Capture, for every buffer set, the stages each stream runs once as a
 * single-stream HIP graph (on a private stream) and replay the graphs from
 * then on: a submitted step becomes one pose copy into a per-set device
 * slot, one graph launch per stream and the ordering counter operations.
 * Must be called before the first submit;
 * options set on the context afterwards do not reach the captured graphs.
 * on = 0 returns to direct launches. Returns OV_EHIP (graphs off) if the
 * runtime refuses the capture. */
int ov_pipe_use_graphs(ov_pipe *pipe, int32_t on);

/* Queue the next step with poses (device, ngrids*12 doubles, must stay
 * unchanged until the step completes). If count_out (device int64) is not
 * NULL it receives the step's query count. Nothing synchronises. */
int ov_pipe_submit(ov_pipe *pipe, const double *poses, int64_t *count_out);

/* Queue n consecutive steps: step i reads its poses at poses + i*pose_stride
 * (device; pose_stride >= ngrids*12 doubles) and, if counts_out (device
 * int64[n]) is not NULL, writes its query count to counts_out[i]. The same
 * as n calls of ov_pipe_submit, without a host round trip per step. */
int ov_pipe_submit_many(ov_pipe *pipe, const double *poses, int64_t pose_stride, int64_t n, int64_t *counts_out);

/* on = 1: ov_pipe_submit_many of more than one step on two or three streams
 * issues each stream's work from a host thread of its own (the calling thread
 * takes the first stream; the others are started for the call and joined
 * before it returns), so that the host's time per step is that of one
 * stream's calls rather than of all of them. The order between the streams
 * is the device-side one in either case, so the results are the same; a
 * thread issues a wait only after the write it waits for has been issued by
 * its thread, so every wait is for work submitted before it. Not
 * used with graphs, in the by-step order or with a stage timed alone
 * (ov_pipe_set_timing), where the calls go out from the calling thread. on = 0 (default): one thread.
 * Returns OV_EINVAL for another value. */
int ov_pipe_set_threads(ov_pipe *pipe, int32_t on);

/* on = 1 (before the first submit; two or three streams, no graphs; waits
 * for the device, as the host then numbers this pipe's steps on from the
 * context's step counter): the by-step order. Step t runs all three stages on stream t mod nsets, one
 * after another, after the step that used that buffer set before; across
 * streams only its back half waits, for the previous step's back half (the
 * warm start), so that one ordering crosses streams per step instead of
 * three, and the front half of a step may run while the back halves of the
 * steps before it do. The results are the same. A stage
 * timed alone waits for the other streams' work so far, and the next step
 * waits for it. on = 0 (default): stream g runs stage group g of every step.
 * Returns OV_EINVAL for another value or one stream, OV_ESTATE after the
 * first submit or with graphs. */
int ov_pipe_set_by_step(ov_pipe *pipe, int32_t on);

/* Make `stream` wait for all work submitted so far. */
int ov_pipe_join(ov_pipe *pipe, void *stream);

/* Time stage `stage` (0 = A hole cut, 1 = B fringe + compaction, 2 = C back
 * half) of the next submitted step and of every `every`-th step after it
 * (every = 0 stops timing) with events on the stream it runs on, up to
 * max_timed steps. With graphs the events bracket the whole graph of that
 * stage's stream. With several streams a timed stage runs alone (it waits
 * for the other streams' earlier work, and the next step waits for it), so
 * its events time its own kernels, not the queueing behind other streams;
 * this costs some overlap on the timed steps. Each timed step also adds two
 * event records to the stream, which cost device time of their own. */
int ov_pipe_set_timing(ov_pipe *pipe, int32_t every, int32_t stage);

/* As ov_pipe_set_timing, with alone = 0: the timed stage keeps its place in
 * the pipeline (no extra waits), so its events include any slowdown from the
 * other streams' kernels running beside it: the duration it has in the
 * steady state. alone = 1 is ov_pipe_set_timing. */
int ov_pipe_set_timing_mode(ov_pipe *pipe, int32_t every, int32_t stage, int32_t alone);

/* Elapsed milliseconds of the timed stages so far (waits for them) into
 * ms_out[0..*n_out) [host], then restarts the record. */
int ov_pipe_stage_times(ov_pipe *pipe, float *ms_out, int32_t max, int32_t *n_out);

/* Wait for the pipeline's streams and free its events. */
int ov_pipe_destroy(ov_pipe *pipe);

#ifdef __cplusplus
}
#endif

#endif /* OVERSET_H */
