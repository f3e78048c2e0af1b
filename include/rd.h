/*
 * rd.h - C ABI of librd, a GPU (AMD Instinct MI355X, gfx950) library for the
 * multidimensional upwind residual-distribution scheme of Paardekooper (2017),
 * "Multidimensional upwind hydrodynamics on unstructured meshes using
 * Graphics Processing Units - I. Two-dimensional uniform meshes".
 *
 * The library advances the two-dimensional Euler equations of an ideal gas
 * (Section 3, conservation form) on a static triangular mesh. Each step
 * Roe-averages the parameter vectors of a triangle's three vertices, builds
 * the flux Jacobians K_i along the inward edge normals and their positive
 * and negative parts (Section 3.2 and Appendix A), forms the triangle
 * residual, distributes it to the vertices with the N, LDA or blended B
 * schemes (Section 3.3), sums the parts per vertex and updates the state with
 * forward Euler or the two-stage Runge-Kutta scheme of Section 3.4, with
 * periodic, non-reflecting (ghost) and reflecting-wall boundaries
 * (Section 3.5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - States are float64, structure of arrays: W[k * n_vertices + i] is
 *    component k of vertex i, k = 0..3 for (rho, rho u, rho v, e) with
 *    e = rho (u^2 + v^2)/2 + p/(gamma - 1).
 *  - Every call returns an rd_status; no C++ exception crosses this ABI.
 *    On a non-OK status rd_last_error() returns a message (thread-local,
 *    valid until the next call from the same thread).
 *  - `on_device` = 0: the pointer is host memory; the call copies and
 *    returns when the copy is complete. `on_device` = 1: the pointer is
 *    device memory of the current HIP device (e.g. a torch tensor's
 *    data_ptr); the work is ordered on the mesh's stream and the call
 *    returns without waiting.
 *  - The library never frees memory it did not allocate. Arrays passed to
 *    rd_mesh_create and host states are copied; the caller keeps ownership.
 *  - One mesh is used by one host thread at a time.
 *  - Kernels never use floating-point atomics: the vertex sums run over a
 *    fixed (ascending-triangle) order, so repeated runs give bitwise
 *    identical results.
 */
#ifndef RD_H
#define RD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rd_mesh rd_mesh;   /* opaque; owns its device buffers */
typedef struct rd_batch rd_batch; /* opaque; owns its device buffers */

typedef enum {
  RD_OK = 0,
  RD_EINVAL = 1,        /* an argument or the mesh is invalid */
  RD_ENOMEM = 2,        /* device or host allocation failed */
  RD_EDEVICE = 3,       /* a HIP runtime call failed */
  RD_ENONPHYS = 4,      /* a state with rho <= 0, p <= 0 or a non-finite value */
  RD_EUNSUPPORTED = 5   /* valid request the library does not provide */
} rd_status;

/* Distribution schemes (Section 3.3): N, LDA, and the blend B with its
 * diagonal Theta; BMAX / BMIN set every Theta_kk to the largest / smallest.
 * BX is the blend of Section 3.3.3 with one scalar theta per triangle from a
 * shock sensor: theta = min(1, s^2 h / L), s = max(0, -L div v / (|v|max -
 * |v|min)), div v of the linear interpolant of the vertex velocities, h =
 * sqrt(2 |T|), |v|max and |v|min over the mesh's vertices at the stage's
 * state (s = 0 when they are equal), L the larger side of the domain (the
 * period on a periodic axis, else the coordinate extent). Two extra
 * vertex passes per stage find |v|max and |v|min. */
typedef enum { RD_N = 0, RD_LDA = 1, RD_B = 2, RD_BMAX = 3, RD_BMIN = 4, RD_BX = 5 } rd_scheme;

/* Lumping of the mass term in the second Runge-Kutta stage (Section 3.4):
 * global (the default), or selective, which adds sum_j (|T| delta_ij / 3 -
 * m^G_ij) (W*_j - W^n_j) / dt, m^G_ij = |T| (1 + delta_ij) / 12 (Galerkin
 * mass), to the N and LDA total parts before they are blended. */
typedef enum { RD_LUMP_GLOBAL = 0, RD_LUMP_SELECTIVE = 1 } rd_lumping;

/* Time integration: forward Euler (the update of Section 3.2) or the
 * two-stage Runge-Kutta scheme of Section 3.4 with global lumping and the
 * mass matrix |T|/3 beta_i. */
typedef enum { RD_EULER1 = 1, RD_RK2 = 2 } rd_time;

/* Arithmetic: FP64 throughout, or the triangle algebra in FP32 with the
 * vertex sums and the state update in FP64 (compensated summation). */
typedef enum { RD_FP64 = 0, RD_FP32_ACC64 = 1 } rd_precision;

typedef struct {
  int64_t n_vertices;      /* > 0 */
  int64_t n_triangles;     /* > 0, 3 * n_triangles < 2^31 */
  const double* x;         /* [n_vertices] host */
  const double* y;         /* [n_vertices] host */
  const int32_t* tri;      /* [3 * n_triangles] host, corners counter-clockwise
                              after unwrapping to the minimum image of corner 0 */
  double period_x;         /* 0: x bounded; > 0: x periodic with this period */
  double period_y;         /* 0: y bounded; > 0: y periodic with this period */
  const uint8_t* ghost;    /* [n_vertices] host or NULL; 1 marks a ghost vertex that
                              keeps its state (non-reflecting / inflow, Section 3.5) */
  int64_t n_wall_edges;    /* >= 0 */
  const int32_t* wall_edges; /* [2 * n_wall_edges] host: (a, b) with the domain on the
                                left of a -> b; reflecting wall of Section 3.5 */
  double gamma;            /* ratio of specific heats, > 1 */
} rd_mesh_desc;

/* Checks a mesh description on the host only (no GPU needed): indices in
 * range, positive unwrapped areas, every vertex in at least one and at most
 * 1023 triangles, valid wall edges. RD_OK or RD_EINVAL. */
rd_status rd_mesh_validate(const rd_mesh_desc* desc);

/* Validates `desc`, precomputes vertex volumes V_i = sum |T|/3 (median dual,
 * Section 3.2 update with global lumping), the vertex -> (triangle, corner)
 * CSR used by the deterministic gather, longest edges for the CFL limit and
 * the wall-edge lists, and allocates the device buffers. `stream` is a
 * hipStream_t (NULL: the null stream). The state is zero until
 * rd_set_state. RD_EINVAL, RD_ENOMEM or RD_EDEVICE on failure (*out = NULL). */
rd_status rd_mesh_create(const rd_mesh_desc* desc, void* stream, rd_mesh** out);

/* Waits for the mesh's stream, frees every buffer. NULL is accepted. */
rd_status rd_mesh_destroy(rd_mesh* mesh);

/* Sizes of a mesh. */
rd_status rd_mesh_info(const rd_mesh* mesh, int64_t* n_vertices, int64_t* n_triangles);

/* Replaces the stream all later work of this mesh is ordered on. */
rd_status rd_set_stream(rd_mesh* mesh, void* stream);

/* Sets the state W [4][n_vertices]. Host input is checked (rho > 0, p > 0,
 * finite: else RD_ENONPHYS and nothing changes); device input is checked on
 * the device and reported by rd_sync. Ghost vertices keep this value. */
rd_status rd_set_state(rd_mesh* mesh, const double* W, int on_device);

/* Copies the current state into W [4][n_vertices]. With on_device = 0 it
 * waits and returns RD_ENONPHYS if a non-physical state was latched
 * (the copy is still made). */
rd_status rd_get_state(rd_mesh* mesh, double* W, int on_device);

/* CFL limit of Section 3.2 at the current state, times `cfl`:
 * cfl * min_i 2 V_i / sum_{T ni i} l_max^T lambda_max^T, with
 * lambda_max^T = max over the corners of |v| + c. Waits for the result. */
rd_status rd_max_dt(rd_mesh* mesh, double cfl, double* dt_out);

/* One time step of size dt > 0 (Sections 3.2-3.4). Enqueues only. */
rd_status rd_step(rd_mesh* mesh, double dt, int scheme, int time, int precision);

/* `n_steps` steps, each with dt = cfl * (CFL limit at the step's start),
 * computed on the device: no host synchronisation. Enqueues only. */
rd_status rd_step_cfl(rd_mesh* mesh, int n_steps, double cfl, int scheme, int time, int precision);

/* Kernel slots of one step, in launch order, as reported by rd_step_timed.
 * Two-pass form: every part goes to HBM, a vertex gather sums it. Tiled
 * form: a tile pass sums the parts of tile-interior vertices in LDS and a
 * shared pass sums those of vertices on tile borders. */
enum {
  RD_K_WALL1 = 0,   /* wall term at W^n (meshes with walls) */
  RD_K_TRI1 = 1,    /* stage-1 (or Euler) triangle pass; two-pass form: also l_max lambda_max per
                       corner; tiled form: tile pass, also interior vertex residuals and CFL bounds */
  RD_K_SHARED1 = 2, /* tiled form: shared-vertex residuals and CFL bounds */
  RD_K_CFL = 3,     /* CFL reduction: per-vertex bounds, block and per-mesh minima -> dt */
  RD_K_GATHER1 = 4, /* two-pass form: stage-1 vertex sums and update; tiled form: Euler update */
  RD_K_WALL2 = 5,   /* wall term at W* (RK2 with walls) */
  RD_K_TRI2 = 6,    /* stage-2 triangle pass (RK2); tiled form: also the interior vertex update */
  RD_K_GATHER2 = 7, /* stage-2 vertex sums and update (RK2); tiled form: shared vertices only */
  RD_NKERNELS = 8
};

/* One step as rd_step_cfl(mesh, 1, ...) does, with a HIP event recorded on
 * the mesh's stream between consecutive kernels; waits, then writes the
 * duration of every kernel in milliseconds to ms[RD_NKERNELS] (0 for
 * kernels the step does not launch). For profiling. */
rd_status rd_step_timed(rd_mesh* mesh, double cfl, int scheme, int time, int precision, double* ms);

/* Form of the step (Sections 3.2-3.4 computed either way). tile_triangles
 * = 0 selects the two-pass form. A value in [32, 1024] selects the tiled
 * form: triangles are ordered along a Morton curve of their centroids and cut
 * into tiles of that many triangles; one workgroup per tile stages the
 * tile's vertex data in LDS and finishes the vertices all of whose
 * triangles are in the tile. Every vertex sums its parts in ascending
 * triangle order in both forms, so results are bitwise identical for every
 * tile size and equal to the two-pass form's up to rounding. RD_EUNSUPPORTED
 * if a tile would need more LDS than one workgroup may use on the device
 * (160 KiB on MI355X). Waits for the mesh's stream. The default is 0. */
rd_status rd_mesh_set_tile(rd_mesh* mesh, int tile_triangles);
rd_status rd_mesh_get_tile(const rd_mesh* mesh, int* tile_triangles);
/* Lumping of the mesh's RK2 steps (rd_lumping; RD_EINVAL for other values).
 * Takes effect with the next step; the members of a batch must agree
 * (rd_batch_run returns RD_EINVAL otherwise). The default is global. */
rd_status rd_mesh_set_lumping(rd_mesh* mesh, int lumping);
rd_status rd_mesh_get_lumping(const rd_mesh* mesh, int* lumping);

/* Shape of the current tiling (all zero in the two-pass form): info[0] tiles,
 * info[1] local vertex records over all tiles (vertices on tile borders
 * count once per tile), info[2] shared vertices, info[3] their parts
 * (shared corners). */
rd_status rd_mesh_tile_info(const rd_mesh* mesh, int64_t info[4]);

/* Autotuner: for each of the n_candidates tile sizes (NULL: 0, 64, 128,
 * 256, 512; unsupported sizes are skipped and report a negative time) runs
 * one warm-up step and n_steps >= 1 timed steps (dt from `cfl`, as
 * rd_step_cfl), writes milliseconds per step to ms_per_step (may be NULL,
 * else n_candidates entries), selects the fastest size for the mesh and
 * returns it in *best; candidates are taken in the given order and a later
 * one replaces the size kept so far only when it is more than 2% faster
 * (about the spread of one timing), so the first candidate (the two-pass
 * form by default) wins near-ties. The mesh's state is restored afterwards.
 * Waits. */
rd_status rd_tune(rd_mesh* mesh, double cfl, int scheme, int time, int precision, int n_steps,
                  const int* candidates, int n_candidates, double* ms_per_step, int* best);

/* Spatial residual at the current state (Section 3.2-3.3, FP64): R_i = sum
 * over the triangles of i (ascending triangle order) of the scheme's part
 * phi_i^T, plus the wall term; R is [4][n_vertices]. phiT (may be NULL)
 * receives the triangle residuals [4][n_triangles]. */
rd_status rd_residual(rd_mesh* mesh, int scheme, double* R, double* phiT, int on_device);

/* Adjoint of one step for a fixed dt (FP64 only): given the state W_n
 * [4][n_vertices] the step started from and lam_np1 = dL/dW^{n+1}, writes
 * lam_n = (dW^{n+1}/dW^n)^T lam_np1. Does not change the mesh's state.
 * Derivatives follow the branch the forward values take; d|x|/dx = 0 at 0.
 * RD_EUNSUPPORTED for the BX scheme and for RK2 with selective lumping.
 * The step is recomputed on the adjoint's own buffers: the mesh's state,
 * signal speeds and non-physical latch are not touched. Two conditions are
 * latched on the device instead: W_n (or its recomputed first stage) is
 * non-physical (RD_ENONPHYS), or a triangle's pivoted solve skipped a column
 * (an exactly stagnant triangle, Section 3.3.1, where the solve is not an
 * inverse and lam_n is not the derivative: RD_EUNSUPPORTED). With
 * on_device = 0 the call waits and returns that status; with on_device = 1
 * it only enqueues and the next rd_sync returns it. Either way the latch is
 * cleared once reported. lam_n must not overlap lam_np1 (lam_np1 is read
 * while lam_n is written). */
rd_status rd_adjoint_step(rd_mesh* mesh, const double* W_n, double dt, int scheme, int time,
                          const double* lam_np1, double* lam_n, int on_device);

/* Allocation-free form of rd_adjoint_step, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation. Same arguments and result as rd_adjoint_step with
 * on_device = 1 (W_n, lam_np1 and lam_n are device pointers [4][n_vertices],
 * stream-ordered on the mesh's stream), computed by the same kernels; it
 * calls no allocator. Its workspace is one fixed array of 128 MiB per GPU
 * (held by the process from its first use on that GPU until exit), which
 * fits meshes of about 125,000 vertices / 250,000 triangles; a larger mesh
 * gives RD_EINVAL with the sizes in rd_last_error. flags: device int[2],
 * cleared by the call, then set by the kernels: flags[0] = 1 when W_n or its
 * recomputed first stage is non-physical, flags[1] = 1 when a triangle's
 * solve skipped a column (exact stagnation, where lam_n is not the
 * derivative); both 0 means lam_n is valid. Only enqueues and returns RD_OK
 * (or an argument error: null pointer, dt, scheme, RD_EUNSUPPORTED for Bx
 * and selective lumping); does not wait. Every call on one GPU shares that
 * GPU's workspace, which keeps the last call's contents: calls that overlap
 * on one GPU (different streams, or threads) race and must be serialised by
 * the caller. */
rd_status rd_adjoint_step_noalloc(rd_mesh* mesh, const double* W_n, double dt, int scheme, int time,
                                  const double* lam_np1, double* lam_n, int* flags);

/* Delaunay triangulation by edge flips (Section 2, the step that ends every
 * refinement iteration), on the current GPU. Input: n_vertices points (x, y
 * host arrays) and a triangulation of them, tri [3 * n_triangles] host
 * (counter-clockwise after minimum-image unwrapping on a periodic axis, as
 * in rd_mesh_desc); every vertex used, every edge in at most two triangles.
 * On return tri holds a Delaunay triangulation of the same points with the
 * same number of triangles (boundary edges, those in one triangle, are kept;
 * triangle t keeps its index, its corners change): every interior edge has
 * its opposite vertex on or outside the circumcircle of each of its
 * triangles, decided by an exact in-circle predicate (FP64 with an error
 * bound, exact expansion arithmetic when that cannot decide; exact while
 * nonzero coordinate differences stay between about 2^-200 and 2^250; on a
 * periodic axis, on each vertex's image nearest to the edge's first vertex:
 * its coordinate, or that coordinate plus or minus the period, rounded to
 * FP64). Edges are flipped in rounds of independent
 * flips, the lowest-numbered illegal edge first wherever two compete, so the
 * result is the same on every run. n_flips and n_rounds (may be NULL)
 * receive the number of flips and rounds. RD_EINVAL for an invalid input
 * (with the checks of rd_mesh_validate), RD_ENOMEM, RD_EDEVICE. Allocates
 * device memory for the call, uses a stream of its own and waits for it. */
rd_status rd_delaunay_flip(int64_t n_vertices, const double* x, const double* y, double period_x, double period_y,
                           int64_t n_triangles, int32_t* tri, int64_t* n_flips, int32_t* n_rounds);

/* Delaunay refinement (Section 2: quality and size tests, point location by
 * walking with an exact orientation test, encroachment of boundary segments,
 * insertion, edge flips; Section 4.1: the parallel insertion set), on the
 * current GPU. Input as rd_delaunay_flip, with room to grow: *n_vertices
 * points in x, y [max_vertices] and *n_triangles triangles in
 * tri [3 * max_triangles] (host arrays). A boundary edge (in one triangle)
 * is a segment that must stay covered by edges; it must be axis-aligned (the
 * domain is a rectangle, or periodic on one or both axes; coordinates on a
 * periodic axis in [0, period)). The mesh is first made Delaunay by flips;
 * then each iteration: every triangle with circumradius r > max_radius s(c)
 * (0: no bound; c its centroid, s the size field below, 1 without one) or
 * r / (shortest edge) > max_ratio (0: no bound, else >= 1;
 * termination is guaranteed for max_ratio >= sqrt 2) proposes its
 * circumcentre, and every triangle whose boundary edge it encroaches on (its
 * opposite corner inside the edge's diametric circle) proposes that edge's
 * midpoint; a proposed point is located by walking from its triangle; a
 * point beyond the boundary, or one that encroaches on a boundary edge of a
 * triangle around the corners of its insertion triangle(s), is moved to that
 * edge's midpoint; points on a vertex are dropped; every point locks the
 * triangles whose circumcircle may hold it (its cavity) with a pseudo-random
 * priority, and the points that hold their whole cavity are inserted; then
 * flips restore the Delaunay property; with morton = 1 the vertices and
 * triangles are renumbered along a Z-order curve whenever the triangle count
 * has grown by a quarter since the last renumbering, and at the end
 * (Section 4.1: keys interleave the coordinates quantised to 32 bits over
 * the period on a periodic axis, else over the input's extent, x in the even
 * bits, and elements are ordered by the top 32 bits of the key; a
 * triangle's key is its centroid's; stable order for equal keys). Stops when
 * no triangle proposes a point. Size field (Section 2: the size bound may vary in
 * space): size_grid [grid_ny][grid_nx] host, positive scale factors at the
 * nodes of a grid over the domain (a periodic axis: grid_n nodes at spacing
 * period / grid_n from 0, wrapping; a bounded axis: grid_n nodes spanning the
 * input's extent), interpolated bilinearly; NULL for s = 1. With
 * morton = 0 original vertices keep their indices and new vertices and
 * triangles are appended. On return *n_vertices, *n_triangles, x, y, tri
 * describe the refined mesh; n_iterations (insertion iterations) and n_flips may be NULL.
 * The result does not depend on scheduling. RD_EINVAL for invalid input,
 * capacities or bounds, and (with the mesh reached so far returned) when
 * more than max_iterations iterations would be needed; RD_ENOMEM when the
 * refined mesh would exceed a capacity (the mesh reached so far is
 * returned) or device allocation fails; RD_EUNSUPPORTED when no proposed
 * point can be inserted, or a circumcentre lies more than a quarter period
 * away on a periodic axis (mesh so far returned); RD_EDEVICE. Allocates
 * about 140 bytes of device memory per triangle of capacity (about 100 more
 * with morton = 1), uses a stream
 * of its own and waits for it. */
rd_status rd_delaunay_refine(int64_t* n_vertices, double* x, double* y, int64_t max_vertices, double period_x,
                             double period_y, int64_t* n_triangles, int32_t* tri, int64_t max_triangles,
                             double max_radius, double max_ratio, const double* size_grid, int32_t grid_nx,
                             int32_t grid_ny, int32_t max_iterations, int32_t morton, int32_t* n_iterations,
                             int64_t* n_flips);

/* Many independent meshes advanced together. The batch keeps its own copy of
 * the meshes' geometry and its own HIP stream (a null stream cannot be
 * captured); rd_batch_run is ordered after pending work on `stream` and on the
 * members' streams, takes each mesh's current state, runs n_steps steps in one
 * captured HIP graph (per-mesh CFL dt each step, computed on the device),
 * writes the states back to the meshes, and makes those streams wait for it.
 * Enqueues only. Meshes must share gamma and device; members periodic on an
 * axis must share the period on that axis, and a member that is not periodic
 * on such an axis must have an extent of at most that period and no triangle or
 * wall edge spanning more than half of it along the axis (RD_EINVAL
 * otherwise). Each mesh's result is bitwise what its own rd_step_cfl would
 * give. A member
 * whose state goes non-physical during the run has its own latch set
 * (reported by rd_sync or rd_get_state on that mesh); the others do not. */
rd_status rd_batch_create(rd_mesh* const* meshes, int n_meshes, void* stream, rd_batch** out);
rd_status rd_batch_run(rd_batch* batch, int n_steps, double cfl, int scheme, int time, int precision);
rd_status rd_batch_destroy(rd_batch* batch);
/* Tile size of the batch's step (as rd_mesh_set_tile; tiles never straddle
 * two meshes, so each member is tiled exactly as it would be alone). */
rd_status rd_batch_set_tile(rd_batch* batch, int tile_triangles);
/* Autotuner of a batch: as rd_tune, timing one replay of the captured
 * n_steps-step graph per candidate; members' states are not changed. */
rd_status rd_batch_tune(rd_batch* batch, double cfl, int scheme, int time, int precision, int n_steps,
                        const int* candidates, int n_candidates, double* ms_per_step, int* best);

/* Waits for the mesh's stream. RD_ENONPHYS if a non-physical state was
 * produced since the last rd_set_state (the flag stays set), RD_EDEVICE on a
 * runtime error; otherwise the adjoint's latched status since it was last
 * reported (see rd_adjoint_step), which is then cleared. */
rd_status rd_sync(rd_mesh* mesh);

/* ---- Three dimensions (tetrahedra) --------------------------------------
 * The method of Section 3 generalised to three dimensions, as the paper's
 * closing discussion describes (a row and a column added to every matrix):
 * state (rho, rho u, rho v, rho w, e), Z = sqrt(rho)(1, u, v, w, h),
 * K_i = (|n_i| / 3) K(n_i / |n_i|) with n_i the inward normal of the face
 * opposite corner i scaled by its area; schemes RD_N, RD_LDA, RD_B, RD_BMAX,
 * RD_BMIN; forward Euler or RK2 (global lumping, vertex volume sum |T| / 4);
 * FP64; periodic boxes (each axis periodic or not; no wall or ghost
 * vertices, so a bounded axis is only meaningful for flows that do not
 * reach it). CFL limit: dt_i = 3 V_i / sum_T S_T lambda_T, S_T the largest
 * face area, lambda_T the largest |u| + c at the corners. */
typedef struct rd3_mesh rd3_mesh; /* opaque; owns its device buffers and stream */

typedef struct {
  int64_t n_vertices;
  int64_t n_tets;
  const double* x; /* [n_vertices] host */
  const double* y;
  const double* z;
  const int32_t* tet; /* [n_tets][4] host; positively oriented after minimum-image unwrapping */
  double period_x;    /* > 0: periodic axis of that length; 0: bounded */
  double period_y;
  double period_z;
  double gamma; /* > 1 */
} rd3_mesh_desc;

/* Validates (indices, 4 n_tets < 2^31, positive volumes, every vertex used),
 * precomputes face normals, volumes and the per-vertex slot order of the
 * sums (ascending tetrahedron), uploads, and creates the mesh's stream.
 * The state is zero until rd3_set_state. RD_EINVAL, RD_ENOMEM, RD_EDEVICE. */
rd_status rd3_mesh_create(const rd3_mesh_desc* desc, rd3_mesh** out);
rd_status rd3_mesh_destroy(rd3_mesh* mesh);
/* State [5][n_vertices] FP64, host (on_device = 0) or device pointer. */
rd_status rd3_set_state(rd3_mesh* mesh, const double* W, int on_device);
rd_status rd3_get_state(rd3_mesh* mesh, double* W, int on_device);
/* CFL limit of the current state times cfl (waits for the stream). */
rd_status rd3_max_dt(rd3_mesh* mesh, double cfl, double* dt);
/* One step with the given dt, or n_steps steps with dt from the CFL limit
 * computed on the device before each step. Enqueue only. */
rd_status rd3_step(rd3_mesh* mesh, double dt, int scheme, int time);
rd_status rd3_step_cfl(rd3_mesh* mesh, int n_steps, double cfl, int scheme, int time);
/* n_steps CFL steps, each kernel bracketed by HIP events on the mesh's
 * stream; ms[0..4] receive the average milliseconds per step of the CFL
 * limit, the first tetrahedron pass, the first vertex pass, the second
 * tetrahedron pass and the second vertex pass (0 for Euler). Waits. */
rd_status rd3_step_timed(rd3_mesh* mesh, int n_steps, double cfl, int scheme, int time, double* ms);
/* Waits for the mesh's stream. RD_ENONPHYS if a state with rho <= 0, p <= 0
 * or a non-finite value was produced since the last rd3_set_state (the
 * latch stays set), RD_EDEVICE on a runtime error. */
rd_status rd3_sync(rd3_mesh* mesh);

/* Message for the last non-OK status returned on this thread. */
const char* rd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RD_H */
