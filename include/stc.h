/*
 * stc.h -- C ABI of the MI355X spherical tree code.
 *
 * Evaluates the velocity of the Lagrangian barotropic vorticity equation
 * (Chen & Jablonowski, Sec. 2, the midpoint-rule particle system)
 *
 *     u_i = -(1/4pi) sum_{j != i} (x_i x x_j) zeta_j A_j / (1 - x_i . x_j)
 *
 * for N particles x_i on the unit sphere, through the spherical tree code of
 * Sec. 3: an icosahedral triangle tree, proxy charges at interpolation points
 * of each triangle (spherical Bernstein-Bezier basis), a dual tree traversal
 * with multipole acceptance criterion theta, and particle-particle (PP),
 * particle-cluster (PC), cluster-particle (CP) and cluster-cluster (CC)
 * interactions.
 *
 * Conventions for every call:
 *  - Pointers named d_* are DEVICE pointers (HIP, gfx950), h_* are HOST
 *    pointers.  The caller owns every pointer it passes; the library never
 *    frees them and keeps none of them after the call returns, except that
 *    stc_upward reads the last d_x given to stc_tree_build (see there).
 *  - Particle positions are (n, 3) FP64, row-major (x0 y0 z0 x1 y1 z1 ...).
 *    zeta, area: (n,) FP64.  Velocities are (n, 3) FP64 in INPUT order.
 *  - Ownership: the library never allocates or frees device memory.  A
 *    context's device buffers (geometry and interpolation tables, sorted
 *    particles, lists, proxy records, RK4 stage state) are carved from one
 *    caller-owned workspace (stc_workspace_size, then stc_create), which
 *    must outlive the context; the direct sums take caller scratch.  The
 *    library owns only the host-side stc_ctx, freed by stc_destroy.
 *  - All pipeline calls are asynchronous on the context's HIP stream.
 *    Host-side argument errors return at once and enqueue nothing.
 *    Device-side conditions raise a flag in device memory that the next
 *    synchronising call (stc_sync, stc_list_counts, stc_copy_*) reports:
 *    STC_ERR_CAPACITY (list capacity exceeded), STC_ERR_NONFINITE (a
 *    particle position, vorticity or area is NaN or infinite); outputs are
 *    then undefined.
 *  - A context is not thread safe.  No call aborts the process or lets a C++
 *    exception escape; stc_last_error() gives a message for the last error.
 */
#ifndef STC_H
#define STC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum stc_status {
    STC_OK = 0,
    STC_ERR_INVALID_ARG = 1, /* bad pointer, size or parameter               */
    STC_ERR_CAPACITY = 2,    /* an interaction list outgrew its capacity      */
    STC_ERR_DEVICE = 3,      /* a HIP runtime call failed                     */
    STC_ERR_STATE = 4,       /* call out of order (e.g. upward before build)  */
    STC_ERR_ALLOC = 5,       /* host allocation failed in stc_create          */
    STC_ERR_WORKSPACE = 6,   /* workspace or scratch buffer too small or
                                misaligned                                    */
    STC_ERR_NONFINITE = 7    /* non-finite position, vorticity or area        */
} stc_status;

enum { STC_FP64 = 0, STC_FP32 = 1 };           /* arithmetic of the PP/PC/CP/CC sums   */
enum { STC_DEN_DOT = 0, STC_DEN_DIST2 = 1 };   /* 1 - x.y (Sec. 2) | |x-y|^2/2 (Sec. 2, alt. kernel) */
enum { STC_LIST_PP = 0, STC_LIST_PC = 1, STC_LIST_CP = 2, STC_LIST_CC = 3 };
enum { STC_FLAG_EAGER_RK4 = 1,                /* stc_rk4 without graph capture */
       STC_FLAG_LEARNED = 2 };                /* learned gating (see stc_set_model) */
enum { STC_MAX_MEMBERS = 64 };                /* members of one batched context */

/* Method parameters (Sec. 3, dual tree traversal).
 *  theta       MAC: a pair is well separated iff (r_t + r_s) / R < theta,
 *              with r the circumradius (largest chord from the circumcentre to
 *              a vertex) and R the chord between circumcentres.  (0, 1].
 *  degree      interpolation degree d, (d+1)(d+2)/2 points per triangle. 1..14.
 *  n_crit      N_T: a triangle has "many" particles iff count > n_crit.  >= 1.
 *  max_level   depth limit of the tree (root faces are level 0).  0..12, or
 *              -1 for the default: two levels below the level at which an
 *              average node of a uniform distribution holds n_crit particles.
 *  precision   STC_FP64, or STC_FP32: PP/PC/CP/CC kernel sums in FP32 with
 *              target-relative coordinates and FP64 accumulation per tile;
 *              proxy charges, interpolation weights and the output stay FP64.
 *  denominator STC_DEN_DOT or STC_DEN_DIST2.
 *  flags       0 or a combination of STC_FLAG_EAGER_RK4, STC_FLAG_LEARNED.
 *  list_capacity entries per interaction list and per traversal frontier;
 *              0 for the default (16 * n_max, at least 65536).
 *  theta_max   learned form only: the wider acceptance parameter whose
 *              separated pairs the network judges (0 = theta).  [theta, 1].
 *
 * The learned form (STC_FLAG_LEARNED; one member): far-field interactions are
 * evaluated per list entry at one of four degrees, 4, 6, 8 or 10 (classes
 * 0..3), and `degree` (one of these) is the fallback degree.  The traversal
 * first collects candidate pairs -- well separated at theta_max with a side
 * of more than n_crit particles -- and a network (stc_set_model) accepts each
 * at a degree class or rejects it; rejected pairs are traversed by the plain
 * method (theta, the fallback degree) from there on, so without a model the
 * result is that of the fixed-degree method.                                */
typedef struct stc_params {
    double theta;
    int32_t degree;
    int32_t n_crit;
    int32_t max_level;
    int32_t precision;
    int32_t denominator;
    int32_t flags;
    int64_t list_capacity;
    double theta_max;
} stc_params;

typedef struct stc_ctx stc_ctx;

/* Launch shape of the two persistent interaction kernels (near side: PP and
 * PC; target proxies: CP and CC): workgroup size (128, 256 or 512 threads;
 * one LDS source tile and one batch of list entries per workgroup hold that
 * many items) and workgroups per compute unit (1..64; the grid is rounded up
 * to a multiple of 8, one slot per XCD).  Default {256, 48, 256, 48}.  The
 * shape changes only the grouping of the FP32/FP64 partial sums, not what is
 * summed. */
typedef struct stc_launch_config {
    int32_t near_threads;
    int32_t near_blocks_per_cu;
    int32_t far_threads;
    int32_t far_blocks_per_cu;
} stc_launch_config;

/* Message for a status code (static string). */
const char* stc_status_string(int32_t status);

/* Fills *p with theta 0.7, degree 8, n_crit 64, max_level -1, FP64, DOT. */
stc_status stc_default_params(stc_params* p);

/* Number of interpolation points (d+1)(d+2)/2 (Sec. 3, interpolation in
 * triangles); 0 if d is out of range. */
int32_t stc_n_basis(int32_t degree);

/* Number of nodes of the complete tree down to max_level: 20 (4^(L+1)-1)/3.
 * Node id of (level l, key k) is 20 (4^l - 1)/3 + k. */
int64_t stc_total_nodes(int32_t max_level);

/* The depth limit stc_create uses for max_level = -1. */
int32_t stc_default_max_level(int64_t n_max, int32_t n_crit);

/* Bytes of device workspace a context for these parameters and up to n_max
 * particles needs (host-only; no device work).  Errors as stc_create. */
stc_status stc_workspace_size(const stc_params* p, int64_t n_max, size_t* bytes);

/* Creates a context for up to n_max particles: builds the triangle geometry
 * of every node down to max_level on the host (FP64, fixed operation order)
 * and the interpolation tables, and uploads them into the caller's
 * workspace d_ws (device memory, 256-byte aligned, at least
 * stc_workspace_size bytes; STC_ERR_WORKSPACE otherwise), from which every
 * device buffer of the context is carved.  The workspace stays the caller's:
 * it must outlive the context and is not touched by anything else while the
 * context lives.  hip_stream is a hipStream_t (NULL = default stream); the
 * call synchronises it once after the uploads.  On success *out owns the
 * host-side context. */
stc_status stc_create(const stc_params* p, int64_t n_max, void* d_ws, size_t ws_bytes, void* hip_stream,
                      stc_ctx** out);

/* Ensembles (batching): a context for up to max_members independent particle
 * sets ("members") evaluated together, one kernel launch per phase for all of
 * them.  The members' particles are concatenated in one array: member m owns
 * rows [h_offsets[m], h_offsets[m+1]) of x, zeta, area and u, with
 * h_offsets a HOST array of members + 1 int64, h_offsets[0] = 0,
 * non-decreasing, h_offsets[members] <= n_max_total.  Members never interact:
 * every member gets its own tree (Sec. 3) and its own lists, and its result is
 * bitwise the one a single-member context with the same parameters gives.
 * max_level = -1 resolves with n_max_member (the largest member expected).
 * Node ids of member m are (m << node_bits) + local id (stc_node_layout).
 * 1 <= max_members <= STC_MAX_MEMBERS; 2 max_level + 5 + bits(max_members)
 * <= 32.  stc_create(p, n, ws, b, s, out) is
 * stc_create_batched(p, 1, n, n, ws, b, s, out); the workspace rules are
 * stc_create's, with its size from stc_workspace_size_batched. */
stc_status stc_workspace_size_batched(const stc_params* p, int32_t max_members, int64_t n_max_member,
                                      int64_t n_max_total, size_t* bytes);
stc_status stc_create_batched(const stc_params* p, int32_t max_members, int64_t n_max_member,
                              int64_t n_max_total, void* d_ws, size_t ws_bytes, void* hip_stream,
                              stc_ctx** out);

/* Node id layout: node id = (member << *node_bits) + local id, local ids
 * 0 .. *nodes_per_member - 1 as stc_total_nodes describes; per-node arrays
 * (stc_copy_tree) have *node_array_len entries.  Any pointer may be NULL. */
stc_status stc_node_layout(const stc_ctx* ctx, int32_t* node_bits, int64_t* nodes_per_member,
                           int64_t* node_array_len);

/* Frees the host-side context (synchronises its stream first); the caller's
 * workspace is free for other use afterwards. */
stc_status stc_destroy(stc_ctx* ctx);

/* Changes the stream later calls are enqueued on. */
stc_status stc_set_stream(stc_ctx* ctx, void* hip_stream);

/* The parameters the context resolved (max_level filled in). */
stc_status stc_get_params(const stc_ctx* ctx, stc_params* out);

/* --- the pipeline (Sec. 3) ------------------------------------------------ */

/* Tree build: locates every particle in the icosahedral triangle tree
 * (exact orientation predicates; a point on a shared edge goes to the lowest
 * root face containing it and, inside a triangle, to a corner child only if
 * strictly inside it), sorts particles by leaf (stable in input index) and
 * finds every node's particle range.  0 <= n <= n_max.  d_x must stay valid
 * and unchanged until the evaluation calls that follow have completed. */
stc_status stc_tree_build(stc_ctx* ctx, int64_t n, const double* d_x);

/* Tree build of an ensemble (see stc_create_batched); the pipeline calls
 * below then work on all its members. */
stc_status stc_tree_build_batched(stc_ctx* ctx, int32_t members, const int64_t* h_offsets,
                                  const double* d_x);

/* Upward pass: charges q_j = zeta_j A_j and, for every node with more than
 * n_crit particles, the proxy charges w_m = sum_j L_m(y_j) q_j (Sec. 3,
 * particle-cluster interaction: the paper's proxy weights omega_k transformed
 * by the inverse transposed Vandermonde matrix).  FP64.  Needs a tree. */
stc_status stc_upward(stc_ctx* ctx, const double* d_zeta, const double* d_area);

/* Dual tree traversal from the 400 root pairs (Sec. 3) -> PP, PC, CP, CC
 * lists, grouped by target.  Needs a tree. */
stc_status stc_traverse(stc_ctx* ctx);

/* Near field: the PP interactions only, u_near = -(1/4pi) x_i x sum_PP.
 * Writes d_u (n,3) (adds to it if accumulate != 0).  Needs upward+traverse. */
stc_status stc_eval_near(stc_ctx* ctx, double* d_u, int32_t accumulate);

/* Far field: the PC, CP and CC interactions with target-side interpolation
 * back to the particles.  Writes or adds to d_u like stc_eval_near. */
stc_status stc_eval_far(stc_ctx* ctx, double* d_u, int32_t accumulate);

/* One full velocity evaluation: tree build, upward pass, traversal, near and
 * far field, written to d_u (n,3) in input order. */
stc_status stc_velocity(stc_ctx* ctx, int64_t n, const double* d_x, const double* d_zeta,
                        const double* d_area, double* d_u);

/* One velocity evaluation of every member of an ensemble, all members in the
 * same launches (tree build, upward pass, traversal, near and far field). */
stc_status stc_velocity_batched(stc_ctx* ctx, int32_t members, const int64_t* h_offsets,
                                const double* d_x, const double* d_zeta, const double* d_area,
                                double* d_u);

/* One stc_velocity(ctx, n, d_x, d_zeta, d_area, d_u) captured in a HIP graph
 * (on the context's own capture stream), replayed by stc_graph_launch on the
 * context's current stream: the same kernels with the same arguments, and
 * the same result as stc_velocity, without per-kernel launch costs on the
 * host.  Host values are fixed at capture: n, the pointers, the launch
 * shapes, the forcing and its time, the network of a learned context; a
 * change of any of them needs a new graph.  The inputs may change in place
 * between replays.  Every replay is bracketed by two events recorded on the
 * launch stream (outside the graph): stc_graph_last_ms gives the last
 * replay's duration (synchronises).  A graph must be destroyed before its
 * context.  Errors as stc_velocity; STC_ERR_DEVICE if capture or
 * instantiation fails; stc_graph_last_ms before any replay: STC_ERR_STATE. */
typedef struct stc_graph stc_graph;
stc_status stc_velocity_graph(stc_ctx* ctx, int64_t n, const double* d_x, const double* d_zeta,
                              const double* d_area, double* d_u, stc_graph** out);
stc_status stc_graph_launch(stc_graph* graph);
stc_status stc_graph_last_ms(stc_graph* graph, double* ms);
stc_status stc_graph_destroy(stc_graph* graph);

/* Bytes of device scratch stc_direct / stc_direct_stream need for m targets
 * over n sources on the current device (0 when the sum is not split; the
 * split depends on the device's compute units and the kernel's occupancy).
 * Host-only.  STC_ERR_INVALID_ARG for bad sizes, precision or denominator. */
stc_status stc_direct_scratch_size(int64_t n, int64_t m, int32_t precision, int32_t denominator,
                                   size_t* bytes);

/* Direct O(N^2) sum (Sec. 2, discrete system) for m targets: d_targets (m,)
 * int64 indices into [0, n), or NULL for all (then m must equal n).  Sources
 * are all n particles, the self term excluded by index.  precision STC_FP64
 * or STC_FP32 (FP32 kernel, FP64 accumulation per tile of 256 sources).
 * d_u is (m, 3).  Asynchronous on hip_stream; needs no context.  When m is
 * too small to fill the GPU the sources are split into chunks whose partial
 * sums (chunks x m x 3 doubles) go to the caller's scratch d_scratch
 * (device memory, 8-byte aligned, scratch_bytes >= stc_direct_scratch_size;
 * STC_ERR_WORKSPACE otherwise; may be NULL when that size is 0); the chunks
 * are added in a fixed order, so the result does not vary between calls.
 * The scratch must not be reused before the call's work has completed. */
stc_status stc_direct(void* hip_stream, int64_t n, const double* d_x, const double* d_zeta,
                      const double* d_area, int64_t m, const int64_t* d_targets,
                      int32_t precision, int32_t denominator, double* d_u,
                      void* d_scratch, size_t scratch_bytes);

/* stc_direct for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Arguments, layout, result and errors as stc_direct, and the result is
 * bitwise that of stc_direct on the same device.  The chunks' partial sums
 * go to a library-owned static device array of 16 MiB per GPU (allocated by
 * the HIP runtime with the library's code object on the first call on a
 * device and held until the process ends) instead of a stream-ordered
 * allocation; this call allocates nothing.  A split that needs more than
 * 16 MiB (chunks x m x 24 bytes; at most 4 x CUs x workgroups per CU x 64
 * x 24 bytes, 12.6 MB on 256 CUs) returns STC_ERR_WORKSPACE and enqueues
 * nothing.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads) race.  Every partial
 * sum is written before it is read, so nothing is cleared between calls. */
stc_status stc_direct_noalloc(void* hip_stream, int64_t n, const double* d_x, const double* d_zeta,
                              const double* d_area, int64_t m, const int64_t* d_targets,
                              int32_t precision, int32_t denominator, double* d_u);

/* Stream function (Sec. 2, stream function and Green's function):
 *   psi_i = (1/4pi) sum_{j != i} zeta_j A_j log(den(x_i, x_j)),
 * den = 1 - x.y or |x - y|^2 / 2 per the context's denominator, through the
 * same tree, proxy charges and lists as the velocity (the method is kernel
 * independent, Sec. 3) with the logarithmic kernel in the PP / PC / CP / CC
 * interactions.  The sign is the one for which Delta psi = zeta (for
 * zero-mean zeta) and u = x x grad psi is the velocity of stc_velocity.
 * d_psi: n FP64 values, input order.  The forcing, if set, applies to the
 * charges as for the velocity.  STC_ERR_INVALID_ARG for a learned context
 * (its gating network judges velocity interactions) and for bad sizes or
 * pointers, as stc_velocity. */
stc_status stc_stream_function(stc_ctx* ctx, int64_t n, const double* d_x, const double* d_zeta,
                               const double* d_area, double* d_psi);

/* The stream function of every member of an ensemble in the same launches,
 * members as for stc_velocity_batched; d_psi: n_total values.  Each member's
 * values are bitwise those of a single-member context. */
stc_status stc_stream_function_batched(stc_ctx* ctx, int32_t members, const int64_t* h_offsets,
                                       const double* d_x, const double* d_zeta, const double* d_area,
                                       double* d_psi);

/* Direct O(N m) stream function at m targets, arguments (scratch included)
 * as stc_direct; d_psi holds m FP64 values. */
stc_status stc_direct_stream(void* hip_stream, int64_t n, const double* d_x, const double* d_zeta,
                             const double* d_area, int64_t m, const int64_t* d_targets, int32_t precision,
                             int32_t denominator, double* d_psi, void* d_scratch, size_t scratch_bytes);

/* Classical RK4 (Sec. 4) for n_steps steps of dt on (x, zeta):
 *   dx/dt = u(x; zeta A),  dzeta/dt = -2 omega u_z  (Sec. 2, discrete system)
 * Every stage is a full stc_velocity (tree rebuilt).  Stage positions are
 * used as computed (off the sphere), so the context must use STC_DEN_DIST2
 * (Sec. 2: the |x-y|^2/2 form stays well defined off the sphere, while
 * 1 - x.y vanishes for close pairs there); otherwise STC_ERR_INVALID_ARG.
 * After each step x <- x / |x|.  d_x, d_zeta are updated
 * in place.  Units are the caller's (dt * omega dimensionless).
 * Unless the context has STC_FLAG_EAGER_RK4, one step is captured once into a
 * HIP graph (on a stream the context creates) and the graph is launched on
 * the context stream once per step; it is re-captured when n, the pointers,
 * dt or omega change.  Results are bitwise those of the eager path. */
stc_status stc_rk4(stc_ctx* ctx, int64_t n, double* d_x, double* d_zeta, const double* d_area,
                   double dt, double omega, int32_t n_steps);

/* --- adaptive mesh refinement (Appendix A; Gaussian vortex, Sec. 4.3) ------ */

/* The particles are the vertices of a triangulation; every triangle of the
 * initial mesh (n_faces triangles over the n0 initial particles, h_faces
 * host int32 (n_faces, 3), counter-clockwise seen from outside) is the root of
 * a refinement tree.  An adaptation pass tests every leaf triangle T (and
 * every refined one whose children are leaves) with its vertices' current
 * positions and vorticities:
 *   C(T) = |A_T (zeta_1 + zeta_2 + zeta_3) / 3| >= eps1  or
 *          max zeta - min zeta >= eps2
 * (A_T the spherical triangle area), merges refined triangles with leaf
 * children where C no longer holds (never below the initial mesh), then
 * splits leaves where C holds into four (edge midpoints (a + b) / |a + b|),
 * at most max_levels below the initial mesh.  Readings where the appendix is
 * silent: the circulation test uses its magnitude; all decisions of a pass
 * use the state at its start, merging before splitting (one level per pass);
 * a midpoint particle is shared by the two triangles of its edge and removed
 * when no leaf has it as a vertex; a new particle takes the mean absolute
 * vorticity zeta + omega_abs z of its edge's ends (omega_abs = 2 Omega, the
 * quantity the particle system carries unchanged) minus omega_abs z at its
 * position; triangles carry their areas (the flow is incompressible): an
 * initial triangle its spherical area at the first pass, the children of a
 * split the parent's carried area in proportion to their spherical areas
 * then, a merged triangle its own again; A_T in the circulation test is the
 * carried area, and the quadrature weights are A_i = sum of carried A_T / 3
 * over the leaves having i as a vertex (valid after the first pass).  The
 * live particles (the tree code's input) are kept in slot order: the
 * initial particles first, in input order. */
typedef struct stc_amr stc_amr;
typedef struct stc_amr_params {
    double eps1, eps2;   /* thresholds of the circulation and variation tests  */
    double omega;        /* Omega of the particle system (the 2 Omega z term)  */
    int32_t max_levels;  /* refinement levels below the initial mesh, 0..6    */
} stc_amr_params;

/* Device workspace bytes of an adaptive mesh and the largest particle count
 * it can reach (*max_particles: every midpoint of max_levels refinements);
 * host-only.  STC_ERR_INVALID_ARG for bad parameters or face indices. */
stc_status stc_amr_workspace_size(const stc_amr_params* p, int64_t n0, int64_t n_faces,
                                  const int32_t* h_faces, size_t* bytes, int64_t* max_particles);

/* Creates the adaptive mesh in the caller's workspace (256-byte aligned,
 * stc_amr_workspace_size bytes; STC_ERR_WORKSPACE otherwise): the slot tables
 * of every triangle and particle refinement can create are built on the host
 * and uploaded; the initial particles are live and every root a leaf.  The
 * particle state is set with stc_amr_set_state.  Synchronises hip_stream. */
stc_status stc_amr_create(const stc_amr_params* p, int64_t n0, int64_t n_faces, const int32_t* h_faces,
                          void* d_ws, size_t ws_bytes, void* hip_stream, stc_amr** out);
stc_status stc_amr_destroy(stc_amr* amr);

/* Writes positions d_x (n, 3) and vorticities d_zeta (n) of the live
 * particles (in the order stc_amr_particles gives; n must be the current
 * count) into the mesh.  Asynchronous. */
stc_status stc_amr_set_state(stc_amr* amr, int64_t n, const double* d_x, const double* d_zeta);

/* One adaptation pass, then the live particles compacted into the arrays
 * stc_amr_particles returns; synchronises (the new particle count). */
stc_status stc_amr_adapt(stc_amr* amr);

/* The live particles: count and device arrays x (n, 3), zeta (n), area (n)
 * inside the mesh's workspace (valid until the next pass; the tree code may
 * read and, through stc_amr_rk4, update them).  No synchronisation. */
stc_status stc_amr_particles(stc_amr* amr, int64_t* n, double** d_x, double** d_zeta, double** d_area);

/* After the last pass: live particles, leaf triangles, triangles merged and
 * split by that pass, and the particle capacity.  Synchronises. */
stc_status stc_amr_stats(stc_amr* amr, int64_t* n_particles, int64_t* n_leaves, int64_t* merged,
                         int64_t* split, int64_t* max_particles);

/* Slot of every live particle (h_slots, up to cap) and the edge ends of the
 * first cap particle slots (h_ends (cap, 2); -1 for initial particles);
 * either may be NULL.  Synchronises. */
stc_status stc_amr_copy_slots(stc_amr* amr, int64_t cap, int32_t* h_slots, int32_t* h_ends);

const char* stc_amr_last_error(const stc_amr* amr);

/* n_steps RK4 steps of the live particles with the tree code of ctx (its
 * parameters; the |x - y|^2 / 2 denominator; capacity >= the mesh's
 * particle capacity), each followed by one adaptation pass.  The steps run
 * eagerly (the particle count changes between steps).  ctx and amr must
 * enqueue on the same stream.  Synchronises once per step. */
stc_status stc_amr_rk4(stc_amr* amr, stc_ctx* ctx, double dt, double omega, int32_t n_steps);

/* RK4 of every member of an ensemble (same dt and omega), each stage one
 * stc_velocity_batched; graph-captured like stc_rk4 (re-captured when the
 * offsets change). */
stc_status stc_rk4_batched(stc_ctx* ctx, int32_t members, const int64_t* h_offsets, double* d_x,
                           double* d_zeta, const double* d_area, double dt, double omega,
                           int32_t n_steps);

/* --- vorticity forcing (Sec. 4.4, polar vortex collapse) ----------------------
 *
 * With a forcing set, every evaluation of the context (stc_upward, hence
 * stc_velocity, the batched calls and every RK4 stage) uses the source charges
 *   q_j = (zeta_j - F_R(x_j, t)) A_j,
 *   F_R = (3/5) omega k^2 A(t) B(lat) cos(k lon),
 *   A(t) = (1 - cos(pi t / T_p)) / 2 on [0, T_p), 1 on [T_p, T_f - T_p),
 *          (1 + cos(pi (t - T_f + T_p) / T_p)) / 2 on [T_f - T_p, T_f), 0 for
 *          t >= T_f and (reading) for t < 0,
 *   B(lat) = s e^(1 - s), s = tan^2(lat1) / tan^2(lat), for lat > 0; 0 for lat <= 0,
 * with lat, lon the latitude and longitude of the direction of x_j (stage
 * points of RK4 are off the sphere).  The particles' own zeta still evolves by
 * dzeta/dt = -2 omega u_z.  Units are the caller's (the paper: days, omega =
 * 2 pi per day, T_p = 4, T_f = 15, lat1 = pi / 3, k = 1 or 2).
 * `time` is t of the next single evaluation and the start time of the next
 * stc_rk4 / stc_rk4_batched call, whose stages see t, t + dt/2, t + dt/2,
 * t + dt of each step; after the call the context's time has advanced by
 * n_steps dt (stc_get_forcing reads it).
 * Errors: STC_ERR_INVALID_ARG (enqueues nothing) unless 0 <= k <= 16, omega
 * finite, 0 < lat1 < pi/2, T_p > 0, T_f >= 2 T_p and time finite.  A NULL f
 * switches the forcing off.  Setting or clearing drops a captured RK4 step. */
typedef struct stc_forcing {
    int32_t k;        /* zonal wavenumber */
    double omega;     /* rotation rate in the amplitude (3/5) omega k^2 */
    double lat1;      /* latitude of maximum forcing, radians */
    double t_ramp;    /* T_p: ramp-up (and ramp-down) time */
    double t_total;   /* T_f: the forcing is zero from T_f on */
    double time;      /* forcing time t (see above) */
} stc_forcing;
stc_status stc_set_forcing(stc_ctx* ctx, const stc_forcing* f);
/* Copies the forcing (with the current time) into *f and 1 / 0 into *on. */
stc_status stc_get_forcing(const stc_ctx* ctx, stc_forcing* f, int32_t* on);
/* F_R(x_i, f->time) of the forcing above at n positions d_x ((n, 3) row-major
 * FP64, any length) into d_out (n FP64), input order; asynchronous on
 * hip_stream (NULL: the null stream).  STC_ERR_INVALID_ARG for an invalid
 * forcing, n < 0, or NULL / unaligned pointers with n > 0. */
stc_status stc_forcing_field(void* hip_stream, const stc_forcing* f, int64_t n, const double* d_x,
                             double* d_out);

/* --- the learned form: gating network ---------------------------------------
 *
 * Network: 12 inputs -> 64 -> 64 -> 4 outputs, ReLU, BF16 weights and
 * activations, FP32 accumulation on the matrix cores.  Parameters are one
 * flat BF16 vector of stc_mlp_param_count() = 5252 values: W1 [12][64]
 * (input f -> hidden h, row-major), b1 [64], W2 [64][64], b2 [64], W3 [64][4],
 * b3 [4].  Inputs: rows of 16 BF16 features (the 12 below, then 4 zeros).
 * Outputs per row: o0 acceptance logit, o1..o3 ordinal logits ("degree above
 * 4", "above 6", "above 8"); a pair is accepted iff o0 > 0, at degree class
 * #{k : o_k > 0}.  Features of a candidate (t, s), R the chord between the
 * circumcentres, r the circumradii, Q_x the sum of |q| over node x, Q over all
 * particles:  [n_t > n_crit], [n_s > n_crit] (1 or 0), level_t / 8, level_s / 8, r_t/R,
 * r_s/R, (r_t + r_s)/R, -log10 R / 2, log10(Q_s/Q)/8 + 1, |sum_s q|/Q_s,
 * log10(|w_s^(4)|_1 / Q_s)/2 (degree-4 proxy charges; 0 for a small source),
 * log10(Q_t/Q)/8 + 1.  Training loss per row: a(y0) BCE(o0, y0) + y0 sum_k
 * h(y_k) BCE(o_k, y_k) (labels y: accept, then the three ordinal targets;
 * a(0) = 8, a(1) = 1, h(1) = 8, h(0) = 1: accepting a reject-labelled pair
 * and choosing a degree below the labelled one weigh eight times).  */

/* The BF16 parameters the traversal of a learned context uses (device
 * pointer, 16-byte aligned, kept until replaced; NULL rejects every candidate,
 * i.e. the fixed-degree method).  The caller keeps the buffer alive. */
stc_status stc_set_model(stc_ctx* ctx, const uint16_t* d_params);

/* Training samples from the current tree (after stc_tree_build and
 * stc_upward of a learned context): the candidates of theta_max, their
 * features (d_features: cap x 16 BF16), for each degree class the largest
 * error over the target particles of the interaction the pair would get at
 * that degree against the exact pair sum (d_errors: cap x 4 FP64, W units:
 * the sum before the cross product), and labels (d_labels: cap x 4 float):
 * accept iff some class has error <= abs_tol, ordinal targets from the
 * smallest such class.  Samples are in (target id, source id) order.  *n_out =
 * number of candidates (samples beyond cap are dropped and STC_ERR_CAPACITY
 * returned).  Synchronises.  The lists of the
 * context are invalid afterwards (evaluate again). */
stc_status stc_learned_samples(stc_ctx* ctx, double abs_tol, int64_t cap, uint16_t* d_features,
                               float* d_labels, double* d_errors, int64_t* n_out);

/* Introspection after a learned traversal or stc_learned_samples: candidate
 * pairs (2 x int64 each, in the order of the sample arrays), network outputs
 * (4 floats; written only when a model is set) and features (16 BF16; after
 * a traversal only when a model is set); any may be NULL.  Synchronises. */
stc_status stc_copy_candidates(stc_ctx* ctx, int64_t cap, int64_t* h_pairs, float* h_out,
                               uint16_t* h_feat, int64_t* n_out);

/* Degree class (0..3) of every entry of list `type`, in stc_copy_list order
 * (all 0 for a single-degree context). */
stc_status stc_copy_list_classes(stc_ctx* ctx, int32_t type, int64_t cap, int32_t* h_class,
                                 int64_t* n_out);

int32_t stc_mlp_param_count(void);

/* Device workspace bytes stc_mlp_grad / stc_mlp_train need for a batch. */
int64_t stc_mlp_workspace_bytes(int64_t n_batch);

/* Network outputs (n x 4 float) for n input rows; asynchronous on hip_stream.
 * d_x, d_out 16-byte aligned. */
stc_status stc_mlp_forward(void* hip_stream, int64_t n, const uint16_t* d_x, const uint16_t* d_params,
                           float* d_out);

/* Gradient (5252 floats, FP32) and loss (1 float) of the mean training loss
 * over the n rows d_index[0..n) of (d_x, d_y) (d_index NULL: rows 0..n);
 * d_y: rows of 4 floats.  The sum over rows runs in a fixed order. */
stc_status stc_mlp_grad(void* hip_stream, int64_t n, const int32_t* d_index, const uint16_t* d_x,
                        const float* d_y, const uint16_t* d_params, float* d_ws, int64_t ws_bytes,
                        float* d_grad, float* d_loss);

/* Label unit of the learned form's training data: 4 pi sqrt(mean_i |u_i|^2)
 * over n velocities d_u (n, 3) FP64 -- the size of W, the sum that the cross
 * product with x turns into u -- written to *d_scale (one FP64, device).
 * Fixed summation order (repeatable).  Asynchronous on hip_stream. */
stc_status stc_label_scale(void* hip_stream, int64_t n, const double* d_u, double* d_scale);

/* Device workspace bytes stc_mlp_calibrate needs for n samples. */
int64_t stc_mlp_calibrate_workspace_bytes(int64_t n);

/* Calibration of a trained network's decisions on n labelled samples (d_x
 * (n, 16) BF16 features, d_y (n, 4) labels as stc_learned_samples writes
 * them): with o the network's outputs (stc_mlp_forward), da is the smallest
 * value of the grid {0} + 200 values geometric in [1e-3, 64] at which at
 * most max_false_accept of all samples are labelled "reject" yet accepted
 * (o0 - da > 0), and dc the smallest at which at most max_under_class of the
 * samples labelled "accept" and accepted get fewer ordinal steps than
 * labelled (#{k: o_k + dc > 0} < y1 + y2 + y3); the grid's largest value if
 * none meets a bar.  d_params_out receives d_params with b3[0] - da and
 * b3[1..3] + dc (FP64 shift, rounded to FP32 then BF16, nearest even), and
 * d_shifts (2 FP64, device) {da, dc}.  d_ws: stc_mlp_calibrate_workspace_bytes
 * of device scratch (STC_ERR_WORKSPACE if smaller); d_x, d_y, d_ws 16-byte
 * aligned.  Asynchronous on hip_stream. */
stc_status stc_mlp_calibrate(void* hip_stream, int64_t n, const uint16_t* d_x, const float* d_y,
                             const uint16_t* d_params, double max_false_accept, double max_under_class,
                             void* d_ws, int64_t ws_bytes, uint16_t* d_params_out, double* d_shifts);

/* Adam training on the GPU: `epochs` passes over the n_samples rows in
 * minibatches of `batch` (a seeded bijection of the rows per epoch), each
 * step a gradient (as stc_mlp_grad) and an Adam update (beta 0.9, 0.999,
 * eps 1e-8, learning rate lr) of the FP32 master weights d_master with
 * moments d_m1, d_m2 (5252 floats each, zero at the start of training), whose
 * BF16 copy is written to d_params (first from d_master, then after every
 * step).  d_index: batch int32 of scratch.  d_loss
 * (optional): one float per step, the minibatch loss before the step.
 * Asynchronous on hip_stream. */
stc_status stc_mlp_train(void* hip_stream, int64_t n_samples, const uint16_t* d_x, const float* d_y,
                         int32_t epochs, int32_t batch, float lr, uint64_t seed, float* d_master,
                         float* d_m1, float* d_m2, uint16_t* d_params, int32_t* d_index, float* d_ws,
                         int64_t ws_bytes, float* d_loss);

/* --- launch shapes ------------------------------------------------------------ */

/* The shape used for a total particle count n_total (size classes are
 * powers of two: the shape applies to every n with the same bit length). */
stc_status stc_get_launch_config(const stc_ctx* ctx, int64_t n_total, stc_launch_config* out);

/* Sets the shape for n_total's size class, or, with n_total < 0, the default
 * for classes without one. */
stc_status stc_set_launch_config(stc_ctx* ctx, int64_t n_total, const stc_launch_config* cfg);

/* Times every candidate shape (workgroup sizes 128/256/512 x 8, 16, 24, 32,
 * 48 or 64 workgroups per CU, for each of the two kernels) on the lists of the last
 * traversal, `repeats` launches each after one warm-up, keeps the fastest
 * for the current size class (the precision and degree are the context's)
 * and writes it to *out.  Needs stc_upward and stc_traverse (or a velocity
 * evaluation) first; synchronises.  The evaluation's output is not touched,
 * internal accumulators are: evaluate again afterwards. */
stc_status stc_autotune(stc_ctx* ctx, int32_t repeats, stc_launch_config* out);

/* --- introspection (these synchronise the context stream) ------------------ */

/* Waits for queued work; reports device-side error flags. */
stc_status stc_sync(stc_ctx* ctx);

/* counts[4]: list lengths PP, PC, CP, CC of the last traversal.  If
 * kernel_evals != NULL, *kernel_evals[0..3] receive the number of kernel
 * evaluations each list implies (PP: n_t n_s, minus n_t on self pairs; PC:
 * n_t n_p; CP: n_p n_s; CC: n_p^2). */
stc_status stc_list_counts(stc_ctx* ctx, int64_t counts[4], int64_t kernel_evals[4]);

/* Copies list `type` as (target id, source id) pairs, sorted by (t, s), into
 * h_pairs (2 * cap int64).  *n_out = list length (may exceed cap: then only
 * cap pairs are written and STC_ERR_CAPACITY is returned).  With h_pairs NULL
 * and cap 0 it only reports the length. */
stc_status stc_copy_list(stc_ctx* ctx, int32_t type, int64_t cap, int64_t* h_pairs,
                         int64_t* n_out);

/* Copies the tree: h_perm (n) = input index of the i-th particle in tree
 * order (indices into the concatenated arrays for an ensemble); h_count
 * (node_cap) = particle count of each node id.  Either may be NULL.
 * node_cap must be >= the node array length (stc_node_layout; for a single
 * member stc_total_nodes(max_level)) if h_count != NULL. */
stc_status stc_copy_tree(stc_ctx* ctx, int64_t n, int32_t* h_perm, int64_t node_cap,
                         int32_t* h_count);

/* Copies the proxy charges w (n_p) of one node (zero if the node has at most
 * n_crit particles). */
stc_status stc_copy_proxy_charges(stc_ctx* ctx, int64_t node_id, double* h_w);

/* Host-only geometry introspection (no device work): vertices (9), the
 * circumcentre (3) and radius (1) of a node (of any member: the local part of
 * the id is used), as used by the traversal. */
stc_status stc_node_geometry(const stc_ctx* ctx, int64_t node_id, double* h_v9, double* h_c3,
                             double* h_r);

/* Host-only: builds the geometry of the complete tree down to max_level
 * without a device (for checks on machines without a GPU).  h_v: 9 doubles
 * per node, h_c: 3, h_r: 1; each array sized for stc_total_nodes(max_level). */
stc_status stc_geometry_tables(int32_t max_level, double* h_v, double* h_c, double* h_r);

/* Host-only: the reference interpolation points (n_p x 3 planar
 * barycentrics) and the inverse reference Vandermonde matrix (n_p x n_p,
 * row k = basis index, column m = point index) for degree d. */
stc_status stc_reference_tables(int32_t degree, double* h_points, double* h_vinv);

/* Phase timing.  stc_set_timing(ctx, k) with k > 0 creates HIP events for k
 * evaluations; each following evaluation (stc_velocity, or the pipeline calls
 * that make one up) records a begin and an end event around each of its
 * phases, on the stream the phase runs on: 0 tree build, 1 upward pass, 2
 * traversal (incl. list sort), 3 near-side interactions (one kernel: PP and
 * PC), 4 target-proxy interactions (one kernel: CP and CC, the values at the
 * target proxy points), 5 interpolation (the coefficients formed from those
 * values, the interpolation to particles) and output.
 * Phase 1 runs on the context's side stream while phase 2 runs (in the
 * learned form until the gating, which waits for it), so the phases of an
 * evaluation need not add up to its duration.  k = 0 turns timing off and
 * frees the events.  stc_phase_times synchronises and returns
 * the summed milliseconds per phase over the recorded evaluations (ms[6]) and
 * their number; recording restarts afterwards.  Evaluations beyond k are not
 * recorded. */
stc_status stc_set_timing(stc_ctx* ctx, int32_t max_evals);

/* As stc_set_timing, but only the phases whose bits are set in phase_mask
 * (bit p = phase p above) are bracketed by events; the others report 0 ms.
 * Each recorded event adds a few microseconds between kernels, so a
 * benchmark that needs one phase's time times only that one. */
stc_status stc_set_timing_phases(stc_ctx* ctx, int32_t max_evals, uint32_t phase_mask);
stc_status stc_phase_times(stc_ctx* ctx, double ms[6], int64_t* n_evals);

/* Message of the last error on this context ("" if none). */
const char* stc_last_error(const stc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* STC_H */
