/*
 * hyperlag.h -- C-ABI of libhyperlag.so: one second-order cell-centred
 * Lagrangian ADER-MOOD time step for neo-Hookean solids on 2D triangle and
 * 3D tetrahedral meshes, computed by HIP kernels on one AMD Instinct GPU
 * (gfx950), in FP64 throughout.
 *
 * Method: Boscheri, Loubere & Maire, "A cell-centered Lagrangian ADER-MOOD
 * finite volume scheme on unstructured meshes for a class of
 * hyper-elasticity models" (arXiv 2104.02139):
 *   - conservation laws and B evolution: Section 2.2 (eqs. cl, trcb);
 *   - neo-Hookean law: Section 2.2.4 (eqs. EOS_neoHook, cstnh);
 *   - geometry and corner vectors: Section 3.1 (eq. def_lcpncp);
 *   - subcell force and nodal solver: Section 3.3 (eqs. subforce,
 *     nodal_solver, Mcp);
 *   - ADER midpoint update and Crank-Nicolson B update: Section 3.4
 *     (eqs. tau_c^n .. subforce^n, firstB, CN_B);
 *   - MOOD detection and cascade: Section 3.5 (eqs. PAD, RDMP), Section
 *     3.7 (Figure sketch);
 *   - time step: Section 3.6 (eqs. CFL, CFL2);
 *   - boundary conditions: Section 3.8 and Appendix B (eq. sBC1).
 *
 * Conventions
 *   - Every call returns hl_status: 0 = HL_OK, < 0 error, > 0 warning.  No
 *     exception crosses the ABI.  hl_status_str() gives the text.
 *   - A failed call leaves the held state unchanged.
 *   - Input arrays are BORROWED for the duration of the call only; the
 *     library copies what it keeps.  "on_device" != 0 means the pointer is
 *     HIP device memory (for instance a torch tensor's data_ptr()),
 *     otherwise host memory.
 *   - All arrays are row-major in the caller's numbering: node vectors
 *     [n_nodes][dim], cell vectors [n_cells][dim], B as [n_cells][nB] with
 *     nB = 6 components (11,22,33,12,13,23) in 3D and nB = 3 components
 *     (11,22,12) in 2D (plane strain, B33 == 1).
 *   - The context owns every device buffer it allocates (hipMalloc) and
 *     frees them in hl_destroy.  All work is enqueued on the stream given
 *     to hl_create (borrowed, may be NULL for the default stream); calls
 *     that return host data synchronise that stream.
 *   - Calls on one context are not thread-safe; distinct contexts are
 *     independent.
 */
#ifndef HYPERLAG_H
#define HYPERLAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hl_ctx hl_ctx;

typedef enum {
    HL_OK = 0,
    HL_WARN_PARACHUTE_INADMISSIBLE = 1, /* a first-order cell is not admissible */
    HL_E_INVALID = -1,                  /* bad argument                          */
    HL_E_DEGENERATE_CELL = -2,          /* a cell with V <= 0 at upload           */
    HL_E_NONCONFORMING = -3,            /* the cells do not form a conforming mesh */
    HL_E_OOM = -4,                      /* device allocation failed              */
    HL_E_HIP = -5,                      /* a HIP runtime call failed             */
    HL_E_STATE = -6                     /* call order (no mesh / no state yet)   */
} hl_status;

/* Scheme parameters (Sections 3.5 and 3.6).  Paper values: c_v = 0.2,
 * c_i = 0.1, delta0 = 1e-4, delta1 = 1e-3, c_cfl = 0.4 (2D) / 0.25 (3D). */
typedef struct {
    double c_cfl;   /* acoustic CFL number                                  */
    double c_v;     /* bound on the relative volume change per step        */
    double c_i;     /* bound on the growth of dt per step                  */
    double delta0;  /* absolute relaxed-DMP tolerance on rho               */
    double delta1;  /* relative relaxed-DMP tolerance on rho               */
    double eps_tol; /* eps = e - |v|^2/2 is troubled below -eps_tol (|e| + |v|^2/2) */
    int32_t detect; /* 0: accept the unlimited second-order candidate      */
    int32_t cascade;/* MOOD cascade (Section 3.5): 2 (or 0) P1 -> P0;
                       3 P1 -> P1 with the Barth-Jespersen limiter -> P0    */
    double shear_a; /* shear energy family (eq. familiy_energies), in
                       [-1, 1/2] (the hyperbolic range): -1 neo-Hookean
                       (the default), 0 the paper's non-linear law          */
    int32_t eos;    /* volumetric part: 0 the energy of eq. EOS_neoHook with
                       K = lambda + 2 mu / 3 (default); 1 the stiffened gas
                       (eq. EOS_stiffened_gas): p = (gamma - 1)(eps - Psi_s)
                       / tau - gamma p_inf with eps = e - |v|^2 / 2 and Psi_s
                       the shear energy, sound speed a^2 = tau (gamma (p +
                       p_inf) + 4 mu / 3), eps reconstructed and advanced by
                       d eps/dt = tau T : grad v in the predictor, a state
                       with p + p_inf <= 0 troubled, hl_state_init at p = 0
                       (e += gamma p_inf tau / (gamma - 1)).  eos 1 needs
                       cascade 0 or 2, gamma > 1, p_inf >= 0               */
    int32_t reserved;
    double sg_gamma;/* stiffened-gas gamma (default 2.2, the droplet test)  */
    double sg_pinf; /* stiffened-gas p_inf (default 1e6)                    */
} hl_params;

/* Per-step report.  Filled by hl_step / hl_step_replay when non-NULL. */
typedef struct {
    double dt_used;      /* dt of the step just taken (mesh 0)              */
    double dt_next;      /* CFL-controlled dt for the next step (mesh 0)    */
    double dt_acoustic;  /* C_CFL min L_c / a_c at t^{n+1}                  */
    double dt_volume;    /* C_v dt min V^{n+1} / |V^{n+1} - V^n|            */
    double mass, mom[3], energy, kinetic, elastic; /* sums over all cells   */
    int64_t n_p0;        /* cells advanced at first order                  */
    int64_t n_flag_first;/* cells flagged on the first candidate            */
    int32_t mood_iters;  /* candidate evaluations (1 = nothing flagged)     */
    int32_t status;      /* 1: some first-order cell is not admissible      */
    int64_t n_limited;   /* cells advanced with limited slopes (cascade 3)  */
    int64_t n_contact;   /* contact candidates held by the plane afterwards */
    int32_t trials;      /* step evaluations (> 1: a contact event redid it) */
    int32_t clipped;     /* 1: dt was cut to a contact impact time          */
    int64_t n_recomputed;/* cell updates redone by the MOOD passes: per pass,
                            the cells sharing a node with a newly flagged
                            cell (Section 3.5: troubled cells go back with
                            their neighbours)                              */
    double gcl_defect;   /* involution monitor of the geometric
                            conservation law (eq. GCL): max over cells of
                            |V(x^{n+1}) - V(x^n) - dt sum_p Cbar_cp . v*_p|
                            / V(x^n), Cbar_cp the Simpson average of the
                            corner vectors over the step (zero up to
                            roundoff for this scheme)                      */
    double detB_defect;  /* max over cells of |sqrt(det B^{n+1}) - J^{n+1}|,
                            J = rho0 tau (eq. test_detB_rho)               */
    int64_t n_detB;      /* cells where that difference is >= L_c^3, L_c the
                            in-sphere diameter at t^{n+1} (eq. test_detB_rho) */
} hl_step_info;

/* Fields for hl_query / hl_upload_field. */
enum {
    HL_X = 0,     /* node positions          [n_nodes][dim]   double       */
    HL_VHAT = 1,  /* carried node velocity   [n_nodes][dim]   double       */
    HL_TAU = 2,   /* specific volume         [n_cells]        double       */
    HL_V = 3,     /* cell velocity           [n_cells][dim]   double       */
    HL_E = 4,     /* specific total energy   [n_cells]        double       */
    HL_B = 5,     /* left Cauchy-Green       [n_cells][nB]    double       */
    HL_VSTAR = 6, /* node velocity of the last step [n_nodes][dim] (query) */
    HL_ORDER = 7, /* cascade level of each cell in the last step: 0
                     unlimited second order, 1 Barth-Jespersen limited,
                     2 first order; [n_cells] uint8 (query)                */
    HL_MASS = 8,  /* cell mass               [n_cells]        double (query) */
    HL_T = 9      /* Cauchy stress [n_cells][6] (11,22,33,12,13,23) in 3D,
                     [n_cells][4] (11,22,12,33) in 2D (query)              */
};

/* Create a context on HIP device `device`; work goes to `hip_stream`
 * (a hipStream_t, borrowed; NULL = default stream). */
hl_status hl_create(hl_ctx **out, int device, void *hip_stream);

/* Free every device buffer and the context.  NULL is accepted. */
hl_status hl_destroy(hl_ctx *ctx);

/* Batch of independent meshes of one dimension in one context: every stage
 * of hl_step runs as one launch over all of them, the CFL reduction gives
 * one dt per mesh (not in the paper: a throughput mode for many small
 * meshes).  node_offsets / cell_offsets: [n_meshes + 1] host arrays, first
 * entry 0, non-decreasing; x0, nwall, normals and the per-cell arrays of
 * hl_state_init are the meshes' arrays concatenated in order; `cells`
 * holds mesh-local node numbers (0 .. nodes of that mesh - 1). */
hl_status hl_mesh_upload_batch(hl_ctx *ctx, int dim, int n_meshes, const int64_t *node_offsets,
                               const int64_t *cell_offsets, const double *x0, const int32_t *cells,
                               const uint8_t *nwall, const double *normals, int on_device);

/* Upload a simplicial mesh (Section 3.1, "Mesh and notation").
 *   dim           2 (triangles) or 3 (tetrahedra)
 *   x0            [n_nodes][dim] initial node positions
 *   cells         [n_cells][dim+1] node indices, every cell positively
 *                 oriented (V > 0), else HL_E_DEGENERATE_CELL; the cells
 *                 must form a conforming mesh, else HL_E_NONCONFORMING
 *                 (the checks of hl_mesh_check)
 *   nwall         [n_nodes] number of slip-wall constraints at the node
 *                 (0 = free, dim = node held fixed), or NULL for none
 *   normals       [n_nodes][dim][dim]: the first nwall[p] rows are the unit
 *                 wall normals of node p (Appendix B symmetry/wall BC), or
 *                 NULL when nwall is NULL
 * Builds the node->corner lists (cells ascending in the internal numbering,
 * see hl_set_numbering, then local node order).  Replaces any previous mesh
 * and discards the state.  n_cells may be 0. */
hl_status hl_mesh_upload(hl_ctx *ctx, int dim, int64_t n_nodes, const double *x0,
                         int64_t n_cells, const int32_t *cells, const uint8_t *nwall,
                         const double *normals, int on_device);

/* Internal numbering of the meshes uploaded from now on (Section 3.9,
 * "Meshing and parallelization": the cells of a partition are numbered for
 * locality).  HL_NUMBERING_SPATIAL (the default) renumbers, within each
 * mesh, the cells along a Hilbert curve through their centroids (J.
 * Skilling's transpose method, 21 bits per axis in 3D, 31 in 2D, one scale
 * for all axes; ties in the caller's order) and the nodes in the order those
 * cells first use them, so that the gathers of the step touch neighbouring
 * memory whatever order the caller's mesh comes in.  HL_NUMBERING_KEEP
 * keeps the caller's numbering.  Either way every array at this interface
 * stays in the caller's numbering; only sums over a node's cells (taken in
 * the internal cell order) change at the level of rounding. */
enum { HL_NUMBERING_KEEP = 0, HL_NUMBERING_SPATIAL = 1 };
hl_status hl_set_numbering(hl_ctx *ctx, int numbering);

/* Check a simplicial mesh on the host, with no context and no GPU (host
 * arrays; the same checks hl_mesh_upload runs, Section 3.1 "Mesh and
 * notation": cells of positive measure that meet face to face):
 *   HL_E_INVALID          node id out of range, non-finite position;
 *   HL_E_DEGENERATE_CELL  a cell with V <= 0 (not positively oriented);
 *   HL_E_NONCONFORMING    a face shared by more than two cells, two cells
 *                         on the same side of a shared face, (3D) a boundary
 *                         edge on an odd number of boundary faces, or a
 *                         node lying on a boundary face (2D: edge) it is not
 *                         a vertex of (a hanging node), within 1e-9 of the
 *                         face's size. */
hl_status hl_mesh_check(int dim, int64_t n_nodes, const double *x0, int64_t n_cells, const int32_t *cells);

/* Conforming red refinement of the uploaded mesh, `levels` times (0..4),
 * computed on the GPU (edge numbering by a device radix sort).  This is the
 * local 1 -> 8 refinement the paper applies to the partitions of a coarse
 * mesh (Section 3.9, "Implementation considerations").  Each tetrahedron
 * becomes 4 corner tetrahedra and 4 tetrahedra of its inner octahedron,
 * split along the octahedron's shortest diagonal (squared length without
 * fused operations, ties to the first of (m01,m23), (m02,m13), (m03,m12));
 * each triangle becomes 4.  Children of cell c are cells 8c .. 8c+7
 * (4c .. 4c+3 in 2D); the midpoint of an edge is a new node numbered after
 * the old ones in the order of the edges' (min node, max node) keys, at
 * 0.5 (x_p + x_q), with the wall normals its two end nodes share.  Every
 * child is positively oriented (the last two nodes are swapped where
 * needed).  Replaces the mesh and discards the state (per-cell inputs of
 * hl_state_init then follow the child order).  Single-mesh contexts. */
hl_status hl_mesh_refine(hl_ctx *ctx, int levels);

/* Dimension and sizes of the held mesh (any pointer may be NULL). */
hl_status hl_mesh_info(hl_ctx *ctx, int *dim, int64_t *n_nodes, int64_t *n_cells);

/* Copy out the held mesh in its reference configuration: x [n_nodes][dim],
 * cells [n_cells][dim+1], nwall [n_nodes], normals [n_nodes][dim][dim];
 * any pointer may be NULL; on_device: the destinations are device memory. */
hl_status hl_mesh_get(hl_ctx *ctx, double *x, int32_t *cells, uint8_t *nwall, double *normals, int on_device);

/* Initial state (Section 4 preamble): tau = 1/rho0, B = I, v_c = v_cell,
 * e = |v_c|^2 / 2, m_c = rho0 V_c, carried node velocity = v_node projected
 * on the directions its walls allow.  Material per cell: rho0, shear
 * modulus mu and Lame lambda (the volumetric energy uses the bulk modulus
 * K = lambda + 2 mu / 3).  p may be NULL for the paper defaults with the
 * 2D/3D CFL number. */
hl_status hl_state_init(hl_ctx *ctx, const double *rho0, const double *mu, const double *lam,
                        const double *v_cell, const double *v_node, const hl_params *p,
                        int on_device);

/* Snapshot of the held state in host memory: positions, carried node
 * velocities, cell state (tau, v, e, B), material, the next dt, the
 * cascade levels of the last step, the contact states and the parameters.
 * blob NULL: *bytes receives the size needed.  Otherwise *bytes is the
 * blob's capacity: HL_E_INVALID (and *bytes set to the size needed) if it
 * is too small.  The blob's layout is internal; it restores only into a
 * context holding the same mesh. */
hl_status hl_state_save(hl_ctx *ctx, void *blob, int64_t *bytes);

/* Restore a snapshot of hl_state_save: the state, material, next dt,
 * cascade levels, contact states and parameters come back, so the next
 * steps repeat bitwise.  HL_E_INVALID if the blob is not a snapshot of the
 * held mesh (size, counts, dimension, connectivity check word); the held
 * state is then unchanged.  Captured graphs are kept when the parameters
 * are the same, else dropped; a recorded adjoint tape is kept. */
hl_status hl_state_restore(hl_ctx *ctx, const void *blob, int64_t bytes);

/* Replace the parameters used by the following steps. */
hl_status hl_set_params(hl_ctx *ctx, const hl_params *p);

/* Boundary loads on faces of the mesh (Section 3.8, Appendix B: boundary
 * conditions; not part of the paper's test problems).  Load l acts on the
 * face of cell cell[l] opposite its local node face[l] (0..dim), which the
 * caller names as a boundary face; kind[l] is
 *   1  prescribed traction: value[l] = the symmetric stress T^BC as
 *      (11, 22, 33, 12, 13, 23) (2D uses 11, 22, 12); every node p of the
 *      face gets T^BC (|f|/dim) n_f on the right-hand side of its nodal
 *      system, n_f the outward unit normal and |f| the face measure at t^n
 *      ((|f|/dim) n_f = -C_ck, k = face[l]);
 *   2  prescribed outward normal velocity: value[l][0] = v_n (the other
 *      entries are ignored); at a node of such faces,
 *      v*_p = M_p^-1 (r_p - pi d_p), d_p = sum over its loaded faces of
 *      (|f|/dim) n_f, with the multiplier pi chosen so that
 *      v*_p . d_p = sum of v_n |f|/dim over the same faces (for one flat
 *      face: v*_p . n = v_n).  Walls and symmetry constraints come first:
 *      at a constrained node the multiplier acts within the allowed
 *      directions P (v = P a, (P^T M_p P) a = P^T (r_p - pi d_p)), and the
 *      load is dropped where P^T d_p vanishes (|P^T d|^2 <= 1e-20 |d|^2).
 * Every node sums its loads in the order of l.  value: [n][6] doubles.
 * n = 0 removes all loads.  Loads persist across steps until replaced or
 * until a new mesh is uploaded; setting them drops captured graphs and any
 * recorded adjoint tape, and hl_forward_record refuses a context that has
 * loads (its adjoint omits them).  HL_E_INVALID for a cell out of range, a
 * face > dim, a kind other than 1 or 2 or a value that is not finite. */
hl_status hl_set_boundary_loads(hl_ctx *ctx, int64_t n, const int32_t *cell, const uint8_t *face,
                                const uint8_t *kind, const double *value, int on_device);

/* Acoustic time step C_CFL min_c L_c / a_c of the current state (eq. CFL2
 * at the first step).  It also becomes the dt used by hl_step(ctx, 0). */
hl_status hl_compute_dt(hl_ctx *ctx, double *dt_out);

/* Allocation-free acoustic time step, for callers that cannot allocate
 * device memory (work under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  The value of hl_compute_dt, C_CFL min_c L_c / a_c with
 * the neo-Hookean sound speed at J = rho0 tau (K = lambda + 2 mu / 3), for a
 * state held in the caller's device memory, with no context:
 *   x [n_nodes][dim], cells [n_cells][dim+1] (int32), rho0, mu, lam, tau
 *   [n_cells]: device pointers, read only; dt_out: one double of device
 *   memory, written.
 * The work is enqueued on hip_stream (NULL: the default stream) of device
 * `device` and the call returns without waiting: dt_out holds the result
 * once the stream has run it.  Partial minima go to a workspace of 512 KiB
 * that the library holds in static device memory on each GPU it runs on
 * (until the process ends): one per 2048 cells, so n_cells <= 134,217,728,
 * else HL_E_INVALID.  Calls that overlap on one GPU share that workspace and
 * race; serialise them (one stream, or events).  A node id out of range
 * gives dt_out = NaN (the arrays are not read on the host).  n_cells = 0
 * gives +inf.  The call allocates nothing. */
hl_status hl_acoustic_dt_noalloc(int device, void *hip_stream, int dim, int64_t n_nodes, const double *x,
                                 int64_t n_cells, const int32_t *cells, const double *rho0, const double *mu,
                                 const double *lam, const double *tau, double c_cfl, double *dt_out);

/* One ADER-MOOD step (Section 3.7): unlimited second-order candidate,
 * detection, first-order recompute of troubled cells until no new cell is
 * flagged, then the CFL reduction for the next dt.  dt > 0 is used as is;
 * dt <= 0 uses the dt computed on the device by the previous step (or by
 * hl_compute_dt), with no host round trip.  Returns
 * HL_WARN_PARACHUTE_INADMISSIBLE (with the step applied) if a first-order
 * cell is not physically admissible. */
hl_status hl_step(hl_ctx *ctx, double dt, hl_step_info *info_or_null);

/* One step of every mesh of a batch with its own dt: dt_per_mesh is
 * [n_meshes] (host or device), or NULL for each mesh's CFL-controlled dt
 * computed on the device by the previous step (eqs. CFL, CFL2). */
hl_status hl_step_batch(hl_ctx *ctx, const double *dt_per_mesh, int on_device,
                        hl_step_info *info_or_null);

/* The next dt of every mesh, [n_meshes] (n_meshes must match). */
hl_status hl_query_dt(hl_ctx *ctx, double *dt_next, int n_meshes, int on_device);

/* One step with a frozen cascade choice: mask[c] is the cascade level of
 * cell c (0 unlimited second order, 1 Barth-Jespersen limited, 2 first
 * order; levels above 2 act as 2); no detection.  mask: [n_cells] uint8. */
hl_status hl_step_replay(hl_ctx *ctx, double dt, const uint8_t *mask, int on_device,
                         hl_step_info *info_or_null);

/* Run each step as a captured hipGraph (one per buffer parity, built on
 * first use): the first candidate, `max_mood_passes` sparse MOOD passes
 * whose kernels read their list sizes from device memory (a pass with
 * nothing to do exits at once) and the CFL reduction.  One host read per
 * step checks for flags left after the captured passes; the fixpoint is
 * then finished eagerly, so results equal the eager path's bitwise.
 * Profiling (hl_profile_enable) and hl_step_replay run eagerly.
 * max_mood_passes: 0..64. */
hl_status hl_use_graph(hl_ctx *ctx, int on, int max_mood_passes);

/* ---- Groups: a 2D and a 3D context stepped together --------------------
 * Batching across dimensions (a family of triangle and tetrahedron meshes,
 * each dimension held as a batch in its own context): hl_group_step runs
 * every stage, MOOD pass and CFL reduction of the two contexts as ONE
 * kernel launch, the launch's blocks split between them, so the family
 * costs the launches of one context.  Each context takes one step with its
 * per-mesh dt held on the device (as hl_step(ctx, 0, ..) or
 * hl_step_batch(ctx, NULL, ..)), with results bitwise equal to stepping the
 * two contexts one after the other.
 * The group borrows the contexts: destroy it before them.  Both contexts
 * need a state and cells, one device and one stream, the neo-Hookean law
 * with the two-level cascade (hl_params.shear_a = -1, eos = 0, cascade 2),
 * the same `detect`, no boundary loads or contact, and, for each stage
 * where both have work, one block size in their schedules (the defaults
 * agree); otherwise HL_E_INVALID with the reason in hl_last_error(). */
typedef struct hl_group hl_group;
hl_status hl_group_create(hl_group **out, hl_ctx *ctx_2d, hl_ctx *ctx_3d);
hl_status hl_group_destroy(hl_group *group);
/* The group's step as a captured hipGraph per pair of buffer parities,
 * with `max_mood_passes` (0..64) paired passes; flags left after them are
 * finished eagerly (as hl_use_graph).  Captured graphs are rebuilt when a
 * context drops its own (new mesh, state, parameters or schedules). */
hl_status hl_group_use_graph(hl_group *group, int on, int max_mood_passes);
/* One step of both contexts; either info may be NULL.  Returns
 * HL_WARN_PARACHUTE_INADMISSIBLE (steps applied) as hl_step does. */
hl_status hl_group_step(hl_group *group, hl_step_info *info_2d_or_null, hl_step_info *info_3d_or_null);

/* Rigid-plane contact, a boundary condition that changes type during the
 * run (Section 3.8, "Boundary condition treatments"; single mesh only).
 * The plane passes through point[dim] with normal[dim] pointing from the
 * obstacle into the body (normalised here).  Each of the n candidate nodes
 * (distinct, in range) is free -- its own walls only -- until it would
 * cross the plane, then held on it as a slip wall (added to its own walls)
 * until its free velocity points away.  hl_step then runs trial steps from
 * t^n:
 *   - a held node whose free velocity (the nodal solution with its own
 *     walls only, from the same corner values) has a positive normal
 *     component is released at t^n and the trial is repeated;
 *   - a free node ending below the plane (gap g = (x - point) . normal,
 *     g1 < 0) reaches it at the fraction s = g0 / (g0 - g1) of the step
 *     (0 if g0 <= 0).  If min s <= 1e-9 those nodes are held at once and
 *     the trial is repeated; otherwise dt is cut to s_min dt and the nodes
 *     with s <= s_min (1 + 1e-9) are held from the next step on;
 *   - after 8 trials the last is accepted and every free node below the
 *     plane is held from the next step on.
 * After a cut step the next dt is min(acoustic, volume, (1 + c_i) dt of
 * the uncut trial).  hl_step_info reports trials, clipped and n_contact;
 * hl_step_replay does not evolve the contact.  point / normal are host
 * arrays; nodes is host or device (on_device).  n = 0 removes the contact
 * and restores every candidate's own walls.  A new mesh drops it;
 * hl_state_init releases every candidate; hl_forward_record refuses a
 * context with contact. */
hl_status hl_set_contact(hl_ctx *ctx, int64_t n, const int32_t *nodes, const double *point,
                         const double *normal, int on_device);

/* Contact state of the candidates in the order given: [n] uint8, 1 = held
 * by the plane (n must match). */
hl_status hl_get_contact(hl_ctx *ctx, uint8_t *state, int64_t n);

/* Stages of the full-mesh part of a step, for launch schedules. */
enum {
    HL_STAGE_PACK = 0,       /* per cell: gather record of the state */
    HL_STAGE_NODE_AGG = 1,   /* per node: least-squares aggregates */
    HL_STAGE_PREDICT = 2,    /* per cell: reconstruction, predictor, corners */
    HL_STAGE_NODE_SOLVE = 3, /* per node: nodal solver */
    HL_STAGE_UPDATE = 4,     /* per cell: update and detection */
    HL_STAGE_COUNT = 5
};

/* Launch schedule of one stage.  Each mesh's entities (cells or nodes) are
 * cut into work items of at most `tile` consecutive entities; items of the
 * largest mesh come first.  One launch per stage covers all meshes of the
 * context: blocks of `block` threads walk the items, each XCD a contiguous
 * eighth of the list; with blocks_per_cu > 0 the launch has that many blocks
 * per compute unit (persistent blocks), with 0 one block per item.  Results
 * do not depend on the schedule (bitwise). */
typedef struct {
    int32_t tile;          /* 1 .. 2^20 */
    int32_t block;         /* 64, 128, 192 or 256 */
    int32_t blocks_per_cu; /* 0 .. 64 */
    int32_t reserved;
} hl_schedule;

/* Set / get the schedule of stage `stage` (HL_STAGE_*).  The defaults are
 * {256, 256, 0} for pack and update, {64, 256, 0} for the node aggregates
 * and {32, 256, 0} for the node solve (8 lanes per node: one pass of 64 or
 * 32 nodes per block).  The predictor's default follows the meshes: {T, T,
 * 0} with T the largest of 256, 128, 64 that still gives at least 8 items
 * per compute unit (counted over both contexts of a group).  With one item
 * per block (blocks_per_cu 0, tile <= block) the predictor's items are cut
 * further where their cells use more distinct nodes than the block's LDS
 * holds (at most 189 in 3D, 255 in 2D, with 256 threads).  Setting one drops
 * captured graphs. */
hl_status hl_set_schedule(hl_ctx *ctx, int stage, const hl_schedule *sched);
hl_status hl_get_schedule(hl_ctx *ctx, int stage, hl_schedule *sched);

/* Autotuner: times each stage on the current mesh and state under every
 * candidate schedule (block 64/128/256, tile 1/2/4 blocks and, for the node
 * stages, also 1/8 and 1/4 of a block, 0/2/4/8 blocks
 * per compute unit; `reps` timed launches each, HIP events on the context's
 * stream) and keeps the fastest per stage.  The state is not changed; the
 * next step rebuilds its work buffers.  best_ms: NULL or [HL_STAGE_COUNT],
 * the chosen schedule's mean launch time.  reps: 1..100. */
hl_status hl_autotune(hl_ctx *ctx, int reps, double *best_ms);

/* ---------------------------------------------------------------------
 * Adjoint (not in the paper: differentiation of the step for parameter
 * identification).  The map from (mu, initial cell velocity, initial node
 * velocity) to the final node positions is differentiated with the dt and
 * the cascade choice of every step frozen as recorded by the forward pass.
 * ------------------------------------------------------------------- */

/* Run nsteps CFL-controlled ADER-MOOD steps from the current state,
 * recording each step's dt and cascade mask and a state checkpoint every
 * ckpt_every steps (device memory owned by the context).  The adjoint
 * covers the two-level cascade and the neo-Hookean law without boundary
 * loads or contact: with cascade 3, shear_a != -1, loads or a contact set
 * this returns HL_E_INVALID. */
hl_status hl_forward_record(hl_ctx *ctx, int nsteps, int ckpt_every);

/* Re-run the recorded steps from the current state with the recorded dt and
 * masks (for finite-difference checks after hl_state_init with other
 * parameters). */
hl_status hl_forward_replay(hl_ctx *ctx);

/* Reverse sweep over the recorded steps (each checkpoint segment replayed
 * forward, then stepped back with hand-written adjoint kernels).
 *   dL_dx_final [n_nodes][dim]  gradient of the loss w.r.t. the final
 *                               node positions (input)
 *   dL_dmu      [n_cells]       gradient w.r.t. the per-cell shear modulus
 *   dL_dvcell   [n_cells][dim]  gradient w.r.t. the initial cell velocity
 *   dL_dvnode   [n_nodes][dim]  gradient w.r.t. the initial node velocity
 * The context is left at the final forward state.  HL_E_STATE without a
 * recorded run; HL_E_INVALID (with hl_last_error set) when the parameters
 * were changed after the recording to ones hl_forward_record refuses
 * (cascade 3, shear_a != -1, eos != 0). */
hl_status hl_adjoint_run(hl_ctx *ctx, const double *dL_dx_final, double *dL_dmu, double *dL_dvcell,
                         double *dL_dvnode, int on_device);

/* Recorded cascade mask [n_cells] and dt [n_meshes] of step `step` (host). */
hl_status hl_tape_get(hl_ctx *ctx, int step, uint8_t *mask, double *dt);

/* Copy a field of the current state to `out` (count = number of elements
 * of the field's type, checked). */
hl_status hl_query(hl_ctx *ctx, int field, void *out, int64_t count, int on_device);

/* Overwrite a state field (HL_X, HL_VHAT, HL_TAU, HL_V, HL_E, HL_B). */
hl_status hl_upload_field(hl_ctx *ctx, int field, const void *in, int64_t count, int on_device);

/* Average duration in milliseconds of the kernel named `name` over the
 * steps taken since the last hl_profile_reset (timed with HIP events on the
 * context's stream when profiling is on).  Names: "node_agg", "predict",
 * "node_solve", "update", "reduce".  *launches receives the launch count. */
hl_status hl_profile_enable(hl_ctx *ctx, int on);
hl_status hl_profile_reset(hl_ctx *ctx);
hl_status hl_profile_get(hl_ctx *ctx, const char *name, double *avg_ms, int64_t *launches);

const char *hl_status_str(hl_status s);

/* Text of the last failed HIP runtime call on this thread (which call,
 * where, and the runtime's message), or "" if none failed. */
const char *hl_last_error(void);

/* What the device reaches with two plain kernels, against which the step
 * kernels' vendor-peak rooflines can be read (not part of the method):
 *   copy_gbs     streaming copy of copy_bytes (>= 1 MiB, a multiple of 16)
 *                between two buffers the call allocates and frees: bytes
 *                read + written per second / 1e9, over 10 launches, the
 *                best of four launch shapes;
 *   fp64_tflops  independent FP64 fused multiply-adds (8 chains of 4096 per
 *                lane, 1 M lanes): 2 flop per FMA, per second / 1e12, over
 *                5 launches.
 * Runs on hip_stream (NULL: the default stream) of `device` and waits for
 * it.  HL_E_INVALID for bad sizes or null outputs, HL_E_OOM when the
 * buffers cannot be allocated. */
hl_status hl_measure_peaks(int device, void *hip_stream, int64_t copy_bytes, double *copy_gbs,
                           double *fp64_tflops);

#ifdef __cplusplus
}
#endif

#endif /* HYPERLAG_H */
