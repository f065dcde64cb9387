/*
 * symx.h -- C-ABI of libsymx.so: per-element energy derivatives, assembly into
 * a 3x3 block-sparse Hessian and implicit-Euler Newton steps on one MI355X.
 *
 * Problem statement (the paper's Sec. 3, Eq. 5): the global degrees of freedom
 * are node positions x (N x 3); every energy set applies one element energy to
 * a list of fixed-size elements (connectivity + per-element parameters); the
 * total energy is the sum over sets and elements, plus the inertia term of the
 * incremental potential (Eq. 2) during time stepping.  The library evaluates
 * the three levels of Sec. 5.2 (energy; energy and gradient; energy, gradient
 * and Hessian), assembles the gradient and a 3x3 block compressed-row Hessian
 * (Sec. 5.3, BCRS), optionally projects every element Hessian to positive
 * semi-definiteness first (Sec. 5.2, Alg. 1 ProjectToPD), and runs the Newton
 * loop of Sec. 7 (block-diagonal PCG with a forcing sequence, backtracking line
 * search, time-step halving on failure).
 *
 * Conventions for every function:
 *   - return value: SYMX_OK or an error status; nothing throws across the ABI.
 *     symx_last_error() gives a thread-local message for the last failure.
 *     On error the outputs are unspecified; no caller buffer is freed.
 *   - "host" pointers are CPU memory; "device" pointers are HIP device memory
 *     (e.g. torch tensor data pointers) on the mesh's device.
 *   - position, velocity and gradient arrays are N x 3 row-major float64
 *     (node-major, x y z), i.e. 3N contiguous doubles.
 *   - calls enqueue on the mesh's HIP stream; a call that returns a host
 *     scalar (energy, report) synchronises that stream before returning.
 *   - one mesh must not be used by two threads at once; different meshes may.
 */
#ifndef SYMX_H
#define SYMX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct symx_mesh_s* symx_mesh;

typedef enum {
  SYMX_OK = 0,
  SYMX_ERR_INVALID_ARG = 1,   /* bad pointer, size, index or option */
  SYMX_ERR_OUT_OF_MEMORY = 2, /* device or pinned host allocation failed */
  SYMX_ERR_DEVICE = 3,        /* a HIP runtime call or kernel launch failed */
  SYMX_ERR_NONFINITE = 4,     /* NaN/Inf met in positions, energy or gradient */
  SYMX_ERR_NOT_CONVERGED = 5, /* Newton did not converge within all halvings */
  SYMX_ERR_LINE_SEARCH = 6,   /* line search failed within all halvings */
  SYMX_ERR_BUDGET = 7,        /* request exceeds a configured memory budget */
  SYMX_PENDING = 8            /* serving: the request has not finished yet */
} symx_status;

/* Arithmetic of the element kernels and of the linear solve. */
typedef enum {
  SYMX_F64 = 0,          /* everything in float64 */
  SYMX_F32 = 1,          /* element kernels, Hessian values and PCG in float32;
                            gradient and energy sums accumulated in float64
                            (a Newton step in this mode is limited by the
                            float32 element gradients: on stiff or strongly
                            stretched meshes it can stall above a tight
                            residual tolerance and halve dt; the refined mode
                            below does not) */
  SYMX_F32_REFINED = 2   /* Newton only: SpMV and PCG in float32 on the float64
                            Hessian rounded to float32; energies, gradient,
                            Newton residual and the iterative refinement of
                            each linear solve in float64 (the refinement
                            residual b - H dx uses the float64 Hessian) */
} symx_precision;

/* Element energies (the paper's App. B and Eq. 13).  Linear tets use
 * E = V psi(F) with F = Ds Dm^-1 and Lame parameters from (young, poisson).
 * Quadratic and cubic tets integrate psi over the element (Eq. 12),
 * E = sum_q w_q |det J_X(xi_q)| psi(J_x J_X^-1), with a symmetric rule: 4
 * points of degree 2 (Hammer, Marlowe and Stroud) for the quadratic tet, 11
 * points of degree 4 (Keast) for the cubic tet.  Their lumped masses follow
 * HRZ lumping (diagonal of the consistent mass scaled to the element mass).
 * Element ids per set are below 2^25. */
typedef enum {
  SYMX_SNH_TET4 = 0,   /* Stable Neo-Hookean, linear tet, 4 nodes                */
  SYMX_STVK_TRI3 = 1,  /* St. Venant-Kirchhoff membrane triangle, 3 nodes        */
  SYMX_HINGE4 = 2,     /* quadratic bending hinge (edge v0-v1, wings v2, v3)     */
  SYMX_NH_TET4 = 3,    /* classic Neo-Hookean (needs det F > 0)                  */
  SYMX_STVK_TET4 = 4,  /* St. Venant-Kirchhoff tet                               */
  SYMX_FCR_TET4 = 5,   /* fixed co-rotational, rotation R lagged per time step   */
  SYMX_ARAP_TET4 = 6,  /* as-rigid-as-possible + volume term, R lagged           */
  SYMX_SNH_TET10 = 7,  /* Stable Neo-Hookean, quadratic tet, 10 nodes: corners
                          0-3, then the mid-edge nodes of edges (0,1), (1,2),
                          (2,0), (0,3), (1,3), (2,3) (App. A).               */
  SYMX_SNH_TET20 = 8   /* Stable Neo-Hookean, cubic tet, 20 nodes: corners 0-3;
                          on edge k = (i, j) of the list above, node 4 + 2k a
                          third of the way from i and node 5 + 2k a third of
                          the way from j; node 16 + c at the centroid of the
                          face opposite corner c (App. A).
                          A mesh holding a quadratic or cubic set holds no
                          other set; no PSD projection, no contacts.         */
} symx_energy_kind;

/* Evaluation flags (the three levels of Sec. 5.2, plus options). */
enum {
  SYMX_EVAL_E = 1,
  SYMX_EVAL_GRAD = 2,
  SYMX_EVAL_HESS = 4,
  SYMX_PROJECT_PSD = 8,   /* project each element Hessian onto the PSD cone   */
  SYMX_PROJECT_FILTER = 32, /* Stable Neo-Hookean tets: rebuild the element
                             Hessian from the density Hessian d2psi/dF2 with
                             its negative eigenvalues set to zero (analytic
                             eigensystem, Smith et al. 2019); every other kind
                             is projected as with SYMX_PROJECT_PSD.  Takes
                             precedence over SYMX_PROJECT_PSD.              */
  SYMX_DIRICHLET = 16     /* zero gradient rows and Hessian rows/columns of
                             fixed nodes, identity diagonal block            */
};

/* One energy applied to a set of elements.  Material data are converted by
 * the library: Lame parameters from (young, poisson) with the 3D formulas. */
typedef struct {
  int32_t kind;            /* symx_energy_kind                                 */
  int64_t n_elem;          /* number of elements, >= 0                         */
  const int32_t* conn;     /* host, n_elem x k node ids in [0, N): k = 3 for the
                              triangle, 10 for the quadratic tet, 20 for the
                              cubic tet, else 4                                */
  const double* young;     /* host, per-element Young's modulus, or NULL       */
  double young_const;      /* Young's modulus when young == NULL               */
  double poisson;          /* Poisson ratio (tets, triangles)                  */
  double thickness;        /* membrane thickness (triangles)                   */
  double bend_kb;          /* bending stiffness k_b (hinges)                   */
  double density;          /* mass density, kg/m^3 (tets, triangles)           */
} symx_energy_desc;

typedef struct {
  int64_t n_nodes;                   /* N >= 1                                 */
  const double* x_rest;              /* host, N x 3 rest positions             */
  int32_t n_energies;                /* 1..4                                   */
  const symx_energy_desc* energies;  /* host, n_energies descriptors           */
  const uint8_t* fixed;              /* host, N flags (1 = Dirichlet) or NULL   */
  void* hip_stream;                  /* hipStream_t to enqueue on; NULL = null stream */
} symx_mesh_desc;

/* Read-only view of the mesh-owned assembled Hessian (device pointers).
 * Values are stored component-major: entry (i, j) of block b is
 * values[(3*i + j) * nnzb + b], as float or double per `precision`.
 * Valid until the next call on the mesh or its destruction. */
typedef struct {
  int64_t n_block_rows;
  int64_t nnzb;
  const int32_t* row_ptr;   /* device, n_block_rows + 1 */
  const int32_t* col_idx;   /* device, nnzb, ascending within each row */
  const void* values;       /* device, 9 * nnzb */
  int32_t precision;        /* SYMX_F64 or SYMX_F32 */
} symx_bsr_view;

typedef struct {
  int64_t n_nodes, nnzb, n_incidences, n_batches;
  int64_t n_elem[4];
  int32_t n_energies, max_row_blocks;
  double total_mass;
} symx_mesh_info;

typedef struct {
  double dt;                 /* nominal time step (s)                           */
  double gravity[3];         /* enters through x_tilde = x + dt v + dt^2 g      */
  double newton_rtol;        /* stop when |g_free| <= rtol * |g_free(x(t))|     */
  int32_t max_newton;        /* Newton iterations per attempt                   */
  int32_t max_pcg;           /* PCG iterations per linear solve                 */
  int32_t project;           /* 0: none, 1: project element Hessians to PSD,
                                2: as SYMX_PROJECT_FILTER                       */
  int32_t precision;         /* symx_precision                                  */
  int32_t max_halvings;      /* dt halvings before giving up                    */
  int32_t regrow_after;      /* successful steps before dt is doubled back      */
  int32_t max_refine;        /* F32_REFINED: refinement passes per solve        */
  double forcing_max;        /* largest forcing term: PCG stops at
                                |r| <= min(forcing_max, sqrt(r_k / r_0)) |b|;
                                in (0, 1)                                       */
} symx_step_params;

typedef struct {
  int32_t status;            /* symx_status of the step                         */
  int32_t newton_iters, pcg_iters, ls_backtracks, dt_halvings, refinements;
  double dt_used;            /* time step actually taken                        */
  double residual0, residual;/* |g_free| at x(t) and at the result (float64)    */
  double energy;             /* incremental potential at the result             */
  double ms_assemble, ms_pcg, ms_linesearch, ms_total;
  double lin_residual;       /* F32_REFINED: the largest relative residual
                                |b - H dx| / |b| of the step's linear solves
                                after refinement, in float64 with the float64
                                Hessian; -1 in the other modes                  */
} symx_step_report;

/* Defaults for symx_step_params: dt 0.01, gravity (0,0,-9.81), rtol 1e-6,
 * max_newton 100, max_pcg 500, project 0, precision SYMX_F64, max_halvings 8,
 * regrow_after 3, max_refine 4, forcing_max 0.5. */
void symx_step_params_default(symx_step_params* p);

/* Build a mesh: copies all host inputs (the caller may free them afterwards),
 * computes rest data (volumes, areas, hinge weights, lumped masses), the block
 * sparsity pattern (block (i,j) exists iff i and j share an element; all
 * diagonal blocks exist), the scatter map and the per-node incidence lists,
 * and uploads them to the current HIP device.  Errors: INVALID_ARG for node
 * ids out of range, degenerate rest elements, more than 255 blocks or 256
 * element incidences on one node; OUT_OF_MEMORY; DEVICE. */
symx_status symx_mesh_create(const symx_mesh_desc* desc, symx_mesh* out);
symx_status symx_mesh_destroy(symx_mesh mesh);
symx_status symx_mesh_get_info(symx_mesh mesh, symx_mesh_info* info);

/* Host copies of the pattern: row_ptr (N+1), col_idx (nnzb) and, if
 * scatter_map is not NULL, the scatter map of every energy set concatenated:
 * for set s, element e, local nodes (a, b) in row-major order, the index of
 * block (conn[e][a], conn[e][b]) in col_idx (n_elem * k * k int32 per set).
 * Any pointer may be NULL to skip that output. */
symx_status symx_mesh_get_pattern(symx_mesh mesh, int32_t* row_ptr, int32_t* col_idx,
                                  int32_t* scatter_map);

/* Lumped node masses (host, N doubles): rho V / 4 per linear tet, rho h A / 3
 * per triangle (the inertia term of Eq. 2); a quadratic tet gives rho V / 36
 * to each corner and 4 rho V / 27 to each edge node, a cubic tet rho V / 193
 * to each corner, 27 rho V / 772 to each edge node and 27 rho V / 193 to each
 * face node (HRZ lumping, V of the straight-sided element). */
symx_status symx_mesh_get_masses(symx_mesh mesh, double* mass_host);

/* Per-element evaluation of one energy set (the low-level element interface
 * of Sec. 5.2 and the local-output option of Sec. 5.3).  x_dev: device N x 3
 * float64 positions.  Outputs are device arrays of the precision's type
 * (float for SYMX_F32, double for SYMX_F64), any of them NULL to skip:
 *   elem_E:    n_elem
 *   elem_grad: n_elem x 3k        (node-major)
 *   elem_hess: n_elem x 3k x 3k   (row-major; projected if SYMX_PROJECT_PSD)
 * flags: SYMX_EVAL_* bits select what is computed; SYMX_PROJECT_PSD. */
symx_status symx_eval_derivatives(symx_mesh mesh, int32_t energy_index, const double* x_dev,
                                  uint32_t flags, int32_t precision, void* elem_E,
                                  void* elem_grad, void* elem_hess);

/* Global evaluation and assembly at positions x_dev (device N x 3 float64):
 *   energy_host: total energy (float64), if flags has SYMX_EVAL_E, else untouched
 *   grad_dev:    device N x 3 float64 gradient, if flags has SYMX_EVAL_GRAD
 *   H_out:       view of the mesh-owned BSR Hessian, if flags has SYMX_EVAL_HESS
 * x_tilde_dev != NULL adds the inertia term m/(2 dt^2)|x - x_tilde|^2 per node
 * (Eq. 2) with time step dt; NULL assembles the elastic energies only.
 * Summation order per block and per gradient row is fixed (energy set, then
 * element id), so results are bitwise reproducible run to run.
 * precision: SYMX_F64 or SYMX_F32. */
symx_status symx_assemble_bsr(symx_mesh mesh, const double* x_dev, const double* x_tilde_dev,
                              double dt, uint32_t flags, int32_t precision, double* energy_host,
                              double* grad_dev, symx_bsr_view* H_out);

/* symx_assemble_bsr for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same evaluation and assembly, allocating nothing.
 *   values_dev: device, 9 * nnzb values of the precision's type (float for
 *     SYMX_F32, double for SYMX_F64), component-major as in symx_bsr_view
 *     (entry (i, j) of block b at values_dev[(3 i + j) nnzb + b]), over the
 *     pattern of symx_mesh_get_pattern; caller-owned; required with
 *     SYMX_EVAL_HESS, otherwise unused (may be NULL).
 *   other arguments as symx_assemble_bsr; results are bitwise those of
 *   symx_assemble_bsr.
 * Scratch: the energy reduction (one partial sum per workgroup of the energy
 * kernels), the total and the non-finite flag live in a static device array
 * of the library, 40,992 doubles (320.25 KiB) per GPU, held until the process
 * ends; its address is taken once per device on the first call.  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (any mesh,
 * any stream) race.  The call synchronises the mesh's stream.
 * Errors: INVALID_ARG for the cases of symx_assemble_bsr, a NULL values_dev
 * with SYMX_EVAL_HESS, meshes with contacts, and SYMX_PROJECT_PSD (and
 * SYMX_PROJECT_FILTER on meshes that are not all Stable Neo-Hookean tets),
 * whose element records need a workspace; BUDGET if the energy needs more
 * partial sums than the array holds (not reached by meshes of at most four
 * sets); NONFINITE as symx_assemble_bsr. */
symx_status symx_assemble_bsr_noalloc(symx_mesh mesh, const double* x_dev,
                                      const double* x_tilde_dev, double dt, uint32_t flags,
                                      int32_t precision, double* energy_host, double* grad_dev,
                                      void* values_dev);

/* One implicit-Euler time step (Eq. 2-3): x_dev, v_dev (device N x 3 float64)
 * hold x(t), v(t) on entry and x(t+dt_used), v(t+dt_used) on success; on
 * failure they are left unchanged.  Newton from x(t); block-Jacobi PCG with
 * forcing term min(forcing_max, sqrt(r_k / r_0)); Armijo backtracking (c = 1e-4,
 * halving, at most 30; energies compared up to 1e-12 |E(x)|, the rounding of
 * their float64 sum); on line-search failure or too many Newton iterations
 * the step restarts with dt/2 (at most max_halvings times); the mesh keeps the
 * reduced dt and doubles it back after regrow_after successful steps.  With
 * max_halvings == 0 there is no step control: the step is taken at exactly
 * params->dt and the mesh's reduced dt and success count are neither used nor
 * changed (so a given dt sequence can be replayed).
 * report may be NULL. */
symx_status symx_newton_step(symx_mesh mesh, double* x_dev, double* v_dev,
                             const symx_step_params* params, symx_step_report* report);

/* Lagged rotations of the fixed co-rotational and ARAP sets (Sec. 6.1: the
 * rotation is held constant over a time step): for every such element, R is
 * the rotation closest to its deformation gradient at positions x_dev (device
 * N x 3 float64), i.e. the maximiser of tr(R^T F) over rotations (from the
 * SVD of F, with the sign of the smallest singular value's direction chosen
 * so that det R = 1).  A new mesh starts from the rotations at rest (R = I);
 * symx_newton_step takes them at x(t) itself; symx_assemble_bsr and
 * symx_eval_derivatives use the current ones.  No-op for meshes without such
 * sets. */
symx_status symx_mesh_update_rotations(symx_mesh mesh, const double* x_dev);

/* Candidate contacts of a conditional barrier (Sec. 5.2, conditional
 * evaluations, Eq. 9; the contact potential of Sec. 5.4): tuples_host holds n
 * x 4 node ids (p, t0, t1, t2), node p against the plane through t0, t1, t2
 * with normal N = (t1 - t0) x (t2 - t0).  With d the signed distance of p to
 * that plane, the energy is -k_c (d - d_hat)^2 ln(d / d_hat) while
 * 0 < d < d_hat, zero for d >= d_hat (inactive: not evaluated, not assembled)
 * and +inf for d <= 0, so that a line search backs off.  The list replaces
 * the previous one and n = 0 removes all contacts: as in the paper's dynamic
 * topology, the caller updates the list (e.g. from a proximity query at each
 * time step) and the couplings follow.  They form a second block-sparse matrix
 * beside the mesh's pattern (rebuilt on the device when the list changes;
 * a list no longer than the one its buffers were sized for reuses them);
 * assembly, energies, the PCG and the Newton step include it.  With
 * projection on, contact element Hessians take the nearest-PSD projection.
 * Node ids in range and distinct within a tuple; k_c, d_hat > 0; not on
 * meshes of quadratic or cubic tets. */
symx_status symx_mesh_set_contacts(symx_mesh mesh, int64_t n, const int32_t* tuples_host,
                                   double k_c, double d_hat);
/* Dynamic topology (Sec. 5.2, dynamic topology; Alg. 1, the rebuild of the
 * sparsity when it changes): a set of elements that replaces the previous
 * dynamic set between steps (set->n_elem = 0 removes it).  Kinds: SYMX_SNH_TET4,
 * SYMX_NH_TET4, SYMX_STVK_TET4 (parameters as for a static set; their lumped
 * masses rho V / 4 are added to the static sets' node masses) or SYMX_HINGE4
 * (no mass).  All host inputs are copied.  The elements' couplings form the
 * mesh's second block matrix, built on the device as for contacts (a list
 * that fits the previous buffers reuses them), and assembly, energies, the
 * PCG and the Newton step include them, summed after the static sets in
 * element order; with projection on, their element Hessians take the
 * nearest-PSD projection.  symx_mesh_get_contact_bsr returns that matrix and
 * symx_mesh_get_masses the combined masses.  A mesh holds either contacts or
 * a dynamic set (INVALID_ARG for the other); INVALID_ARG also for another
 * kind, node ids out of range or repeated within an element, degenerate rest
 * elements, and meshes of quadratic or cubic tets. */
symx_status symx_mesh_set_dynamic_elements(symx_mesh mesh, const symx_energy_desc* set);

/* How the contact barrier's activation (Eq. 9) is evaluated.
 *   SYMX_CONTACT_COMPACT (default): an activation pass flags the candidates
 *     with d < d_hat, a scan compacts them, and only they are evaluated.
 *   SYMX_CONTACT_BRANCH: the activation is a branch inside the generated
 *     element function (Sec. 5.2, branching): every candidate is evaluated,
 *     and an inactive one takes the zero arm with an if/else, so it costs the
 *     distance and nothing more; no compaction.
 * Both give the same energy, gradient and contact matrix (up to rounding
 * order of the barrier's arithmetic). */
typedef enum { SYMX_CONTACT_COMPACT = 0, SYMX_CONTACT_BRANCH = 1 } symx_contact_mode;
/* Select the mode for the mesh's contacts (kept across symx_mesh_set_contacts
 * calls; INVALID_ARG for another value). */
symx_status symx_mesh_set_contact_mode(symx_mesh mesh, int32_t mode);

/* View of the contact matrix (or of the dynamic elements' matrix) of the
 * last assembly (device pointers, the layout of symx_bsr_view,
 * n_block_rows = N, blocks of inactive candidates zero), at `precision`.
 * Without contacts or dynamic elements nnzb = 0. */
symx_status symx_mesh_get_contact_bsr(symx_mesh mesh, int32_t precision, symx_bsr_view* view);

/* Kernel timing for measurement: with profiling on, every kernel launch of
 * the mesh carries start/stop HIP events on the mesh's stream
 * (hipExtLaunchKernelGGL), which time the kernel itself.  set_profiling
 * resets all counters.  get_kernel_time returns the number of launches of one
 * kernel whose device time was at least min_ms, and their summed time (PCG
 * kernels enqueued past convergence only check a flag and return; a small
 * min_ms separates them).  kernel_names writes the known names, comma
 * separated, into buf (host, buf_len bytes).  Names: row_assemble_gH,
 * row_assemble_H, row_assemble_g, energy, reduce, elem_eval, elem_filtered,
 * project_psd, incidence_positions, elem_rows_projected, elem_rows_filtered,
 * lagged_rotations, pcg_init, pcg_spmv, pcg_update, residual64, dot64,
 * x_tilde, lincomb64, velocity, check_finite, accumulate (those launched
 * since profiling was enabled). */
symx_status symx_mesh_set_profiling(symx_mesh mesh, int32_t enable);
symx_status symx_mesh_get_kernel_time(symx_mesh mesh, const char* name, double min_ms,
                                      int64_t* launches, double* total_ms);
symx_status symx_mesh_kernel_names(symx_mesh mesh, char* buf, int64_t buf_len);

/* ---- serving: time-step requests of many scenes on one GPU -------------------
 * Requests wait in a FIFO queue and are admitted when one of max_slots slots
 * is free and the request's estimated device footprint fits in what is left
 * of hbm_budget_bytes.  Each slot has its own worker thread and HIP stream;
 * admitted requests run concurrently (their kernels overlap on the device),
 * and the PCG iterations of the requests that are solving at the same time
 * are batched: one SpMV and one update launch per iteration cover all their
 * meshes (each with its own grid and arrays), so kernel boundaries are the
 * only synchronisation and one host synchronisation serves the whole batch.
 * A request is one implicit-Euler time step (as symx_newton_step) of its own
 * scene; the result does not depend on the other requests in flight (it is
 * bitwise the result of symx_newton_step on that scene alone).
 * Device memory comes from a pool owned by the server, and the block pattern
 * of a scene stays on the device after its request: a later request with the
 * same node count, energy kinds and connectivity reuses it (only positions,
 * materials and masses are rebuilt).  Idle patterns count against the budget
 * and are evicted, least recently used first, when a request needs room. */
typedef struct symx_server_s* symx_server;
typedef struct {
  uint64_t budget_bytes, in_use_bytes, peak_bytes;
  uint64_t pattern_cache_bytes;      /* idle cached patterns                    */
  int64_t queued, completed;
  int64_t pattern_hits, pattern_misses;
  int64_t pcg_batches;               /* batched PCG launch sequences            */
  int64_t pcg_chunks;                /* request chunks they carried             */
  int32_t active, peak_active, max_slots;
  uint64_t peak_device_bytes;        /* most device memory the server's pool
                                        handed out at once (admission charges
                                        estimates; this is what was used)   */
} symx_server_stats;

/* Create a server on the current HIP device; max_slots in 1..64. */
symx_status symx_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, symx_server* out);
/* Queue a request.  All host inputs are copied; x_host, v_host are N x 3
 * float64.  Returns SYMX_ERR_BUDGET if the scene can never fit the budget.
 * *ticket identifies the request. */
symx_status symx_server_submit(symx_server server, const symx_mesh_desc* scene,
                               const double* x_host, const double* v_host,
                               const symx_step_params* params, int64_t* ticket);
/* Result of a request: SYMX_PENDING while it runs (wait = 0), otherwise the
 * step's status, with x_out, v_out (host N x 3, may be NULL), the report and
 * times_ms[5] = {submitted, started, mesh ready on the device, step done and
 * result on the host, finished (device memory released)} in ms since server
 * creation (may be NULL).  A finished ticket is released by this call. */
symx_status symx_server_poll(symx_server server, int64_t ticket, int32_t wait, double* x_out,
                             double* v_out, symx_step_report* report, double* times_ms);
symx_status symx_server_get_stats(symx_server server, symx_server_stats* stats);
/* Device footprint the server charges against its budget for a scene solved
 * at `precision` (an upper bound of the mesh and Newton workspace, with the
 * records of per-element projection; a request without projection is charged
 * that much less). */
symx_status symx_server_estimate_bytes(const symx_mesh_desc* scene, int32_t precision,
                                       uint64_t* bytes);
/* Waits for running requests, abandons queued ones, frees the server. */
symx_status symx_server_destroy(symx_server server);

const char* symx_status_string(symx_status status);
const char* symx_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SYMX_H */
