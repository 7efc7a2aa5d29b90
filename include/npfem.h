/*
 * npfem.h - C ABI of the MI355X npFEM solver library (libnpfem.so).
 *
 * The library advances deformable blood cells (surface meshes) by one implicit-Euler time
 * step (arXiv 1911.03062, supplementary material, npFEM subsection: the velocity update,
 * Newton's second law with implicit Euler, its minimisation form g(x) and the quasi-Newton
 * iteration x^{k+1} = x^k - H~ grad g(x^k)). The elemental energies are projective-dynamics
 * constraints (triangle strain and area, edge bending, cell volume) and H~ is the inverse
 * of the constant matrix L (Hessian of the quadratic part of g), so one iteration is one
 * local (projection) step plus one global (linear solve) step.
 *
 * Units: um, us, fg, pN. Arrays of vertex data are structure-of-arrays [3][V_total]
 * (x coordinates of every vertex of the batch, then y, then z); the vertices of one cell
 * are contiguous and cells follow each other in batch order.
 *
 * Errors: every call returns an npfem_status; no exception crosses the ABI. Validation
 * errors are reported synchronously. npfem_last_error() returns a thread-local message for
 * the last non-OK status of the calling thread.
 *
 * Threads: cell types are immutable after creation and may be shared by batches and
 * threads. A batch must not be stepped from two threads at once.
 */
#ifndef NPFEM_H
#define NPFEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NPFEM_OK = 0,
  NPFEM_E_INVALID = -1,    /* bad argument (null pointer, size, precision, form)            */
  NPFEM_E_MESH = -2,       /* mesh not closed/manifold/consistently oriented, degenerate
                              triangle, unused vertex, or rest volume <= 0                  */
  NPFEM_E_NOT_SPD = -3,    /* the system matrix failed to factorise                          */
  NPFEM_E_DT = -4,         /* step dt differs from the cell type's factorised dt             */
  NPFEM_E_NOMEM = -5,      /* host or device allocation failed                               */
  NPFEM_E_HIP = -6,        /* a HIP runtime call failed (message names it)                   */
  NPFEM_E_NONFINITE = -7,  /* a step produced a non-finite position or velocity              */
  NPFEM_E_UNSUPPORTED = -8 /* the requested form/precision/type size is not available        */
} npfem_status;

/* Surface mesh of one cell type (host memory, borrowed for the duration of the call). */
typedef struct {
  int32_t n_vertices;
  int32_t n_triangles;
  const double* rest_xyz;  /* [n_vertices][3], um: the stress-free shape                   */
  const int32_t* tri;      /* [n_triangles][3], counter-clockwise seen from outside        */
} npfem_mesh;

/* Material constants (parameter table of the supplementary material). */
typedef struct {
  double density;       /* fg/um^3: lumped mass m = density * V0 / n per vertex            */
  double shear_B;       /* pN/um: strain-constraint weight per unit rest area              */
  double area_C;        /* pN/um: area-constraint weight per unit rest area                */
  double skalak_D;      /* pN/um: stored; no role in the projective-dynamics energies      */
  double k_bend;        /* pN um: bending-constraint weight                                */
  double k_vol;         /* pN/um: volume-constraint weight per vertex                      */
  double strain_min;    /* singular-value clamp of the strain projection (1, 1 = polar)    */
  double strain_max;
  double pbd_kappa;     /* position-based velocity damping in [0, 1] (0 = off): per cell,   */
                        /* v_n -> v_n + kappa (v_cm + w x r - v_n) before the prediction,   */
                        /* keeping the rigid part (centre-of-mass velocity v_cm, angular     */
                        /* velocity w about the centre of mass) of the velocity field        */
  double v_max;         /* um/us, velocity cap (0 = off): after a step, a vertex velocity   */
                        /* longer than v_max is scaled to length v_max, direction kept       */
                        /* (positions unchanged); the truncation of the solid velocities     */
                        /* for a stable immersed-boundary coupling (Fluid-structure          */
                        /* interaction subsection)                                           */
  double rayleigh_alpha;/* 1/us, Rayleigh damping C = alpha M + beta K (0, 0 = off), K the    */
  double rayleigh_beta; /* us,   constant strain + area + bending stiffness: M~ = M + h C     */
                        /* enters y_n = x_n + h M~^-1 (M v_n + h F_ext) and the mass term of */
                        /* g, and L = M~/h^2 + k_vol I + K (npFEM subsection); both forms    */
  int32_t membrane;     /* NPFEM_MEMBRANE_PD: strain + area constraint energies (default);    */
                        /* NPFEM_MEMBRANE_SKALAK: the Skalak strain energy                   */
                        /* W = (B/4)(I1^2 + 2 I1 - 2 I2) + (C/4) I2^2 per unit rest area      */
                        /* (B = shear_B, C = area_C), quasi-Newton direction -L^-1 grad g     */
                        /* with a backtracking line search on g per cell (steps 1, 1/2, ...,  */
                        /* 1/256, Armijo constant 1e-4). Plain form only, without Rayleigh   */
                        /* beta; other combinations report NPFEM_E_UNSUPPORTED               */
} npfem_material;

enum { NPFEM_MEMBRANE_PD = 0, NPFEM_MEMBRANE_SKALAK = 1 };

typedef struct npfem_celltype npfem_celltype;   /* opaque, library-owned */
typedef struct npfem_batch npfem_batch;         /* opaque, library-owned */

/* Read-only description of a cell type (host-side setup results). */
typedef struct {
  int32_t n_vertices, n_triangles, n_hinges;
  int32_t bandwidth;        /* max |i - j| over the nonzeros of L                           */
  double rest_volume;       /* V0, um^3                                                      */
  double rest_area;         /* um^2                                                          */
  double vertex_mass;       /* fg                                                            */
  double dt;                /* us, the dt L was factorised for                               */
  int32_t tri_rounds;       /* rounds of the per-wave triangle schedule (fused form)         */
  int32_t hinge_rounds;     /* rounds of the per-wave hinge schedule (fused form)            */
} npfem_celltype_info;

/* Solver forms (npfem_batch_create `form`). */
enum {
  NPFEM_FORM_PLAIN = 0,  /* one cell at a time: predict, K x (local, global), finalise are
                            separate kernel launches per cell; FP64 or FP32                 */
  NPFEM_FORM_FUSED = 1   /* every cell of the batch in one launch per step: local + global
                            iterations fused in LDS, global step as a dense-inverse product
                            on the matrix cores (split fp16 operands, FP32 accumulation);
                            FP32 state, FP64 volume/area reductions                         */
};

/*
 * Build a cell type on the host (no GPU call): validate the mesh, compute the rest frames
 * of the triangles, the bending stencils of the interior edges, the rest volume V0, the
 * uniform lumped mass, assemble L = (m/h^2 + k_vol) I + sum_t (B + C) A_t G_t^T G_t
 * + sum_e k_bend a_e a_e^T, factorise it (Cholesky, FP64) and form its inverse.
 * `dt` (us) is fixed for the type: stepping with another dt is an error.
 * Errors: NPFEM_E_INVALID, NPFEM_E_MESH, NPFEM_E_NOT_SPD, NPFEM_E_NOMEM.
 */
npfem_status npfem_create_celltype(const npfem_mesh* mesh, const npfem_material* material,
                                   double dt, npfem_celltype** out);
void npfem_celltype_destroy(npfem_celltype* type);
npfem_status npfem_celltype_get_info(const npfem_celltype* type, npfem_celltype_info* out);
/* Copy the assembled FP64 system matrix L into host memory [n][n] (row-major). */
npfem_status npfem_celltype_get_matrix(const npfem_celltype* type, double* L_out);

/*
 * Create a batch of n_cells cells; cell c has type type_of_cell[c] (host array of handles,
 * borrowed). precision is 32 or 64 (64 only with NPFEM_FORM_PLAIN). vertex_offsets, if not
 * NULL, receives [n_cells + 1] int64 offsets of each cell in the vertex axis (host memory).
 * Allocates the batch's device work list and workspace on the current HIP device.
 * Errors: NPFEM_E_INVALID, NPFEM_E_UNSUPPORTED, NPFEM_E_NOMEM, NPFEM_E_HIP.
 */
npfem_status npfem_batch_create(int32_t n_cells, npfem_celltype* const* type_of_cell,
                                int32_t precision, int32_t form, npfem_batch** out,
                                int64_t* vertex_offsets);
void npfem_batch_destroy(npfem_batch* batch);
int64_t npfem_batch_vertex_count(const npfem_batch* batch);

/*
 * Advance every cell of the batch by one time step of length dt with n_pd_iters
 * quasi-Newton (local/global) iterations, asynchronously on `stream` (a hipStream_t;
 * NULL = default stream).
 *   x, v        device, in/out, [3][V_total] float (precision 32) or double (64):
 *               positions (um) and velocities (um/us), overwritten with x_{n+1}, v_{n+1};
 *   ext_forces  device, in, [3][V_total], external force per vertex (pN), same precision;
 *   cell_volume_area  optional device double [n_cells][2]: enclosed volume and surface
 *               area of each cell at x_{n+1} (FP64 reductions), or NULL.
 * Buffers are caller-owned and borrowed for the duration of the enqueued work.
 * n_pd_iters = 0 returns the prediction y_n (x_n + h v_n + h^2 F/m without damping).
 * Errors: NPFEM_E_INVALID (null buffer, n_pd_iters < 0), NPFEM_E_DT, NPFEM_E_HIP.
 * A non-finite result is flagged on the device; npfem_batch_check reports it.
 */
npfem_status npfem_step(npfem_batch* batch, void* x, void* v, const void* ext_forces,
                        double dt, int32_t n_pd_iters, void* stream,
                        double* cell_volume_area);

/*
 * npfem_step with collision energies (particle-in-kernel technique, supplementary material):
 * for every vertex i with contact_w[i] > 0, the energy (contact_w[i]/2) ||x_i - p_i||^2 toward
 * its projection point p_i (the desired location given by the closest foreign particle) is
 * added to g, so grad g gains contact_w[i] (x_i - p_i); the system matrix is unchanged. The
 * caller finds the contacts and zeroes ext_forces at contacting vertices (the technique
 * replaces the fluid force there). The iteration contracts while contact_w stays well below
 * the diagonal of L (m/h^2 + ...: about 3.6e4 pN/um for the RBC of the workloads).
 *   contact_p  device, in, [3][V_total] projection points (um), batch precision;
 *   contact_w  device, in, [V_total] weights (pN/um), 0 = no contact, batch precision.
 * Both NULL: exactly npfem_step. Errors: as npfem_step, and NPFEM_E_INVALID when only one of
 * the two is given. Not recorded by npfem_graph_create.
 */
npfem_status npfem_step_contacts(npfem_batch* batch, void* x, void* v, const void* ext_forces,
                                 double dt, int32_t n_pd_iters, void* stream,
                                 double* cell_volume_area, const void* contact_p,
                                 const void* contact_w);

/*
 * Restrict the following npfem_step calls of a fused-form batch to a subset of its cells
 * (continuous batching: the union of the cells of the requests admitted to one tick).
 * cell_ids: host array of n distinct cell ids of the batch, read during the call; NULL or
 * n < 0 restores the list of all cells; n = 0 makes steps do nothing. The group work list is
 * built on the host and copied asynchronously on `stream` into one of two device lists, so a
 * step enqueued on the same stream after this call uses it while the previous list may still
 * be in use by an earlier step. Cells outside the subset are not read or written. A graph
 * made by npfem_graph_create keeps its own copy of the list current at its creation.
 * Errors: NPFEM_E_INVALID (id out of range or repeated), NPFEM_E_UNSUPPORTED (plain form),
 * NPFEM_E_HIP.
 */
npfem_status npfem_batch_set_active(npfem_batch* batch, const int32_t* cell_ids, int32_t n,
                                    void* stream);

/*
 * Fused-form layouts. A fused step gives each wave of a workgroup `cells_per_wave` cells of one
 * type (the workgroup takes 4 x cells_per_wave cells) and 64 / cells_per_wave lanes per cell
 * for the element rounds; every value that fits the kernel's LDS and register budget has its
 * own element schedule. These calls choose among them (by hand, or by timing with
 * npfem_batch_autotune); results of different layouts agree to rounding (the element
 * summation order differs).
 *
 * npfem_celltype_cells_per_wave: writes up to max_out feasible values (largest first; the
 * first is the default of new batches) to out (host, may be NULL) and returns their number,
 * or a negative status.
 */
int32_t npfem_celltype_cells_per_wave(const npfem_celltype* type, int32_t* out, int32_t max_out);
/* Layout of `type` in a fused-form batch (host out). Errors: NPFEM_E_INVALID (type not in the
 * batch), NPFEM_E_UNSUPPORTED (plain form). */
npfem_status npfem_batch_get_cells_per_wave(const npfem_batch* batch, const npfem_celltype* type,
                                            int32_t* cells_per_wave);
/* Switch `type` to another feasible layout. Synchronises the device, rebuilds the batch's work
 * lists and makes the all-cells list current (an active list set earlier is dropped).
 * Errors: NPFEM_E_INVALID, NPFEM_E_UNSUPPORTED (plain form, or not a layout of the type),
 * NPFEM_E_NOMEM, NPFEM_E_HIP. */
npfem_status npfem_batch_set_cells_per_wave(npfem_batch* batch, const npfem_celltype* type,
                                            int32_t cells_per_wave);
/* Time every feasible layout of every type of the batch (warm-up step, then `reps` steps of
 * n_pd_iters iterations on `stream`, with only that type's cells active, on library-allocated
 * scratch state: each cell at its rest shape under small pseudo-random forces) and keep the
 * fastest per cell. Then, with those layouts, time the variants of the global step alone the
 * batch supports (npfem_global_solve, `reps` calls each over the whole batch) and keep the
 * fastest for NPFEM_SOLVE_AUTO. The fused step itself always applies L^-1 as the dense product on the
 * matrix cores. Synchronises the device; the caller's state buffers are not touched. The
 * all-cells list is current afterwards. Errors: NPFEM_E_INVALID (n_pd_iters or reps < 1),
 * NPFEM_E_UNSUPPORTED (plain form), NPFEM_E_NOMEM, NPFEM_E_HIP. */
npfem_status npfem_batch_autotune(npfem_batch* batch, int32_t n_pd_iters, int32_t reps,
                                  void* stream);

typedef struct npfem_graph npfem_graph;         /* opaque, library-owned */

/*
 * Record n_steps consecutive steps of the batch (each exactly as npfem_step with the same
 * x, v, dt and n_pd_iters; step s uses ext_forces[s]) into a HIP graph and instantiate it,
 * so that a fixed sequence of steps can be replayed with one launch. x, v, every
 * ext_forces[s] (host array of n_steps device pointers, read during the call) and
 * cell_volume_area (optional, written by every step) are device buffers whose addresses are
 * baked into the graph: they must stay allocated while the graph exists, and their contents
 * at replay time are what the steps read. For the fused form the graph holds its own copy of
 * the batch's current active-cell list (npfem_batch_set_active), so later changes of the list
 * do not affect it. Recording happens on a private stream of the batch's device and enqueues
 * no work. The graph holds no reference to `batch` after creation beyond its device data:
 * destroy the graph before the batch. Errors: NPFEM_E_INVALID (null argument, n_steps < 1,
 * n_pd_iters < 0), NPFEM_E_DT, NPFEM_E_NOMEM, NPFEM_E_HIP.
 */
npfem_status npfem_graph_create(npfem_batch* batch, void* x, void* v,
                                const void* const* ext_forces, int32_t n_steps, double dt,
                                int32_t n_pd_iters, double* cell_volume_area,
                                npfem_graph** out);
/* Enqueue one replay of the recorded steps on `stream` (a hipStream_t; NULL = default).
 * Errors: NPFEM_E_INVALID, NPFEM_E_HIP. Non-finite results are flagged as for npfem_step. */
npfem_status npfem_graph_launch(npfem_graph* graph, void* stream);
/* Release the graph (waits for its replays to finish). NULL is ignored. */
void npfem_graph_destroy(npfem_graph* graph);

/*
 * Median filter of external forces (Fluid-structure interaction subsection): for every cell of
 * the batch and every vertex, each component of the force becomes the median of that
 * component over the vertex and its one-ring neighbours (vertices sharing an edge with it);
 * the median of an even count is the mean of the two middle values. Attenuates isolated
 * spikes of the coupling forces before they enter a step. Asynchronous on `stream`.
 *   f_in, f_out  device, [3][V_total] of the batch's precision (float 32 / double 64); either
 *                the same buffer (filtered in place) or non-overlapping.
 * Buffers are caller-owned and borrowed for the duration of the enqueued work. Every cell of
 * the batch is filtered, whatever npfem_batch_set_active selected.
 * Any vertex degree is handled. Errors: NPFEM_E_INVALID (null batch or buffer),
 * NPFEM_E_UNSUPPORTED (a cell so large that its forces plus one 4-byte index per vertex exceed
 * 64 KiB: above 4096 vertices in FP32, 2340 in FP64), NPFEM_E_HIP.
 */
npfem_status npfem_filter_forces(npfem_batch* batch, const void* f_in, void* f_out, void* stream);

/*
 * Particle-in-kernel (PIK) contact detection (main text, near-contact handling; supplementary
 * material, particle-in-kernel technique): produces the contact_p / contact_w inputs of
 * npfem_step_contacts from the positions alone. For every vertex i of the batch, the colliding
 * neighbour is the closest vertex j of ANOTHER cell with |x_i - x_j| < radius (the kernel
 * sphere); distances are compared as squared distances ((dx dx + dy dy) + dz dz), every
 * operation rounded in the batch precision (no fused multiply-add), strictly below
 * radius^2, and among equal distances the smallest vertex index j wins. With a neighbour:
 * contact_p[:, i] = x_j + separation * n_j, n_j the unit outward normal of j's cell at j
 * (the normalised sum of its incident triangles' doubled area vectors), and
 * contact_w[i] = weight. Without: contact_p[:, i] = x_i and contact_w[i] = 0. Asynchronous
 * on `stream`; every cell of the batch takes part, whatever npfem_batch_set_active selected.
 *   x          device, in, [3][V_total] positions (um), batch precision;
 *   radius     kernel radius (um), finite, > 0; positions should stay within 1e4 radii of the
 *              origin (the grid's cell coordinates are rounded products x / (1.001 radius));
 *   separation distance (um) of the projection point from the neighbour, finite, >= 0;
 *   weight     contact weight (pN/um) written for contacting vertices, finite, >= 0;
 *   contact_p  device, out, [3][V_total], batch precision (may not overlap x);
 *   contact_w  device, out, [V_total], batch precision.
 * The first call allocates the batch's search workspace (a grid-bucket table of 2^k >= 2 V_total
 * buckets and about 80 bytes per vertex); calls on one batch must not overlap in time.
 * Errors: NPFEM_E_INVALID (null batch or buffer, radius / separation / weight out of range),
 * NPFEM_E_UNSUPPORTED (more than 2^29 vertices in the batch), NPFEM_E_NOMEM, NPFEM_E_HIP.
 */
npfem_status npfem_detect_contacts(npfem_batch* batch, const void* x, double radius,
                                   double separation, double weight, void* contact_p,
                                   void* contact_w, void* stream);

/*
 * The global step alone: out[:, cell] = L^-1 rhs[:, cell] for every cell of the batch and each
 * of its 3 coordinate columns, L the cell type's constant system matrix (supplementary
 * material, npFEM subsection: the prefactored Hessian approximation H~ of the quasi-Newton
 * update x - H~ grad g, shared by every cell of a type). Three ways of applying it:
 *   NPFEM_SOLVE_DENSE   the dense precomputed L^-1 (FP64-derived) times the right-hand sides
 *                       of each group of same-type cells on the fp16 matrix cores with split
 *                       operands (each FP32 value as a hi + lo pair of fp16 values, 22
 *                       significant bits; FP32 accumulation), as the fused step does;
 *                       fused-form (FP32) batches only;
 *   NPFEM_SOLVE_BANDED  forward and back substitution with the banded Cholesky factor
 *                       (FP64-computed, used in the batch precision), one lane per column;
 *                       either form and precision, band widths up to 65;
 *   NPFEM_SOLVE_GEMV    the dense L^-1 (FP64-derived, in the batch precision) times each
 *                       cell's right-hand sides on the vector ALU, a few cells per
 *                       workgroup; either form and precision, meshes whose staged
 *                       right-hand sides fit 64 KiB of LDS (n <= 1365 in FP32, 682 in FP64);
 *   NPFEM_SOLVE_AUTO    the fastest variant the batch supports as npfem_batch_autotune last
 *                       timed them on this batch (before any autotune: dense for fused,
 *                       banded for plain batches).
 *   rhs, out  device, [3][V_total] in the batch precision (may be the same buffer);
 * every cell takes part, whatever npfem_batch_set_active selected. Asynchronous on `stream`.
 * Errors: NPFEM_E_INVALID (null batch or buffer, unknown variant), NPFEM_E_UNSUPPORTED (dense on
 * a plain-form batch; a band wider than 65; GEMV staging above 64 KiB), NPFEM_E_HIP.
 */
enum { NPFEM_SOLVE_DENSE = 0, NPFEM_SOLVE_BANDED = 1, NPFEM_SOLVE_AUTO = 2, NPFEM_SOLVE_GEMV = 3 };
npfem_status npfem_global_solve(npfem_batch* batch, int32_t solve, const void* rhs, void* out,
                                void* stream);
/* The variant NPFEM_SOLVE_AUTO uses for `batch` (NPFEM_SOLVE_DENSE, _BANDED or _GEMV) into
 * *solve. Errors: NPFEM_E_INVALID (null argument). */
npfem_status npfem_batch_get_global_solve(const npfem_batch* batch, int32_t* solve);

/*
 * Allocation-free variant of npfem_detect_contacts, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as npfem_detect_contacts (bitwise the same outputs), but
 * the search workspace lives in a static device array of 64 MiB that the library holds on each
 * GPU it runs on until the process ends, instead of memory allocated for the batch. The call
 * makes no device allocation and no host-device copy; the first call on a GPU looks up the
 * array's device address. It serves batches of at most 524 288 (2^19) vertices (about 2 000
 * red cells); larger batches fail with NPFEM_E_UNSUPPORTED before any device work.
 * Every call on one GPU, from any batch, thread or stream, shares the one workspace, and each
 * call rewrites it from scratch: calls that overlap in time on one GPU race and give
 * undefined results. Serialise them (one stream, or events between streams).
 */
npfem_status npfem_detect_contacts_noalloc(npfem_batch* batch, const void* x, double radius,
                                           double separation, double weight, void* contact_p,
                                           void* contact_w, void* stream);

/*
 * Synchronise `stream` and report NPFEM_E_NONFINITE if any step since the last check
 * produced a non-finite position or velocity (the flag is then cleared), NPFEM_E_HIP on a
 * device error, NPFEM_OK otherwise.
 */
npfem_status npfem_batch_check(npfem_batch* batch, void* stream);

/* Thread-local message of the calling thread's last non-OK status ("" if none). */
const char* npfem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NPFEM_H */
