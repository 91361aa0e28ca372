/*
 * fsgmg — field-split additive-Schwarz geometric multigrid + FGMRES for the
 * linearized monolithic fluid-structure-interaction system on MI355X (gfx950).
 *
 * Method: Calandrini, Aulisa, Ke, "A field-split preconditioning technique for
 * fluid-structure interaction problems with applications in biomedicine":
 *   - the system is ordered as J2 (Section 3.2, eq. matrix_J2): unknowns
 *     d^s d^f p^s | u^s u^f p^f, equations S A V | K F W;
 *   - outer GMRES preconditioned by one geometric-multigrid V-cycle
 *     (Section 3.2): damped Richardson on levels l >= 1, direct solve on l = 0;
 *   - the Richardson smoother is the additive field-split preconditioner P_2
 *     (eq. FS) whose field blocks are solved by additive Schwarz AS_1 / AS_2
 *     (Vanka saddle-point blocks, overlapping ALE blocks, Jacobi on the
 *     lumped kinematic mass), last-writer additive update (Section 3.2);
 *   - prolongation = natural injection, restriction = the equation-routed
 *     R_2 of Section 3.3 (not P^T).
 *
 * Vector layout of a level (all vectors crossing this ABI are the finest
 * level, FP64, device memory unless stated otherwise):
 *   [ d (dim*N2, node-major) | p^s (Nps) | u (dim*N2) | p^f (Npf) ]
 * N2 = Q2 nodes, numbered x-fastest; p^s / p^f = Q1 vertices of solid / fluid
 * elements in vertex order.  Offsets are returned by level_info().
 *
 * Ownership: the handle owns every matrix, transfer, block inverse and
 * Krylov work vector.  Their device memory comes from the fsgmg_allocator
 * given to setup_hierarchy (e.g. a framework's caching allocator), or from
 * hipMalloc on the handle's device when none is given; the handle returns
 * all of it through the same allocator in hierarchy_destroy (and earlier
 * when a rebuild replaces a buffer).  Two small pinned host buffers for
 * Hessenberg read-backs come from hipHostMalloc.
 * Vector arguments are caller-owned and must not alias each other.
 * Streams: all device work is enqueued on the stream given to
 * setup_hierarchy (NULL = default stream).  vcycle_apply, apply_operator and
 * assemble_load are asynchronous; gmres_solve and adjoint_solve return after
 * the convergence decision.  Handles are not thread-safe.
 * Errors: every call returns an fsgmg_status; no exception crosses the ABI;
 * last_error() gives a message for the last failing call on a handle.
 */
#ifndef FSGMG_H
#define FSGMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsgmg_hierarchy* fsgmg_h;

typedef enum {
  FSGMG_OK = 0,
  FSGMG_NOT_CONVERGED = 1, /* x holds the last iterate, info is filled */
  FSGMG_EINVAL = -1,       /* bad argument (sizes, NULL, NaN/Inf in b)  */
  FSGMG_EHIP = -2,         /* a HIP runtime call failed                */
  FSGMG_ESINGULAR = -3,    /* a zero pivot in a block or coarse matrix */
  FSGMG_ENOMEM = -4,       /* device or host allocation failed         */
  FSGMG_ESTATE = -5        /* call not valid in this state (e.g. no blocks
                              built yet, or a device call on a host-only
                              handle)                                  */
} fsgmg_status;

typedef enum { FSGMG_FP64 = 0, FSGMG_FP32 = 1, FSGMG_BF16 = 2 } fsgmg_prec;

/* Device memory for a handle.  alloc(bytes, stream, user) returns device
 * memory of at least `bytes` bytes, 256-byte aligned, usable on `stream`
 * (the stream given to setup_hierarchy), or NULL when it has none (the call
 * then fails with FSGMG_ENOMEM).  free(ptr, stream, user) takes back a
 * pointer alloc returned; the library calls it only after every launch of
 * the handle that may use the memory has finished, so an allocator may hand
 * the memory out again at once.  Both are called from the thread that
 * calls into the library, never during a HIP graph capture.  alloc and
 * free must both be set (or the whole struct be NULL). */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, void* stream, void* user);
  void* user;
} fsgmg_allocator;

/* Multigrid cycle (Section 3.2 admits any): V, W (two coarse cycles per
 * level), F (an F-cycle then a V-cycle on the coarser level). */
typedef enum { FSGMG_CYCLE_V = 0, FSGMG_CYCLE_W = 1, FSGMG_CYCLE_F = 2 } fsgmg_cycle;

/* Schwarz update of the smoother (Section 3.2): additive (every block takes
 * the residual of the iterate the sweep starts from, entry i from the last
 * block containing it) or multiplicative (block after block, each taking
 * the residual of the latest iterate and writing all of its entries). */
typedef enum { FSGMG_SCHWARZ_ADDITIVE = 0, FSGMG_SCHWARZ_MULTIPLICATIVE = 1 } fsgmg_schwarz;

/* Nested structured mesh (Section 3.3: every level is the midpoint
 * refinement of a conforming coarse mesh, regions are the same on every
 * level).  Faces: 0 x-min, 1 x-max, 2 y-min, 3 y-max, 4 z-min, 5 z-max.
 * bc_d[face][region]: 0 natural, 1 d = 0.  bc_u[face][region]: 0 natural,
 * 1 u = 0, 2 parabolic inflow of peak inflow_peak over the fluid extent of
 * the face.  A tag applies to every node of the face that belongs to an
 * element of that region.  region: 0 fluid, 1 solid. */
typedef struct {
  int dim;                     /* 2 (quadrilaterals) or 3 (hexahedra)     */
  int n_levels;                /* >= 1; level 0 = coarse mesh             */
  int nc[3];                   /* coarse elements per axis                */
  const double* breaks[3];     /* host, nc[a]+1 reference breakpoints     */
  const int8_t* region;        /* host, prod(nc) tags, x fastest          */
  int mapping;                 /* 0 identity, 1 circular bulge, 2 smooth  *
                                * cos^2 bulge tangent to the wall (2D),   *
                                * 3 square (x, y) section [0,1]^2 onto a  *
                                * disc (tube along z)                     */
  double map_params[8];        /* bulge: centre x, radius, blend y0, y1;  *
                                * disc: centre x, centre y, radius        */
  int8_t bc_d[6][2];
  int8_t bc_u[6][2];
  double inflow_peak;
} fsgmg_mesh_desc;

/* Linearized physics (Section 2.2 at the stress-free state, frozen advecting
 * velocity w): solid G = E/(2(1+nu)), 1/lambda_L = (1+nu)(1-2nu)/(E nu);
 * Newtonian fluid mu; density rho; dt > 0 finite adds one backward-Euler
 * step (K_ds = -K_us/dt and rho M/dt inertia), dt <= 0 or inf is steady.
 * supg != 0 enables SUPG (eqs. tausupg, lambda_k).  ale_k: 0 k = 1/V of the
 * coarse element containing the point, 1 k = 1.  k_mass: 0 lumped, 1
 * consistent kinematic mass.  w: host array (finest N2 x dim) or NULL.
 * theta (with a finite dt): weight of the steady terms of the momentum rows
 * (the solid-side d rows and the fluid u rows), the rest of a step's
 * operator unchanged: 1 (or 0, the zero-initialized default) is backward
 * Euler, 1/2 Crank-Nicolson for the momentum balance with backward
 * differences for the other time derivatives (Section 2.2); the explicit
 * part -(1 - theta) of those terms joins the time operator of time_rhs.
 * Range [0, 1], else EINVAL. */
typedef struct {
  double E, nu, mu, rho, dt;
  int supg, ale_k, k_mass;
  const double* w;
  double theta;
} fsgmg_physics;

/* Smoother: cores of core[0] x core[1] elements per region, Vanka halo of
 * `halo` element layers (1 = the paper's selection rule), nu_pre / nu_post
 * Richardson sweeps with damping omega, block inverses and level operators
 * of the V-cycle in `prec` (FSGMG_BF16 stores block inverses in bfloat16
 * and keeps FP32 level operators).  The coarse solve's inverse and its
 * accumulation are always FP64; in an FP32 / BF16 cycle its right-hand side
 * is the FP32 restriction and its result is rounded to FP32 for the
 * prolongation, like every other vector inside that cycle.
 * use_graph != 0 captures each FGMRES Arnoldi step (V-cycle, operator
 * product, Gram-Schmidt, Hessenberg read-back) and the V-cycle of
 * vcycle_apply as HIP graphs on first use; they are kept by a later
 * build_fs_as_blocks with the same options (refactoring into the same
 * buffers, as after update_params) and captured again after any other.
 * Graphs are bypassed while kernel_timing records.
 * iface_mult (0 or 1 = off): for each region, a tile row of cores touching
 * another region across a face normal to axis 1 absorbs the next
 * iface_mult - 1 tile rows away from that interface, giving enlarged
 * interface blocks (layered walls only: the regions must be constant along
 * the other axes, else FSGMG_EINVAL).
 * monolithic != 0 builds the comparator of the paper instead of the field
 * split (the AS formula of Section 3.2, P^s_1j / P^f_1j): one Vanka block per
 * core and region over its displacements, velocities and pressures together,
 * u^s included; the rest of the V-cycle is unchanged.
 * cycle: fsgmg_cycle used by vcycle_apply, gmres_solve and adjoint_solve
 * (the transposed cycle is the exact transpose of the chosen one).
 * schwarz: fsgmg_schwarz.  The multiplicative sweep colours the blocks of
 * each level (greedy first fit in block order; blocks conflict when they
 * share an unknown or the operator couples them either way, an entry
 * counting when an affine piece of the operator holds it above 1e-14 of
 * that piece's largest magnitude in the row), runs the colours in order,
 * each colour's blocks at once on the residual of the latest iterate, then
 * the unknowns in no block (which must be mutually uncoupled, else
 * FSGMG_EINVAL); the damping omega scales the whole sweep's correction.  The
 * blocks are then stored colour by colour (export_blocks shows that order),
 * with full inverses (every row of a block is written).  The transposed
 * sweep runs the reverse order with transposed block solves.
 * sweep_form: 0 = chosen per level by the autotuner (see tuning_info),
 * 1 = a residual SpMV before each forward sweep, 2 = forward sweeps that
 * form their blocks' residual rows inside the smoother launch (additive:
 * alternating between two iterate buffers; multiplicative: in place, colour
 * by colour).  Transposed sweeps always take the residual SpMV.
 * interchange != 0 builds the cascade the paper names as future work
 * (Section 5: its GMG and FS boxes swapped): GMRES preconditioned by the
 * field split P_2 of eq. FS, block diagonal over the groups [d, p^s] and
 * [u, p^f], each diagonal block approximated by one multigrid cycle on that
 * block.  Both blocks' cycles share the levels, so they run as one cycle on
 * the field split's diagonal blocks of every level operator (entries that
 * couple the two groups removed), with the restriction kept inside each
 * group (without R_2's routing of fine fluid-momentum rows into coarse
 * solid-momentum rows), the same prolongation and FS-AS smoother, and the
 * direct solve of level 0's diagonal blocks; FGMRES keeps the whole
 * operator.  Sweeps use the SpMV form (sweep_form 2: EINVAL); the
 * transposed cycle, adjoint_solve and the k-column calls are not built for
 * it (EINVAL). */
typedef struct {
  int core[3];
  int halo;
  int nu_pre, nu_post;
  double omega;
  fsgmg_prec prec;
  int use_graph;
  int iface_mult;
  int monolithic;
  int cycle;
  int schwarz;
  int sweep_form;
  int interchange;
} fsgmg_smoother_opts;

/* FGMRES(restart), right preconditioned, x0 = 0, CGS2; converged when the
 * true residual ||b - A x||_2 <= rtol ||b||_2. */
typedef struct {
  int restart;       /* 1..64 */
  int max_restarts;
  double rtol;
} fsgmg_krylov_opts;

typedef struct {
  int iters;          /* Arnoldi steps                                     */
  int restarts;
  int converged;
  double rel_res_true;
  double* history;    /* host, optional: Givens estimates / ||b||         */
  int history_cap;
  int history_len;
  double t_solve_ms;  /* wall time of the call                           */
  int vcycles;        /* multigrid cycles applied (one per Arnoldi step)  */
  double t_setup_ms;  /* wall time of the handle's setup_hierarchy        */
  double t_blocks_ms; /* wall time of its last build_fs_as_blocks         */
} fsgmg_solve_info;

/* Build the mesh hierarchy (Section 3.3: nested midpoint refinements with
 * the same regions on every level), assemble every level operator in the
 * J2 ordering (Sections 2.2 and 3.1, eq. matrix_J2; re-discretized,
 * Dirichlet rows/columns eliminated symmetrically), the transfers (Section
 * 3.3) and the coarse FP64 inverse (the direct solve on level 0 of Section
 * 3.2).  mesh, phys and the host arrays they point to are read during the
 * call only.  alloc: device memory for the handle (NULL: hipMalloc).
 * device >= 0: upload to that HIP device and use `stream`; device == -1:
 * host-only handle (export_* and dof_map queries only).  *out receives the
 * handle also on failure (read last_error, then hierarchy_destroy); EINVAL
 * for an invalid description or parameters, ENOMEM, EHIP. */
fsgmg_status setup_hierarchy(const fsgmg_mesh_desc* mesh, const fsgmg_physics* phys,
                             const fsgmg_allocator* alloc, int device, void* stream,
                             fsgmg_h* out);

/* Build the FS-AS block index sets (Section 3.2: the field split P_2 of
 * eq. FS, its blocks solved by additive Schwarz AS_1 / AS_2 with the Vanka
 * selection rule and the last-writer owner map), gather every block's principal submatrix, invert it on the
 * device by Gauss-Jordan with partial pivoting (in FP64 for FP64 inverses,
 * in FP32 for FP32 and BF16 inverses) and keep the owned rows in
 * opts->prec.
 * ESINGULAR (block id in last_error) on a zero pivot.  On a host-only handle
 * only the index sets are built. */
fsgmg_status build_fs_as_blocks(fsgmg_h h, const fsgmg_smoother_opts* opts);

/* z = M^{-1} r (transpose = 0) or z = M^{-T} r (transpose = 1): one cycle of
 * the geometric multigrid preconditioner of Section 3.2 (damped Richardson
 * with the FS-AS smoother on levels >= 1, restriction R_2 and prolongation
 * of Section 3.3, direct solve on level 0); the transpose runs every step
 * transposed in reverse order.  r, z: device FP64, finest level, r != z.
 * Asynchronous on the handle's stream.  ESTATE before build_fs_as_blocks,
 * ESINGULAR when a pending coarse rebuild met a zero pivot. */
fsgmg_status vcycle_apply(fsgmg_h h, const double* r, double* z, int transpose);

/* The cycle of vcycle_apply (Section 3.2; additive smoother; transpose != 0:
 * its exact transpose) on k right-hand sides at once, 1 <= k <= 64: r and z are device
 * FP64 arrays of N * k entries, unknown-major (entry (i, c) at i * k + c: a
 * contiguous N x k row-major matrix), caller-owned, r != z.  Column c of z
 * equals vcycle_apply of column c of r (same transpose flag) up to rounding
 * (every launch works on all k columns; the block applies run on the matrix
 * cores, the transposed one with transposed copies of the block inverses
 * made on first use after each factorization).
 * Work buffers of N_l * k entries per level are allocated on the first call
 * with a larger k and kept.  EINVAL for k out of range, the multiplicative
 * smoother or a Schwarz block of more than 1024 unknowns, ESTATE before
 * build_fs_as_blocks. */
fsgmg_status vcycle_apply_batch(fsgmg_h h, const double* r, double* z, int k, int transpose);

/* Solve A x = b on the finest level: GMRES (Section 3.2's outer solver, here
 * FGMRES(restart) with CGS2) right-preconditioned by one cycle of
 * vcycle_apply per iteration.  b, x: device FP64, finest level, b != x; x is
 * overwritten (x0 = 0).  Returns after the convergence decision; info (host,
 * optional) receives iterations, restarts, the true relative residual,
 * times and the residual history.  NOT_CONVERGED leaves the last iterate in
 * x; EINVAL for NaN/Inf in b or bad options; ESTATE before
 * build_fs_as_blocks. */
fsgmg_status gmres_solve(fsgmg_h h, const double* b, double* x,
                         const fsgmg_krylov_opts* opts, fsgmg_solve_info* info);

/* FGMRES of gmres_solve on k right-hand sides at once (1 <= k <= 64, additive
 * smoother): b and x are device FP64 arrays of N * k entries, unknown-major
 * (entry (i, c) at i * k + c), caller-owned, b != x, x overwritten (x0 = 0).
 * Every column has its own Krylov basis, Givens rotations and convergence
 * test, exactly as gmres_solve; every operator product, cycle
 * (vcycle_apply_batch) and Gram-Schmidt pass works on all k columns at once.
 * infos: host array of k entries (history is not recorded) or NULL.
 * Returns FSGMG_OK when every column converged, FSGMG_NOT_CONVERGED if some
 * did not; the other errors as vcycle_apply_batch. */
fsgmg_status gmres_solve_batch(fsgmg_h h, const double* b, double* x, int k,
                               const fsgmg_krylov_opts* opts, fsgmg_solve_info* infos);

/* adjoint_solve on k right-hand sides at once: gmres_solve_batch with A^T
 * and the transposed cycle (same arguments, layout and errors). */
fsgmg_status adjoint_solve_batch(fsgmg_h h, const double* c, double* lam, int k,
                                 const fsgmg_krylov_opts* opts, fsgmg_solve_info* infos);

/* Solve A^T lam = c (the adjoint of the linearized system of Sections 2.2
 * and 3.1) by gmres_solve's FGMRES with A^T and the transposed cycle of
 * vcycle_apply as right preconditioner.  Same arguments, layout, return and
 * errors as gmres_solve; A^T and the transposed block inverses are built on
 * first use. */
fsgmg_status adjoint_solve(fsgmg_h h, const double* c, double* lam,
                           const fsgmg_krylov_opts* opts, fsgmg_solve_info* info);

/* b = F (L f) + lift: the momentum load rho (f_h, phi) of the weak form of
 * Section 2.2 (+ its SUPG counterpart, eq. tausupg) for a nodal body force
 * f (device, finest N2 x dim), Dirichlet rows set to their values and the
 * Dirichlet lift applied (F zeroes Dirichlet rows).  Asynchronous. */
fsgmg_status assemble_load(fsgmg_h h, const double* f_nodal, double* b);

/* gf = (F L)^T lam: the adjoint of assemble_load's linear part (the load of
 * Section 2.2), i.e. the gradient of lam^T b with respect to the nodal body
 * force (device, finest N2 x dim output, lam of the finest level size). */
fsgmg_status load_adjoint(fsgmg_h h, const double* lam, double* gf);

/* y = A_l x or A_l^T x on level `level`: the linearized operator J2 of eq.
 * matrix_J2 (Sections 2.2, 3.1) re-discretized on that level, FP64, device
 * vectors of that level's size, x != y.  Asynchronous. */
fsgmg_status apply_operator(fsgmg_h h, int level, const double* x, double* y, int transpose);

/* out[0] = -(F lam)^T dA/dE x, out[1] = -(F lam)^T dA/dmu x on the finest
 * level: the parameter gradients of a functional through the adjoint of the
 * system of Section 2.2 (E enters the solid stress through G and lambda_L,
 * mu the fluid stress and the Dirichlet lift; unreduced derivative, SUPG
 * tau frozen); lam, x device; out host (synchronizes). */
fsgmg_status param_grad(fsgmg_h h, const double* lam, const double* x, double out[2]);

/* param_grad for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels in the same order, so the same out[] bit for bit, with
 * the product dA/dtheta x, the reduction partials and the three sums in a
 * file-scope device array of 32 MiB instead of the handle's lazily
 * allocated buffers; it calls no allocating routine.  Limit: the finest
 * level's unknowns N must satisfy 8 N + 256 KiB <= 32 MiB (N up to about
 * 4.1 M), else EINVAL.  Each GPU holds one such array until the process
 * ends, shared by every call on that GPU: calls that overlap on one GPU
 * (several host threads or streams) race and must be serialized by the
 * caller.  Synchronizes the handle's stream; EHIP when the array's device
 * address cannot be obtained; other errors as param_grad. */
fsgmg_status param_grad_noalloc(fsgmg_h h, const double* lam, const double* x, double out[2]);

/* Recombine every level operator and the Dirichlet lift for new (E, mu)
 * from the stored affine pieces of the Section 2.2 operator (it is affine in
 * G, 1/lambda_L and mu; SUPG tau frozen at setup).  Invalidates the
 * blocks: call build_fs_as_blocks again.  The coarse inverse is rebuilt on
 * a stream of the library's own, after the new level-0 values on the
 * handle's stream, without waiting for it (the call returns at once, and a
 * following block refactorization runs beside it); the next cycle or solve
 * waits for it and returns FSGMG_ESINGULAR if the coarse matrix turned out
 * singular. */
fsgmg_status update_params(fsgmg_h h, double E, double mu);

/* Picard step of the nonlinear loop (Section 2.2: the paper linearizes each
 * time step by Newton's method; here the convection and SUPG terms are
 * re-linearized about the latest velocity): re-assemble every level
 * operator, the Dirichlet lift, the load operator and the time operator
 * about the advecting velocity w = the velocity part of x (finest level
 * vector in device memory, in host memory for a host-only handle; w at the
 * finest Q2 nodes, injected at the coarse levels' nodes), with the current
 * (E, mu); the operators' patterns do not change.  The first call
 * assembles on the host (one thread per level) and keeps, per level, the
 * sums of the terms that do not depend on w (host memory of four values
 * per operator entry and a 32-bit slot per advective term), adding the
 * convection and SUPG terms element colour by element colour, so the
 * values equal a fresh setup's about the same w bit for bit.  Later calls
 * on a 2D device hierarchy with the additive smoother (not interchanged)
 * run on the device: the elements' terms in the host's order and
 * arithmetic, gathered onto the kept sums in the host's order, so the
 * values agree with the host's to rounding (the host copies are fetched
 * when a host consumer such as export_csr needs them); otherwise on the
 * host as the first.  Asynchronous on the device except for the check of
 * the velocity.  Invalidates the blocks (call build_fs_as_blocks again) and
 * rebuilds the coarse inverse as update_params does.  EINVAL for a hierarchy set up without an advecting
 * velocity (physics.w = NULL) or a velocity with NaN / Inf. */
fsgmg_status update_advection(fsgmg_h h, const double* x);

/* b = F (L f) + g lift + F T x_prev: the right-hand side of one backward-
 * Euler step (the time discretization of Section 2.2) of the linearized
 * system, for the nodal body force f (device, finest N2 x dim), the
 * Dirichlet data scaled by g (every nonzero prescribed value is inflow, so
 * g is the pulsatile inflow factor) and the previous state x_prev (device,
 * finest level).  T holds the operator's terms that carry 1/dt (inertia,
 * the kinematic coupling of the solid, the SUPG time term) on the free
 * rows (and, for theta < 1, -(1 - theta) times the steady terms of the
 * momentum rows); F zeroes Dirichlet rows, which receive g times their data.  b must
 * not alias x_prev or f.  EINVAL for a steady hierarchy (dt <= 0 or inf).
 * Asynchronous. */
fsgmg_status time_rhs(fsgmg_h h, const double* f_nodal, double g, const double* x_prev,
                      double* b);

/* One run of the time-periodic outer loop of Sections 2.2 and 4: `steps`
 * backward-Euler steps t_i = t0 + i dt (dt of the hierarchy) with the
 * pulsatile inflow factor g(t) = 1 + inflow_amp sin(2 pi t) (the 2D
 * aneurysm inflow of Section 4.1 has amplitude 0.75), each time step solved
 * by up to picard_max Picard steps: update_advection about the latest
 * iterate (the previous state for the first), build_fs_as_blocks with the
 * handle's current smoother options, time_rhs and gmres_solve (x0 = 0);
 * a time step ends early once ||x_s - x_{s-1}|| <= picard_tol ||x_s||
 * (picard_tol = 0: always picard_max steps). */
typedef struct {
  int steps;            /* time steps (>= 1)                             */
  double t0;            /* time of the initial state                     */
  int picard_max;       /* nonlinear steps per time step (>= 1)          */
  double picard_tol;    /* relative change that ends a time step (>= 0)  */
  double inflow_amp;    /* amplitude of the pulsatile inflow factor      */
} fsgmg_period_opts;

/* Section 4's statistics of the run: s_max the mean number of nonlinear
 * steps per time step, N the mean GMRES iterations per linear solve, rho
 * the mean per-iteration residual reduction (r_N / r_0)^(1 / N_i,s) of the
 * solves (true residuals, r_0 = ||b||); wall times of the host assembly,
 * the block factorizations, the solves (right-hand side, FGMRES, change
 * norms) and the whole call. */
typedef struct {
  int steps;            /* time steps completed                          */
  int solves;           /* linear solves                                 */
  int max_iters;
  double N, rho, s_max;
  double t_assemble_ms, t_factor_ms, t_solve_ms, t_total_ms;
} fsgmg_period_info;

/* x (device, finest level): the state at t0 on entry, at t0 + steps dt on
 * return.  iters / changes (host, optional, steps x picard_max, row-major;
 * -1 / NaN where a time step ended early): each linear solve's iterations
 * and relative change.  Requires a hierarchy set up with a finite dt and an
 * advecting velocity (EINVAL) whose blocks were built once (ESTATE).
 * Returns NOT_CONVERGED when a solve misses rtol (x then holds that
 * solve's iterate, info covers the steps so far); any other error leaves x
 * as on entry.  Synchronizes. */
fsgmg_status period_solve(fsgmg_h h, const fsgmg_period_opts* opts,
                          const fsgmg_krylov_opts* krylov, const double* f_nodal, double* x,
                          int32_t* iters, double* changes, fsgmg_period_info* info);

/* Test hook that makes FSGMG_ESINGULAR observable with valid data: the next
 * build_fs_as_blocks replaces the gathered matrix of Schwarz block `block`
 * (export_blocks numbering) of level `level` (1 .. L-1) by zeros before
 * inverting it, so that block's first pivot is zero and the call returns
 * FSGMG_ESINGULAR naming it in last_error; every kernel still runs to its
 * normal end (the zero-pivot exit leaves an identity column permutation
 * for the owned-row extraction).  The hook applies once; block < 0 clears
 * it.  A block id beyond the level's blocks never matches (no effect).
 * EINVAL for a level out of range. */
fsgmg_status debug_zero_block(fsgmg_h h, int level, int64_t block);

/* out[0..8] = N, N2, Nps, Npf, off_ps, off_u, off_pf, nnz(A_l), dim. */
fsgmg_status level_info(fsgmg_h h, int level, int64_t out[9]);

/* What each unknown of level `level` is (the J2 unknowns of eq. matrix_J2 in
 * the vector layout above).  *n: in, the length of the output arrays; out,
 * the level's number of unknowns N (call with every array NULL to get it).
 * Per unknown i (host arrays, each optional): field[i] 0 = d, 1 = p^s,
 * 2 = u, 3 = p^f; comp[i] the vector component (0 for pressures); node[i]
 * the Q2 node (d, u) or Q1 vertex (pressures) index, both x-fastest on the
 * level's node / vertex lines; xyz[3 i .. 3 i + 2] the physical coordinates
 * of that node (z = 0 in 2D).  EINVAL for a bad level or arrays shorter
 * than N.  Valid on host-only handles. */
fsgmg_status dof_map(fsgmg_h h, int level, int64_t* n, int32_t* field, int32_t* comp,
                     int32_t* node, double* xyz);

/* Host copies of setup data (inspection and tests).  which: 0 reduced level
 * operator A_l, 1 prolongation P_l (level l from l-1, Dirichlet-masked),
 * 2 restriction R_l (level l-1 from l, equation-routed, Dirichlet-masked),
 * 3 load operator L of the finest level (N x dim*N2), 4 time operator T of
 * the finest level (N x N, Dirichlet rows empty; finite dt only).  Call with NULL
 * arrays to get sizes in dims[0..2] = rows, cols, nnz. */
fsgmg_status export_csr(fsgmg_h h, int level, int which, int64_t dims[3],
                        int64_t* rowptr, int32_t* col, double* val);

/* Host copy of a level vector: which 0 = Dirichlet lift (finest), 1 =
 * Dirichlet mask (1.0 / 0.0). */
fsgmg_status export_vector(fsgmg_h h, int level, int which, double* out);

/* Block index sets of level l: sizes[0] = number of blocks, sizes[1] = total
 * entries; ptr (nblk+1), dofs (total, sorted per block), owner (N, -1 if
 * none). */
fsgmg_status export_blocks(fsgmg_h h, int level, int64_t sizes[2], int64_t* ptr,
                           int32_t* dofs, int32_t* owner);

/* Colours of the multiplicative sweep on level l >= 1: *ncolours (0 for the
 * additive smoother) and, if colour_ptr is not NULL, colour_ptr[0..ncolours]
 * = index of the first block of each colour in export_blocks order (the
 * last entry is the number of blocks).  ESTATE before build_fs_as_blocks. */
fsgmg_status block_colours(fsgmg_h h, int level, int64_t* ncolours, int64_t* colour_ptr);

/* Measurement: enable != 0 starts recording HIP events on the handle's
 * stream around selected launches (cleared on start); enable == 0 stops,
 * synchronizes and returns per kind the number of launches and their summed
 * duration: 0 smoother sweep on the finest level, 1 residual SpMV of the
 * V-cycle on the finest level, 2 outer FP64 SpMV of FGMRES, 3 restriction +
 * prolongation between the two finest levels (vcycle_apply_batch records its
 * K-column block applies as kind 0 and its K-column residuals as kind 1).
 * counts / total_ms may be NULL. */
fsgmg_status kernel_timing(fsgmg_h h, int enable, int64_t counts[4], double total_ms[4]);

/* Measurement: the read-only streaming rate of the device, as the ceiling a
 * read-dominated kernel is held against.  A buffer of `bytes` (>= 1 MiB,
 * from the handle's allocator, freed on return) is read once per launch
 * with 16-byte loads by a grid of 2,048 workgroups, `reps` times after one
 * warm-up; *gbs = bytes / median launch time (HIP events on the handle's
 * stream), in GB/s.  Synchronizes; ENOMEM without room for the buffer. */
fsgmg_status stream_read_ceiling(fsgmg_h h, int64_t bytes, int reps, double* gbs);

/* Launch shapes chosen by the autotuner that build_fs_as_blocks runs on the
 * device (HIP-event timing of each candidate launch on the level's own data,
 * median of five, each after a read pass over a 512 MB scratch buffer that
 * evicts the caches as the finer levels do inside a cycle; the buffer is
 * allocated for the autotuning only, and without room for it the candidates
 * are timed warm; kept by later builds with the same block structure and
 * precision):
 * out[0] = lanes per row of the level's V-cycle SpMV (1, 2, 4, 8, 16),
 * out[1] = smoother workgroup width (256, 512, 1024; negative = the same
 * width with non-temporal loads of the block inverses; 0 on level 0),
 * out[2] = lanes per row of the outer FP64 product, out[3] / out[4] = lanes
 * per output of the restriction from / prolongation to this level (0 on
 * level 0), out[5] = 1 when the level's forward sweeps form their residual
 * inside the smoother launch from per-block copies of the operator rows
 * (one launch per sweep) instead of a residual SpMV before each sweep (0 on
 * level 0), out[6] = workgroups sharing one block in the SpMV-form forward
 * sweep (1, 2, 4 or 8; each takes a contiguous share of the block's rows;
 * 0 on level 0).  ESTATE before the first device block build. */
fsgmg_status tuning_info(fsgmg_h h, int level, int32_t out[7]);

const char* last_error(fsgmg_h h);
void hierarchy_destroy(fsgmg_h h);

#ifdef __cplusplus
}
#endif
#endif /* FSGMG_H */
