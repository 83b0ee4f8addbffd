/* sem.h -- C ABI of the MI355X hot path of the stabilised nodal spectral
 * element method for fully nonlinear potential-flow water waves
 * (Engsig-Karup, Eskilsson & Bigoni, arXiv:1512.02548).
 *
 * Model (paper Sec. 2): the free-surface elevation eta(x,t) and surface
 * potential phi~(x,t) evolve by the Zakharov equations; the vertical surface
 * velocity w~ comes from the Laplace problem for the potential, solved in the
 * sigma-transformed domain (x, sigma) in [0,L] x [0,1] with
 * sigma = (z + h)/(eta + h), Dirichlet phi = phi~ at the surface and the
 * natural (impermeable) condition at the bed and at walls.
 *
 * Discretisation (Sec. 3): Nx columns x Nz layers of quadrilaterals, each cut
 * into two order-P nodal triangles (warp-and-blend nodes); quadrature-free
 * element operators built from D_r, D_s and M = (V V^T)^{-1}; global L2
 * projections for gradients; over-integrated free-surface right-hand side;
 * classical RK4; per-element modal filter.
 *
 * Conventions
 *  - Array arguments are DEVICE pointers to contiguous FP64 data unless the
 *    comment says HOST.  All device work is ordered on `stream` (a
 *    hipStream_t passed as void*; NULL = the default stream).
 *  - Surface arrays have length ns and are ordered by x.  Volume arrays have
 *    length n in the library's node numbering, exposed by
 *    sem_mesh_node_coords.
 *  - The caller owns every buffer.  The library allocates no device memory:
 *    sem_mesh_query reports the workspace size, the caller allocates it and
 *    hands it to sem_mesh_bind.  The library never frees caller memory.
 *  - Errors are return codes; no exceptions cross the ABI and nothing is
 *    printed.  sem_last_error() gives a thread-local message.  Argument
 *    errors are detected before any launch.  Device-detected conditions
 *    (DOMAIN, NONFINITE, BREAKDOWN, NOCONV) are accumulated in a device
 *    status word and returned when the call ends; every call that returns
 *    such a status synchronises `stream`.
 *  - A mesh is used by one stream at a time (its workspace holds scratch
 *    state); distinct meshes may run concurrently on distinct streams.
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_mesh sem_mesh;
typedef struct sem_batch sem_batch;

typedef enum {
  SEM_OK = 0,
  SEM_E_INVAL = 1,      /* bad argument (host-checked, nothing launched)      */
  SEM_E_NOMEM = 2,      /* workspace too small                                */
  SEM_E_DOMAIN = 3,     /* some water column height d = eta + h <= 0 (Sec. 2)  */
  SEM_E_NOCONV = 4,     /* Krylov solver hit max_iter before rtol             */
  SEM_E_BREAKDOWN = 5,  /* Krylov breakdown (zero Arnoldi norm with r != 0)   */
  SEM_E_NONFINITE = 6,  /* NaN or Inf detected                                */
  SEM_E_DEVICE = 7      /* HIP runtime error                                  */
} sem_status;

typedef enum {
  SEM_PREC_FP64 = 0,     /* plain FP64 Krylov solve                            */
  SEM_PREC_FP32_IR = 1,  /* FP64 iterative refinement, FP32 inner solves       */
  SEM_PREC_BF16_IR = 2   /* FP64 iterative refinement, BF16-stored inner solve */
} sem_precision;

typedef enum {
  SEM_RECOVER_DX = 0,    /* 1D: f[ns] -> f_x[ns]  (M' f_x = S_x f, Sec. 3.1.3)         */
  SEM_RECOVER_W = 1      /* 2D: Phi[n], eta[ns] -> w~[ns] (M w = S_z Phi, Sec. 3.1.3) */
} sem_recover_kind;

typedef enum {
  SEM_OP_STIFFNESS = 0,  /* y = A u, quadrature-free Laplace operator (Sec. 3.1.2, 3.2) */
  SEM_OP_MASS2D = 1,     /* y = M u, 2D mass of the computational domain             */
  SEM_OP_PRECOND = 2,    /* y = B u, Laplace preconditioner (surface rows zero)      */
  SEM_OP_SZ = 3          /* y = S_z u (vertical-derivative projection right side)    */
} sem_operator;

typedef struct {
  int32_t nx, nz;              /* quads in x (>= 1), layers in sigma (1..256)       */
  int32_t order;               /* polynomial order P, 1..8                          */
  int32_t periodic;            /* 1: periodic in x; 0: impermeable walls            */
  double length;               /* L > 0                                             */
  double g;                    /* gravity (9.81)                                    */
  const double *h, *h_x;       /* HOST, ns: still-water depth and slope at the surface nodes */
  const double *sigma_levels;  /* HOST, nz+1 increasing from 0 to 1, or NULL = uniform */
  int32_t filter_ic;           /* modal filter: modes >= ic scaled by filter_sigma (ic >= 2) */
  double filter_sigma;         /* 1.0 = filter off                                  */
  int32_t overint_order;       /* Pf >= P: GLL(Pf) fine grid for the FS right side; Pf == P: none */
  int32_t restart;             /* GMRES restart length, 0 = default (30)            */
  int32_t variant;             /* stiffness kernel: 0 = matrix cores (MFMA), 1 = reference vector-ALU kernel */
  int32_t tiles_per_block;     /* element tile of the stiffness kernel: 16-element MFMA tiles per workgroup
                                  (1..4; the columns per workgroup follow), 0 = chosen from the tank size */
} sem_mesh_desc;

typedef struct {
  int64_t n, ns, n_free, n_elem;
  int32_t np, nblocks;
  uint64_t workspace_bytes;    /* bytes the caller must allocate (256-byte aligned) */
} sem_mesh_info;

typedef struct {
  double rtol;          /* ||b - A x||_2 <= rtol ||b||_2 (free nodes)              */
  int32_t max_iter;     /* total Krylov iterations (inner iterations for IR)       */
  int32_t prec;         /* sem_precision                                           */
  double inner_rtol;    /* IR: relative tolerance of each inner solve, loosened to
                           min(1/2, rtol ||b|| / (2 ||r||)) when that is larger
                           (the last refinement only needs what is left)    */
  int32_t max_refine;   /* IR: maximum outer refinements                           */
  int32_t warm_start;   /* 1: phi holds the initial guess on entry                 */
  int32_t lookahead;    /* Krylov steps the host may queue ahead of the device (>=1) */
  int32_t predict;      /* RK4 steps only: 0..6 past steps extrapolated into each
                           stage solve's start vector (0: the previous stage's Phi) */
} sem_solve_opts;

typedef struct {
  int32_t iters;        /* Krylov iterations (all inner iterations under IR)   */
  int32_t refinements;  /* outer IR steps (0 for FP64)                         */
  double rel_residual;  /* final ||r||/||b|| (FP64 true residual under IR)     */
  double seconds;       /* wall time of the call (host clock, synchronised);
                           for the stage solves of sem_rk4_step, the device
                           time between the solve's first and last launches
                           (events on the stream: the step does not wait for
                           the device around its stage solves)              */
  int32_t status;       /* sem_status of this solve                            */
  int32_t reserved;
} sem_solve_stats;

/* Build the host-side description of a tank (reference element, mesh tables,
 * preconditioner blocks).  Host work only; no device call. */
sem_status sem_mesh_create(const sem_mesh_desc* desc, sem_mesh** out);
sem_status sem_mesh_query(const sem_mesh* mesh, sem_mesh_info* out);
/* Upload constants into caller memory `workspace` (device, >= workspace_bytes,
 * 256-byte aligned) on `stream`.  Must precede every device call. */
sem_status sem_mesh_bind(sem_mesh* mesh, void* workspace, size_t bytes, void* stream);
/* HOST outputs, length n: x and sigma of every volume node. */
sem_status sem_mesh_node_coords(const sem_mesh* mesh, double* x_host, double* sigma_host);
/* HOST output, length ns: volume index of each (x-ordered) surface node. */
sem_status sem_mesh_surface_nodes(const sem_mesh* mesh, int64_t* idx_host);
void sem_mesh_destroy(sem_mesh* mesh);

/* The reference-element operators every mesh of order P is built from (host
 * work only; all outputs HOST, row-major, any may be NULL):
 *  r, s [Np]: warp-and-blend nodes of the reference triangle (Sec. 3.1.4);
 *  Dr, Ds, M [Np x Np]: V_r V^{-1}, V_s V^{-1}, (V V^T)^{-1} (Sec. 3.1.4);
 *  F [(P+1) x (P+1)]: the 1D modal filter V^ diag(sigma) V^{-1} with modes
 *    >= ic scaled by sigma_f (Sec. 3.4; ic >= 2);
 *  I [(Pf+1) x (P+1)]: interpolation from GLL(P) to GLL(Pf) and
 *  Mf [(Pf+1) x (Pf+1)]: the fine mass matrix (Sec. 3.3).
 * Np = (P+1)(P+2)/2; 1 <= P <= 10, P <= Pf <= 32. */
sem_status sem_reference_operators(int32_t P, int32_t Pf, int32_t ic, double sigma_f, double* r, double* s,
                                   double* Dr, double* Ds, double* M, double* F, double* I, double* Mf);

/* Geometric factors of the sigma-map at every element node (Sec. 2, the
 * Jacobian and K = J J^T / det J with q = (1-sigma) h_x - sigma eta_x):
 * stores G = |J| Lam K Lam^T and 1/d in the workspace.  eta, eta_x: [ns]. */
sem_status sem_set_surface(sem_mesh* mesh, const double* eta, const double* eta_x, void* stream);

/* y = op(u) on full-length vectors [n] with the factors of the last
 * sem_set_surface (diagnostic access to the operators of Secs. 3.1.2-3.2). */
sem_status sem_apply(sem_mesh* mesh, sem_operator op, const double* u, double* y, void* stream);

/* Benchmark support: launch the element kernel of `op` reps times back to
 * back on `stream` (same inputs, no host synchronisation in between) and
 * return the mean duration per launch in *ms_host, measured with HIP events
 * recorded on `stream`.  prec is a sem_precision: FP64 takes double vectors,
 * FP32_IR and BF16_IR the inner-solve kernels on float vectors (stiffness and
 * preconditioner only).  Output y as for sem_apply (its shared vertical lines
 * hold only one block's contribution: use sem_apply for values). */
sem_status sem_apply_timed(sem_mesh* mesh, sem_operator op, int32_t prec, const void* u, void* y,
                           int32_t reps, float* ms_host, void* stream);

/* Laplace problem of Sec. 3.1.2 for the surface state (eta, eta_x, phi~):
 * A_FF Phi_F = -A_FS phi~, Phi_S = phi~.  phi [n]: in = initial guess when
 * opts->warm_start, out = Phi including the surface values.  stats may be
 * NULL. */
sem_status sem_laplace_solve(sem_mesh* mesh, const double* eta, const double* eta_x,
                             const double* phi_s, double* phi, const sem_solve_opts* opts,
                             sem_solve_stats* stats, void* stream);

/* Gradient recovery by global L2 projection (Sec. 3.1.3).
 * SEM_RECOVER_DX: in = f [ns], eta unused (may be NULL), out = f_x [ns].
 * SEM_RECOVER_W:  in = Phi [n], eta [ns], out = w~ [ns]. */
sem_status sem_gradient_recover(sem_mesh* mesh, sem_recover_kind kind, const double* in,
                                const double* eta, double* out, void* stream);

/* Velocity in the whole volume (Sec. 3.1.3, eqs. representationU, velocpot,
 * velocpot2; the chain rule of the sigma-map of Sec. 2): u = d phi/dx and
 * w = d phi/dz at every node [n], each from the global L2 projection
 * M u = S_u Phi, M w = S_z Phi with
 *   S_u = int (d_x Phi + sigma_x d_sigma Phi) N_i,  S_z = int (1/d) d_sigma Phi N_i,
 * sigma_x = ((1 - sigma) h_x - sigma eta_x)/d, over the computational domain.
 * Phi [n] (a Laplace solution for the surface eta [ns], eta_x [ns]); u or w
 * may be NULL.  The surface values of w are the w~ of SEM_RECOVER_W. */
sem_status sem_recover_kinematics(sem_mesh* mesh, const double* Phi, const double* eta,
                                  const double* eta_x, double* u, double* w, void* stream);

/* Over-integrated Galerkin right-hand side of the free-surface equations
 * (Secs. 3.1.1, 3.3) followed by the M' solves: (deta_dt, dphi_dt) [ns]. */
sem_status sem_free_surface_rhs(sem_mesh* mesh, const double* eta, const double* eta_x,
                                const double* phi_x, const double* w_s, double* deta_dt,
                                double* dphi_dt, void* stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * right-hand side as sem_free_surface_rhs, bitwise, with its scratch (the
 * element right-hand sides and their node sums, 2 nx (P+1) + 2 ns doubles)
 * in a static device array of SEM_NOALLOC_SCRATCH_BYTES per device instead
 * of the mesh workspace.  Allocates nothing and never synchronises: the call
 * only enqueues on `stream` and returns.  SEM_E_INVAL for a tank whose
 * scratch exceeds the array or when the current device is not the one the
 * mesh was bound on.  All calls on one device share the array, so calls
 * that overlap on one device (concurrent streams or threads) race; order
 * them on one stream.  The array keeps the last call's contents; every
 * value is written before it is read. */
#define SEM_NOALLOC_SCRATCH_BYTES (4u << 20)
sem_status sem_free_surface_rhs_noalloc(sem_mesh* mesh, const double* eta, const double* eta_x,
                                        const double* phi_x, const double* w_s, double* deta_dt,
                                        double* dphi_dt, void* stream);

/* One classical RK4 step of (eta, phi~) [ns] followed by the modal filter
 * (Secs. 3.1.1, 3.4).  phi_ws [n] carries the warm start of the Laplace
 * solves across calls.  Transactional: on error eta and phi_s are left
 * unchanged.  stats: HOST array of 4 (one per stage) or NULL.
 *
 * Stage start vectors: each stage solve starts from the previous stage's
 * Phi (in phi_ws) plus the change from the previous stage to this one,
 * extrapolated over the same stage of the last opts->predict completed steps
 * of this mesh (a polynomial in the step index of that degree).  The mesh's
 * workspace keeps that record; it restarts when dt changes and after
 * sem_rk4_reset_history.  The start vector never changes the stopping test,
 * only the iteration count. */
sem_status sem_rk4_step(sem_mesh* mesh, double* eta, double* phi_s, double* phi_ws, double dt,
                        const sem_solve_opts* opts, sem_solve_stats* stats, void* stream);

/* Wave generation and absorption zones (Sec. 2.2): each surface variable q
 * gets the source (1 - gamma(x)) tau^-1 (q_a(x, t) - q) with tau = dt.
 * sem_set_relaxation stores the weights 1 - gamma at the surface nodes
 * (HOST [ns], each in [0, 1]; NULL switches the zones off); host work, kept
 * across binds.  sem_rk4_step_forced is sem_rk4_step with the source added
 * to every stage's slopes; qa (DEVICE [3][2][ns]) holds the targets
 * (eta_a, phi~_a) at t, t + dt/2 and t + dt.  SEM_E_INVAL when no weights
 * are set.  Meshes with weights set are rejected by sem_batch_create. */
sem_status sem_set_relaxation(sem_mesh* mesh, const double* weight_host);
sem_status sem_rk4_step_forced(sem_mesh* mesh, double* eta, double* phi_s, double* phi_ws, double dt,
                               const double* qa, const sem_solve_opts* opts, sem_solve_stats* stats,
                               void* stream);

/* Forget the recorded stage solutions of `mesh` (ordered on `stream`): call
 * when the state passed to the next step was not reached by the previous
 * steps on this mesh (a new initial condition). */
sem_status sem_rk4_reset_history(sem_mesh* mesh, void* stream);

/* Batching: many independent tanks (each bound to its own workspace)
 * advanced by one call.  A tank's results do not depend on which other tanks
 * are in the batch.  per_tank_status / per_tank_iters: HOST arrays of `count`
 * (may be NULL); active_host (may be NULL = all) selects the tanks of a call.
 * Each tank step is transactional as in sem_rk4_step; the call returns the
 * first failing status.
 *
 * nstreams = 0, lockstep (Secs. 3.1.1-3.1.3 for every tank at once): the
 * Laplace solves of all tanks run as one restarted GMRES in lockstep; every
 * kernel launch of an Arnoldi step covers the workgroups of all tanks, and a
 * tank whose cycle has ended leaves the launches at once.  Each tank keeps
 * its own Krylov scalars, so its arithmetic is the single-tank solve's.
 * Needs periodic or walled tanks with nx >= 2 (exact still-water inverse)
 * and the matrix-core stiffness kernel; FP64 solves.  sem_batch_create
 * allocates the work-item tables (device) and the progress words (pinned
 * host) and uploads them on `stream`.  The meshes must stay bound, unchanged,
 * while the batch exists.  The batch runs on a stream of its own (default
 * priority), ordered after the caller's `stream` on entry; the caller's
 * stream waits for it on return.
 *
 * nstreams >= 1, concurrent: the tanks are spread over `nstreams` worker
 * threads, each driving its own HIP stream (created here, default priority),
 * each tank running sem_rk4_step.  Work recorded on the caller's `stream`
 * before the call is visible to the workers and the caller's stream waits
 * for all of them. */
sem_status sem_batch_create(sem_mesh* const* meshes, int32_t count, int32_t nstreams, void* stream,
                            sem_batch** out);
sem_status sem_batch_rk4_step(sem_batch* batch, double* const* eta, double* const* phi_s,
                              double* const* phi_ws, const double* dt_host,
                              const uint8_t* active_host, const sem_solve_opts* opts,
                              int32_t* per_tank_status_host, int32_t* per_tank_iters_host,
                              void* stream);
/* Lockstep batches only: the Laplace problem of every active tank, as
 * sem_laplace_solve (phi[t] holds the start vector when opts->warm_start). */
sem_status sem_batch_laplace_solve(sem_batch* batch, const double* const* eta,
                                   const double* const* eta_x, const double* const* phi_s,
                                   double* const* phi, const uint8_t* active_host,
                                   const sem_solve_opts* opts, int32_t* per_tank_status_host,
                                   int32_t* per_tank_iters_host, void* stream);
/* Lockstep batches: issue each Arnoldi step as one HIP graph launch (1, the
 * default; captured on first use per step and precision) or as direct kernel
 * launches (0).  Results are the same either way. */
sem_status sem_batch_graphs(sem_batch* batch, int32_t enable);
/* Number of Arnoldi steps captured as graphs so far (0 when capture is not
 * possible and the steps run as direct launches). */
sem_status sem_batch_graph_count(const sem_batch* batch, int32_t* captured_host);
void sem_batch_destroy(sem_batch* batch);

/* Benchmark hook: mean device time (ms, HOST) of one batched stiffness
 * element launch over every tank of `order` in a lockstep batch (all tanks
 * live, no masking), prec 0 = FP64, 1 = FP32, 2 = FP32 with bfloat16
 * factors, over `reps` launches after a warm-up launch.  Overwrites the
 * tanks' scratch vectors. */
sem_status sem_batch_apply_timed(sem_batch* batch, int32_t order, int32_t prec, int32_t reps, float* ms_host,
                                 void* stream);

/* Self-test of the matrix-core instructions' lane layout: runs one 16x16x4
 * FP64 and one FP32 MFMA on known operands in the mesh's scratch space and
 * returns the largest deviation from the expected product in *max_err_host
 * (0 when the layout the kernels assume holds).  raw_host (HOST, 512
 * doubles, may be NULL) receives lane*4+v for FP64 then for FP32. */
sem_status sem_selftest_mfma(sem_mesh* mesh, double* max_err_host, double* raw_host, void* stream);

/* Live timing of the stiffness-apply kernel inside the Krylov iterations
 * (the operator of Secs. 3.1.2 and 3.2): while enabled, every stiffness
 * launch of the GMRES iterations of sem_laplace_solve / sem_rk4_step (and the
 * batch step), in whatever precision the iterations run, is bracketed by HIP
 * events on the solve's stream; launches queued after convergence, which
 * return at once, are not counted.  While enabled the Arnoldi steps use the
 * plain apply with a separate inner-product launch (otherwise the products
 * are fused into the stiffness launch), so that the timing is the apply's
 * alone.  enable = 1 starts (and clears) the accumulation, 0 stops it.  sem_kernel_timing_read returns the number of
 * counted launches and their summed duration in milliseconds (HOST
 * pointers).  Timing adds event records to the stream; leave it off in
 * production. */
sem_status sem_kernel_timing(sem_mesh* mesh, int32_t enable);
sem_status sem_kernel_timing_read(const sem_mesh* mesh, int64_t* launches_host, double* total_ms_host);

const char* sem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SEM_H */
