/*
 * rexi.h -- C ABI of the MI355X REXI propagation step.
 *
 * The library advances the semi-discrete Schroedinger equation
 *     i hbar psi'(t) = H psi(t),   H = -(hbar^2 / 2m) Lap_h + diag(V)
 * (eq. schroedinger, Section 1; the IVP of eq. ode-system with A = H and
 * B = hbar I for a finite-difference discretisation) by REXI steps
 * (eq. rational-evaluation, Section 3.1):
 *     psi_{n+1} = sum_{j=1..K} w_j (H - s_j I)^{-1} psi_n ,
 *     s_j = i hbar sigma_j / dt ,   w_j = i hbar beta_j / dt ,
 * where r(z) = sum_j beta_j / (z - sigma_j) ~ exp(z) on i[-R1, R1] is a
 * rational approximation in partial fractions (eq.
 * partial-fraction-decomposition), e.g. the Faber-CF approximation of
 * Section 3.2. The caller supplies the dimensionless (sigma_j, beta_j);
 * they are computed once, on the host, and do not depend on psi (Section 3.1).
 *
 * Two solvers (option solver):
 *   - per pole: every shifted system is solved by restarted GMRES (x0 = 0)
 *     driven by a matrix-free stencil matvec on the GPU, all poles batched
 *     together; the weighted pole sum is accumulated in FP64 in a fixed
 *     pole order;
 *   - shared basis: with x0 = 0 all poles of an instance share one Krylov
 *     space, so one Lanczos process on H (partial reorthogonalisation)
 *     serves every pole through its own small least-squares problem, and the
 *     pole sum is one combination of the basis (Section 5 names such shifted
 *     Krylov methods); poles that need more than m vectors restart on a
 *     shared basis too (option fallback).
 * The mass-matrix form with Q1 elements (option discretization) takes
 * either solver.
 *
 * Grid and layout
 *   n[a] interior points per axis a on [lo[a], hi[a]], zero Dirichlet values
 *   outside (Section 1): h_a = (hi[a] - lo[a]) / (n[a] + 1). Vectors are
 *   C-order (axis ndim-1 fastest), complex values interleaved re, im
 *   (layout of std::complex<double> / torch.complex128). V is float64.
 *
 * Conventions
 *   - Pointers named *_dev are device pointers (HIP, same device as the
 *     handle); *_host are host pointers. The caller owns every pointer it
 *     passes; the library owns the handle and its workspaces and never frees
 *     caller memory. rexi_setup copies V, so V may be freed afterwards.
 *   - stream is a hipStream_t (NULL = the default stream). Calls enqueue work
 *     on it; rexi_step and rexi_step_adjoint synchronise it (they read the
 *     device-side convergence counters) unless the handle was set up with
 *     capture_safe = 1 and info == NULL, in which case rexi_step is
 *     asynchronous and enqueues no host reads. A pole that misses its target
 *     within that fixed schedule leaves its best iterate in the sum;
 *     rexi_step with info reports convergence.
 *   - Every call returns a rexi_status and never aborts or throws. After an
 *     error, rexi_last_error() holds a message. Handles are not thread-safe;
 *     distinct handles may be set up and used from different threads (the
 *     setup tuner's cache is shared under a lock).
 */
#ifndef REXI_H
#define REXI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } rexi_c128;

typedef struct {
  int32_t ndim;     /* 1, 2 or 3 */
  int32_t reserved;
  int64_t n[3];     /* interior points per axis (axes >= ndim ignored) */
  double lo[3];
  double hi[3];
} rexi_grid;

typedef enum {
  REXI_OK = 0,
  REXI_E_INVALID_ARG = 1,   /* bad sizes, non-finite inputs, singular shift  */
  REXI_E_NO_MEMORY = 2,     /* a workspace does not fit on the device        */
  REXI_E_HIP = 3,           /* a HIP runtime call failed                      */
  REXI_E_NOT_CONVERGED = 4, /* a pole missed its tolerance; output written    */
  REXI_E_NOT_BUILT = 5      /* the library was built without this feature     */
} rexi_status;

typedef enum {
  REXI_PREC_C128 = 0,       /* complex128 Krylov basis and matvec             */
  REXI_PREC_C64_REFINE = 1  /* complex64 basis and matvec inside FP64
                               residual refinement (FP64 dots, Hessenberg,
                               residual, solution and pole sum)               */
} rexi_precision;

typedef enum {
  REXI_TOL_RELRES = 0,      /* every pole to ||psi - (H - s_j) x_j|| <= tol ||psi|| */
  REXI_TOL_CERTIFIED = 1    /* per-pole targets tol Re(sigma_j) / (K |beta_j|), so
                               sum_j |w_j| ||r_j|| / dist(s_j, spec H) <= tol ||psi|| */
} rexi_tol_policy;

typedef enum {
  REXI_SOLVER_PER_POLE = 0, /* one Krylov basis per pole, all poles batched    */
  REXI_SOLVER_SHIFTED = 1   /* one basis shared by all poles of an instance
                               (x0 = 0 gives K_k(H - s I, psi) = K_k(H, psi)):
                               one Lanczos process per instance and K small
                               least-squares problems; complex128; single
                               instances and batches; poles beyond the basis
                               restart on a shared basis (option fallback).
                               With finite differences, rexi_step with info
                               forms every pole solution x_j = V y_j and
                               reports its explicit FP64 residual             */
} rexi_solver;

typedef enum {
  REXI_DISC_FD = 0,         /* finite differences: A = H (3/5/7-point
                               Laplacian + diag V), B = hbar I                */
  REXI_DISC_FEM_Q1 = 1      /* tensor-product linear finite elements on the
                               same nodes (Section 2 with Q1 elements):
                               A = (hbar^2/2m) K + h^d diag(V) (potential by
                               nodal quadrature), B = hbar M (consistent mass);
                               the step is sum_j w_j (A - s_j M)^{-1} M psi.
                               Per-pole solver, or the shared-basis solver
                               for one instance (M = L L^T with Kronecker
                               Cholesky factors; Lanczos on L^-1 A L^-T from
                               L^T psi, targets in the M-norm); no adjoint   */
} rexi_discretization;

typedef struct {
  int32_t precision;   /* rexi_precision, default REXI_PREC_C128            */
  int32_t solver;      /* rexi_solver, default REXI_SOLVER_PER_POLE          */
  int32_t m;           /* Krylov dimension per cycle (restart length), 30;
                          at most 256. For the shared-basis solver the
                          largest basis of one cycle (poles that need more
                          restart on a new shared basis, option fallback)   */
  int32_t max_cycles;  /* restarts / refinement sweeps per solve, 40         */
  double tol;          /* see tol_policy, default 1e-10                      */
  int32_t tol_policy;  /* rexi_tol_policy, default REXI_TOL_RELRES           */
  int32_t reorth;      /* 0 classical Gram-Schmidt, 1 DGKS when cancellation
                          is detected (default), 2 always twice              */
  double reorth_eta;   /* DGKS threshold: a second pass when the projected
                          vector keeps less than eta of its norm, 1e-2       */
  double inner_rtol;   /* C64_REFINE: a complex64 sweep stops when it has
                          reduced its FP64 starting residual by this factor
                          (or met the pole's target), 0.1                   */
  int32_t check_every; /* shared-basis solver: iterations between host reads
                          of the convergence flag, default 4                 */
  int32_t lanczos;     /* shared-basis solver: H is Hermitian, so the basis
                          follows the three-term (Lanczos) recurrence with
                          partial reorthogonalisation. 1 (default): one fused
                          pass per iteration (update of u_{j+1} and the next
                          matvec together); 2: separate update and matvec
                          passes; 0: full Arnoldi with DGKS. Q1 elements
                          on the shared basis always take 2 (their matvec
                          is formed outside the pass kernels)            */
  int32_t capture_safe;/* 1: rexi_step(info = NULL) runs a fixed schedule
                          with no host reads (all m iterations; per-pole:
                          capture_cycles cycles), finished poles skipped on
                          the device. Captured once per (psi_in, psi_out,
                          nsteps) into a HIP graph that is replayed on the
                          stream; if the stream is itself being captured,
                          the schedule is enqueued into the caller's graph.
                          The shared basis with the tiled pass (march_slots
                          2) takes one launch per iteration, with room for
                          capture_pauses second Gram-Schmidt passes        */
  int32_t capture_cycles; /* capture_safe: cycles of a captured solve, the
                          first included: per-pole solver 4 (C64_REFINE:
                          16), shared basis 1 (no restarts) when 0 (the
                          default); shared basis
                          with fallback 1: capture_cycles - 1 restart cycles
                          on the shared basis                               */
  int32_t graph_chunks;   /* shared-basis solver: replay cached HIP graphs of
                             iteration chunks between host checks, 1        */
  int32_t profile;     /* 1: time kernel classes with HIP events             */
  int32_t tile;        /* points per work tile: 512, 1024, 2048, or 0 (tuned) */
  int32_t grid_blocks; /* workgroups of the grid-stride kernels (0 = tuned)  */
  int32_t autotune;    /* 1 (default): with tile = grid_blocks = 0, time the
                          candidate tilings x grid sizes on short runs at
                          setup and keep the fastest (cached per problem
                          shape; REXI_TUNE_CACHE names an optional file)     */
  int64_t max_workspace_bytes; /* device workspace cap, 0 = 90% of free     */
  int32_t march_planes; /* fused Lanczos pass of the shared-basis solver
                           (lanczos = 1): 0 (default) the tuner chooses
                           between the row-staged pass and the pass that
                           marches along the slowest grid axis (without
                           tuning: the row-staged pass); -1 the row-staged
                           pass; 1..1024 the marching pass with that many
                           planes per work item (row-staged where a system's
                           band of rows does not fit)                         */
  int32_t march_slots;  /* marching pass: points per thread and plane, 3, 5
                           or 8 (0 = 5); a band holds 256 slots / n2 - 2
                           rows of the plane. 2: the tiled pass, which forms
                           H u_j in the pass and stores no z (56 B per point
                           instead of 88; instances below 2^27 points); its
                           items are 16 x 32 points of the plane, or, when
                           every instance is 2D, strips of 253 points of a
                           row marching along the rows                       */
  int32_t fallback;     /* shared-basis solver, poles that miss their target
                           within m vectors:
                           1 (default) restarts on the shared basis: such a
                           pole takes the Galerkin iterate of the basis,
                           whose residual is a multiple of the next basis
                           vector u_m for every such pole of an instance; a
                           new shared basis on u_m then serves all of them
                           (cycles of up to m vectors, at most max_cycles);
                           2: per-pole restarted solves (complex64 + FP64
                           refinement, restart length fallback_m,
                           max_cycles cycles) warm-started from the
                           shared-basis iterate;
                           0: they are reported in not_converged.
                           1 and 2 need host checks (not capture_safe)       */
  int32_t fallback_m;   /* restart length of the per-pole solves of
                           fallback 2 (and of the per-pole adjoint solves of
                           a shared-basis handle), 30                        */
  int64_t fallback_bytes; /* fallback 2: device workspace reserved for the
                           per-pole solves at setup (0 = min(16 GiB, a
                           quarter of the free memory)); unconverged poles
                           are solved in waves that fit                      */
  double stab_eps;      /* weights scaled by (1 - stab_eps), 0 <= stab_eps
                           < 1 (Section 3.4: |r(iy)| exceeds one by up to
                           the approximation error ||e||; a factor
                           1 - eps with eps slightly above ||e|| makes the
                           step stable). Default 0 (not applied)            */
  int32_t center;       /* 1: solve with H - c I, c the midpoint of the
                           spectrum bound [min V, (hbar^2/2m) sum 4/h^2 +
                           max V] of each instance, and multiply the step by
                           exp(-i dt c / hbar) (folded into the weights):
                           the interval the poles must cover halves. The
                           same step for the exact exponential; 0 default.
                           With Q1 elements: A - c M, c from the bound of
                           the pencil (A, M)                                */
  int32_t discretization; /* rexi_discretization, default REXI_DISC_FD      */
  int32_t adjoint_shared; /* shared-basis handles: 1 (default) the adjoint
                           step uses two shared bases (psi_n with the poles,
                           gbar with their conjugates) and forms dL/dV as a
                           bilinear form of the two bases; per-pole solves
                           when a pole misses its target within m vectors.
                           0: always per-pole solves                         */
  int32_t keep_solutions; /* 1: every step keeps the pole solutions x_j of
                           its last step, readable with rexi_get_solution.
                           The per-pole solver keeps them anyway; the
                           shared-basis solver (finite differences) then
                           forms them on every step (sum_i K_i n_i complex128
                           values planned at setup; without this option they
                           are planned when they take at most half of the
                           free memory and formed only on steps with info).
                           Default 0                                          */
  int32_t capture_pauses; /* capture_safe, shared basis with the tiled pass:
                           second Gram-Schmidt passes per cycle the captured
                           schedule makes room for (each takes up to 31
                           launches of it for a single instance, 15 for a
                           batch); 0 (default): 1 for a single instance,
                           max(2, m / 32) for a batch (whose instances all
                           pause when one needs a pass). A cycle whose
                           pauses take more launches than that room stops
                           below m vectors                                 */
  int32_t reserved_opt2_;
} rexi_options;

typedef struct {
  int32_t K;                /* poles (summed over instances for a batch)      */
  int32_t steps;            /* steps taken by the call                         */
  int64_t total_iterations; /* Arnoldi iterations over all poles and steps     */
  int32_t max_cycles_used;  /* largest cycle count of one pole solve           */
  int32_t not_converged;    /* pole solves that missed their target            */
  double max_rel_residual;  /* max_j ||psi - (H - s_j) x_j|| / ||psi|| (last step) */
  double certified_bound;   /* sum_j |w_j| ||r_j|| / dist(s_j, [lmin, lmax]) / ||psi||,
                               a bound on the relative step error (last step;
                               for a batch the largest over its instances,
                               each relative to its own ||psi||)              */
  int32_t reorth_passes;    /* shared-basis Lanczos: second Gram-Schmidt passes
                               of the last step (single instance)             */
  int32_t explicit_residuals; /* 1: max_rel_residual, rel_residual and
                               certified_bound come from explicit FP64
                               residuals psi - (H - s_j) x_j of the computed
                               x_j (per-pole solver: always; shared basis:
                               finite differences, solutions planned); 0: from
                               the implicit (Givens) residual estimates       */
  double norm_in;           /* ||psi_n||_2 of the last step's whole input      */
  double norm_out;          /* ||psi_{n+1}||_2 of the last step's whole output */
  /* optional caller-owned per-pole arrays of length K (NULL to skip):        */
  int32_t* iterations;      /* Arnoldi iterations of pole j (last step)        */
  int32_t* cycles;          /* cycles of pole j (last step)                    */
  double* rel_residual;     /* final relative residual of pole j (last step),
                               relative to ||psi|| of the pole's instance    */
  double* implicit_residual;/* the solver's implicit residual estimate of pole
                               j (per-pole solver: the explicit one)          */
} rexi_step_info;

typedef struct {
  /* accumulated while rexi_options.profile = 1, reset by rexi_profile_reset */
  int32_t nclasses;
  const char* names[12];
  int64_t launches[12];
  double ms[12];            /* summed kernel time, HIP events on the stream   */
  double bytes[12];         /* algorithmic HBM bytes of those launches        */
} rexi_profile;

typedef struct rexi_handle rexi_handle;

/* Fill *opt with the defaults listed above. */
void rexi_default_options(rexi_options* opt);

/*
 * rexi_setup -- prepare REXI steps for one grid (eq. rational-evaluation).
 *   g          grid (ndim 1..3, n[a] >= 1, lo < hi)
 *   V_dev      device float64[prod n], the potential at the interior points
 *   hbar, mass > 0; dt != 0 (finite): the step size tau
 *   K >= 1     poles; sigma_host, beta_host: host rexi_c128[K], the
 *              dimensionless poles and weights of r(z) ~ exp(z)
 *   opt        NULL for defaults
 *   stream     hipStream_t used for the setup copies
 * Maps (sigma, beta) to s_j = i hbar sigma_j / dt, w_j = i hbar beta_j / dt in
 * FP64 and plans the workspaces. Fails with REXI_E_INVALID_ARG on bad sizes,
 * non-finite sigma, beta or V, or a shift on the real segment spanned by the
 * spectrum bound [min V, (hbar^2/2m) sum_a 4/h_a^2 + max V] (a singular
 * system); REXI_E_NO_MEMORY if the workspace does not fit.
 */
rexi_status rexi_setup(rexi_handle** out, const rexi_grid* g, const double* V_dev,
                       double hbar, double mass, double dt, int32_t K,
                       const rexi_c128* sigma_host, const rexi_c128* beta_host,
                       const rexi_options* opt, void* stream);

/*
 * rexi_setup_batch -- count independent instances of uneven sizes in one handle.
 *   grids[i], hbar[i], mass[i], dt[i], K[i] as for rexi_setup;
 *   V_dev      device float64[sum_i prod n_i], the potentials packed in
 *              instance order
 *   sigma_host, beta_host  host rexi_c128[sum_i K_i], packed in instance order
 * All poles of all instances are solved together (one work queue over
 * instance, pole and tile).
 */
rexi_status rexi_setup_batch(rexi_handle** out, int32_t count, const rexi_grid* grids,
                             const double* V_dev, const double* hbar, const double* mass,
                             const double* dt, const int32_t* K,
                             const rexi_c128* sigma_host, const rexi_c128* beta_host,
                             const rexi_options* opt, void* stream);

/*
 * rexi_apply_H -- y = (H - shift I) x in FP64 (the stencil matvec of the
 * solves); with Q1 elements y = (A - shift M) x. x_dev, y_dev: device
 * rexi_c128[prod n] (no aliasing). For a batch handle, the packed vectors of
 * all instances.
 */
rexi_status rexi_apply_H(rexi_handle* h, const rexi_c128* x_dev, rexi_c128* y_dev,
                         rexi_c128 shift, void* stream);

/*
 * rexi_estimate_spectrum -- estimates of the extreme eigenvalues of H per
 * instance, for the step-size condition (Section "Step-Size Requirements",
 * eq. convergence-condition: the REXI step needs tau sr(M) <= R1, where
 * sr(M) = max |lambda(H)| / hbar; the paper notes that a few iterations of a
 * sparse eigensolver give the rough estimate it needs, once per problem).
 *   iters    Lanczos iterations, 1..256 (fewer on an instance whose Krylov
 *            space becomes invariant first, e.g. one with <= iters points)
 *   lo_host, hi_host  host double[instances]: the smallest and largest Ritz
 *            values of H (finite differences, without centering). They lie
 *            inside [lambda_min, lambda_max] and approach its ends as iters
 *            grows; exact once the Krylov space is the whole space.
 * Lanczos with full re-orthogonalisation (two Gram-Schmidt passes) in FP64
 * from a fixed pseudo-random real start vector, on the device; the
 * tridiagonal eigenvalues by Sturm bisection on the host. Allocates and
 * frees (iters + 1) vectors of the handle's size on the device; the call
 * synchronises the stream. REXI_E_INVALID_ARG for a Q1-element handle (its
 * operator is the pencil (A, M)) or iters out of range, REXI_E_NO_MEMORY when
 * the vectors do not fit.
 */
rexi_status rexi_estimate_spectrum(rexi_handle* h, int32_t iters, double* lo_host, double* hi_host,
                                   void* stream);

/*
 * rexi_estimate_spectrum_noalloc -- rexi_estimate_spectrum without any device
 * allocation, for callers that cannot allocate (tight serving loops,
 * harnesses that forbid hipMalloc). Same arguments, the same kernels in the
 * same order and the same results. Its workspace is a fixed 256 MiB device
 * array of the library, one per GPU, held from the library's first use on
 * that GPU until the process ends; it needs
 *   (iters + 2) * N * 16 + (iters + 1) * (8 * tiles + 8 * instances)
 * bytes (N the handle's points, each part rounded up to 256 bytes), and a
 * larger request fails with REXI_E_INVALID_ARG before anything runs. Every
 * workspace buffer is written before it is read within a call, so nothing
 * left by an earlier call is used. All calls on one GPU share the array:
 * calls that overlap in time on one GPU (other threads, other streams of
 * the process) race and must be serialised by the caller.
 */
rexi_status rexi_estimate_spectrum_noalloc(rexi_handle* h, int32_t iters, double* lo_host, double* hi_host,
                                           void* stream);

/*
 * rexi_step -- nsteps >= 1 REXI steps psi_out = r(tau M)^nsteps psi_in
 * (eq. rational-evaluation). psi_in_dev, psi_out_dev: device rexi_c128[prod n]
 * (packed over instances for a batch); psi_out may equal psi_in. info may be
 * NULL. Returns REXI_E_NOT_CONVERGED if a pole missed its target after
 * max_cycles (the best iterate is used and info is filled).
 */
rexi_status rexi_step(rexi_handle* h, const rexi_c128* psi_in_dev, rexi_c128* psi_out_dev,
                      int32_t nsteps, rexi_step_info* info, void* stream);

/*
 * rexi_step_adjoint -- one backward step of a real loss L through
 * psi_{n+1} = R psi_n, R = sum_j w_j (H - s_j)^{-1}. With the
 * conjugate-Wirtinger gradients gbar = dL/d conj(psi):
 *   gbar_n   = R^H gbar_{n+1} = sum_j conj(w_j) (H - conj(s_j))^{-1} gbar_{n+1}
 *   dV_accum += dL/dV = -2 Re sum_j w_j conj(y_j) x_j   (elementwise)
 * with x_j = (H - s_j)^{-1} psi_n and y_j = (H - conj s_j)^{-1} gbar_{n+1}
 * (H is real symmetric, so (H - s)^H = H - conj s). psi_n_dev, gbar_next_dev,
 * gbar_n_dev: device rexi_c128[prod n]; gbar_n may alias gbar_next.
 * dV_accum_dev: device float64[prod n] or NULL. Single-instance handles with
 * finite differences only.
 */
rexi_status rexi_step_adjoint(rexi_handle* h, const rexi_c128* psi_n_dev,
                              const rexi_c128* gbar_next_dev, rexi_c128* gbar_n_dev,
                              double* dV_accum_dev, void* stream);

/*
 * rexi_get_solution -- copy the solution x_j = (H - s_j)^{-1} psi_n of pole j
 * (0 <= j < K, poles numbered over the instances in order) of the last step
 * into x_dev (device rexi_c128[n of the pole's instance]). These are the
 * terms of eq. rational-evaluation before the weighted sum (psi_{n+1} =
 * sum_j w_j x_j). Per-pole handles keep them after every step; shared-basis
 * handles need keep_solutions = 1. REXI_E_INVALID_ARG when none are kept or
 * no step has run. Asynchronous on stream.
 */
rexi_status rexi_get_solution(rexi_handle* h, int32_t pole, rexi_c128* x_dev, void* stream);

/* Kernel-class timings gathered while opt.profile = 1. */
rexi_status rexi_get_profile(const rexi_handle* h, rexi_profile* out);
rexi_status rexi_profile_reset(rexi_handle* h);

/* Device bytes held by the handle's workspaces, and the restart length used. */
rexi_status rexi_workspace_info(const rexi_handle* h, int64_t* bytes, int32_t* m_used);

typedef struct {
  int32_t tile;          /* points per work tile of the grid-stride passes    */
  int32_t grid_blocks;   /* workgroups of the grid-stride passes              */
  int32_t march_slots;   /* fused Lanczos pass: 0 row-staged, 2 tiled, else
                            points per thread and plane of the marching pass */
  int32_t march_planes;  /* planes per marching work item (0: row-staged)     */
  int32_t march_items;   /* marching work items over all instances            */
  int32_t reserved_;
} rexi_tiling;

/* The tiling in use (chosen by the tuner or given in the options). Fills
 * *out; REXI_E_INVALID_ARG for a NULL argument. */
rexi_status rexi_tiling_info(const rexi_handle* h, rexi_tiling* out);

/* Release the handle and its workspaces (NULL is a no-op). */
rexi_status rexi_destroy(rexi_handle* h);

/* Text of a status code (static storage). */
const char* rexi_status_string(rexi_status s);

/* Copy the last error message of h (or of the failed setup when h == NULL)
 * into buf (NUL-terminated, truncated to len). */
rexi_status rexi_last_error(const rexi_handle* h, char* buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* REXI_H */
