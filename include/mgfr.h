/*
 * mgfr.h -- C ABI of the MI355X f(R) field solver.
 *
 * The library computes, on one AMD Instinct MI355X (gfx950), the per-step
 * solve of the Hu-Sawicki f(R) scalar field of Puchwein, Baldi & Springel
 * (2013), "Modified Gravity-GADGET":
 *
 *   1. cloud-in-cell mass assignment of particles onto a periodic mesh
 *      (Sec. 3.1);
 *   2. the non-linear field equation for u = ln(f_R / fbar_R) (Sec. 3.2,
 *      Eqs. fR_u, u_field_eq, u_discrete_field_eq) solved by FAS multigrid
 *      V-cycles with red-black Newton-Gauss-Seidel smoothing (Sec. 3.3,
 *      Eq. iterative_correction, Eq. fine_correction, steps 1-8);
 *   3. the fifth force a_MG = (c^2/2) grad f_R (Sec. 2, Eq. modgrav_accel)
 *      interpolated back to the particles.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every array argument is a DEVICE pointer owned by the caller; the
 *   library never frees or keeps it beyond the call.  Work is enqueued on
 *   the HIP stream given to mgfr_create (a hipStream_t passed as void*;
 *   NULL = the legacy default stream).  Calls return when their results are
 *   ready on that stream (mgfr_solve synchronises once per V-cycle to test
 *   convergence; the other calls do not synchronise).
 * - Meshes are N^3 float64 arrays in C order: index (i*N + j)*N + k with i
 *   along x, k along z (fastest).  Cell (i,j,k) covers [ih,(i+1)h) x ... with
 *   h = box/N, centre ((i+1/2)h, ...).  Boundaries are periodic.
 * - Positions are float32 [np][3] comoving Mpc/h; any real value is wrapped
 *   into the box.
 * - The library owns only its context workspace (level hierarchy, scratch),
 *   allocated in mgfr_create and freed in mgfr_destroy.  mgfr_solve,
 *   mgfr_assign_density and mgfr_fifth_force allocate nothing.
 * - Return codes: 0 OK, 1 not converged (outputs valid), negative = error;
 *   on error the message is available from mgfr_last_error() (thread-local)
 *   and caller buffers may have been partly written only where stated.
 * - One context must not be used from two host threads at once.
 */
#ifndef MGFR_H
#define MGFR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGFR_OK 0
#define MGFR_NOT_CONVERGED 1
#define MGFR_ERR_ARG (-1)       /* invalid argument (message says which) */
#define MGFR_ERR_HIP (-2)       /* a HIP runtime call failed */
#define MGFR_ERR_NONFINITE (-3) /* NaN/Inf in an input or in the iteration */
#define MGFR_ERR_OOM (-4)       /* device allocation failed */

#define MGFR_PROLONG_LINEAR 0 /* parent value + central-difference gradient (Sec. 3.3) */
#define MGFR_PROLONG_INJECT 1 /* straight injection (Sec. 3.3) */

#define MGFR_FP64 0  /* every level and sweep in float64 */
#define MGFR_MIXED 1 /* float32 correction V-cycles inside a float64 defect-correction loop */

#define MGFR_NN_NONE 0   /* initial guess = the u passed in */
#define MGFR_NN_COARSE 1 /* initial guess from the learned network at the N/4 level, corrected
                            on the coarse levels (mgfr_params.coarse_cycles) */

#define MGFR_MAX_HIST 256

/* Problem and solver parameters (Sec. 2 model, Sec. 3.3 solver). */
typedef struct mgfr_params {
    double box;      /* comoving box side L in Mpc/h, > 0 */
    double a;        /* scale factor, > 0 */
    double omega_m;  /* matter density parameter, > 0 */
    double omega_l;  /* vacuum density parameter, >= 0 */
    double fr0_abs;  /* |fbar_R0| > 0 (the paper's fbar_R0 is negative) */
    int n;           /* Hu-Sawicki exponent n >= 1 (the paper runs n = 1) */
    int mesh;        /* N: cells per side, a power of two, 8 <= N <= 1024 (the 1024^3 solve needs ~60 GB) */
    int refine_levels; /* refinement levels above the base mesh (Sec. 3.3): 0 for mgfr_create
                          (uniform mesh), 1 or 2 for mgfr_amr_create */
    double tol;      /* accept when max|f - L(u)| / D <= tol, D = max|f| (Sec. 3.3 step 8); > 0 */
    int pre_smooth;  /* red-black sweeps before restriction, >= 0 */
    int post_smooth; /* red-black sweeps after the correction, >= 0 */
    int coarse_sweeps; /* sweeps on the coarsest grid (the 4^3 level; on refined levels of the
                          adaptive solver, their one-cell-per-block sublevel), >= 1 */
    int max_vcycles; /* V-cycle limit, >= 0 */
    int prolong;     /* MGFR_PROLONG_LINEAR or MGFR_PROLONG_INJECT */
    int precision;   /* MGFR_FP64 or MGFR_MIXED */
    int nn_mode;     /* MGFR_NN_NONE or MGFR_NN_COARSE */
    double max_du;   /* limit on |Newton step| per cell update; <= 0 disables the limit */
    int coarse_cycles; /* MGFR_NN_COARSE only: V-cycles of the N/4 problem (from the network's
                          prediction) and then of the N/2 problem (from the prolonged N/4 solution)
                          before the prolonged N/2 solution starts the solve at N; 0 = prolong the
                          prediction directly.  >= 0 */
} mgfr_params;

/* Per-solve report. */
typedef struct mgfr_stats {
    int status;       /* the return code of the solve */
    int vcycles;      /* V-cycles run (FP64) or inner V-cycles (mixed) */
    int outer_iters;  /* float64 defect-correction iterations (mixed), else = vcycles */
    int fell_back;    /* 1 if the mixed/learned solve restarted as plain FP64 from u = 0 */
    double res0;      /* relative max residual of the initial guess */
    double res;       /* relative max residual of the returned u */
    double scale;     /* D, the residual normalisation */
    double l2res;     /* relative rms residual of the returned u */
    double res_hist[MGFR_MAX_HIST]; /* relative max residual after each (outer) cycle */
    double t_solve_ms;   /* device time of the solve between two HIP events */
    double t_sweep_ms;   /* summed HIP-event time of finest-level smoothing launches (timing on) */
    int n_sweep_launches; /* number of launches in t_sweep_ms */
    double t_nn_ms;      /* HIP-event time of the network warm start, if any */
    int smooth_used;     /* pre-smoothing sweeps of the last cycle (mgfr_set_adaptive_smoothing may raise them) */
} mgfr_stats;

typedef struct mgfr_ctx mgfr_ctx;

/* Background quantities of Sec. 2 for these parameters: |fbar_R(a)|,
 * beta = a^2 (H0/c)^2 / |fbar_R(a)| in (h/Mpc)^2 and C = Omega_m a^-3 + 4 Omega_L.
 * Host only; returns MGFR_ERR_ARG on invalid parameters. */
int mgfr_background(const mgfr_params *p, double *fbar, double *beta, double *C);

/* Validate p and allocate the level hierarchy for an N^3 mesh on the current
 * HIP device.  stream: hipStream_t as void* (NULL = default stream).
 * Errors: MGFR_ERR_ARG, MGFR_ERR_OOM, MGFR_ERR_HIP; *out is NULL on error. */
int mgfr_create(const mgfr_params *p, void *stream, mgfr_ctx **out);

/* Free the context (NULL is allowed). */
void mgfr_destroy(mgfr_ctx *ctx);

/* Change the stream later calls enqueue on. */
int mgfr_set_stream(mgfr_ctx *ctx, void *stream);

/* Turn per-launch HIP-event timing of the finest-level smoothing kernel on
 * or off (reported in mgfr_stats.t_sweep_ms). */
int mgfr_set_timing(mgfr_ctx *ctx, int on);

/* Float64 sweeps: smallest level size N at which a red-black sweep runs as
 * one fused, out-of-place kernel (both colours per launch, LDS-staged tiles);
 * smaller levels use one in-place kernel per colour.  Default 512; 0 = never;
 * otherwise n >= 64.  Results agree to rounding either way. */
int mgfr_set_fused_min_mesh(mgfr_ctx *ctx, int n);

/* Float32 correction sweeps of the mixed-precision solve: smallest level size
 * N at which each colour runs as the plane-marching pass kernel (row tiles of
 * cell pairs staged in LDS, exponentials evaluated once per cell); smaller
 * levels use the plain one-thread-per-cell kernel.  Default 128; 0 = never;
 * otherwise n >= 128.  Both apply the same update in the same red-black
 * order; results agree to float32 rounding. */
int mgfr_set_colour_min_mesh(mgfr_ctx *ctx, int n);

/* Float32 correction sweeps on the levels that use the pass kernels (see
 * mgfr_set_colour_min_mesh): on = 1 runs each red-black sweep (Sec. 3.3) as
 * one fused, out-of-place kernel that updates the red cells of plane i + 1
 * and then the black cells of plane i while marching over the planes, so
 * that e, u and r are read once per sweep instead of once per colour; on = 0
 * (default) runs one pass kernel per colour.  The same updates in the same
 * red-black order; results agree to float32 rounding.  The second correction
 * buffer is allocated by mgfr_create for mixed-precision contexts, so this
 * call allocates nothing.  Errors: MGFR_ERR_ARG for on not 0 or 1. */
int mgfr_set_fused_sweep32(mgfr_ctx *ctx, int on);

/* Relaxation factor omega of the float32 correction sweeps of the
 * mixed-precision solve: each Newton-Gauss-Seidel update (Sec. 3.3, Eq.
 * iterative_correction) is scaled by omega (1: the paper's plain update;
 * 1 < omega < 2: over-relaxation).  The float64 outer loop judges
 * convergence, so the answer does not depend on omega, only the number of
 * V-cycles.  Once the float64 residual grows during a solve, the remaining
 * cycles of that solve use omega = 1.  Default 1.  The float64 solve always
 * uses 1 (refined levels: mgfr_amr_set_relaxation32).  Errors: MGFR_ERR_ARG
 * unless 0 < omega < 2. */
int mgfr_set_relaxation32(mgfr_ctx *ctx, double omega);

/* Float32 correction V-cycles per float64 residual check of the mixed
 * solve, at most max_inner (1..4; default 1, one cycle per check).  With
 * max_inner > 1 the solve runs that many cycles between checks while the
 * residual, reduced at the rate the last check measured, would still be
 * above tol after one more cycle; near the tolerance it checks after every
 * cycle again.  Each cycle is a whole FAS V-cycle of the correction equation,
 * so only the float64 residual passes are skipped; stats.vcycles counts the
 * correction cycles, stats.outer_iters and res_hist the checks.
 * Errors: MGFR_ERR_ARG for max_inner outside [1, 4]. */
int mgfr_set_inner_cycles(mgfr_ctx *ctx, int max_inner);

/* Adaptive smoothing for stalling solves (FP64 and mixed): when a residual
 * check is not below the one two checks earlier, the pre- and post-smoothing
 * sweeps of the following cycles double, up to max_sweeps; each solve starts
 * again from the parameters' counts.  0 (default) keeps the fixed V(pre,post)
 * cycle of the paper.  Meant for deep screened cores at large |f_R0|, where
 * red-black Newton sweeps can leave neighbouring cells alternating between
 * the screened and the unscreened branch and a fixed V(4,4) cycle stalls.
 * The answer is judged by the same residual.  stats.smooth_used reports the
 * count in use at the end.  Errors: MGFR_ERR_ARG unless max_sweeps is 0 or
 * between max(pre_smooth, post_smooth) and 32. */
int mgfr_set_adaptive_smoothing(mgfr_ctx *ctx, int max_sweeps);

/* Cloud-in-cell assignment (Sec. 3.1) of np particles onto the N^3 mesh and
 * delta = m / m_bar - 1 with m_bar the mean cell mass of the assignment.
 * pos: float32 [np][3]; mass: float64 [np] or NULL for equal masses;
 * delta: float64 [N^3] output.  np >= 1.  Non-finite positions give
 * MGFR_ERR_NONFINITE (delta then holds unspecified values). */
int mgfr_assign_density(mgfr_ctx *ctx, const float *pos, const double *mass, int64_t np,
                        double *delta);

/* Allocation-free variant of mgfr_assign_density, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It needs no context: mesh (a power of two,
 * 8 <= mesh <= 1024) and box (> 0, Mpc/h) describe the periodic N^3 mesh, and
 * the work is enqueued on `stream` (a hipStream_t as void*, NULL = default).
 * pos, mass, np and delta as for mgfr_assign_density; particles are visited in
 * index order (no binning).  delta (caller-owned, float64 [N^3]) first holds
 * the cell masses and is then normalised in place.  The library allocates
 * nothing: the reduction workspace (2048 partial sums, the total mass and the
 * non-finite flag; 16.4 KB) is a fixed array in device memory, one per GPU,
 * held until the process ends and reset by every call.  Calls that overlap on
 * one GPU (two host threads, or two streams in flight) race on that array and
 * must be serialised by the caller.  The call synchronises `stream` once to
 * read the total mass and the flag.
 * Errors: MGFR_ERR_ARG (NULL pointers, np < 1, mesh not a power of two in
 * [8, 1024], box), MGFR_ERR_NONFINITE (non-finite position or mass, or a
 * total mass that is not positive), MGFR_ERR_HIP. */
int mgfr_assign_density_noalloc(int mesh, double box, void *stream, const float *pos, const double *mass,
                                int64_t np, double *delta);

/* Workspace for particle binning (Sec. 3.1 assignment, Sec. 2 force): three
 * uint32 arrays of max_np entries, the per-tile counts and first slots, a
 * list of work units and a scan's scratch, owned by the context, freed by
 * mgfr_destroy or by a later call with a larger max_np (which synchronizes
 * the stream first).  With it, mgfr_assign_density for np <= max_np orders
 * the particle indices by the 8^3-cell tile of their lower CIC corner (a
 * counting sort; the order within a tile may differ between calls),
 * accumulates each tile's particles in on-chip memory and adds the 9^3
 * window to the mesh; mgfr_fifth_force for the same np then visits the
 * particles in that order (any order gives the same forces; only the speed
 * depends on it).  Without it (or for larger np) both work in particle index
 * order.  max_np <= 2^31 - 1; MGFR_ERR_OOM if the allocation fails. */
int mgfr_reserve_particles(mgfr_ctx *ctx, int64_t max_np);

/* 1 (default): use the binning workspace when it is large enough; 0: never. */
int mgfr_set_binning(mgfr_ctx *ctx, int on);

/* Initial guess for mgfr_solve from the screened limit of the field
 * equation (Sec. 2, Eqs. fR_field_eq and dR_fR): where the Laplacian of f_R
 * is negligible the equation reduces to the local balance
 * dR = 8 pi G d rho, i.e. exp(-u/(n+1)) = 1 + Omega_m a^-3 delta / C(a).
 * Overdense cells get that u, the others u = 0:
 *   u = -(n+1) log1p(Omega_m a^-3 max(delta, 0) / C(a)).
 * It is exact for a constant overdensity and close to the solution in
 * screened cores; the solve still iterates to the same tolerance, so only
 * the number of V-cycles depends on it.
 * delta: float64 [N^3] input; u: float64 [N^3] output (may not alias delta).
 * Enqueued on the context's stream; MGFR_ERR_ARG for NULL pointers. */
int mgfr_screened_guess(mgfr_ctx *ctx, const double *delta, double *u);

/* Effective mass density of the effective-mass formulation (Sec. 3.4, Eq.
 * effective_density), in units of the mean matter density:
 *   delta_eff = delta/3 - dR / (24 pi G rho_bar)
 *             = delta/3 - C(a) expm1(-u/(n+1)) / (3 Omega_m a^-3),
 * with dR from Eq. dR_fR.  It is delta/3 where the field is unscreened and
 * tends to 0 in screened regions; for a converged u it equals the flux term
 * of the field equation divided by 3 beta Omega_m a^-3.
 * delta, u: float64 [N^3] inputs; out: float64 [N^3] output (may alias
 * neither input).  Enqueued on the context's stream; MGFR_ERR_ARG for NULL
 * pointers. */
int mgfr_effective_density(mgfr_ctx *ctx, const double *delta, const double *u, double *out);

/* Power-spectrum diagnostic of the effective mass (Sec. 3.4; the paper's
 * power-spectrum comparison, Sec. 5): the ratio of the power spectrum of
 * delta + delta_eff to that of delta in shells of |k| ((4/3)^2 where the
 * fifth force is unscreened, 1 where it is screened).
 * P(k_i) = L^3/N^6 * mean over the modes of shell i of |DFT(f)|^2, shell i =
 * the integer wave vectors n with i - 1/2 <= |n| < i + 1/2, k_i = 2 pi i / L.
 * delta, delta_eff: float64 [N^3] device inputs; nbins in [1, N/2];
 * k, ratio: float64 [nbins] host outputs; p_delta (P of delta) and counts
 * (modes per shell): float64 [nbins] host outputs or NULL.  A diagnostic, not
 * part of the per-step path: it allocates a workspace (three N^3 float64
 * arrays) and an FFT plan (hipFFT) for the call, synchronizes the stream and
 * frees them.  Errors: MGFR_ERR_ARG (NULL, nbins), MGFR_ERR_OOM, MGFR_ERR_HIP. */
int mgfr_power_ratio(mgfr_ctx *ctx, const double *delta, const double *delta_eff, int nbins, double *k,
                     double *ratio, double *p_delta, double *counts);

/* Solve L(u) = f for u (Sec. 3.2 Eq. u_discrete_field_eq; Sec. 3.3).
 * delta: float64 [N^3] density contrast (input, unchanged);
 * u: float64 [N^3], in: initial guess (zeros = the background, or the
 *    previous step's solution, Sec. 3.3 step 2), out: the solution;
 * dfr: float64 [N^3] or NULL, out: delta f_R = fbar_R (e^u - 1);
 * st: may be NULL.
 * Returns MGFR_OK when the relative max residual is <= tol,
 * MGFR_NOT_CONVERGED after max_vcycles (u, dfr valid), MGFR_ERR_NONFINITE
 * if delta or the iteration is not finite. */
int mgfr_solve(mgfr_ctx *ctx, const double *delta, double *u, double *dfr, mgfr_stats *st);

/* Fifth force a_MG = c^2/(2a) grad_x f_R (Sec. 2, Eq. modgrav_accel; c in
 * km/s, x comoving Mpc/h, so acc is in (km/s)^2 h/Mpc), with f_R = fbar_R e^u,
 * the gradient a two-point central difference at cell centres, interpolated
 * to the particles with cloud-in-cell weights.
 * u: float64 [N^3]; pos: float32 [np][3]; acc: float32 [np][3] output. */
int mgfr_fifth_force(mgfr_ctx *ctx, const double *u, const float *pos, int64_t np, float *acc);

/* Chained time steps (the paper's solve is one per time step and starts from
 * the previous step's u, Sec. 3.3 step 2).  These calls carry a particle-mesh
 * step around the solve; the Newtonian part is the standard PM force, not a
 * step of the paper's method.
 *
 * mgfr_set_scale_factor: change a (the background of Sec. 2 is recomputed on
 * the host; nothing is reallocated).  MGFR_ERR_ARG unless a > 0.
 *
 * mgfr_pm_accel: peculiar acceleration of the particles, acc = -(1/a) grad_x Psi
 * with Psi = phi + (c^2/2) fbar e^u, where lap_x phi = (3/2) Omega_m H0^2 delta / a
 * (H0 = 100 km/s per Mpc/h) is solved by FFT with the eigenvalues of the
 * periodic 7-point Laplacian (zero mean), and the second term is the fifth
 * force of mgfr_fifth_force (Sec. 2, Eq. modgrav_accel); u == NULL gives the
 * Newtonian acceleration alone.  Same gradient and cloud-in-cell gather as
 * mgfr_fifth_force; units (km/s)^2 h/Mpc.  delta, u: float64 [N^3]; pos,
 * acc: float32 [np][3].  The first call makes two FFT plans and an
 * N^2 (N/2+1) complex workspace, kept by the context.
 *
 * mgfr_kick_drift: mom += acc kick, then pos += mom drift, every component in
 * float64 as fused multiply-adds from the float32 values and stored as float32;
 * positions wrapped into [0, box).  acc may be NULL (drift only); pos, mom,
 * acc float32 [np][3], in place.  With p = a^2 dx/dt the equations of motion
 * are dp/da = g / H(a) and dx/da = p / (a^3 H(a)); the caller chooses the
 * kick and drift integrals of a step. */
int mgfr_set_scale_factor(mgfr_ctx *ctx, double a);
int mgfr_pm_accel(mgfr_ctx *ctx, const double *delta, const double *u, const float *pos, int64_t np, float *acc);
int mgfr_kick_drift(mgfr_ctx *ctx, float *pos, float *mom, const float *acc, int64_t np, double kick, double drift);

/* One kick-drift-kick step from the context's a = a0 to a1 > a0 with the
 * midpoint rule, am = (a0 + a1)/2, H(a) = 100 sqrt(Omega_m a^-3 + Omega_L):
 *   mom += acc (am - a0) / H((a0 + am)/2);  pos += mom (a1 - a0) / (am^3 H(am));
 *   a = a1; delta = assignment of pos; u = solve from the u passed in (the
 *   previous step's solution, Sec. 3.3 step 2); acc = mgfr_pm_accel(delta, u, pos);
 *   mom += acc (a1 - am) / H((am + a1)/2).
 * pos, mom, acc: float32 [np][3] in/out (acc in: the acceleration at a0);
 * delta: float64 [N^3] output; u: float64 [N^3] in/out; st: the solve's stats.
 * Returns the solve's status (MGFR_NOT_CONVERGED keeps going) or an error. */
int mgfr_pm_step(mgfr_ctx *ctx, float *pos, float *mom, float *acc, int64_t np, double a1, double *delta, double *u,
                 mgfr_stats *st);

/* Per-step entry points (Sec. 3.3), used to check single steps.
 * mgfr_ngs_sweep: `sweeps` red-black sweeps on the finest level, u updated
 * in place, f = the source of L(u) = f.  mgfr_vcycle: one V-cycle on u with
 * source f.  mgfr_residual: r = f - L(u) on the finest level. */
int mgfr_ngs_sweep(mgfr_ctx *ctx, double *u, const double *f, int sweeps);
int mgfr_vcycle(mgfr_ctx *ctx, double *u, const double *f);
int mgfr_residual(mgfr_ctx *ctx, const double *u, const double *f, double *r);

/* ---------------------------------------------------------------------
 * Learned warm start (not part of the paper's method).  A 3-level 3D U-Net
 * (16/32/64 channels, 3^3 periodic convolutions, bfloat16 weights and
 * activations, float32 accumulation) maps delta on a periodic S^3 mesh, with
 * the scale factor and |f_R0| as constant input channels, to u on that mesh.
 * With nn_mode = MGFR_NN_COARSE, mgfr_solve restricts delta to the N/4 mesh
 * (means of 4^3 cells), predicts u there, prolongs it twice with the linear
 * reconstruction of Sec. 3.3 and uses the result as the initial guess; the
 * multigrid iteration then runs to the same tolerance as without it.
 * The network object owns its weights, Adam moments and activation
 * workspace (allocated in mgfr_net_create); the solver context only borrows
 * it.  Arrays are device pointers unless stated; bf16 tensors are
 * channels-last [B][S][S][S][C] with voxel index ((b S + z) S + y) S + x.
 * --------------------------------------------------------------------- */
typedef struct mgfr_net mgfr_net;

/* He-normal weights from `seed`, zero biases; workspace for up to
 * max_voxels = B * S^3 voxels per call (a multiple of 4096). */
int mgfr_net_create(int seed, int64_t max_voxels, void *stream, mgfr_net **out);
void mgfr_net_destroy(mgfr_net *net);
int mgfr_net_set_stream(mgfr_net *net, void *stream);
/* Number of float32 parameters (conv weights [27][Cout][Cin] then biases, layer by layer, then the head). */
int64_t mgfr_net_num_params(const mgfr_net *net);
/* Copy the float32 master parameters to / from a HOST buffer of mgfr_net_num_params floats;
 * set_params also resets the Adam state. */
int mgfr_net_get_params(mgfr_net *net, float *host);
int mgfr_net_set_params(mgfr_net *net, const float *host);
/* Checkpoint to / restore from a file: the master parameters, the Adam moments
 * and step count, after a header naming the layer shapes.  load rejects a file
 * of another layout (MGFR_ERR_ARG) and leaves the network unchanged then. */
int mgfr_net_save(mgfr_net *net, const char *path);
int mgfr_net_load(mgfr_net *net, const char *path);
/* u = network(delta) for B volumes of side S (power of two, 32 <= S <= 1024).
 * delta, u: float64 [B][S^3]; cond: HOST float64 [B][2] = (a, |f_R0|) per volume. */
int mgfr_net_predict(mgfr_net *net, const double *delta, int B, int S, const double *cond, double *u);
/* Copy one intermediate tensor of the last forward pass (predict, train_step
 * or grads) into the DEVICE buffer dst of exactly `count` elements, on the
 * network's stream, synchronised before return.  index, in forward order
 * (channels; side for an input of side S):
 *    0 features x0 (16; S)        1 conv1a (16; S)    2 conv1b = skip 1 (16; S)
 *    3 pool (16; S/2)             4 conv2a (32; S/2)  5 conv2b = skip 2 (32; S/2)
 *    6 pool (32; S/4)             7 conv3a (64; S/4)  8 conv3b (64; S/4)
 *    9 up + skip 2 (96; S/2)     10 conv4a (32; S/2) 11 conv4b (32; S/2)
 *   12 up + skip 1 (48; S)       13 conv5a (16; S)   14 conv5b (16; S)
 *   15 head output y = u / 5 (float32 [B][S^3]).
 * Indices 0-14 are bf16 channels-last tensors.  MGFR_ERR_ARG for an index out
 * of range, a count that is not the tensor's size, or no forward pass yet. */
int mgfr_net_activation(mgfr_net *net, int index, void *dst, int64_t count);
/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the mean squared error
 * between the network output and u_target / 5; *loss (host, nullable) gets the loss
 * before the step.  Returns MGFR_ERR_NONFINITE if the loss is not finite. */
int mgfr_net_train_step(mgfr_net *net, const double *delta, const double *u_target, int B, int S,
                        const double *cond, float lr, float *loss);
/* Loss and its gradient with respect to every parameter (HOST float32 [num_params]),
 * without updating the weights. */
int mgfr_net_grads(mgfr_net *net, const double *delta, const double *u_target, int B, int S,
                   const double *cond, float *loss, float *grad_host);
/* Attach (or detach with NULL) the network used by nn_mode = MGFR_NN_COARSE.
 * A network the context created with mgfr_nn_init is destroyed first. */
int mgfr_set_net(mgfr_ctx *ctx, mgfr_net *net);

/* The same network owned by the context (the ctx-level calls of the
 * boundary).  mgfr_nn_init creates it (He-normal weights from seed, capacity
 * max((N/4)^3, 8 * 64^3) voxels), attaches it for nn_mode = MGFR_NN_COARSE
 * and replaces any attached network; mgfr_destroy destroys it.  The others
 * act on the attached network (either kind) on the context's stream, with
 * the arguments of the mgfr_net_* call of the same name.  mgfr_nn_predict
 * writes to u0 (device float64 [N^3]) the initial guess a solve with
 * nn_mode = MGFR_NN_COARSE starts from when coarse_cycles = 0: delta
 * restricted to N/4 by 4^3 means, the network's u there, prolonged twice
 * (Sec. 3.3 reconstruction); it needs N >= 128.  MGFR_ERR_ARG without a
 * network. */
int mgfr_nn_init(mgfr_ctx *ctx, int seed);
int mgfr_nn_train_step(mgfr_ctx *ctx, const double *delta, const double *u_target, int B, int S,
                       const double *cond, float lr, float *loss);
int mgfr_nn_predict(mgfr_ctx *ctx, const double *delta, double *u0);
int mgfr_nn_save(mgfr_ctx *ctx, const char *path);
int mgfr_nn_load(mgfr_ctx *ctx, const char *path);

/* Single convolution layers on bf16 tensors (the network's building blocks),
 * on `stream`, no synchronisation:
 *   fwd:         y[v][o] = act(sum_{t,c} x[v+off(t)][c] w[t][o][c] + bias[o]), periodic;
 *                w bf16 [27][Cout][Cin], bias float32 [Cout] or NULL, relu 0/1;
 *                y bf16 and/or y32 float32 outputs [V][Cout] (either may be NULL).
 *                Cin % 8 == 0, Cout % 16 == 0, both <= 96, S >= 8 a power of two.
 *   bwd_data:    dx[v][c] = sum_{t,o} dz[v-off(t)][o] w[t][o][c]; wt_work: bf16 scratch
 *                of 27*Cin*Cout elements (caller-owned); Cin % 16 == 0.
 *   bwd_weight:  dw[t][o][c] += sum_v dz[v][o] x[v+off(t)][c] (float32, accumulated with
 *                atomics, so summation order varies); db[o] += sum_v dz[v][o] if db != NULL. */
int mgfr_conv3d_fwd(const void *x, int B, int S, int Cin, const void *w, const float *bias, int Cout,
                    int relu, void *y, float *y32, void *stream);
int mgfr_conv3d_bwd_data(const void *dz, int B, int S, int Cout, const void *w, int Cin, void *wt_work,
                         void *dx, void *stream);
int mgfr_conv3d_bwd_weight(const void *x, const void *dz, int B, int S, int Cin, int Cout, float *dw,
                           float *db, void *stream);

/* ---------------------------------------------------------------------
 * Adaptive refinement (Sec. 3.3 steps 9-12, one-way interface) on a
 * block-structured mesh.  The base mesh N0 = p->mesh is solved by the
 * uniform solver (p->precision applies there); refinement levels
 * l = 1..p->refine_levels (1 or 2) have N0 2^l cells per side and consist of
 * 8^3-cell blocks: a cell of level l-1 holding more than 8 particles
 * (nearest-grid-point count, unit masses) refines the aligned 4^3 group of
 * cells around it.  Level-2 blocks also refine the level-1 blocks within two
 * level-1 cells of them.  Masses follow Sec. 3.1 on the composite mesh:
 * each particle is a cube with the side of the finest cell containing it,
 * every leaf cell it overlaps (of any level) receives the overlapping
 * fraction of its mass, and each coarser cell covered by a finer level the
 * sum of its daughters; delta_l = m / mbar_l - 1 with mbar_l the total mass
 * over N_l^3.  Each level starts from, and keeps as fixed ghost
 * values around its blocks, the linear prolongation of its parent's
 * solution, and is solved by float64 FAS V-cycles over its blocks at
 * 1/1, 1/2, 1/4 and 1/8 resolution (coarse cells outside the blocks hold the
 * solution at that resolution).  The object owns all level storage, sized at
 * creation for at most max_blocks blocks per level.
 * --------------------------------------------------------------------- */
typedef struct mgfr_amr mgfr_amr;

/* p->refine_levels in {1, 2}; 32 <= p->mesh <= 512; 1 <= max_blocks <= 2^22. */
int mgfr_amr_create(const mgfr_params *p, int64_t max_blocks, void *stream, mgfr_amr **out);
void mgfr_amr_destroy(mgfr_amr *amr);

/* Relaxation factor of the float32 correction sweeps of a mixed-precision
 * adaptive solve (the base solve and every refined level; see
 * mgfr_set_relaxation32, with the same reset to 1 once a level's float64
 * residual grows).  Default 1.  Errors: MGFR_ERR_ARG unless 0 < omega < 2. */
int mgfr_amr_set_relaxation32(mgfr_amr *amr, double omega);
/* pos: float32 [np][3] (unit masses); u0: float64 [N0^3] output (base solution) or
 * NULL; st: HOST array of refine_levels + 1 stats (level 0 = base) or NULL.
 * Refinement flags are built on the device and only the block maps reach
 * the host; then the composite masses are assigned (binned when
 * mgfr_amr_reserve_particles covers np).
 * A non-finite position (or one beyond 1e15 Mpc/h) gives MGFR_ERR_NONFINITE.
 * Returns the worst level status (MGFR_NOT_CONVERGED if a level hit
 * max_vcycles); MGFR_ERR_ARG if a level needs more than max_blocks blocks. */
int mgfr_amr_solve(mgfr_amr *amr, const float *pos, int64_t np, double *u0, mgfr_stats *st);
/* Workspace for the binned composite assignment (Sec. 3.1): four uint32
 * arrays of max_np entries plus the radix sort's scratch, owned by the amr
 * object (max_np = 0 frees it).  A solve with np <= max_np sorts the particles
 * by the aligned 8^3 group of cells of their level holding their lower CIC
 * corner, accumulates each run in an LDS window and adds the window to the
 * level with one atomic per touched cell; the few particles whose cube
 * overlaps leaves of several levels keep the per-particle path.  Without it
 * (or for larger np) every particle adds its eight weights with global
 * atomics.  Both give the same masses up to the order of the float64 sums.
 * Errors: MGFR_ERR_ARG for max_np < 0 or > 2^31 - 1, MGFR_ERR_OOM. */
int mgfr_amr_reserve_particles(mgfr_amr *amr, int64_t max_np);
/* Composite fields of the last solve on the uniform mesh of the finest level,
 * side N0 2^refine_levels (the paper's power-spectrum comparison of adaptive
 * and fixed meshes, Sec. 5.1, needs the adaptive solution on one grid):
 * every cell takes delta and the effective density of Sec. 3.4,
 * delta_eff = delta/3 - C(a) expm1(-u/(n+1)) / (3 Omega_m a^-3), of the finest
 * level covering it, so a coarser leaf's values fill its sub-cells (its mass
 * spread over its volume).  delta, delta_eff: device float64 arrays of that
 * size.  Feed them to mgfr_power_ratio of a context of that mesh. */
int mgfr_amr_composite(mgfr_amr *amr, double *delta, double *delta_eff);
/* Blocks of level l (1..refine_levels) after the last solve, -1 on error. */
int64_t mgfr_amr_num_blocks(const mgfr_amr *amr, int level);
/* origins: HOST int32 [nblocks][3] block origins in level cells (multiples of 8);
 * u: device float64 [nblocks][8][8][8] level solution (either may be NULL). */
int mgfr_amr_get_level(mgfr_amr *amr, int level, int32_t *origins, double *u);

/* Last error message of this host thread ("" if none). */
const char *mgfr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MGFR_H */
