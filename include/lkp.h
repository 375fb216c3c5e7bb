/*
 * lkp -- higher-order lattice-kinetic Poisson solver for AMD Instinct MI355X (gfx950).
 *
 * Method: Mendoza, Succi, Herrmann, "High-Order Kinetic Relaxation Schemes as
 * High-Accuracy Poisson Solvers".  A periodic Poisson problem lap(Phi) = -s
 * is solved as the steady state of the diffusion equation with source
 * (Sec. 2, Eq. DIFFU), itself the small-Knudsen limit of a BGK kinetic equation
 * (Eq. boltzmann).  On a lattice of Q discrete velocities v_i each sweep does,
 * for every cell x (Sec. 4 and 5):
 *
 *     stream (pull):    f_i(x)    = f*_i(x - v_i)              (periodic)
 *     moment:           Phi(x)    = sum_i f_i(x)
 *     collide + source: f*_i'(x)  = (1 - omega) f_i(x) + omega phi_i Phi(x) + chi_i S(x)
 *
 * with omega = 1 / tau_lb, the separable equilibrium phi(v) Phi (Eq. equilibrium2)
 * and source chi(v) S whose Hermite coefficients cancel the unwanted moments up
 * to order N (Eq. CON; Eqs. omega:eq, chi:eq, omega:eq3, chi:eq3), and the
 * strong source S = s c_s^2 (tau_lb - 1/2) (Sec. 5).  The answer is Phi at the
 * fixed point of the sweep.
 *
 * Conventions for every call:
 *  - Fields are periodic, stored x fastest: index (z * ny + y) * nx + x.
 *    Population state is Q planes of n = nx*ny*nz cells ("SoA"), plane i
 *    holding velocity i of lkp_lattice_info's table.
 *  - All calls return lkp_status (LKP_OK = 0); no exception crosses the ABI.
 *    lkp_last_error() gives a thread-local message for the last failure.
 *  - Device pointers are HIP device pointers valid on the handle's device;
 *    "host" pointers are ordinary process memory.
 *  - A handle is not thread-safe; all its GPU work is enqueued on the stream
 *    given at creation (NULL = the default stream).  Calls that return data
 *    to the host synchronise that stream.
 */
#ifndef LKP_H
#define LKP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lkp_status {
  LKP_OK = 0,
  LKP_ERR_ARG = 1,            /* invalid argument (shape, pointer, option) */
  LKP_ERR_LATTICE_ORDER = 2,  /* order N not 1/3/5/7, or above the set's maximum, or dim mismatch */
  LKP_ERR_UNSTABLE = 3,       /* tau_lb below the set/order stability limit */
  LKP_ERR_SOURCE_MEAN = 4,    /* |mean(s)| > 1e-12 max|s| and subtract_mean == 0 */
  LKP_ERR_OOM = 5,            /* device allocation failed */
  LKP_ERR_HIP = 6,            /* a HIP runtime call failed */
  LKP_ERR_NOT_CONVERGED = 7,  /* lkp_solve reached max_sweeps */
  LKP_ERR_DIVERGED = 8,       /* non-finite values or sustained growth */
  LKP_ERR_STATE = 9,          /* call not valid in the handle's current state */
  LKP_ERR_UNSUPPORTED = 10    /* combination not built (e.g. lattice/precision) */
} lkp_status;

/* Velocity sets.  1D sets: Appendix A.  2D: tensor products of the 1D sets
 * (the paper's "tensorial" extension, Sec. 4) and the standard
 * nearest-neighbour D2Q5 / D2Q9.  3D: D3Q111 (Appendix A, Table vector2).
 * Generated sets (quadrature conditions of Sec. 4, smallest stable): D2Q37,
 * D2Q77, D3Q107. */
typedef enum lkp_lattice {
  LKP_D1Q5 = 0,   /* N <= 3 */
  LKP_D1Q9 = 1,   /* N <= 5 */
  LKP_D1Q13 = 2,  /* N <= 7 */
  LKP_D2Q5 = 3,   /* N = 1, standard LB */
  LKP_D2Q9 = 4,   /* N <= 3 */
  LKP_D2Q25 = 5,  /* N <= 3 */
  LKP_D2Q81 = 6,  /* N <= 5 */
  LKP_D2Q169 = 7, /* N <= 7 */
  LKP_D3Q111 = 8, /* N <= 5 */
  LKP_D2Q37 = 9,  /* N <= 5: generated minimal 2D set (quadrature conditions of Sec. 4) */
  LKP_D2Q77 = 10, /* N <= 7: generated minimal 2D set stable at N = 7 */
  LKP_D3Q107 = 11, /* N <= 5: generated minimal 3D set stable at N = 5 (shells 0, (1,0,0),
                      (1,1,0), (1,1,1), (2,0,0), (2,1,0), (2,2,0), (3,0,0), (3,1,1), (2,2,2)) */
  LKP_NUM_LATTICES = 12
} lkp_lattice;

typedef enum lkp_precision {
  LKP_F64 = 0,    /* FP64 populations, FP64 everything */
  LKP_F32 = 1,    /* FP32 populations and sweep (FP64 moment sum and norms), no refinement */
  LKP_F32_IR = 2,    /* FP32 inner sweeps inside FP64 iterative refinement on the population state */
  LKP_BF16DEV_IR = 3 /* ablation: inner sweeps store each population as phi_i Phi + n_i with the
                      * deviation n_i in BF16 and Phi in FP32 (4Q + 12 bytes per cell and sweep
                      * instead of 12Q for FP32), inside the same FP64 refinement; the first
                      * inner solve is the plain BF16-deviation sweep.  Not available in the
                      * tau_lb = 1 stencil form (there n_i = chi_i S exactly) nor in groups. */
} lkp_precision;

/* At tau_lb = 1 (omega = 1) the collision forgets the populations: after a
 * sweep f*_i = phi_i Phi + chi_i S, so the next moment is the scalar stencil
 * Phi' = sum_i phi_i Phi(x - v_i) + sum_i chi_i S(x - v_i).  Handles then keep
 * Phi alone and sweep with that stencil (same answer, same sweep count, far
 * fewer bytes); populations are rebuilt on request and cannot be set.  This
 * flag keeps the population sweep instead. */
#define LKP_FLAG_POPULATION_SWEEP 1
/* One population buffer swept in place (F64, F32; for F32_IR the inner
 * corrections): consecutive sweeps alternate between two storage layouts of
 * the same buffer (a sweep that gathers from and scatters to neighbours, then
 * one that reads and writes its own cell), which halves the population
 * memory.  Phi and the convergence history are bitwise those of the
 * two-buffer sweep.  Populations and the residual stay available; the
 * velocity-group split is not tuned; such handles cannot join a group. */
#define LKP_FLAG_IN_PLACE 2

typedef struct lkp_problem_desc {
  int32_t dim;              /* 1, 2 or 3; must equal the lattice's dimension */
  int32_t lattice;          /* lkp_lattice */
  int64_t n[3];             /* nx, ny, nz; axes beyond dim must be 1; each >= 1;
                               nx*ny*nz < 2^29 (a population plane stays below 4 GiB) */
  int32_t order;            /* expansion order N: 1, 3, 5 or 7 (Sec. 4) */
  int32_t precision;        /* lkp_precision */
  double tau_lb;            /* lattice relaxation time; used when knudsen <= 0 */
  double knudsen;           /* > 0: tau_lb = 1/2 + Kn * L / c_s, L = smallest box side
                               (Kn = lambda / L, Sec. 2, with lambda = c_s (tau_lb - 1/2)) */
  const double *source;     /* s in lap(Phi) = -s (Sec. 5, Eq. poisson1: s = rho/eps),
                               nx*ny*nz FP64 values; copied at creation, the caller
                               keeps ownership */
  int32_t source_on_device; /* 1: `source` is a device pointer */
  int32_t subtract_mean;    /* 1: remove the mean of s instead of rejecting it */
  int32_t allow_unstable;   /* 1: skip the tau_lb stability check */
  int32_t flags;            /* LKP_FLAG_* bits */
  void *stream;             /* hipStream_t for all of this handle's work; NULL = default */
  double drift[3];          /* uniform drift u (lattice units per sweep) of the
                               advection-diffusion variant, the extension named at the
                               end of the paper (Sec. 6); all zero = the paper's diffusion
                               scheme.  The equilibrium becomes that of a Gaussian moved by
                               u, to second order in u:
                                 phi_i += w_i [ (v_i.u)/c_s^2 + ((v_i.u)^2 - c_s^2 |u|^2)/(2 c_s^4) ]
                               (mass, first moment u and second moment c_s^2 delta + u u), so
                               a sweep is a time step of d_t Phi + u.grad Phi = D lap Phi + D s,
                               D = c_s^2 (tau_lb - 1/2), and the fixed point solves
                               lap Phi - (u/D).grad Phi = -s.  Components beyond dim must be 0
                               and |u|^2 < c_s^2 (else LKP_ERR_ARG / LKP_ERR_UNSTABLE unless
                               allow_unstable).  A drifted handle always sweeps populations
                               (also at tau_lb = 1) and cannot join a group.  Zero-initialise
                               the whole description so that older callers get u = 0. */
  void *workspace;          /* NULL: the handle allocates its device state itself.  Else a
                               device pointer, 256-byte aligned, to workspace_bytes bytes of
                               the current device that hold the whole state (populations,
                               source, Phi buffers, reduction partials): lkp_create carves
                               them from it and allocates no device memory for the state.
                               The caller keeps ownership, must not touch the range and must
                               keep it alive until lkp_destroy returns.  Readbacks that convert
                               precision (lkp_get_phi / lkp_get_populations / lkp_set_populations
                               to or from host memory) may still allocate staging buffers. */
  int64_t workspace_bytes;  /* size of `workspace`; at least lkp_footprint_bytes(d), else
                               LKP_ERR_ARG; must be 0 when workspace is NULL */
} lkp_problem_desc;

typedef struct lkp_handle lkp_handle;

/* Create a problem (the discrete BGK scheme of Sec. 2, Eq. boltzmann, on the
 * set and equilibrium order of Sec. 4, source term of Sec. 5): validates the description, computes the set's
 * weights, c_s^2, phi_i, chi_i (long double, rounded once), scales the source
 * S = s c_s^2 (tau_lb - 1/2), places the device state (two population
 * buffers, S, Phi buffers, reduction partials) and sets f* = 0.
 * Ownership: without a workspace the handle owns all device memory it
 * allocates; with one, the state lives in the caller's range.  Release with
 * lkp_destroy.  Errors: LKP_ERR_ARG (also a workspace that is misaligned, too
 * small, or given without a size), LKP_ERR_LATTICE_ORDER, LKP_ERR_UNSTABLE,
 * LKP_ERR_SOURCE_MEAN, LKP_ERR_OOM, LKP_ERR_HIP; *out is NULL on failure. */
lkp_status lkp_create(const lkp_problem_desc *d, lkp_handle **out);

/* Release every resource of the handle (NULL is accepted): waits for its
 * stream, frees what it allocated and leaves a caller's workspace alone. */
lkp_status lkp_destroy(lkp_handle *h);

/* Device bytes of the state lkp_create places for `d`: the size of every
 * buffer, each starting at a 256-byte boundary, i.e. the smallest workspace
 * that `d` accepts (0 if `d` is invalid; the last error is left as it was). */
int64_t lkp_footprint_bytes(const lkp_problem_desc *d);

/* The slowest decay the sweep of `d` allows: the largest modulus of the
 * one-sweep amplification over the grid's modes other than the mass mode
 * (Fourier analysis of the sweep of Sec. 4 and 5; the stability analysis of
 * the same modes decides LKP_ERR_UNSTABLE), written to *rho.  It peaks at the
 * kinetic value |1 - 1/tau_lb|, at a corner mode (every wavevector component
 * 0 or pi) or at the longest wave along an axis, and those are the modes
 * taken.  lkp_solve never estimates the distance to the fixed point with a
 * contraction below it.  Host only (no device call, `source` not read).
 * Errors: as lkp_create's validation (LKP_ERR_ARG, LKP_ERR_LATTICE_ORDER,
 * LKP_ERR_UNSTABLE). */
lkp_status lkp_contraction_bound(const lkp_problem_desc *d, double *rho);

typedef struct lkp_solve_opts {
  double tol_rel_l2;    /* > 0: stop when the estimated relative L2 distance of Phi to the
                           fixed point, |D| rho^m / (1 - rho^m) / |Phi|, is <= tol_rel_l2.
                           D: the change of Phi over the last m sweeps (with tol_rel_l2
                           alone, a population solve compares with the Phi stored before
                           each chunk, m = the chunk; otherwise m = 1); rho: the largest of
                           the last four per-sweep contractions measured between checks and
                           of lkp_contraction_bound (refinement: the last correction scaled
                           by the residual's shrink since it, and at least what its inner
                           solve estimated it left) */
  double tol_maxchange; /* > 0: stop when max_x |Phi_t - Phi_{t-1}| < tol_maxchange */
  int64_t max_sweeps;   /* hard cap on sweeps done by this call (> 0) */
  int32_t check_every;  /* sweeps between convergence checks (>= 1) */
  int32_t max_outer;    /* LKP_F32_IR: cap on refinement steps (0 = 20) */
  double ir_inner_tol;  /* LKP_F32_IR: relative accuracy of each inner solve; 0 = adaptive,
                           0.3 tol_rel_l2 / (current estimated error), within [1e-7, 0.1] */
  int32_t use_graph;    /* 1: replay the chunk of sweeps as a captured hipGraph */
  int32_t reserved;
} lkp_solve_opts;

typedef struct lkp_solve_report {
  int64_t sweeps;        /* sweeps done by this call (inner sweeps for F32_IR) */
  int64_t total_sweeps;  /* sweeps since creation */
  int32_t outer;         /* refinement steps (F32_IR) */
  int32_t status;        /* same as the return value */
  double max_change;     /* max |Phi_t - Phi_s| at the last check: s = t - 1, or, for a
                            population solve with tol_rel_l2 alone, the sweep of the Phi
                            stored before the check's chunk (the change over the chunk) */
  double l2_change;      /* ||Phi_t - Phi_s||_2 at the last check (s as above) */
  double phi_l2;         /* ||Phi||_2 */
  double mass;           /* sum_x Phi */
  double est_rel_err;    /* estimated relative L2 distance to the fixed point */
  double rate;           /* per-sweep contraction rho used by the estimate */
  double wall_s;         /* wall time of the call */
  double glups;          /* 1e-9 * cells * sweeps / wall_s */
} lkp_solve_report;

/* Sweep until the stopping rule of `o` holds (Sec. 5: the steady state of the
 * iteration is the Poisson solution).  The convergence norms are FP64
 * wavefront reductions on the GPU, read back once per check.  The state stays
 * resident, so a later call resumes; for F64 and F32 handles the convergence
 * history (last check's change, measured contraction) carries over too, so the
 * first check of a resumed call already yields an error estimate (it restarts
 * after lkp_set_populations / lkp_set_equilibrium).  Refinement handles resume
 * from the residual of the current FP64 state.  Returns LKP_ERR_NOT_CONVERGED
 * at max_sweeps, LKP_ERR_DIVERGED on non-finite values or growth.  `rep` may be
 * NULL. */
lkp_status lkp_solve(lkp_handle *h, const lkp_solve_opts *o, lkp_solve_report *rep);

/* Advance exactly `sweeps` sweeps (>= 0): each is one step of the discrete
 * BGK relaxation with source (Sec. 2, Eq. boltzmann, with the equilibrium and
 * source shapes of Sec. 4 and the scaled source of Sec. 5): pull-stream,
 * moment Phi = sum_i f_i, collide.  No stopping test; the last sweep stores
 * Phi.  Errors: LKP_ERR_ARG (sweeps < 0), LKP_ERR_STATE (the handle is
 * resident in a group: the group steps it), LKP_ERR_HIP. */
lkp_status lkp_step(lkp_handle *h, int64_t sweeps);

typedef struct lkp_residual_report {
  double max_change;      /* max |Phi_{t+1} - Phi_t|: one-sweep change of the moment, the
                             discrete Poisson residual in the scheme's own units */
  double l2_change;       /* ||Phi_{t+1} - Phi_t||_2 */
  double pop_residual_l2; /* ||T f* + g - f*||_2 over all populations (FP64) */
  double phi_l2;          /* ||Phi_t||_2 */
  double mass;            /* sum_x Phi_t */
  int64_t sweeps;         /* sweeps since creation */
} lkp_residual_report;

/* Residual of the current state in FP64 on the GPU, without advancing it:
 * the distance from the steady state that Sec. 4 and 5 take as the Poisson
 * solution (all time derivatives zero, Sec. 3), measured as one sweep's change
 * of Phi and of the populations.  Needs at least one sweep done
 * (LKP_ERR_STATE otherwise); `r` is written only on success. */
lkp_status lkp_residual(lkp_handle *h, lkp_residual_report *r);

/* Phi of the last sweep (post-stream moment, Sec. 2: Phi = sum_i f_i), n FP64
 * values into caller-owned memory.  LKP_ERR_STATE before the first sweep or
 * after lkp_set_populations. */
lkp_status lkp_get_phi(lkp_handle *h, double *dst, int32_t dst_is_device);

/* Copy the post-collision population state (Q*n FP64, plane-major, plane i =
 * velocity i) out of / into the handle; FP32 states are converted. */
lkp_status lkp_get_populations(lkp_handle *h, double *dst, int32_t dst_is_device);
lkp_status lkp_set_populations(lkp_handle *h, const double *src, int32_t src_is_device);

/* Constants of a set at order N (host memory, caller-owned; any pointer may be
 * NULL): Q, dim, velocities v[Q][3], weights w, phi_i, chi_i and c_s^2.  Arrays
 * must hold at least 169 (x3 for v) entries. */
lkp_status lkp_lattice_info(int32_t lattice, int32_t order, int32_t *Q, int32_t *dim,
                            int32_t *v, double *w, double *phi, double *chi, double *cs2);

typedef struct lkp_handle_info {
  int32_t lattice, order, dim, Q, precision, velocity_groups;
  int32_t scalar_stencil;   /* 1: omega = 1 stencil form (state is Phi) */
  int32_t in_place;         /* 1: one population buffer swept in place (LKP_FLAG_IN_PLACE) */
  int32_t stencil_tile;     /* 3D stencil form: tile variant chosen by timing, output tile
                               64 x 4CY x BZ: 0..5 velocity by velocity with (CY, BZ) =
                               (2,32) (2,16) (2,8) (4,16) (4,8) (1,16); 6..9 separable (sums
                               over +-x, then +-y offsets, then one weight per offset
                               magnitude) with (2,32) (2,16) (1,16) (4,16).  The variants of
                               one family give the same bits, the families agree to rounding;
                               else -1 */
  int32_t stencil_remap;    /* 3D stencil form: 0 hardware block order, R > 0 runs of R
                               blocks per XCD; else -1 */
  int64_t n[3];
  double tau_lb, omega, cs2;
  int64_t total_sweeps;
  int64_t footprint_bytes;
} lkp_handle_info;

lkp_status lkp_get_info(lkp_handle *h, lkp_handle_info *info);

/* The handle's equilibrium and source shapes phi_i, chi_i (Sec. 4, Eqs.
 * omega:eq, chi:eq, omega:eq3, chi:eq3, with the drift terms of a drifted
 * handle) in the order of lkp_lattice_info's velocities: Q FP64 values each
 * into host arrays (either may be NULL).  Errors: LKP_ERR_ARG. */
lkp_status lkp_get_coefficients(lkp_handle *h, double *phi, double *chi);

/* Time-dependent use (the sweep as a time step of the diffusion or
 * advection-diffusion equation, Sec. 2 and 6): set the post-collision state
 * to the equilibrium f*_i = phi_i Phi_0 of the field Phi_0 (n FP64 values,
 * host or device, caller-owned), computed on the device straight into the
 * handle's state, in its layout and precision (a host field is staged through
 * the handle's own Phi buffer): no device memory is allocated, so it works at
 * any size the handle holds.  Then advance with lkp_step and read lkp_get_phi.
 * Errors: LKP_ERR_ARG, LKP_ERR_UNSUPPORTED (tau_lb = 1 stencil form),
 * LKP_ERR_HIP. */
lkp_status lkp_set_equilibrium(lkp_handle *h, const double *phi0, int32_t phi0_is_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the FP64
 * residual sweep of lkp_residual for a population state held in caller-owned
 * device buffers, with no handle and no allocation.  Its per-block partial
 * norms use a fixed array in device memory (12 MiB per GPU, held until the
 * process ends), so it serves grids of at most 2^24 cells (LKP_ERR_ARG
 * beyond).  Everything is enqueued on `stream` (hipStream_t, NULL = default):
 * two kernel launches, no copy, no synchronisation.  Calls on one GPU share
 * that array: calls that overlap on one GPU (several streams, threads) race.
 *   lattice, order, n[3], tau_lb: as in lkp_problem_desc (explicit tau_lb, no drift)
 *   f:        Q*n FP64 post-collision populations (device, plane i = velocity i)
 *   S:        n FP64 scaled source S = s c_s^2 (tau_lb - 1/2) (device)
 *   phi_prev: n FP64 (device) Phi of the sweep that produced f, or NULL (zeros)
 *   phi_out:  n FP64 (device) output: Phi of the next sweep (the moment of f streamed)
 *   r_out:    Q*n FP32 (device) output: residual populations r = T f + g - f, or NULL
 *   norms_out: 6 FP64 (device) output: max |Phi' - Phi_prev|, sum (Phi' - Phi_prev)^2,
 *             sum Phi'^2, sum Phi', count of non-finite values, sum r^2 (lkp_residual
 *             reports the square roots of the second, third and sixth).
 * Errors (nothing is enqueued): LKP_ERR_ARG, LKP_ERR_LATTICE_ORDER, LKP_ERR_HIP. */
lkp_status lkp_residual_noalloc(int32_t lattice, int32_t order, const int64_t n[3], double tau_lb,
                                const double *f, const double *S, const double *phi_prev,
                                double *phi_out, float *r_out, double *norms_out, void *stream);

/* Wait for all of the handle's queued work. */
lkp_status lkp_sync(lkp_handle *h);

/* Thread-local message of the last failing call ("" if none). */
const char *lkp_last_error(void);

/* ------------------------------------------------------------------------
 * Serving: many resident problems advanced together.
 *
 * A group holds problems of one class (lattice, order, precision) that share
 * the group's stream.  lkp_group_step advances every running member by the
 * same number of sweeps in batched launches: each launch covers up to a few
 * dozen members, and its blocks are dealt member after member so small grids
 * still fill the GPU.  The FP32 + refinement residual and update steps run
 * per member.  Members are checked with exactly the rules lkp_solve applies
 * (the group's sweeps per step playing the role of check_every), so a
 * member's sweeps, answer and retirement are the same alone (lkp_solve with
 * check_every = sweeps per step and the same velocity-group split) and in any
 * mix.  Membership changes between steps; the caller retires converged
 * members (lkp_get_phi, then lkp_group_remove or lkp_destroy).
 * ------------------------------------------------------------------------ */
typedef struct lkp_group lkp_group;

typedef enum lkp_member_state {
  LKP_MEMBER_RUNNING = 0,
  LKP_MEMBER_CONVERGED = 1,
  LKP_MEMBER_FAILED = 2     /* diverged, or max_sweeps reached: see status */
} lkp_member_state;

typedef struct lkp_member_report {
  lkp_handle *handle;
  int32_t state;            /* lkp_member_state */
  int32_t status;           /* LKP_OK, or the error that stopped the member */
  int64_t sweeps;           /* sweeps since the member was added */
  int32_t outer;            /* refinement steps (F32_IR) */
  int32_t reserved;
  double est_rel_err;       /* estimated relative L2 distance to the fixed point */
  double max_change;        /* max |Phi_t - Phi_{t-1}| at the last check (plain sweeps) */
  double phi_l2;            /* ||Phi||_2 */
} lkp_member_report;

/* Create an empty group for (lattice, order, precision) on `stream`
 * (hipStream_t; NULL = default).  The group owns only its bookkeeping. */
lkp_status lkp_group_create(int32_t lattice, int32_t order, int32_t precision, void *stream,
                            lkp_group **out);

/* Admit a created handle of the group's class and stream, with its stopping
 * options (tol_rel_l2 / tol_maxchange / max_sweeps as in lkp_solve; the
 * group's sweeps per step replace check_every).  The handle's convergence
 * state starts afresh; while resident it cannot be driven by lkp_solve or
 * lkp_step.  Errors: LKP_ERR_ARG (class or stream mismatch, already in a
 * group), LKP_ERR_STATE. */
lkp_status lkp_group_add(lkp_group *g, lkp_handle *h, const lkp_solve_opts *o);

/* Remove a member (its state and device memory stay with the handle). */
lkp_status lkp_group_remove(lkp_group *g, lkp_handle *h);

/* Advance every running member by `sweeps` (>= 2) sweeps with one check at
 * the end, then report every member (running, converged or failed) into
 * out[0 .. *count) (out may be NULL when capacity is 0).  Enqueues on the
 * group's stream and synchronises it once for the read-back of all members'
 * norms (48 bytes each).
 * The batched sweeps and norm reductions of a step are replayed from a
 * captured hipGraph when the step launches exactly (byte for byte, launch
 * parameters included) what an earlier captured step launched: a step whose
 * launches repeat those of the two steps before it is captured, up to 8
 * graphs per group are kept (least recently used evicted).  Results are bitwise those of the
 * eager launches.  The environment variable LKP_GROUP_GRAPH=0, read at
 * lkp_group_create, disables capture for the group. */
lkp_status lkp_group_step(lkp_group *g, int32_t sweeps, lkp_member_report *out, int32_t capacity,
                          int32_t *count);

/* The group's velocity-group split P of its batched sweeps.  At the first step
 * with enough work to time (2^18 cells over the running members) the group
 * times every built split of its batched sweep (F32_IR: the correction
 * sweep) on its members' own buffers (the state is unchanged) and keeps the
 * fastest, cached for the class (set, precision) in the process; every split
 * gives the same bits, so answers are the same alone and in any mix.
 * LKP_SPLIT forces a split, LKP_AUTOTUNE=0 keeps the default. */
lkp_status lkp_group_split(const lkp_group *g, int32_t *velocity_groups);

/* Counters of the group's captured steps: graphs captured and steps replayed
 * from a graph since creation (either pointer may be NULL). */
lkp_status lkp_group_graph_stats(const lkp_group *g, int64_t *captures, int64_t *replays);

/* Destroy the group; members are released from it, not destroyed. */
lkp_status lkp_group_destroy(lkp_group *g);

#ifdef __cplusplus
}
#endif

#endif /* LKP_H */
