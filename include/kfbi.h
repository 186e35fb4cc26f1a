/*
 * kfbi.h -- C ABI of the MI355X (gfx950) kernel-free boundary integral
 * (KFBI) time-stepping library.
 *
 * The library solves, on an irregular 2-D domain Omega inside the box
 * B = [-L, L]^2 (paper section 3.2),
 *
 *     lap u - kappa u = f  in Omega,   u = g  on Gamma = dOmega     (eq. 3.13)
 *
 * through the second-kind boundary integral equation
 * 1/2 phi + W phi + Y f = g (eq. 3.17) for the double-layer density phi,
 * u = W phi + Y f (eq. 3.18), where every application of W and Y is the
 * solution of an interface problem on the Cartesian grid (eqs. 3.24, 3.27,
 * 3.30): jump corrections at irregular nodes (section 3.2.4), a five-point
 * (Delta_h - kappa) solve on B with u = 0 on dB (eq. 3.31), and extraction
 * of the interior limit at the boundary collocation points (section 3.2.6).
 * GMRES solves the integral equation.  On top of it the implicit time steps
 * of section 3.1 -- Crank-Nicolson for the heat equation (eqs. 3.1-3.4),
 * the implicit theta-scheme for the wave equation (eqs. 3.5-3.7) and Strang
 * splitting for the Schroedinger equation (eqs. 3.8-3.12) -- each reduce to
 * one such solve.
 *
 * Conventions for every call
 *   - Grid arrays are (M+1) x (M+1), row-major with x fastest:
 *     element (i, j) at index j*(M+1) + i, node (x_i, y_j) = (-L + i h,
 *     -L + j h), h = 2L/M.  Boundary arrays have Nb entries ordered by the
 *     collocation parameter theta_k = 2 pi k / Nb.
 *   - Arrays passed to the solve and step calls are DEVICE pointers owned by
 *     the caller; real domains use float64, complex domains interleaved
 *     complex128 (re, im), as torch stores them.  The library never frees or
 *     retains caller memory.  Arrays of the copy_* calls are HOST pointers.
 *   - All device work of a domain is enqueued on the stream given at
 *     creation (NULL = the default stream).  A call returns after its work
 *     is enqueued and the scalars it reports have been read back.
 *   - Every call returns a kfbi_status; on failure kfbi_last_error() gives a
 *     thread-local message.  No C++ exception crosses this interface.
 */
#ifndef KFBI_H
#define KFBI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KFBI_OK = 0,
    KFBI_EINVAL = 1,   /* bad argument (null pointer, size, mode)            */
    KFBI_EDOMAIN = 2,  /* interface within 3h of the box, or too few points  */
    KFBI_ENOMEM = 3,   /* device allocation failed                           */
    KFBI_ENOCONV = 4,  /* GMRES hit max_iter; outputs and stats still valid  */
    KFBI_EDEVICE = 5,  /* a HIP runtime call failed                          */
    KFBI_ENOTSUP = 6   /* combination not supported                          */
} kfbi_status;

typedef enum { KFBI_CURVE_DISK = 0, KFBI_CURVE_ELLIPSE = 1, KFBI_CURVE_STAR = 2 } kfbi_curve_kind;
typedef enum { KFBI_REAL = 0, KFBI_COMPLEX = 1 } kfbi_scalar;
typedef enum { KFBI_PREC_FP64 = 0, KFBI_PREC_MIXED = 1 } kfbi_precision;
typedef enum { KFBI_HEAT = 0, KFBI_WAVE = 1, KFBI_SCHRODINGER = 2 } kfbi_equation;
typedef enum { KFBI_BC_DIRICHLET = 0, KFBI_BC_NEUMANN = 1 } kfbi_boundary_condition;
/* Operator splitting of the Schroedinger step (section 3.1; the comparison
 * of section 4.1, Example 7).  STRANG: S^A(tau/2) S^B(tau) S^A(tau/2), the
 * three-step algorithm after eq. 3.12, second order, kappa = 2i/tau.
 * GODUNOV: S^A(tau) S^B(tau), first order: the closed-form Crank-Nicolson
 * B-step of eq. 3.10 over tau applied to u^n, then the backward-Euler A-step
 * of eq. 3.11 over tau, lap u^{n+1} - (i/tau) u^{n+1} = -(i/tau) u**,
 * kappa = i/tau. */
typedef enum { KFBI_SPLIT_STRANG = 0, KFBI_SPLIT_GODUNOV = 1 } kfbi_split;

/* Domain description (section 3.2.4 grid, Procedure 1 of section 3.3).
 * Curves, counter-clockwise in theta in [0, 2 pi):
 *   DISK     (cx + R cos t, cy + R sin t)
 *   ELLIPSE  (cx + a cos t, cy + b sin t)
 *   STAR     (cx, cy) + (r0 + amp sin(lobes t)) (cos t, sin t), amp < r0
 * M: grid intervals per axis, a power of two with 16 <= M <= 4096.
 * Nb: number of collocation points, 8 <= Nb <= 16384. */
typedef struct {
    double L;
    int32_t M;
    int32_t Nb;
    int32_t kind;        /* kfbi_curve_kind */
    int32_t lobes;
    double cx, cy;
    double R;
    double a, b;
    double r0, amp;
    int32_t scalar;      /* kfbi_scalar: element type of every array */
    int32_t precision;   /* kfbi_precision: default grid-solve precision */
    void *stream;        /* hipStream_t; NULL = default stream */
} kfbi_domain_desc;

typedef struct {
    int32_t M, Nb;
    double L, h;
    int32_t n_inside;     /* grid nodes inside Omega                        */
    int32_t n_irregular;  /* interior nodes with a 4-neighbour on the other
                             side of Gamma (section 3.2.4)                  */
    int32_t n_edges;      /* grid edges crossed by Gamma                    */
    int32_t scalar;       /* kfbi_scalar of the domain: element type of its
                             arrays (float64 or interleaved complex128)    */
    uint64_t device_bytes;/* device memory held by the domain               */
    uint64_t device_bytes_max; /* what it holds once every solve has run:
                             the per-kappa operator tables and the FP32 tables
                             of mixed precision, allocated on first use,
                             included (the figure for admission budgets)    */
} kfbi_domain_info;

typedef struct {
    double tol;           /* stop when ||b - K phi|| / ||b|| <= tol; default 1e-10 */
    int32_t max_iter;     /* maximum GMRES iterations (Arnoldi steps); default 500 */
    int32_t restart;      /* GMRES restart length m, 1..64; default 50             */
    int32_t fixed_iters;  /* > 0: run exactly this many iterations (parity mode)   */
    int32_t precision;    /* -1: the domain's default; else kfbi_precision         */
    int32_t flags;        /* KFBI_SOLVE_* bits; 0 by default                       */
    int32_t pad;
    double gamma;         /* Richardson parameter (KFBI_SOLVE_RICHARDSON); <= 0: 1  */
} kfbi_solve_opts;

/* kfbi_solve_opts.flags: return as soon as GMRES has finished on the device.
 * The final grid solve (u_grid_out, phi_inout) and the stepper's right-hand
 * side update are then still queued on the domain stream: they complete in
 * stream order before any later work on that stream, and the host must
 * synchronise the stream before reading them.  stats are valid on return
 * except device_ms, which is -1. */
#define KFBI_SOLVE_ASYNC 1

/* kfbi_solve_opts.flags, batched solves only: keep the default launch shape
 * of the tridiagonal kernel instead of timing the candidates (see
 * kfbi_batch_tuning).  The choice never changes results. */
#define KFBI_BATCH_NO_TUNE 2

/* kfbi_solve_opts.flags: solve the second-kind equation (eq. 3.17) by the
 * Richardson iteration of eq. 3.21, phi_{k+1} = (1 - gamma/2) phi_k +
 * gamma (g - Yf - W phi_k) = phi_k + gamma (b - K phi_k), instead of GMRES,
 * from the same initial density and to the same stopping test
 * (||b - K phi|| <= tol ||b||; fixed_iters > 0: exactly that many updates).
 * stats.iters counts the updates.  FP64 (complex128) only: with the mixed
 * precision the call returns KFBI_ENOTSUP; single solves and steps only
 * (batched calls return KFBI_ENOTSUP). */
#define KFBI_SOLVE_RICHARDSON 4

typedef struct {
    int32_t iters;        /* GMRES iterations (matrix-vector products in Arnoldi) */
    int32_t converged;
    double rel_resid;     /* final ||b - K phi|| / ||b|| estimate                  */
    int32_t refinements;  /* outer FP64 refinement sweeps (mixed precision)        */
    int32_t pad;
    double device_ms;     /* device time of the call (HIP events)                  */
} kfbi_solve_stats;

typedef struct kfbi_domain kfbi_domain;
typedef struct kfbi_stepper kfbi_stepper;
typedef struct kfbi_batch kfbi_batch;

/* Thread-local description of the last failure. */
const char *kfbi_last_error(void);

/* Procedure 1 (section 3.3; parallel form in section 3.4.2): build the grid,
 * classify every node as inside/outside (strict polynomial test, a node on
 * Gamma is outside), list irregular nodes in increasing linear index, find
 * every grid edge crossed by Gamma and its intersection, place Nb
 * collocation points and factor their six-point extraction stencils
 * (section 3.2.6).  All of it runs in device kernels.
 * Errors: EINVAL (bad sizes), EDOMAIN (Gamma within 3h of dB, or the
 * interface too close to the box), ENOMEM, EDEVICE. */
int kfbi_domain_create(const kfbi_domain_desc *desc, kfbi_domain **out);

/* Frees the domain's device memory.  Caller buffers are never touched. */
int kfbi_domain_destroy(kfbi_domain *dom);

int kfbi_domain_get_info(const kfbi_domain *dom, kfbi_domain_info *out);

/* Node classes, (M+1)^2 host bytes: bit 0 = inside, bit 1 = irregular. */
int kfbi_domain_copy_classification(const kfbi_domain *dom, uint8_t *host_out);

/* Collocation points z_k, host array of 2*Nb doubles (x0, y0, x1, y1, ...). */
int kfbi_domain_copy_boundary(const kfbi_domain *dom, double *host_out);

/* Outward unit normals n = (t_y, -t_x) at the collocation points (section
 * 3.2.5; the direction of du/dn in kfbi_neumann_solve), host array of 2*Nb
 * doubles (nx0, ny0, nx1, ny1, ...). */
int kfbi_domain_copy_normals(const kfbi_domain *dom, double *host_out);

/* Crossed edges: host arrays of n_edges entries each.  pq[2e], pq[2e+1] are
 * the linear indices of the edge's inside and outside node; xyt[3e..3e+2]
 * are the intersection (x, y) and its curve parameter theta. */
int kfbi_domain_copy_edges(const kfbi_domain *dom, int32_t *pq, double *xyt);

/* The five-point solve of eq. (3.31) alone: (Delta_h - kappa) U = rhs at
 * the interior nodes, U = 0 on dB.  rhs and u_out are device grid arrays
 * (boundary entries of rhs are ignored; those of u_out are written 0).
 * kappa = kappa_re + i kappa_im; kappa_im must be 0 for a real domain. */
int kfbi_grid_solve(kfbi_domain *dom, double kappa_re, double kappa_im,
                    const void *rhs, void *u_out);

/* One interface-problem evaluation (Procedure 2; eqs. 3.30 and the table
 * after it with Phi = phi, Psi = 0, F = f~): jumps (section 3.2.5),
 * corrections (section 3.2.4), grid solve, extraction (section 3.2.6).
 * f_grid (nullable: f = 0) is f on the grid, used at inside nodes only
 * (eq. 3.25); f_gamma is f's trace on Gamma at the collocation points
 * (required when f_grid is given); phi (nullable: 0) the density.
 * u_grid_out (nullable) receives the grid solution, uplus_out (nullable)
 * the interior limit U+ at the collocation points. */
int kfbi_interface_apply(kfbi_domain *dom, double kappa_re, double kappa_im,
                         const void *f_grid, const void *f_gamma,
                         const void *phi, void *u_grid_out, void *uplus_out);

/* Solve lap u - kappa u = f in Omega, u = g on Gamma (eq. 3.13) through the
 * integral equation (3.17) by GMRES and the representation (3.18).
 * f_grid (nullable) / f_gamma as for kfbi_interface_apply; g_gamma the
 * Dirichlet data at the collocation points; u_grid_out the grid solution
 * (meaningful at inside nodes); phi_inout (nullable) the warm start on
 * entry and the density on exit.  opts nullable (defaults), stats nullable.
 * The Krylov vectors of one domain are held by one workgroup of 512 threads,
 * 16 entries each: solves (and steps) need Nb <= 8192 and return
 * KFBI_ENOTSUP above it.
 * Returns ENOCONV when max_iter is reached first (outputs still written). */
int kfbi_helmholtz_solve(kfbi_domain *dom, double kappa_re, double kappa_im,
                         const void *f_grid, const void *f_gamma,
                         const void *g_gamma, void *u_grid_out, void *phi_inout,
                         const kfbi_solve_opts *opts, kfbi_solve_stats *stats);

/* Solve lap u - kappa u = f in Omega, du/dn = g_N on Gamma (n the outward
 * normal) through the second-kind equation (3.19) for the density psi of
 * u = Yf - V psi (eq. 3.20).  Each application of its operator is one
 * interface problem (3.29) ([u] = 0, [u_n] = psi, the table after eq. 3.30)
 * read out as the interior normal derivative at the collocation points: the
 * first-order coefficients of the six-point fit of section 3.2.6.
 * gn_gamma: du/dn at the collocation points; f_grid / f_gamma as for
 * kfbi_helmholtz_solve; u_grid_out the grid solution (inside nodes);
 * psi_inout (nullable) warm start on entry and density on exit; trace_out
 * (nullable) receives U+, the solution's interior limit at the collocation
 * points.  opts and stats as for kfbi_helmholtz_solve (GMRES or the
 * Richardson form of eq. 3.22; FP64 or mixed precision).  kappa = 0 is
 * refused (KFBI_EINVAL: the solution is then not unique); KFBI_ENOTSUP when
 * Nb exceeds 8192 (real) or 4096 (complex) or the domain's correction
 * windows cannot be merged.  Returns ENOCONV as kfbi_helmholtz_solve. */
int kfbi_neumann_solve(kfbi_domain *dom, double kappa_re, double kappa_im,
                       const void *f_grid, const void *f_gamma,
                       const void *gn_gamma, void *u_grid_out, void *psi_inout,
                       void *trace_out, const kfbi_solve_opts *opts, kfbi_solve_stats *stats);

/* Time-step parameters (section 3.1).
 *   HEAT: c u_t = lap u + s; Crank-Nicolson, kappa = 2c/tau (c = diffusivity,
 *         0 means 1).
 *   WAVE: u_tt = lap u; implicit theta-scheme (eq. 3.5), kappa = 1/(theta
 *         tau^2); theta in (0, 1/2].
 *   SCHRODINGER: i u_t = lap u + v u + w |u|^2 u (eq. 2.2); Strang splitting,
 *         kappa = 2i/tau, or Godunov splitting, kappa = i/tau (split, see
 *         kfbi_split; any other value is KFBI_EINVAL); the carried state is
 *         u* for Strang and u^n for Godunov; v_grid / v_gamma are device arrays (float64) of the
 *         potential on the grid and at the collocation points (nullable: 0),
 *         copied by kfbi_stepper_create (which waits for the copy), so they
 *         need not outlive the call.
 * The domain must be REAL for HEAT and WAVE, COMPLEX for SCHRODINGER.
 * bc: KFBI_BC_DIRICHLET (g of each step is u on Gamma) or KFBI_BC_NEUMANN
 * (g is du/dn; each step solves eq. 3.19 and carries the recurrence on
 * Gamma with the extracted trace U+ of the new solution). */
typedef struct {
    double tau;
    double theta;
    double diffusivity;
    double w;
    const void *v_grid;
    const void *v_gamma;
    int32_t bc;
    int32_t split;       /* SCHRODINGER only: kfbi_split (0, Strang, by default) */
} kfbi_step_params;

int kfbi_stepper_create(kfbi_domain *dom, int32_t equation,
                        const kfbi_step_params *params, kfbi_stepper **out);
int kfbi_stepper_destroy(kfbi_stepper *st);

/* Initial state "by initial boundary condition" (Procedure 3a):
 * u0 and lap u0 on the grid and on Gamma (all required); for WAVE also
 * u^{-1} and lap u^{-1} (the state one step before t = 0), else NULL. */
int kfbi_stepper_init(kfbi_stepper *st, const void *u0_grid, const void *lap_u0_grid,
                      const void *u0_gamma, const void *lap_u0_gamma,
                      const void *uprev_grid, const void *lap_uprev_grid,
                      const void *uprev_gamma, const void *lap_uprev_gamma);

/* Checkpoint and restart of a stepper.  The state of the time scheme is the
 * carried right-hand-side term of its recurrence on the grid and on Gamma
 * (heat: G, eq. 3.4; wave: F^{n+1} and F^n, the recurrence after eq. 3.7;
 * Schroedinger: u*, the algorithm after eq. 3.12) plus the density of the
 * last solve, which warm-starts the next one.  The blob is opaque: a 64-byte
 * header (equation, M, Nb, scalar type, boundary condition, tau, kappa)
 * followed by those arrays
 * in the domain's element type.  dst / src are caller-owned device buffers
 * of at least kfbi_stepper_state_bytes() bytes.  get_state and set_state
 * synchronise the domain stream.  set_state accepts only a blob written by
 * a stepper with the same equation, grid, collocation count, scalar type,
 * boundary condition and kappa (else KFBI_EINVAL). */
int kfbi_stepper_state_bytes(const kfbi_stepper *st, uint64_t *bytes);
int kfbi_stepper_get_state(kfbi_stepper *st, void *dst, uint64_t bytes);
int kfbi_stepper_set_state(kfbi_stepper *st, const void *src, uint64_t bytes);

/* One Crank-Nicolson step t^n -> t^{n+1} (eqs. 3.2-3.4): g_next is u on
 * Gamma at t^{n+1} (du/dn for a Neumann stepper); src_grid / src_gamma
 * (nullable) hold s^n + s^{n+1}.  u_grid_out receives u^{n+1}. */
int kfbi_step_heat(kfbi_stepper *st, const void *g_next_gamma, const void *src_grid,
                   const void *src_gamma, void *u_grid_out,
                   const kfbi_solve_opts *opts, kfbi_solve_stats *stats);

/* One theta-scheme step (eqs. 3.5-3.7 and the F recurrence after them). */
int kfbi_step_wave(kfbi_stepper *st, const void *g_next_gamma, void *u_grid_out,
                   const kfbi_solve_opts *opts, kfbi_solve_stats *stats);

/* One Schroedinger step: the Strang three-step algorithm after eq. 3.12, or
 * the Godunov step S^A(tau) S^B(tau) of a stepper created with
 * KFBI_SPLIT_GODUNOV (see kfbi_split). */
int kfbi_step_schrodinger(kfbi_stepper *st, const void *g_next_gamma, void *u_grid_out,
                          const kfbi_solve_opts *opts, kfbi_solve_stats *stats);

/* Batched modified-Helmholtz solves (eq. 3.13 through eqs. 3.17-3.18, one
 * problem per member domain).  A batch holds n domains of one scalar type
 * (all REAL or all COMPLEX) that share one stream; every kernel launch of a
 * batched solve runs the blocks of all members, each member with its own
 * GMRES state, so members of different grid sizes, curves and kappa advance
 * together and finished members drop out on the device.  Members must have
 * M >= 64 and Nb <= 8192 (real) or 4096 (complex); a domain may belong to
 * several batches but must not be used by two calls at once.
 * kfbi_batch_create copies the launch tables to the device (it
 * synchronises the stream); kfbi_batch_destroy frees only the batch's own
 * memory.  Errors: KFBI_EINVAL (null or empty, mixed streams, mixed scalar
 * types), KFBI_ENOTSUP (M < 64, too large), KFBI_ENOMEM. */
int kfbi_batch_create(kfbi_domain *const *doms, int32_t n, kfbi_batch **out);
int kfbi_batch_destroy(kfbi_batch *b);

/* n solves, member q with kappa = kappa_re[q] + i kappa_im[q] (kappa_im
 * NULL: real kappa; nonzero entries need a complex batch) and the device
 * arrays f_grid[q] (grid, f at inside nodes), f_gamma[q] and g_gamma[q] (Nb
 * values on Gamma), of the batch's element type; u_grid_out[q] (grid) and
 * phi_inout[q] (density: warm start in, result out) may be NULL as arrays
 * or entries.  kappa_re, f_grid, ... are host arrays of n entries.  opts as
 * for kfbi_helmholtz_solve (the precision field selects FP64 or the FP32 /
 * complex64 inner solves for all members); stats, if not NULL, receives n
 * entries, device_ms the time of the whole batch.  Returns KFBI_ENOCONV when
 * some member reached max_iter (all outputs are still written). */
int kfbi_batch_helmholtz(kfbi_batch *b, const double *kappa_re, const double *kappa_im,
                         const void *const *f_grid, const void *const *f_gamma,
                         const void *const *g_gamma, void *const *u_grid_out, void *const *phi_inout,
                         const kfbi_solve_opts *opts, kfbi_solve_stats *stats);

/* One time step of every active member stepper: the Crank-Nicolson step of
 * kfbi_step_heat (eq. 3.4) or the theta-scheme step of kfbi_step_wave
 * (eqs. 3.5-3.7) in a real batch, the splitting step of
 * kfbi_step_schrodinger in a complex batch, with the members'
 * modified-Helmholtz solves batched as in kfbi_batch_helmholtz.  st[q] is
 * an initialised stepper on member q's domain (heat or wave: real batch;
 * Schroedinger: complex batch).  active (host, n bytes; NULL: all) selects the
 * members that step; for each, g_next[q] is g on Gamma at the new time and
 * u_grid_out[q] (grid) receives u; a heat member may pass its sources as
 * kfbi_step_heat does (src_grid[q], src_gamma[q]; the arrays or entries may
 * be NULL).  Members not active are untouched (state and outputs).  st,
 * g_next, ... are host arrays of n entries; the results are on the batch
 * stream in stream order.  stats (n entries, zero for members not active)
 * as kfbi_batch_helmholtz.  Errors: KFBI_EINVAL (null, stepper not on the
 * member's domain, not initialised, equation not of the batch's scalar
 * type), KFBI_ENOTSUP
 * (a Neumann stepper: batched steps are Dirichlet only), KFBI_ENOCONV
 * (some member reached max_iter; its step still completes). */
int kfbi_batch_step(kfbi_batch *b, kfbi_stepper *const *st, const uint8_t *active,
                    const void *const *g_next, const void *const *src_grid, const void *const *src_gamma,
                    void *const *u_grid_out, const kfbi_solve_opts *opts, kfbi_solve_stats *stats);

/* Launch shape of the tridiagonal kernel (the y-direction solves of the
 * five-point system, section 3.4) per class of members with equal M.  The
 * first kfbi_batch_helmholtz of each precision (unless KFBI_BATCH_NO_TUNE)
 * times, on the members' own tables, every shape that computes the same
 * values (1, 2 or 4 sine modes per 64-, 128- or 256-lane workgroup, and 8
 * per 512 lanes in the register-row kernel; the sparse input staged in LDS
 * or read from HBM; the right-hand side and solution held in an LDS tile or
 * in registers) and keeps the fastest.  Writes min(cap, rows) rows of 6 int32 {M, kind (0: sparse FP64,
 * 1: with dense input FP64, 2: sparse FP32), modes per workgroup, staged,
 * tuned, register rows} to rows (may be NULL when cap is 0), the time of the
 * kept shape in microseconds per launch of the class (or -1 when untuned) to
 * us (may be NULL), and the row count to n_rows.  Errors: KFBI_EINVAL.
 * The environment variable KFBI_TRIDIAG_KERNEL = "tile" or "rows", when set,
 * limits this timing and that of single domains (at a domain's first solve)
 * to the LDS-tile or the register-row kernel, "tile:<mb>" / "rows:<mb>" also
 * to mb modes per workgroup, and "<kernel>:<mb>:<s>" also to the sparse input
 * staged in LDS (s = 1) or not (s = 0) (for tests and diagnosis; the values
 * are the same). */
int kfbi_batch_tuning(const kfbi_batch *b, int32_t cap, int32_t *rows, double *us, int32_t *n_rows);

/* Per-kernel device timing (instrumentation for benchmarks).  When enabled,
 * every launch of the listed kernels of this domain is bracketed by two HIP
 * events on the domain stream; launches after the solve had finished on the
 * device are not counted (in the mixed-precision schedule the grid-solve
 * launches of the precision a slot did not use are counted as launches of
 * near-zero length).  kfbi_profile_enable(dom, 1)
 * resets the counters; kfbi_profile_read waits for the outstanding events
 * and fills KFBI_K_COUNT entries: launches, summed event time and summed
 * algorithmic bytes (the bytes the kernel must move by design: its dense
 * inputs and outputs, not cache re-reads). */
enum {
    KFBI_K_TRIDIAG_SPARSE = 0,  /* y-solve, right-hand side synthesised from corrections */
    KFBI_K_TRIDIAG_DENSE = 1,   /* y-solve reading a dense x-transformed right-hand side */
    KFBI_K_DST = 2,             /* dense DST-I along x                                   */
    KFBI_K_IDST = 3,            /* dense inverse DST-I along x to the grid               */
    KFBI_K_EVAL_NODES = 4,      /* grid solution at extraction-stencil nodes             */
    KFBI_K_CORRECTIONS = 5,
    KFBI_K_EXTRACT = 6,
    KFBI_K_ARNOLDI = 7,
    KFBI_K_COUNT = 8
};
typedef struct {
    int64_t launches;
    double total_ms;
    double bytes;
} kfbi_kernel_prof;

int kfbi_profile_enable(kfbi_domain *dom, int32_t on);
int kfbi_profile_read(kfbi_domain *dom, kfbi_kernel_prof *out);

/* Replay timing: `reps` back-to-back launches of one FP64 grid-solve kernel
 * of this domain on its current internal buffers, between two HIP events on
 * the domain stream; writes the average launch duration (ms) and the
 * algorithmic bytes of one launch.  kind: KFBI_K_TRIDIAG_SPARSE (the
 * corrections of the last solve's density -> mode-space solution, the form
 * used in every matrix-vector product), KFBI_K_TRIDIAG_DENSE (dense right-hand side ->
 * mode-space solution) or KFBI_K_EVAL_NODES (mode-space solution -> stencil
 * values), KFBI_K_CORRECTIONS (the corrections of the last solve's density
 * by the merged per-kappa operator, as in every matrix-vector product) or
 * KFBI_K_ARNOLDI (the GMRES control kernel: the same Arnoldi
 * step on column min(5, last column) of the last solve's basis, repeated in
 * a replay mode that leaves the control block as it was).  Needs a completed solve on the domain (it reuses
 * the last kappa's coefficients and the last solve's data); overwrites the
 * domain's internal scratch only.  Blocks until the launches have finished.
 * Errors: KFBI_EINVAL (null pointer, reps outside 1..100000, other kind, no
 * solve yet), KFBI_ENOTSUP (corrections or control kernel of a domain
 * without the device-driven schedule). */
int kfbi_profile_replay(kfbi_domain *dom, int32_t kind, int32_t reps, double *avg_ms,
                        double *bytes_per_launch);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * five-point solve as kfbi_grid_solve, with the same arguments and results,
 * but its two mode-space intermediates (R^ and U^, (M-1)^2 elements each)
 * live in a device array the library holds once per GPU, of
 * KFBI_NOALLOC_SCRATCH_BYTES (16 MiB), from its first use on that GPU until
 * the process ends; the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine) and needs a domain made by
 * kfbi_domain_create (whose set-up looks up the array's address on the
 * domain's device).  Limit: 2 (M-1)^2 w bytes <= the array (w = 8 real,
 * 16 complex: M <= 1024 real, M <= 512 complex), else KFBI_ENOTSUP with a
 * message.  Every call on a GPU shares that GPU's array and leaves its
 * contents to the next: calls that overlap on one GPU (other streams, other
 * host threads) race and must be serialised by the caller.  Nothing in the
 * array needs to start at zero: each call writes every entry before it reads
 * it.  Errors: KFBI_EINVAL (null argument, complex kappa on a real domain),
 * KFBI_ENOTSUP (too large), KFBI_EDEVICE. */
#define KFBI_NOALLOC_SCRATCH_BYTES (16u << 20)
int kfbi_grid_solve_noalloc(kfbi_domain *dom, double kappa_re, double kappa_im,
                            const void *rhs, void *u_out);

#ifdef __cplusplus
}
#endif
#endif /* KFBI_H */
