/*
 * mrcm.h - C ABI of the MI355X (gfx950) library for the Darcy solve of the
 * Multiscale Robin Coupled Method (MRCM).
 *
 * The problem (paper, section 2, eq. (Darcy)): u = -lambda(s) K grad p,
 * div u = q in Omega, p = p_b on the Dirichlet part of the boundary and
 * u.n = u_b on the Neumann part.  The method (section 3, eqs. (mrc1),
 * (mrc2), (beta)): split Omega into equal rectangular subdomains, solve one
 * Robin problem per subdomain and interface basis function, couple the
 * pieces through weak flux and pressure continuity on the skeleton, and
 * return one fine-scale pressure and a conservative fine-scale flux.
 *
 * Discretisation: cell-centred two-point fluxes on a uniform Cartesian
 * grid (the quadrature form of lowest-order mixed elements), with the
 * Robin face law F = T_R (p_c - g), T_R = |f| kappa_c / (d + alpha H),
 * g = P_H - beta U_H (n . n_i), beta = alpha H / kappa_c.
 *
 * Index conventions (all arrays flat, row-major, float64):
 *   cell (i, j), i along x        -> j*nx + i                 (nx*ny)
 *   x-face at x = i*hx in row j   -> j*(nx+1) + i             ((nx+1)*ny)
 *   y-face at y = j*hy in col i   -> j*nx + i                 (nx*(ny+1))
 *   boundary sides                -> 0 W (x=0), 1 E, 2 S (y=0), 3 N
 *   interfaces: vertical (between subdomains (I,J),(I+1,J)) first as
 *   J*(SX-1)+I, then horizontal (between (I,J),(I,J+1)) as nV + J*SX + I;
 *   dofs of interface e: e*(nP+nU) + [P_0..P_{nP-1}, U_0..U_{nU-1}].
 * The fixed skeleton normal points +x / +y, i.e. out of the subdomain with
 * the smaller index (section 3).
 *
 * Every entry point returns an int status (0 = MRCM_OK) and never throws.
 * A context is not re-entrant: use one per host thread.  All device work
 * is issued on the context's HIP stream.
 */
#ifndef MRCM_H
#define MRCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrcm_ctx mrcm_ctx; /* opaque; owns all of its device memory */

enum {
  MRCM_OK = 0,
  MRCM_E_INVAL = 1,   /* an argument is out of range; the context is unchanged */
  MRCM_E_NOMEM = 2,   /* device or host allocation failed */
  MRCM_E_HIP = 3,     /* a HIP runtime call failed (message in mrcm_last_error) */
  MRCM_E_NOT_SPD = 4, /* a local or interface pivot was not positive/nonzero */
  MRCM_E_NO_CONV = 5, /* an iterative refinement did not converge and no fallback is left */
  MRCM_E_STATE = 6,   /* calls out of order (e.g. fine_flux before solve) */
  MRCM_E_UNSUPPORTED = 7 /* a valid combination this build has no kernel for */
};

enum { MRCM_BC_NEUMANN = 0, MRCM_BC_DIRICHLET = 1 };

/* Interface spaces: piecewise-constant functions on the fine faces of each
 * interface (section 3).  LINEAR: the two nodal linear functions for
 * pressure and for flux (2 + 2 dofs per interface; the polynomial space of
 * section 3.1 with no channel).  EDGE_SOLUTION: two non-polynomial functions
 * per space built at setup from a 1-D two-point problem along each interface
 * on the absolute permeability (reduces to LINEAR for uniform K); the paper
 * does not define this space (its own physics-based spaces are those of
 * eqs. (new_basis1)-(new_basis6)), so it is a reading of "spaces built from
 * local edge solutions".  FULL: every fine-edge indicator (m + m dofs). */
enum { MRCM_SPACE_LINEAR = 0, MRCM_SPACE_EDGE_SOLUTION = 1, MRCM_SPACE_FULL = 2, MRCM_SPACE_PHYSICS = 3 };

/* Precision of the local (subdomain) factorisations.  The interface system
 * is always solved in FP64.  FP32_IR: FP32 factors and solves of the
 * diagonally scaled local system, FP64 residuals and iterative refinement
 * until the last correction is below 1e-12 of the solution, per-subdomain
 * FP64 fallback when refinement stalls (16 x 16 subdomains with 2 + 2 dofs,
 * 32 x 32 subdomains with 4 dofs; other sizes MRCM_E_UNSUPPORTED).
 * SURROGATE (16 x 16, 2 + 2 dofs): the basis functions of each
 * subdomain are predicted by the convolutional network set with
 * mrcm_set_surrogate and accepted only if every column's FP64 residual in
 * the local problem is below 1e-6 of its right-hand side; every other
 * subdomain is solved by the FP64 path. */
enum { MRCM_PREC_FP64 = 0, MRCM_PREC_FP32_IR = 1, MRCM_PREC_SURROGATE = 2 };

typedef struct {
  int32_t nx, ny; /* cells; > 0 */
  double lx, ly;  /* domain [0,lx] x [0,ly]; > 0 */
} mrcm_grid;

typedef struct {
  int32_t kind[4];        /* per side W,E,S,N: MRCM_BC_NEUMANN or MRCM_BC_DIRICHLET */
  const double* value[4]; /* host arrays: W,E: ny values (bottom to top), S,N: nx values
                             (left to right).  Dirichlet: boundary pressure p_b;
                             Neumann: outward normal velocity u_b.  NULL = all zero. */
} mrcm_bc;

typedef struct {
  double mu_w, mu_o; /* phase viscosities; lambda(s) = s^2/mu_w + (1-s)^2/mu_o
                        (eq. (fluxos1) with k_rw = s^2, k_ro = (1-s)^2, section 5) */
} mrcm_fluid;

/* Phase times are read from the GPU's constant-rate clock by the kernels that
   open and close each phase, so timing adds no work to the stream. */
typedef struct {
  double ms_local;       /* last solve: assemble + factor + basis solves + traces */
  double ms_interface;   /* last solve: interface system (FP64) */
  double ms_flux;        /* last fine_flux: compose + stitch + conservation */
  int32_t n_sub;         /* subdomains */
  int32_t n_dof;         /* interface unknowns */
  int32_t ir_iters_max;  /* FP32_IR: largest refinement count over subdomains */
  int32_t fallbacks;     /* FP32_IR / SURROGATE: subdomains re-solved in FP64 */
  double interface_residual; /* max_i |b - A x|_i / max_i (|b_i| + sum_j |A_ij x_j|)
                                of the interface solve (a normwise backward error) */
  double ms_surrogate;   /* SURROGATE: network inference + residual gate */
  int32_t interface_ir_steps; /* refinement steps of the interface solve (taken while
                                 max |b - A x| > tol max |b|, at most max_steps: see
                                 mrcm_set_interface_refinement) */
  double interface_gflop;      /* algorithmic work of one interface solve (elimination
                                  of the nested-dissection fronts, back substitution,
                                  extend-add), GFLOP; fixed by the plan */
  int32_t interface_launches;  /* kernel launches of one interface solve */
} mrcm_stats;

/* Set up a solver for one grid, permeability field and decomposition
 * (section 3: non-overlapping subdomains, interface spaces, Robin alpha).
 *  out        : receives the new context (caller destroys it).
 *  g          : grid; nx % sub_nx == 0 and ny % sub_ny == 0 required.
 *  perm       : host, nx*ny absolute permeabilities K > 0 (finite).
 *  sub_nx/ny  : subdomain size in cells; this build requires
 *               sub_nx == sub_ny in {4, 8, 16, 32}.
 *  space      : MRCM_SPACE_*; p_dofs/u_dofs must match the space (2, 2 for
 *               LINEAR and EDGE_SOLUTION, sub_nx each for FULL, 4, 4 for
 *               PHYSICS).  PHYSICS: the channel and barrier spaces of section
 *               3.1, eqs. (new_basis1)-(new_basis6), built per interface from
 *               K: faces whose conductance (harmonic mean of K across the
 *               face) is at least 10 times the interface's median form
 *               channels, at most a tenth of it barriers; at most 2 channels
 *               and 1 barrier are kept (the widest); a space with no
 *               structure of its kind is linear.  The 4 + 4 dofs per
 *               interface are slots: the interface's pressure functions
 *               first, then its flux functions; unused slots are fixed to 0.
 *               FP64 only (the generic kernels).
 *  alpha_per_interface : host, one alpha > 0 per interface (eq. (beta)), or
 *               NULL to use alpha_scalar everywhere.
 *  bc, source : boundary data (deep-copied) and q per unit area (host,
 *               nx*ny, NULL = 0).  With no Dirichlet side the pressure is
 *               defined up to a constant: the first pressure dof of
 *               interface 0 is fixed to zero in place of its (dependent)
 *               flux-continuity equation and the returned cell pressure is
 *               shifted to zero mean.
 *  fluid      : viscosities for mrcm_update_mobility from saturation.
 *  precision  : MRCM_PREC_*.
 *  hip_stream : hipStream_t to issue work on, or NULL for a library-owned
 *               stream.
 * Host inputs are copied before return.  Errors: MRCM_E_INVAL (bad sizes,
 * non-positive or non-finite K or alpha, bad space/dof combination),
 * MRCM_E_UNSUPPORTED, MRCM_E_NOMEM, MRCM_E_HIP.  The default mobility is
 * lambda = 1 (single phase). */
int mrcm_setup(mrcm_ctx** out, const mrcm_grid* g, const double* perm, int32_t sub_nx,
               int32_t sub_ny, int32_t space, int32_t p_dofs, int32_t u_dofs,
               const double* alpha_per_interface, double alpha_scalar, const mrcm_bc* bc,
               const double* source, const mrcm_fluid* fluid, int32_t precision,
               void* hip_stream);

/* Set the total mobility used by the next mrcm_solve: kappa = lambda K
 * (section 3).  values: nx*ny saturations in [0,1] (values_are_lambda = 0;
 * lambda is evaluated on the GPU with eq. (fluxos1)) or mobilities > 0
 * (values_are_lambda = 1).  on_device = 1: values is a device pointer read
 * by a kernel on the context's stream; it must stay valid and unchanged
 * until the next mrcm_solve returns (work that produced it on another
 * stream must be complete).  on_device = 0: host array, copied before
 * return.  Values are validated on
 * the GPU during the next solve: a non-finite or non-positive lambda makes
 * that solve fail with MRCM_E_INVAL. */
int mrcm_update_mobility(mrcm_ctx* ctx, const double* values, int32_t values_are_lambda,
                         int32_t on_device);

/* Solve the MRCM system for the current mobility (eqs. (mrc1), (mrc2)):
 * local Robin problems and basis functions for all subdomains, then the
 * FP64 interface system.  Asynchronous except for a final status read.
 * Errors: MRCM_E_INVAL (a mobility not finite and positive), MRCM_E_NOT_SPD
 * (a zero, negative or non-finite pivot), MRCM_E_NO_CONV (the interface
 * residual is still above its failure bound after the allowed refinement
 * steps, see mrcm_set_interface_refinement: the elimination does not
 * pivot, so a nearly singular pivot shows here);
 * after any error the context has no solution (mrcm_fine_flux returns
 * MRCM_E_STATE) until a solve succeeds. */
int mrcm_solve(mrcm_ctx* ctx);

/* Stopping rule of the FP32 + FP64 refinement of the local solves
 * (MRCM_PREC_FP32_IR; spec precision extension, local problems of
 * eq. (mrc1)): refinement stops once the largest correction of a subdomain is
 * at most tol of its largest solution value, or after max_steps steps; a
 * subdomain that ends above tol (or met a bad FP32 pivot) is re-solved by the
 * FP64 path and counted in mrcm_stats.fallbacks.  Defaults: 8 steps, 1e-12
 * (near FP64 accuracy: the stitch's cell balances rest on it).
 * max_steps = 0 sends every subdomain to the FP64 re-solve.  Takes effect at
 * the next solve.  Errors: MRCM_E_INVAL unless 0 <= max_steps <= 64 and
 * 0 < tol < 1; MRCM_E_STATE for another precision. */
int mrcm_set_refinement(mrcm_ctx* ctx, int32_t max_steps, double tol);

/* Stopping rule of the iterative refinement of the FP64 interface solve
 * (eq. (mrc2)): after the direct solve, refinement steps are taken while
 * max |b - A x| > tol S, S = max_i (|b_i| + sum_j |A_ij x_j|), at most
 * max_steps; if the residual is then above fail_tol S the solve fails with
 * MRCM_E_NO_CONV.  Measured against S (a normwise backward error), the
 * residual that FP64 rounding leaves is about eps wherever the solution
 * is accurate, also where |A| |x| is far above |b|.  Defaults: 3 steps;
 * tol 1e-14 (FP64 and SURROGATE), 1e-12 (FP32_IR); fail_tol 1e-10.  Takes
 * effect at the next solve.  Errors: MRCM_E_INVAL unless
 * 0 <= max_steps <= 16, 0 < tol < 1 and 0 < fail_tol < 1. */
int mrcm_set_interface_refinement(mrcm_ctx* ctx, int32_t max_steps, double tol, double fail_tol);

/* Adaptive Robin parameter (section 3.1, last paragraph; section 5.5):
 * alpha_channel on every interface crossed by a high-permeability channel
 * (the classification of MRCM_SPACE_PHYSICS, made for every space) and
 * alpha_other elsewhere; replaces the alpha given to mrcm_setup.  Takes
 * effect at the next solve.  Errors: MRCM_E_INVAL unless both are finite
 * and > 0. */
int mrcm_set_adaptive_alpha(mrcm_ctx* ctx, double alpha_channel, double alpha_other);

/* Gravity variant of the pressure equation (section 5.5, eqs. (Darcy_wg) and
 * (fluxos1_wg)): u = -K (lambda grad p - lambda_g g grad h), gravity along
 * y, with gravity = g dh/dy (a constant; 0 switches the variant off) and
 * lambda_g = lambda_w rho_w + lambda_o rho_o.  The local matrices are those
 * without gravity; the term enters the data of the local problems (the
 * particular solution) and every face flux: on a half cell of
 * transmissibility t and centre-to-face distance d the flux carries
 * t d gravity (lambda_g / lambda) (n . e_y), the face pressure is
 * eliminated between the two half cells as in the two-point law, a Robin
 * face carries T_R d gravity (lambda_g / lambda) (n . e_y), and Neumann faces
 * keep their prescribed total flux.  With the variant on, the mobility must
 * come from a saturation (mrcm_update_mobility / mrcm_step with
 * values_are_lambda = 0), which also sets lambda_g / lambda per cell.
 * Allocates one array of nx * ny doubles on the first call that enables
 * gravity.  Errors: MRCM_E_INVAL for values that are not finite;
 * MRCM_E_UNSUPPORTED for MRCM_PREC_SURROGATE.  With gravity on, the
 * transport calls (mrcm_transport_step, mrcm_si_step, mrcm_sfi_step) return
 * MRCM_E_UNSUPPORTED (their water flux has no gravity segregation term),
 * mrcm_update_mobility / mrcm_step with lambda values return MRCM_E_INVAL,
 * and a solve before any saturation was given returns MRCM_E_STATE. */
int mrcm_set_gravity(mrcm_ctx* ctx, double gravity, double rho_w, double rho_o);

/* Reconstruct fine-scale output from the last solve:
 *  p  : nx*ny composed multiscale cell pressure (basis functions combined
 *       with the interface solution, section 3);
 *  ux : (nx+1)*ny normal velocity in +x on x-faces;
 *  uy : nx*(ny+1) normal velocity in +y on y-faces.
 * Velocities are the stitched field: on skeleton faces the average of the
 * two one-sided Robin fluxes, inside every subdomain the fluxes of a
 * Neumann re-solve with that interface flux, so that every cell balances.
 *  on_device : 1 if p/ux/uy are device pointers (written in place by the
 *              kernels; distinct, non-overlapping, 8-byte aligned), 0 for
 *              host arrays (copied from the context's buffers); any of them
 *              may be NULL to skip it.
 *  max_cell_imbalance : if not NULL receives max over cells of
 *              |net outflow - q|V|| / max |face flux|.
 * Synchronous: outputs are valid on return.  MRCM_E_STATE before the first
 * successful solve.  The stitch of a subdomain with no Dirichlet face is a
 * Neumann problem whose data sum to zero up to the rounding of the composed
 * solution; that defect is removed evenly from its cells (a uniform source
 * correction at rounding level), so it appears in max_cell_imbalance
 * divided by the subdomain's cell count. */
int mrcm_fine_flux(mrcm_ctx* ctx, double* p, double* ux, double* uy, int32_t on_device,
                   double* max_cell_imbalance);

/* mrcm_fine_flux for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, outputs, synchronisation and errors, and it allocates
 * nothing.  Its scratch (the stitch's per-subdomain statistics and their
 * reduction, 3 doubles per subdomain) is a static device array of the
 * library, one per GPU, held until the process ends, sized for at most
 * 65536 subdomains (1.5 MB): larger contexts get MRCM_E_INVAL.  Every call on
 * one GPU uses that GPU's array, so calls that overlap on one GPU (contexts
 * on different streams or threads) race; the array keeps the last call's
 * contents, and every value a call reads from it that call has written. */
int mrcm_fine_flux_static(mrcm_ctx* ctx, double* p, double* ux, double* uy, int32_t on_device,
                          double* max_cell_imbalance);

/* One step of the pressure solve in one call: the mobility update, the
 * solve and the fine-scale reconstruction, with one synchronisation where
 * mrcm_update_mobility + mrcm_solve + mrcm_fine_flux take two or three.
 *  values, values_are_lambda, values_on_device : as mrcm_update_mobility
 *              (values = NULL keeps the current mobility; a host array is
 *              read before the call returns);
 *  p, ux, uy, outputs_on_device, max_cell_imbalance : as mrcm_fine_flux.
 * The reconstruction is enqueued before the solve's status is known; if
 * the interface solve needs refinement it is refined (one synchronisation
 * per step) and the reconstruction is done again.  Results, statistics and
 * errors are those of the three calls; on an error the outputs are
 * unspecified.  MRCM_E_STATE for a MRCM_PREC_SURROGATE context without a
 * network.  Synchronous: outputs are valid on return. */
int mrcm_step(mrcm_ctx* ctx, const double* values, int32_t values_are_lambda,
              int32_t values_on_device, double* p, double* ux, double* uy,
              int32_t outputs_on_device, double* max_cell_imbalance);

/* ------------------------------------------------------------------------
 * Implicit transport of the water saturation (section 4): one implicit
 * Euler step of eq. (BL2D) with first-order upwind fluxes
 * (eqs. (BL2D_Newton2), (fluxes_impli), (up_fluxes_impli)), solved by
 * Newton's method (eqs. (BL2D_Newton8), (BL2D_Newton7)) with the
 * inflection-point strategy: every iterate is kept in [0, 1] and an update
 * that crosses the inflection point of f is halved.  Each Newton system is
 * solved by BiCGSTAB on the Jacobi-scaled Jacobian to a relative residual
 * of 1e-12 (at most 400 iterations).
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t newton_iters;    /* Newton iterations taken */
  int32_t linear_iters;    /* BiCGSTAB iterations, summed over them */
  int32_t converged;       /* 1 if the last change was <= eta */
  int32_t linear_failures; /* Newton iterations whose linear solve stopped short */
  double last_change;      /* L2 norm sqrt(sum V (s^{nu+1} - s^nu)^2) of the last change */
  double ms;               /* wall time of the call */
} mrcm_transport_stats;

/* One transport step from s_old to s_new with the face velocities ux, uy of
 * the last Darcy solve (frozen over the step, eq. (BL2D_Newton)).
 *  s_old, s_new : device, nx*ny saturations (distinct, non-overlapping);
 *                 s_new receives the new time level.
 *  ux, uy       : device, the +x / +y face velocities in the layout of
 *                 mrcm_fine_flux ((nx+1)*ny and nx*(ny+1)); the face flux is
 *                 velocity times face length.
 *  dt           : time step (> 0); porosity is scaled out (time in pore
 *                 volumes).
 *  s_inflow     : saturation of the water entering through boundary faces
 *                 with inflow (eq. (BL2D), inlet condition), in [0, 1].
 *                 Sources of the context: an injector (q > 0) injects water
 *                 only; a producer (q < 0) produces the mixture, f(s) q.
 *  eta          : Newton stops when the L2 norm of the change is <= eta
 *                 (section 5 uses 1e-6).
 *  max_newton   : iteration cap (1 .. 1000).
 *  stats        : may be NULL.
 * Synchronous.  Errors: MRCM_E_INVAL (bad arguments; nothing is written),
 * MRCM_E_NO_CONV (no convergence within max_newton: s_new holds the last
 * iterate), MRCM_E_HIP. */
int mrcm_transport_step(mrcm_ctx* ctx, const double* s_old, double* s_new, const double* ux,
                        const double* uy, double dt, double s_inflow, double eta, int32_t max_newton,
                        mrcm_transport_stats* stats);

/* One step of the sequential implicit scheme (section 4): the transport
 * step from s_old with the velocities (ux, uy) of the last Darcy solve
 * (u^n), then the Darcy solve (mrcm_step) with the new saturation, which
 * writes p, ux, uy (u^{n+1}) in place.  All arrays are device arrays in the
 * layouts of mrcm_transport_step and mrcm_fine_flux (p may be NULL).  Start
 * a run with mrcm_step on s^0 to get u^0.  Errors: those of the two calls;
 * stats (may be NULL) are the transport's. */
int mrcm_si_step(mrcm_ctx* ctx, const double* s_old, double* s_new, double* p, double* ux,
                 double* uy, double dt, double s_inflow, double eta, int32_t max_newton,
                 mrcm_transport_stats* stats);

typedef struct {
  int32_t outer_iters;   /* Darcy + transport iterations */
  int32_t newton_iters;  /* Newton iterations, summed over the transport solves */
  int32_t converged;     /* 1 if the last change was below outer_tol */
  double last_change;    /* max |s^{k+1} - s^k| of the last outer iteration */
  double ms;             /* wall time of the call */
} mrcm_sfi_stats;

/* One step of the sequential fully implicit scheme (section 5.4): from
 * s^{n+1,0} = s_old, repeat the Darcy solve with the current iterate and the
 * transport step from s_old with its velocities, until the largest change
 * of the saturation between successive outer iterations is below outer_tol
 * (the paper: 1e-4, with eta = 1e-6) or max_outer iterations.  s_new
 * receives the last iterate; p, ux, uy the Darcy solution of the iterate
 * before it (device arrays, as in mrcm_si_step; p may be NULL).  Errors:
 * MRCM_E_INVAL, MRCM_E_NO_CONV (outer loop or a transport solve), and those
 * of mrcm_step. */
int mrcm_sfi_step(mrcm_ctx* ctx, const double* s_old, double* s_new, double* p, double* ux,
                  double* uy, double dt, double s_inflow, double eta, int32_t max_newton,
                  double outer_tol, int32_t max_outer, mrcm_sfi_stats* stats);

/* Statistics of the last solve / fine_flux. */
int mrcm_get_stats(const mrcm_ctx* ctx, mrcm_stats* stats);

/* Number of interface unknowns and of subdomains, and the column count R
 * (1 + 4*(nP+nU)) of the per-subdomain basis-function block. */
int mrcm_get_sizes(const mrcm_ctx* ctx, int32_t* n_dof, int32_t* n_sub, int32_t* n_cols);

/* Inspection of intermediate results of the last solve (host outputs,
 * synchronous).  Used by parity tests of the individual steps.
 *  mrcm_get_interface_solution : n_dof values (P_H, U_H coefficients).
 *  mrcm_get_local_blocks : n_sub * (R-1) * R values.  Block of subdomain
 *     sd, row r, column c at [sd*(R-1)*R + r*R + c]: rows and the first R-1
 *     columns follow the subdomain's W, E, S, N interfaces (nP+nU each,
 *     zero for sides on the domain boundary); column R-1 holds the
 *     right-hand side.  Rows of flux (U) dofs are the negated
 *     pressure-continuity equations: a block is then symmetric except for
 *     the couplings between the pressure and flux dofs of one edge, which
 *     are antisymmetric and cancel between the edge's two subdomains, so
 *     that the assembled interface matrix is symmetric.
 *  mrcm_get_basis : n_sub * R * sub_nx*sub_ny values, column-major per
 *     subdomain: [sd][col][l] with local cell l = ly*sub_nx + lx; column 0
 *     is the particular solution, column 1 + side*(nP+nU) + k the basis
 *     function of that dof.
 * MRCM_E_STATE before the first successful solve. */
int mrcm_get_interface_solution(mrcm_ctx* ctx, double* coeffs);
int mrcm_get_local_blocks(mrcm_ctx* ctx, double* blocks);
int mrcm_get_basis(mrcm_ctx* ctx, double* basis);

/* ------------------------------------------------------------------------
 * Learned surrogate of the local basis functions (not part of the paper's
 * method; an approximation that the residual gate of MRCM_PREC_SURROGATE
 * checks against the local problems of eq. (mrc1)).
 *
 * Network: four 3x3 convolutions, 5 -> 32 -> 32 -> 32 -> 16 channels on the
 * 16 x 16 cells of a subdomain, ReLU after the first three; BF16 weights and
 * activations, FP32 accumulation and FP32 master weights (Adam).  Tensors
 * are channels-last: inputs BF16 [batch][256][8] (channels 5..7 zero),
 * outputs and targets FP32 [batch][256][16].  Only 16 x 16 subdomains with
 * 2 + 2 interface dofs are supported.
 * Parameters (FP32, n = mrcm_cnn_num_params): for each layer l = 1..4 the
 * weights [Cout][9 taps][Cin padded] (layer 1: Cin padded to 8 and taps
 * padded to 10) followed by the Cout biases.
 * ------------------------------------------------------------------------ */
typedef struct mrcm_cnn mrcm_cnn;

/* New network with He-normal weights from `seed`, zero biases, zero Adam
 * state; workspace for batches up to max_batch.  hip_stream: NULL = own. */
int mrcm_cnn_create(mrcm_cnn** out, int32_t max_batch, uint64_t seed, void* hip_stream);
int mrcm_cnn_num_params(const mrcm_cnn* net, int32_t* n);
/* Copy the FP32 parameters out of / into the network (host arrays). */
int mrcm_cnn_get_params(mrcm_cnn* net, float* params);
int mrcm_cnn_set_params(mrcm_cnn* net, const float* params);
/* Forward pass (device pointers); synchronous. */
int mrcm_cnn_forward(mrcm_cnn* net, const void* inputs, float* outputs, int32_t batch);
/* Mean squared error against targets and its gradient with respect to the
 * parameters (device inputs, host results; grads may be NULL). */
int mrcm_cnn_loss_grad(mrcm_cnn* net, const void* inputs, const float* targets, int32_t batch,
                       float* loss, float* grads);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on one batch; *loss
 * (may be NULL) receives the batch loss before the step. */
int mrcm_cnn_train_step(mrcm_cnn* net, const void* inputs, const float* targets, int32_t batch,
                        float lr, float* loss);
void mrcm_cnn_destroy(mrcm_cnn* net);

/* Network inputs of every subdomain for the context's current mobility
 * (device BF16 [n_sub][256][8]); synchronous. */
int mrcm_surrogate_inputs(mrcm_ctx* ctx, void* inputs);
/* Training targets from the last successful solve (device FP32
 * [n_sub][256][16]); synchronous.  MRCM_E_STATE before a solve. */
int mrcm_surrogate_targets(mrcm_ctx* ctx, float* targets);
/* Copy the network's current parameters into a context set up with
 * MRCM_PREC_SURROGATE (required before its first solve). */
int mrcm_set_surrogate(mrcm_ctx* ctx, mrcm_cnn* net);

/* Residual gate of a MRCM_PREC_SURROGATE context: a predicted subdomain is
 * accepted only if every basis column x satisfies ||b - A x||_2 <= tol ||b||_2
 * in its local problem (FP64 residual; default tol = 1e-6).  Note that the
 * FP32 rounding of an exact basis function alone leaves a relative residual
 * of order 1e-6 on 16 x 16 subdomains.  MRCM_E_INVAL unless 0 < tol < inf. */
int mrcm_set_gate_tolerance(mrcm_ctx* ctx, double tol);

/* mrcm_solve of a MRCM_PREC_SURROGATE context with the basis functions
 * predicted elsewhere: predictions is a device array FP32 [n_sub][256][16]
 * in the network's output form (mrcm_surrogate_targets) that must stay
 * valid until the call returns.  The same residual gate and FP64 fallback
 * apply; no network needs to be set. */
int mrcm_solve_with_predictions(mrcm_ctx* ctx, const float* predictions);

/* Text of the last error on this context (never NULL). */
const char* mrcm_last_error(const mrcm_ctx* ctx);

/* Release the context and all its device memory.  NULL is ignored. */
void mrcm_destroy(mrcm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MRCM_H */
