/*
 * chn.h -- C ABI of the MI355X (gfx950) channel-flow RK3 hot path.
 *
 * The library advances the velocity-vorticity formulation of incompressible
 * channel flow (the paper's Appendix A: evolution equations for
 * chi = lap(u2) and omega2 = d3 u1 - d1 u3 plus the mean profiles U1, U3, with
 * a semi-implicit low-storage three-stage Runge-Kutta scheme), using
 *   - Fourier expansions in x and z with 3/2-rule dealiased products
 *     (Section 2.1), evaluated by the library's own FFT kernels;
 *   - seven-point compact finite differences on a non-uniform wall-normal
 *     mesh and banded Helmholtz/Poisson solves per Fourier mode with
 *     Dirichlet end rows (Appendix B);
 *   - constant mass flux through a time-varying mean pressure gradient
 *     (Section 2.1),
 * and provides the low-storage stage of Section 3.1: sharp Fourier cut-off
 * filtering of the velocities, the filtered products F(u_i u_j) and the
 * sub-grid stress tau_ij = F(u_i u_j) - F(u_i) F(u_j).
 *
 * Conventions shared by every entry point
 *   - All device pointers are caller-owned.  The library never allocates
 *     device memory: the caller passes one workspace of
 *     chn_workspace_bytes(cfg) bytes, 256-byte aligned, and keeps it alive
 *     until chn_destroy.  Host memory used internally is freed by chn_destroy.
 *   - Every call is ordered on the HIP stream given in the config and returns
 *     before the GPU work has finished, except where noted ("synchronises").
 *   - Spectral fields are complex128, interleaved (re, im), in layout
 *     [n2][n1/2][n3]: wall-normal node y, streamwise mode kx = 0..n1/2-1, and
 *     spanwise mode kz in FFT slot order over n3 slots; slot n3/2 (the
 *     Nyquist mode) is ignored on input and zero on output.  The kx = 0 line
 *     of a real field must be Hermitian in kz.  Physical wavenumbers are
 *     a = 2 pi kx / lx and b = 2 pi kz / lz; the channel is y in [-1, 1].
 *   - Errors: CHN_EINVAL for invalid sizes or pointers (the context is left
 *     unchanged), CHN_EDEVICE for a HIP runtime error (sticky: every later
 *     call on that context returns it), CHN_ESTATE for a call made before
 *     chn_set_state, CHN_EUNSTABLE when a sub-step's CFL number was not
 *     finite or above CHN_CFL_LIMIT (see chn_step_rk3).
 *     chn_last_error gives a message for the last failing call.
 *   - A context is bound to one stream and is not thread-safe.
 */
#ifndef CHN_H
#define CHN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chn_ctx chn_ctx;

typedef enum {
  CHN_OK = 0,
  CHN_EINVAL = 1,
  CHN_ENOMEM = 2,
  CHN_EDEVICE = 3,
  CHN_ESTATE = 4,
  CHN_EUNSTABLE = 5,
  CHN_EUNSUPPORTED = 6
} chn_status;

/* CHN_FP64: every kernel computes in float64.
 * CHN_MIXED: Fourier transforms, products and the filter stage compute in
 * float32 (with float64 accumulation of plane means); the compact
 * derivatives, banded Helmholtz/Poisson solves, mean-flow modes and
 * mass-flux correction stay float64. */
typedef enum { CHN_FP64 = 0, CHN_MIXED = 1 } chn_precision;

typedef struct {
  int32_t n1, n2, n3;   /* collocation counts in x, y (walls included), z.
                           n1, n3 even; 3*n1/2 and 3*n3/2 must factor into
                           2s and 3s; 9 <= n2 <= 2048. */
  double lx, lz;        /* periods in x and z, in units of the half height */
  double re_b;          /* bulk Reynolds number; nu = 1 / re_b */
  double mass_flux;     /* target integral of U1 over y (2 for unit bulk velocity) */
  int32_t precision;    /* chn_precision */
  const double *y;      /* HOST pointer to n2 ascending nodes, y[0] = -1,
                           y[n2-1] = 1; NULL selects y_j = tanh(g s_j)/tanh(g),
                           s_j uniform on [-1, 1], with the largest g in
                           {2, 1.75, ..., 0.5} whose compact operators have
                           cond_1(A2, Dirichlet rows) <= 1e4 and
                           cond_1(A1) <= 1e5 (chn_get_mesh returns it) */
  void *stream;         /* hipStream_t the context runs on (NULL = default stream) */
  int32_t planes_only;  /* nonzero: a plane-phase context (one GPU's slab of x-z
                           planes): only chn_plane_products, the schedule and
                           timing calls are available, and the workspace holds
                           only the transform buffers of plane_chunk planes */
  int32_t plane_chunk;  /* planes per plane-phase launch (0: all n2; required
                           for planes_only) */
} chn_config;

/* Per-step diagnostics, filled by chn_step_rk3 for its last step. */
typedef struct {
  double f_mean;        /* mean pressure gradient of the last sub-step (Section 2.1) */
  double mass_flux;     /* integral of U1 over y after the step */
  double cfl_max;       /* dt * max(|u1|/dx + |u2|/dy_j + |u3|/dz) on the padded grid
                           (dx = lx/n1, dz = lz/n3, dy_j the smaller gap next to node
                           j), from the velocities entering the step's last sub-step;
                           on CHN_EUNSTABLE the value that tripped the guard */
  double utau_lo, utau_hi; /* sqrt(nu |dU1/dy|) at the two walls after the step */
  double max_abs_div;   /* max over modes and nodes of |i a u1 + D1 u2 + i b u3| of the
                           velocity fields the next sub-step's transforms read (float32
                           on CHN_MIXED, so about 1e-7 of the velocities there; they are
                           formed from continuity, so rounding only on CHN_FP64) */
  float ms_phase[5];    /* milliseconds of the last step per phase (HIP events on the
                           context's stream): z inverse, x pass, z forward, pencil
                           kernel, other launches (velocity recovery, per-dt tables) */
  int32_t fail_step;    /* -1, or the step (0-based, within the call) ... */
  int32_t fail_substep; /* ... and sub-step whose CFL tripped the guard */
} chn_step_info;

/* Stability limit of the guard: a sub-step whose CFL number (as in
 * chn_step_info) is above it or not finite is not applied. */
#define CHN_CFL_LIMIT 2.0

/* Bytes of device workspace needed for cfg (0 if cfg is invalid). */
size_t chn_workspace_bytes(const chn_config *cfg);

/* Builds the compact operators of Appendix B on the mesh (rows solved in
 * extended precision, maximum order, stencils truncated at the walls), the
 * quadrature weights of the mass flux, and the FFT tables, and uploads them
 * into d_workspace.  Synchronises.  *out receives the context.
 * The wall-normal systems are factored without pivoting, so the mesh is
 * checked first (Appendix B notes that the compact rows need care near the
 * walls): CHN_EINVAL, with the two numbers in chn_last_error(NULL), if the
 * 1-norm condition number of A1 or of A2 with Dirichlet end rows exceeds
 * 1e6 (the maximum-order seven-point stencils degenerate for some local
 * stretchings, e.g. the tanh mesh with g = 2 on 33 to 65 nodes; well-posed
 * meshes give 1e2 to 1e4).  Not checked for planes_only contexts. */
chn_status chn_create(const chn_config *cfg, void *d_workspace, size_t ws_bytes, chn_ctx **out);

/* Frees host-side state; the workspace stays the caller's. */
chn_status chn_destroy(chn_ctx *ctx);

/* Copies an initial state in: d_v (= u2) and d_omega2 spectral fields,
 * d_u1mean and d_u3mean float64[n2] mean profiles (all device pointers).
 * chi = (D2 - k^2) v is formed inside with the compact D2.  The (0,0) and
 * Nyquist modes of v and omega2 are ignored. */
chn_status chn_set_state(chn_ctx *ctx, const double *d_v, const double *d_omega2,
                         const double *d_u1mean, const double *d_u3mean);

/* Advances nsteps full RK3 steps of size dt (three sub-steps each, the
 * paper's Appendix A/C sequence: velocities and vorticities, dealiased
 * u x omega, non-linear forcings, explicit viscous terms, implicit
 * Helmholtz steps with the influence-matrix treatment of u2, mean modes with
 * constant mass flux).  Synchronises once, at the end of the call.
 * Instability guard, on every sub-step whether or not info is given: the
 * x pass gathers the sub-step's CFL number on the device; if it is not
 * finite (a NaN or Inf anywhere in the velocities) or above CHN_CFL_LIMIT,
 * that sub-step and every later one of the call leave the state untouched
 * and the call returns CHN_EUNSTABLE, with the step and sub-step in
 * chn_last_error (and in info).  The state is then as at the start of the
 * failing sub-step: for sub-step 0 that is the start of the failing step;
 * for sub-steps 1 and 2 it is the state between two sub-steps of that step
 * (no copy of the state is kept per step).  If info is not NULL it is
 * filled for the last step.  Steps whose per-dt tables and phase fields are
 * already current (all but the first after chn_set_state, a change of dt,
 * or a call that reuses their scratch) are replayed from a HIP graph of one
 * step, captured once per dt and schedule (kernel launches only; the graph
 * runs on the context's stream, the capture on a stream of the context's
 * own).  Replayed and launched steps give the same bits. */
chn_status chn_step_rk3(chn_ctx *ctx, double dt, int32_t nsteps, chn_step_info *info);

/* enable = 0: chn_step_rk3 launches every sub-step's kernels itself (no
 * graph); 1 (the default): steady steps are replayed from the captured
 * graph.  Frees the graph when disabled. */
chn_status chn_step_graph_enable(chn_ctx *ctx, int32_t enable);

/* Field selectors for chn_get_fields. */
enum {
  CHN_F_V = 1u << 0,      /* u2 (spectral) */
  CHN_F_OMEGA2 = 1u << 1, /* omega2 (spectral) */
  CHN_F_CHI = 1u << 2,    /* chi = lap(u2) (spectral) */
  CHN_F_U1 = 1u << 3,     /* u1 (spectral; (0,0) mode = U1) */
  CHN_F_U3 = 1u << 4,     /* u3 (spectral; (0,0) mode = U3) */
  CHN_F_OMEGA1 = 1u << 5, /* omega1 (spectral) */
  CHN_F_OMEGA3 = 1u << 6, /* omega3 (spectral) */
  CHN_F_U1MEAN = 1u << 7, /* U1, float64[n2] */
  CHN_F_U3MEAN = 1u << 8  /* U3, float64[n2] */
};

/* Writes the selected fields of the current state, in bit order, to the
 * device pointers d_out[0], d_out[1], ... (one per set bit).  u1, u3 and the
 * vorticities are recovered from v and omega2 by continuity and the compact
 * D1 (the first steps of every sub-step). */
chn_status chn_get_fields(chn_ctx *ctx, uint32_t mask, double *const *d_out);

/* The dealiased non-linear term on its own: from the six spectral fields
 * d_in[0..5] = u1, u2, u3, omega1, omega2, omega3 (device pointers, spectral
 * layout), forms H = u x omega on the 3n1/2 x 3n3/2 grid of every plane and
 * writes its truncated transforms d_out[0..2] = H1, H2, H3 (spectral layout,
 * forward transform scaled by 1/(P1 P3)).  Computes in the context's
 * precision (inputs and outputs stay float64). */
chn_status chn_nonlinear(chn_ctx *ctx, const double *const *d_in, double *const *d_out);

/* The low-storage stage (Section 3.1) on the current state.  With the
 * retained set K = {0 <= kx <= kcx, |kz| <= kcz} (kcx < n1/2, kcz < n3/2):
 *   d_ubar  [3][n2][kcx+1][2kcz+1] complex: F(u_i) for i = 1, 2, 3,
 *   d_uubar [6][n2][kcx+1][2kcz+1] complex: F(u_i u_j), pairs 11,12,13,22,23,33,
 *           the products formed on an f1 x f3 grid of each plane with
 *           f1 > n1 - 2 + kcx, f3 > n3 - 2 + kcz (2,3-smooth, at most the
 *           3/2 padded grid), on which every retained product mode is exact,
 *   d_tau   [6][n2][q3][q1] float64: tau_ij = F(u_i u_j) - F(u_i) F(u_j)
 *           evaluated on the uniform q1 x q3 grid of each plane,
 * kz in FFT slot order (0..kcz, then -kcz..-1).  q1 > 2 kcx, q3 > 2 kcz,
 * both even and factoring into 2s and 3s.  d_tau may be NULL.  Outputs are
 * complex float64 / float64 DEVICE arrays owned by the caller.  The inputs
 * are the velocity coefficients the time step holds in the context's
 * transform precision (CHN_MIXED: float32, with float32 inverse transforms);
 * the products, forward transforms, mean terms and stresses are float64 on
 * both precisions.  The state, the time step's phase fields and its
 * factor tables are left unchanged.  CHN_EINVAL for a cut-off or q grid
 * outside these ranges or a NULL output; CHN_EUNSUPPORTED where the
 * workspace cannot hold the retained products or the q grid. */
chn_status chn_filter_and_stress(chn_ctx *ctx, int32_t kcx, int32_t kcz, int32_t q1, int32_t q3,
                                 double *d_ubar, double *d_uubar, double *d_tau);

/* Filtered enstrophy of Section 3.1 (the tenth variable of the database):
 * F(omega_i omega_i), the sharp cut-off (0 <= kx <= kcx, |kz| <= kcz) of
 * omega_1^2 + omega_2^2 + omega_3^2 formed on the f1 x f3 grid of
 * chn_filter_and_stress from the vorticity of the current state (omega1,
 * omega3 by continuity and compact D1, the mean vorticity D1 U3, -D1 U1
 * included).  d_out: DEVICE, complex float64 [n2][kcx+1][2kcz+1], kz in
 * slot order as for chn_filter_and_stress; owned by the caller.  The
 * vorticity coefficients in the context's transform precision (CHN_MIXED:
 * float32 omega1, omega3 of the time step and omega2 rounded to float32,
 * float32 inverse transforms); the sum of squares, forward transforms and
 * mean terms in float64.  CHN_EINVAL for a cut-off outside
 * 0 <= kcx < n1/2, 0 <= kcz < n3/2 or a NULL pointer; CHN_ESTATE before
 * chn_set_state; CHN_EUNSUPPORTED on a planes_only context or where the
 * workspace cannot hold the retained products.  Uses the scratch of
 * chn_filter_and_stress; the state is unchanged. */
chn_status chn_filtered_enstrophy(chn_ctx *ctx, int32_t kcx, int32_t kcz, double *d_out);

/* On-the-fly statistics (Section 3: the runs' one-point statistics and the
 * two-dimensional spectra E_ii(kx, x2, kz) = <u_i u_i*>): adds, for the
 * current state, |u_i(kx, y, kz)|^2 of every stored mode except the mean
 * mode (0,0) to d_spec (DEVICE, float64 [3][n2][n1/2][n3], i = 1, 2, 3) and
 * the mean profiles U1(y), U3(y) to d_mean (DEVICE, float64 [2][n2]).  Both
 * buffers are owned by the caller, who zeroes them before the first call and
 * divides by the number of calls.  A stored kx > 0 mode stands for +kx and
 * -kx, so the plane-mean squared fluctuation is
 * sum_kz (E(0, kz) + 2 sum_{kx>0} E(kx, kz)).  Read from the velocity fields
 * the step already produces, in the context's transform precision (float32
 * values on CHN_MIXED).  CHN_EINVAL for a NULL pointer; CHN_ESTATE before
 * chn_set_state; CHN_EUNSUPPORTED on a planes_only context. */
chn_status chn_accumulate_statistics(chn_ctx *ctx, double *d_spec, double *d_mean);

/* Filtered pressure of Section 3.1 from the database variables: on every
 * retained mode (0 <= kx <= kcx, |kz| <= kcz) the Poisson equation
 * d_kk p = -d_i d_j F(u_i u_j), in the A-form of the implicit steps
 * ((B2 - k^2 A2) p = A2 r in the interior rows, r = -d_i d_j F(u_i u_j) with
 * the compact D1, D2 in y), with the wall rows D1 p = nu D2 F(v) (the filtered
 * wall-normal momentum equation at a wall; full compact wall rows of D1 and
 * D2); the mean mode P(y) = -F(u_2 u_2)(0, 0).  d_uubar, d_ubar: DEVICE, as
 * written by chn_filter_and_stress for the same kcx, kcz; d_p: DEVICE,
 * complex float64 [n2][kcx+1][2kcz+1] (kz in slot order), owned by the
 * caller.  Float64 on both precisions; uses the context's tables and scratch,
 * not its state.  CHN_EINVAL for a NULL pointer or a cut-off outside
 * 0 <= kcx < n1/2, 0 <= kcz < n3/2; CHN_EUNSUPPORTED on a planes_only context. */
chn_status chn_filtered_pressure(chn_ctx *ctx, int32_t kcx, int32_t kcz, const double *d_uubar,
                                 const double *d_ubar, double *d_p);

/* Dealiased products of Section 2.1 on every plane (the plane phase of the
 * sub-step): d_in[0..5] = u1, u2, u3, omega1, omega2, omega3 and d_out[0..2] =
 * H1, H2, H3 of H = u x omega, DEVICE pointers in the layout
 * [n2][n1/2][n3] but in the context's transform precision: complex64 for
 * CHN_MIXED, complex128 for CHN_FP64.  d_in[4] may be NULL (omega2 is then
 * formed as i b u1 - i a u3).  Outputs are truncated to the retained modes
 * (Nyquist slot zero) and scaled as the forward transform of Section 2.1.
 * Works on every context; the only compute call of a planes_only context. */
chn_status chn_plane_products(chn_ctx *ctx, const void *const *d_in, void *const *d_out);

/* For callers that cannot allocate device memory at the time of the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): chn_plane_products with the transform intermediate held in a
 * static device array of the library (64 MiB per GPU, reserved when the
 * library is loaded and held until the process ends) instead of the
 * context's workspace; the planes go through it in chunks of as many planes
 * as it holds.  Same arguments, layouts, results and errors as
 * chn_plane_products, plus CHN_EUNSUPPORTED when one plane of the
 * intermediate (6 * 3n3/2 * n1/2 complex values of the context's transform
 * precision) exceeds 64 MiB.  The call allocates nothing and creates no
 * events (chn_timing_enable does not apply to it).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (from different
 * streams or threads) race and give wrong results. */
chn_status chn_plane_products_static(chn_ctx *ctx, const void *const *d_in, void *const *d_out);

/* Copies the context's n2 wall-normal nodes (the configured mesh, or the
 * default one) to the HOST array y. */
chn_status chn_get_mesh(chn_ctx *ctx, double *y);

/* Copies the library's compact-difference tables to host arrays (each
 * n2 x 7, row i holding M[i][i-3..i+3]) and the mass-flux quadrature weights
 * (n2).  Any pointer may be NULL.  Synchronises. */
chn_status chn_get_operators(chn_ctx *ctx, double *a1, double *b1, double *a2, double *b2,
                             double *quad);

/* Near-wall mesh optimisation of Appendix B (a host routine: no context, no
 * GPU).  The homogeneous problem of the implicit steps, (B2 - k* A2) g = 0
 * in the interior rows with g = 1 at y = -1 and g = 0 at y = 1, has the
 * analytic solution sinh(q (1 - y)) / sinh(2 q), q = sqrt(k*); for layers
 * thinner than the first cells the compact solution departs from it near
 * the wall.  The first m interior nodes y_1..y_m (and their mirror images
 * y_{n2-2}..y_{n2-1-m}) are moved to minimise
 *   L = ||g - g_ana||_2 + penalty ||(y_1..y_m) - (y_ref_1..y_ref_m)||_2
 * by steepest descent in spacing-scaled coordinates: central-difference
 * gradient (step 1e-6 of the local spacing), step length halved from twice
 * the last accepted one until the mesh is strictly increasing, L strictly
 * decreases, the Armijo condition with 1e-4 holds, every ratio of adjacent
 * spacings lies in [1/2, 2], and the trial mesh's A2 and A1 each have a
 * 1-norm condition number at most 10 times the reference mesh's (so the
 * compact operators stay well posed); at most max_iter
 * steps, fewer when the step length falls below 1e-30.  The compact rows
 * are the quad-precision ones of the library's operators.
 *   y_ref:      HOST, n2 nodes, strictly increasing, y_ref[0] = -1,
 *               y_ref[n2-1] = 1, exactly symmetric (y[n2-1-i] = -y[i]).
 *   m:          free nodes per wall, 1 <= m, 2 m + 2 <= n2 (the paper moves
 *               20, with the wall node 21).
 *   kstar:      modified wavenumber k^2 + 1/(beta nu dt) of the layer, > 0.
 *   penalty:    C >= 0 (the paper uses about 1e-3).
 *   y_out:      HOST, n2 nodes, written on CHN_OK (may be y_ref itself:
 *               y_ref is copied before anything is written).
 *   err_ref, err_opt, iterations: HOST scalars (each may be NULL):
 *               ||g - g_ana||_2 on y_ref and on y_out, accepted steps.
 * Errors: CHN_EINVAL for invalid arguments (nothing written), CHN_EUNSTABLE
 * if a banded solve breaks down or gives a non-finite error.  Thread-safe
 * (no global state).  Runs on the calling thread. */
chn_status chn_optimise_mesh(const double *y_ref, int n2, int m, double kstar, double penalty,
                             int max_iter, double *y_out, double *err_ref, double *err_opt,
                             int *iterations);

/* ---------------------------------------------------------------- ensembles
 * An ensemble advances n independent channels of uneven sizes together:
 * every phase of the RK3 sub-step is one batched launch per channel group
 * (a work list of (channel, block) items, larger channels first, and one
 * argument block per channel in device memory), and one RK3 step of the
 * whole ensemble is a captured HIP graph replayed nsteps times.  The graph
 * has two branches, one per group: the channels with the most wall-normal
 * nodes, and the rest (with one n2 for all: channels dealt in turn, the
 * second branch starting one plane phase later), so one group's pencil
 * phase overlaps the other's plane phase; each channel's results are those
 * of a single context with the same radix sets.  All configurations must
 * share the precision and the stream.  The ensemble runs on two private
 * streams ordered after and before the configured stream by events.  Same
 * conventions as single contexts (caller-owned workspace). */
typedef struct chn_ens chn_ens;

/* Workspace bytes for n channels (0 if any configuration is invalid). */
size_t chn_ens_workspace_bytes(int32_t n, const chn_config *cfgs);

/* Creates the n channel contexts inside d_workspace and the batched
 * launch tables.  Synchronises. */
chn_status chn_ens_create(int32_t n, const chn_config *cfgs, void *d_workspace, size_t ws_bytes,
                          chn_ens **out);
chn_status chn_ens_destroy(chn_ens *ens);

/* Context handle of channel i (for chn_set_state, chn_get_fields,
 * chn_filter_and_stress, ...); owned by the ensemble. */
chn_ctx *chn_ens_context(chn_ens *ens, int32_t i);

/* chn_set_state on channel i of the ensemble (same arguments, layouts and
 * errors; CHN_EINVAL for i outside 0..n-1, with chn_ens_last_error set). */
chn_status chn_ens_set_state(chn_ens *ens, int32_t i, const double *d_v, const double *d_omega2,
                             const double *d_u1mean, const double *d_u3mean);

/* Advances every channel nsteps RK3 steps; dt is a HOST array of n step
 * sizes.  Every channel must have a state (chn_set_state).  Synchronises at
 * the end; the instability guard of chn_step_rk3 runs per channel (a
 * channel whose sub-step trips it stops there, the others go on), and the
 * call then returns CHN_EUNSTABLE naming the first such channel in
 * chn_ens_last_error. */
chn_status chn_ens_step(chn_ens *ens, const double *dt, int32_t nsteps);

const char *chn_ens_last_error(const chn_ens *ens);

/* Kernel kinds reported by chn_timing_read. */
enum {
  CHN_K_RECOVER = 0, /* velocities/vorticities from v, omega2 (pencils) */
  CHN_K_ZINV = 1,    /* padded inverse transform in z (planes) */
  CHN_K_XPASS = 2,   /* inverse x transforms, u x omega, forward x transforms */
  CHN_K_ZFWD = 3,    /* forward transform in z with truncation */
  CHN_K_ADVANCE = 4, /* forcings, implicit steps, influence matrix, mean modes */
  CHN_K_FILTER = 5,  /* kernels of the low-storage stage */
  CHN_K_COUNT = 6
};

/* Per-kernel timing.  With enable != 0 every later kernel launch of the
 * context is bracketed by two HIP events recorded on the context's stream;
 * enabling or disabling discards earlier records. */
chn_status chn_timing_enable(chn_ctx *ctx, int32_t enable);

/* Sum of the recorded durations (ms) and the number of launches of one
 * kernel kind since chn_timing_enable.  Synchronises. */
chn_status chn_timing_read(chn_ctx *ctx, int32_t kind, double *total_ms, int32_t *count);

/* ---------------------------------------------------------------- schedule
 * How the plane phase (the padded transforms and products of Section 2.1)
 * is cut into workgroups.  x_rows: rows of the x pass per workgroup, 2
 * (six transform lines in LDS at once) or 1 (lines staged one at a time
 * through LDS, values held in registers: the only choice for long rows).
 * z_lines: lines per z-pass workgroup (more lines give longer coalesced
 * segments of the transposed stores, fewer give more workgroups and less
 * LDS per workgroup).  y_chunk: planes per launch (smaller chunks keep the
 * z-padded intermediate of a chunk in the last-level cache between the three
 * kernels; at most the plane_chunk of a planes_only context).  Results agree
 * to rounding between schedules. */
typedef struct {
  int32_t x_rows;
  int32_t z_lines;
  int32_t y_chunk;      /* planes per launch of the three plane kernels */
  int32_t fixed_radix;  /* 1: transforms whose length has a compile-time radix
                           schedule (576 points) use it; 0: the runtime plan */
  int32_t z_pipeline;   /* 1: the z passes issue the next field's loads before
                           transforming the current one (and the z inverse forms
                           omega2 from the u1, u3 values it loaded), where a
                           field of z_lines lines fits their staging registers;
                           0: one field at a time */
  int32_t radix_set;    /* bit 0 for the x transforms, bit 1 for the z
                           transforms: 0 = Stockham passes of radix 8, then 4,
                           2, 3; 1 = the fewest passes with radices up to 16
                           (6, 9, 12 and 16 computed in registers: 576 points
                           in 3 passes instead of 4, 1296 in 3 instead of 6).
                           fixed_radix applies to 576-point lines in either
                           set (8, 8, 3, 3 or 9, 8, 8) */
} chn_plan;

/* Current schedule (chn_create picks 2 rows when they fit, 16 lines capped
 * by registers and LDS, plane_chunk or all planes, and radix set 0 with its
 * compile-time schedules). */
chn_status chn_get_plan(chn_ctx *ctx, chn_plan *plan);

/* Sets the schedule; CHN_EINVAL (context unchanged) if it does not fit the
 * grid or the device's LDS.  Channels of an ensemble keep the schedule
 * their batched tables were built with (chn_ens_create gives a channel the
 * composite radices in a direction where they take fewer passes), and a
 * different radix set on one of them is CHN_EUNSUPPORTED (the autotuner then
 * keeps the channel's set). */
chn_status chn_set_plan(chn_ctx *ctx, const chn_plan *plan);

/* Autotuner: times the plane phase (reps repetitions after one warm-up) for
 * every schedule that fits with the classic radices, then with the
 * composite radix sets at the chosen planes per launch, keeps the fastest
 * and writes it to *chosen (may be NULL).  Only scratch buffers are
 * written; the state is untouched.  Synchronises.  The choice is kept in a
 * cache file, one JSON object per line keyed by the device architecture,
 * n1 x n2 x n3, the precision and the planes per launch the context
 * allows; a later call for the same key applies the cached schedule
 * without timing.  The file is
 * $CHN_TUNE_CACHE, else $XDG_CACHE_HOME/chn_tune.jsonl, else
 * $HOME/.cache/chn_tune.jsonl; CHN_TUNE_CACHE set to an empty string turns
 * the cache off.  An unreadable or unwritable file only disables caching. */
chn_status chn_autotune(chn_ctx *ctx, int32_t reps, chn_plan *chosen);

/* Message of the last failing call on ctx (or of the last failing
 * chn_create if ctx is NULL). */
const char *chn_last_error(const chn_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* CHN_H */
