/*
 * cmhd.h -- C ABI of the MI355X (gfx950) coronal MHD time step.
 *
 * One call of cmhd_rk3_step advances the compressible resistive MHD system in
 * vector potential A, velocity u, ln rho and ln T by one low-storage
 * third-order Runge-Kutta step, with the boundary set of Bourdin (2019,
 * arXiv:1908.08557): periodic horizontal directions, a photospheric lower
 * boundary that nudges u and A toward a driver (Sect. 2.3, eq. 5; Sect. 2.1),
 * an inverted potential-field extrapolation below the photosphere
 * (Sect. 2.4), density fixed to its initial profile and hydrostatic
 * temperature ghosts (Sect. 2.5, eq. 8), a closed upper boundary with
 * symmetric temperature and hydrostatic density (Sect. 4.1, eqs. 11-13), a
 * potential-field upper boundary computed by 2-D Fourier transforms
 * (Sect. 4.2, eqs. 16-17) and swamp layers (Sect. 4.3, eqs. 18-20).
 * B = curl A in the Weyl gauge (Sect. 2.4, eqs. 6-7).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State layout.  One device buffer of float64 holding the eight fields
 *   Ax, Ay, Az, ux, uy, uz, ln rho, ln T (in this order), each an array
 *   [nz+6][ny][nx] with x fastest.  Plane index kz = k + 3 holds height
 *   z_k = z0 + k dz for k = -3 .. nz+2: three ghost planes below and above
 *   the interior.  x and y are periodic and stored without ghosts.  The
 *   buffer holds cmhd_state_elems() doubles.  In solar mode the planes
 *   k = -3..-1 of ux and uy are part of the state (they evolve under the
 *   nudging term of eq. 5 alone); every other ghost plane is derived and is
 *   overwritten by cmhd_fill_ghosts.
 * Units.  Whatever consistent units the caller uses; mu0, R and gamma are
 *   parameters.
 * Ownership.  The context is allocated by cmhd_init_grid and freed by
 *   cmhd_destroy.  All device memory is owned by the caller: the state and
 *   the workspace bound with cmhd_bind_workspace.  The library never frees a
 *   caller pointer and keeps no pointer to a state buffer between calls.
 * Streams.  Every kernel of a context runs on its stream (cmhd_set_stream);
 *   calls return before the work completes unless stated otherwise.  A
 *   context must not be used from two host threads at once.
 * Errors.  Every function returns a cmhd_status; on failure
 *   cmhd_last_error() describes the cause and no kernel was launched.
 */
#ifndef CMHD_H
#define CMHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CMHD_OK = 0,
  CMHD_EINVAL = -1,      /* invalid argument (sizes, parameters, pointers) */
  CMHD_EDEVICE = -2,     /* a HIP runtime call failed */
  CMHD_ENONFINITE = -3,  /* a non-finite value was found (cmhd_check_finite) */
  CMHD_EDT = -4,         /* the time step from the CFL limits is zero or not finite
                            although the state is finite (cmhd_cfl_dt) */
  CMHD_ESTATE = -5,      /* call out of order (e.g. no workspace bound) */
  CMHD_EWORKSPACE = -6   /* workspace too small */
} cmhd_status;

typedef enum { CMHD_FP64 = 0, CMHD_FP32_SPLIT = 1 } cmhd_precision;
typedef enum { CMHD_ZBC_PERIODIC = 0, CMHD_ZBC_SOLAR = 1 } cmhd_zbc;

#define CMHD_MAX_RAD 16
#define CMHD_MAX_NC_TABLE 1024   /* nz + 6 <= this when the Newtonian cooling is on */

typedef struct cmhd_ctx cmhd_ctx;

/* Grid.  nx, ny: powers of two in [16, 1024] (the Fourier boundary works on
 * power-of-two rows of at most 1024 points; the tiles are 16 x 16), nz >= 8.
 * dx = Lx/nx, dy = Ly/ny.  Solar z is vertex-centred: dz = (z1-z0)/(nz-1),
 * z_0 = z0 is the photosphere and z_{nz-1} = z1 the top boundary point (the
 * boundary layers j = 0 of Sect. 2.3 and nz of Sect. 4.1).  Periodic z:
 * dz = (z1-z0)/nz.
 * prec = CMHD_FP32_SPLIT evaluates the right-hand side in float32 (stencil
 * differences of the float64 state are formed in float64 first) while the
 * state, the Runge-Kutta register and update, the ghost rules, the Fourier
 * transforms and the conduction coefficient kappa0 T^5/2 stay float64. */
typedef struct {
  int nx, ny, nz;
  double Lx, Ly, z0, z1;
  int zbc;   /* cmhd_zbc */
  int prec;  /* cmhd_precision */
} cmhd_grid;

/* Physical and numerical parameters (all in the caller's units).
 *  gamma, R, mu0     ideal gas p = rho R T, c_v = R/(gamma-1); mu0 J = curl B
 *  eta, nu           magnetic diffusivity, kinematic viscosity (constant)
 *  D_rho             mass diffusivity of Sect. 2.5
 *  kappa0            Spitzer coefficient: heat flux kappa0 T^5/2 b (b.grad T)
 *  g_z               signed vertical gravity (negative: pointing down)
 *  Bext              uniform field added to curl A
 *  B_floor           |B| regularisation of the field direction b = B/|B|_r
 *  eta_s, chi_s, chi_rho, z_s, z_t   swamp layers, eqs. (18)-(20), with the
 *                    cubic step w(z) from z_s to z_t (Sect. 4.3)
 *  tau_u             inverse time of the u_h nudging, eq. (5)
 *  tau_A             inverse time of the A_h nudging at the photosphere
 *  t_ramp            duration of the linear driver switch-on (Sect. 2.3);
 *                    <= 0: no ramp
 *  f_bot             contrast factor of the inverted potential field below
 *                    the photosphere (Sect. 2.4, one fifth in the paper)
 *  n_rad, rad_lnT, rad_lnL   optically thin loss Q = rho^2 exp(lnL(ln T))
 *                    with lnL piecewise linear through the breakpoints and
 *                    constant outside; n_rad = 0 switches it off
 *  T_rad_lo, T_rad_hi smoothstep in ln T that switches the loss on
 *  c_adv, c_diff, c_nudge   Courant factors of cmhd_cfl_dt
 *  nc_tau            inverse time of the chromospheric Newtonian cooling
 *                    (Sect. 3.1, eqs. 9-10): d ln T/dt gains
 *                    -nc_tau c_rho c_z (1 - Ts / T) with the target
 *                    Ts = sqrt(T0(z) T'(rho)), T'(rho) = T0(z') where
 *                    rho0(z') = rho (linear in ln rho0 between the nodes of
 *                    the initial profiles given to cmhd_init_grid, clamped
 *                    outside); 0 switches it off
 *  nc_lnrho_magn, nc_lnrho_width   c_rho = 1 while ln rho is within
 *                    magn - width natural-log orders of the photospheric
 *                    ln rho0(z0), a sine down to 0 at magn orders
 *  nc_z_max, nc_z_width   c_z = 1 below nc_z_max - nc_z_width, a sine down
 *                    to 0 at nc_z_max
 * Periodic z ignores the swamp, nudging and boundary parameters. */
typedef struct {
  double gamma, R, mu0, eta, nu, D_rho, kappa0, g_z;
  double Bext[3];
  double B_floor;
  double eta_s, chi_s, chi_rho, z_s, z_t;
  double tau_u, tau_A, t_ramp, f_bot;
  int n_rad;
  double rad_lnT[CMHD_MAX_RAD], rad_lnL[CMHD_MAX_RAD];
  double T_rad_lo, T_rad_hi;
  double c_adv, c_diff, c_nudge;
  double nc_tau, nc_lnrho_magn, nc_lnrho_width, nc_z_max, nc_z_width;
} cmhd_params;

/* Create a context.  lnrho0_z: host array of nz+6 doubles, the initial
 * ln rho profile at z_k, k = -3..nz+2; its three lowest entries are the
 * density imposed below the photosphere ('fg', Sect. 2.5) and entry 3 the
 * photospheric value held fixed.  lnT0_z: host array of nz+6 doubles, the
 * initial ln T profile at the same heights; only the Newtonian cooling reads
 * it (then lnrho0_z must decrease strictly with height, the reference
 * stratification of Sect. 3.1) and it may be NULL when params->nc_tau == 0.
 * Both are copied.  stream: a hipStream_t (NULL = the null stream).  *out
 * receives the context.  EINVAL on bad sizes or parameters, EDEVICE when no
 * gfx950 device is current. */
cmhd_status cmhd_init_grid(const cmhd_grid* grid, const cmhd_params* params,
                           const double* lnrho0_z, const double* lnT0_z, void* stream,
                           cmhd_ctx** out);

/* As cmhd_init_grid on a non-uniform z grid (Introduction: the production
 * grid refines from ~800 km in the corona to ~100 km in the lower
 * atmosphere).  z: host [nz+6], the heights z_k of the planes k = -3..nz+2,
 * strictly increasing (copied); grid.z0 and grid.z1 are ignored (the
 * interior runs from z_0 to z_{nz-1}); solar boundaries only.  The sixth-order
 * stencils act in the plane index k and are scaled by the metric of the
 * mapping: d/dz = (1/z') d/dk, d2/dz2 = (1/z'^2) d2/dk2 - (z''/z'^3) d/dk,
 * with z' and z'' the same stencils applied to the heights.  The ghost rules
 * use the actual heights: eq. (8) below and the potential fields at the
 * ghost heights; the upper density follows the recursion of eq. (15) (the
 * mirror form of eq. 13 needs symmetric grid distances).  The time step uses
 * each plane's own spacing min(dx, dy, z'_k).  z = NULL is cmhd_init_grid.
 * The tangent and adjoint steps differentiate the same discrete map. */
cmhd_status cmhd_init_grid_z(const cmhd_grid* grid, const cmhd_params* params, const double* z,
                             const double* lnrho0_z, const double* lnT0_z, void* stream,
                             cmhd_ctx** out);

/* Number of doubles of one state buffer: 8*(nz+6)*ny*nx. */
size_t cmhd_state_elems(const cmhd_ctx* ctx);

/* Bytes of device workspace the context needs: two state buffers for the
 * intermediate Runge-Kutta stages, the Runge-Kutta register, the driver
 * targets and the Fourier scratch.  The caller allocates it (aligned to 256
 * bytes) and binds it; it must outlive every later call. */
size_t cmhd_workspace_bytes(const cmhd_ctx* ctx);
cmhd_status cmhd_bind_workspace(cmhd_ctx* ctx, void* dev_ptr, size_t bytes);

/* Change the stream of all later launches. */
cmhd_status cmhd_set_stream(cmhd_ctx* ctx, void* stream);

/* Photospheric driver (solar mode).  uh: device [2][ny][nx], the target
 * horizontal velocity u* of eq. (5).  Then exactly one of
 *   ah: device [2][ny][nx], the nudging target A_h* of A_x, A_y, or
 *   bz: device [ny][nx], a vertical field from which A_h* is computed so
 *       that d_x A_y - d_y A_x = B_z (eq. 7) in Fourier space (mean and
 *       Nyquist modes set to zero); EINVAL if its net flux exceeds
 *       1e-12 * sum |B_z| (Sect. 2.1: balanced flux).
 * may be non-NULL (both NULL keeps the previous A_h*).  The inputs are
 * copied on the context stream; the caller may free them once that stream
 * has passed this call. */
cmhd_status cmhd_set_driver(cmhd_ctx* ctx, const double* uh, const double* bz,
                            const double* ah);

/* Photospheric driver as two snapshots (Sect. 2.3: the coronal run reads
 * granulation snapshots and interpolates between them in time).  uh0, uh1:
 * device [2][ny][nx], u* at times t0 < t1 (both finite), copied on the
 * context stream.  From then on the target of eq. (5) at a substage time t is
 * u*_0 + w (u*_1 - u*_0), w = (t - t0) / (t1 - t0) clipped to [0, 1],
 * formed by a small kernel before every substage.  A_h* is not changed.  A
 * later cmhd_set_driver returns to a single target.  With a snapshot pair the
 * tangent and adjoint steps accept no driver perturbation or cotangent
 * (duh, uhbar must be NULL; CMHD_EINVAL otherwise).  EINVAL for NULL
 * snapshots or t1 <= t0. */
cmhd_status cmhd_set_driver_snapshots(cmhd_ctx* ctx, const double* uh0, double t0,
                                      const double* uh1, double t1);

/* Fill every derived ghost plane of the device state in place (solar: the
 * rules listed at the top; periodic: plane copies).  t is unused today (the
 * rules do not depend on time) and kept for time-dependent boundaries. */
cmhd_status cmhd_fill_ghosts(cmhd_ctx* ctx, double* state, double t);

/* Advance the device state in place by one RK3 step from time *t.  dt > 0:
 * use it; dt <= 0: compute it first with cmhd_cfl_dt (one device-to-host
 * copy, synchronous).  On return *t has advanced by the step and *dt_used
 * (if non-NULL) holds it.  The derived ghosts of the state are refreshed on
 * entry and are stale on return; the interior and the ux, uy lower ghost
 * planes hold the new state.  Needs a bound workspace (ESTATE).
 * With dt > 0 the call only launches kernels on the context stream (and,
 * while profiling is enabled, records events there): no allocation, copy,
 * memset or host synchronisation, so it may be captured into a HIP graph.  The switch-on ramp and the snapshot
 * weight are evaluated on the host from *t at the call and are fixed in a
 * captured graph. */
cmhd_status cmhd_rk3_step(cmhd_ctx* ctx, double* state, double* t, double dt,
                          double* dt_used);

/* Evaluate the right-hand side once at time t: fills the derived ghosts of
 * the state, then writes dF/dt into rhs (device, state layout and size) at
 * every interior point and, in solar mode, at the ux, uy lower ghost rows;
 * the other entries of rhs are left unchanged.  Needs a bound workspace. */
cmhd_status cmhd_eval_rhs(cmhd_ctx* ctx, double* state, double t, double* rhs);

/* Time step from the Courant, diffusion, radiative-cooling and nudging
 * limits over the interior (fills the ghosts first).  Synchronous. */
cmhd_status cmhd_cfl_dt(cmhd_ctx* ctx, double* state, double* dt_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight stepping loops, harnesses that forbid allocation): the time
 * step of cmhd_cfl_dt for a state whose ghost planes are already filled
 * (cmhd_fill_ghosts; this call does not fill them), with the reduction
 * scratch in a fixed array inside the library (256 bytes per GPU, kept until
 * the process ends) instead of the bound workspace.  It allocates nothing and
 * needs no workspace, except on a non-uniform z grid (whose z table lives in
 * the workspace: CMHD_ESTATE without one).  Any grid the context accepts is
 * accepted (the scratch holds three maxima whatever the size).  The
 * context's GPU must be current (CMHD_ESTATE otherwise).  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race and may return a wrong dt.  Synchronous. */
cmhd_status cmhd_cfl_dt_noalloc(cmhd_ctx* ctx, const double* state, double* dt_out);

/* Copy the fields selected by mask (bit f = field f) to dst, packed in field
 * order as [nsel][nz][ny][nx] (with_ghosts = 0) or [nsel][nz+6][ny][nx].
 * dst_on_host != 0: dst is host memory and the call is synchronous. */
cmhd_status cmhd_get_fields(cmhd_ctx* ctx, const double* state, unsigned mask,
                            double* dst, int dst_on_host, int with_ghosts);

/* The inverse of cmhd_get_fields: copy the fields selected by mask (bit f =
 * field f) from src into the device state, src packed in field order as
 * [nsel][nz][ny][nx] (with_ghosts = 0: the interior planes; the ghost planes
 * keep their values) or [nsel][nz+6][ny][nx] (with_ghosts != 0: every plane,
 * which restores the u_x, u_y ghost rows that are state in solar mode).
 * src_on_host != 0: src is host memory and the call is synchronous; else the
 * copies are queued on the context stream. */
cmhd_status cmhd_set_fields(cmhd_ctx* ctx, double* state, unsigned mask, const double* src,
                            int src_on_host, int with_ghosts);

/* B_z = d_x A_y - d_y A_x + Bext_z on the horizontal plane at height z,
 * linear between the two enclosing grid planes, into device dst [ny][nx]. */
cmhd_status cmhd_bz_plane(cmhd_ctx* ctx, const double* state, double z, double* dst);

/* Non-zero when every interior value of the state is finite (synchronous).
 * Returns CMHD_ENONFINITE otherwise. */
cmhd_status cmhd_check_finite(cmhd_ctx* ctx, const double* state);

/* ---- tangent-linear and adjoint step (differentiation of cmhd_rk3_step) ----
 * The step is differentiated as the discrete map it is, at fixed t and dt:
 *   y = Step(x, u*)    (x: the state entries, i.e. the interior of every
 *                       field and, in solar mode, the ux, uy lower ghost rows;
 *                       u*: the driver target of eq. (5))
 * The pointwise right-hand side is differentiated with forward-mode dual
 * numbers; the stencil, ghost-rule, Fourier-filter and Runge-Kutta transposes
 * are written out.  Entries of x, dx, ybar that are not state entries are
 * ignored; those of dy and xbar are returned as zero.  Calls need a bound
 * adjoint workspace (ESTATE otherwise) and recompute the forward substages
 * into the step workspace.  x is not modified except for its derived ghosts. */
size_t cmhd_adjoint_workspace_bytes(const cmhd_ctx* ctx);
cmhd_status cmhd_bind_adjoint_workspace(cmhd_ctx* ctx, void* dev_ptr, size_t bytes);

/* dy = (d Step/d x) dx + (d Step/d u*) duh.  duh: device [2][ny][nx] or NULL
 * (no driver perturbation).  dx, dy: device, state layout. */
cmhd_status cmhd_rk3_step_jvp(cmhd_ctx* ctx, double* x, double t, double dt, const double* dx,
                              const double* duh, double* dy);

/* xbar = (d Step/d x)^T ybar (overwritten); uhbar += (d Step/d u*)^T ybar
 * (device [2][ny][nx], accumulated; may be NULL). */
cmhd_status cmhd_rk3_step_vjp(cmhd_ctx* ctx, double* x, double t, double dt, const double* ybar,
                              double* xbar, double* uhbar);

/* xbar += (d B_z-plane / d x)^T bzbar for the plane of cmhd_bz_plane at height
 * z (the loss of a magnetogram fit at that height). */
cmhd_status cmhd_bz_plane_vjp(cmhd_ctx* ctx, double z, const double* bzbar, double* xbar);

/* Kernel timing.  While enabled, every substage (cmhd_rk3_step,
 * cmhd_eval_rhs and the forward recomputation of the adjoint) records pairs
 * of HIP events on the context stream around its two parts, selected by
 * cmhd_prof_kernel: the fused stencil/RHS/RK kernel (CMHD_PROF_SUBSTAGE) and
 * the boundary work that precedes it (CMHD_PROF_GHOSTS: ghost fill with the
 * Fourier filters, driver target, nudged ghost rows).  cmhd_profile_read
 * synchronises the stream, returns for the selected part the summed duration
 * in milliseconds and the number of timed regions since its last read, and
 * resets them; an unknown selector is CMHD_EINVAL.  Enabling and disabling
 * keep pending records. */
typedef enum { CMHD_PROF_SUBSTAGE = 0, CMHD_PROF_GHOSTS = 1 } cmhd_prof_kernel;
cmhd_status cmhd_profile_enable(cmhd_ctx* ctx, int enable);
cmhd_status cmhd_profile_read(cmhd_ctx* ctx, int which, double* ms, int* launches);

const char* cmhd_last_error(const cmhd_ctx* ctx);
void cmhd_destroy(cmhd_ctx* ctx);

/* ---- photospheric granulation driver (Sect. 2.3, eqs. 1-4) ----
 * A 2-D run on the photospheric pixel grid that produces driver snapshots
 * u*(x, y) for cmhd_set_driver / cmhd_set_driver_snapshots.  Granules of
 * radius r_gran whose radial outflow extends, through the lane zone, to
 * r_lane fill the plane by random sequential addition: a pixel (x_i = i dx,
 * y_j = j dy) is free when every living centre lies at least r_excl away, and
 * each birth takes the floor(u n)-th free pixel in raster order (y slowest)
 * for the next uniform u of the caller's pool, n the number of free pixels,
 * until none is free.  A granule born at t0 has lifetime
 * T = t_gran (1 + life_var xi_T), amplitude v_max = v0 (1 + amp_var xi_v),
 * t_max = T sqrt(|ln(v_min / v_max)|) (eq. 1), v_min = vmin_frac v0, speed
 * v(t) = v_max exp(-((t - t0 - t_max) / T)^2) (eq. 2), and ceases to exist at
 * the first update with t > t0 + 2 t_max (where v has fallen below v_min).
 * Its velocity is v(t) g(r) r_hat, g = r / r_gran inside r_gran,
 * (1 + cos(pi (r - r_gran) / (r_lane - r_gran))) / 2 in the lane zone, 0
 * beyond, nearest periodic image; the fields of all granules add up.  The
 * snapshot is that granular field plus f_rot times its rotational
 * (divergence-free) part filtered by exp(-(2 |k| / k_N)^4) (eq. 3; k = 0 and
 * the Nyquist row and column dropped, k_N = pi / max(dx, dy)), rescaled to
 * the rms of the granular field (eq. 4).  With an external velocity field the
 * centres move with it (forward Euler since the previous update, bilinear
 * sample at the centre, positions wrapped into [0, L)).
 * Random draws are inputs: the caller's pools unif (uniforms in [0, 1), one
 * per birth) and xi (variations in [-1, 1], two per birth: xi_T, xi_v).
 * Ownership and streams as for the MHD context: the caller allocates and
 * binds the workspace; kernels run on the object's stream. */
typedef struct cmhd_gran_params {
  int nx, ny;               /* pixel grid, powers of two in [16, 1024] */
  double Lx, Ly;            /* periodic extent */
  double r_gran;            /* granule radius (0.8 Mm) */
  double r_lane;            /* outer edge of the lane zone (1.04 Mm), > r_gran */
  double r_excl;            /* no birth closer to a living centre (0.64 Mm) */
  double t_gran;            /* mean lifetime T_gran (5 min) */
  double v0;                /* mean amplitude (1.028 km/s) */
  double vmin_frac;         /* v_min / v0 (0.78), below 1 - amp_var */
  double life_var;          /* lifetime variation (0.10), in [0, 1) */
  double amp_var;           /* amplitude variation (0.15), in [0, 1) */
  double f_rot;             /* vorticity factor (5) */
} cmhd_gran_params;

typedef struct cmhd_gran cmhd_gran;

/* Create an empty population.  stream: hipStream_t of every later launch.
 * EINVAL on bad sizes or parameters. */
cmhd_status cmhd_gran_create(const cmhd_gran_params* params, void* stream, cmhd_gran** out);

/* Device workspace: the granule table (up to the hexagonal packing bound
 * Lx Ly / (sqrt(3)/2 r_excl^2) granules), two complex Fourier planes and
 * reduction scratch.  Caller-allocated, 256-byte aligned, bound once. */
size_t cmhd_gran_workspace_bytes(const cmhd_gran* g);
cmhd_status cmhd_gran_bind_workspace(cmhd_gran* g, void* dev_ptr, size_t bytes);

/* Advance the population to time t (not before the previous update): advect
 * the centres with vext_host ([2][ny][nx] host memory, or NULL: centres stay
 * put), remove the granules that have ended, refill.  Births consume
 * unif[0..], xi[0..] (host memory, n_pool uniforms and 2 n_pool variations);
 * *births receives their number.  Host work only (sequential; no workspace
 * needed): the next cmhd_gran_velocity copies the granule table to the
 * device.  EINVAL when the pool runs out (the granules born until then are
 * kept). */
cmhd_status cmhd_gran_update(cmhd_gran* g, double t, const double* vext_host, const double* unif,
                             const double* xi, long long n_pool, long long* births);

/* Driver snapshot at time t from the current population into device
 * uh [2][ny][nx]: granular field, eq. (3) enhancement, eq. (4) rescaling
 * (a zero field when there is no granule).  Needs a bound workspace.
 * Asynchronous, except for the copy of the granule table after an update. */
cmhd_status cmhd_gran_velocity(cmhd_gran* g, double t, double* uh);

/* Host copy of the living granules, rows (x, y, t0, T, v_max, t_max) in birth
 * order, at most cap rows; *n receives the population size. */
cmhd_status cmhd_gran_list(const cmhd_gran* g, double* host, int cap, int* n);

const char* cmhd_gran_last_error(const cmhd_gran* g);
void cmhd_gran_destroy(cmhd_gran* g);

#ifdef __cplusplus
}
#endif
#endif /* CMHD_H */
