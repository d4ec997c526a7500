/*
 * ugks.h -- C ABI of the MI355X (gfx950) implementation of the 2D unified gas-kinetic
 * scheme (UGKS) time step.
 *
 * The problem follows the paper "Performance Comparison on Parallel CPU and GPU Algorithms
 * for Unified Gas-Kinetic Scheme" (Liu, Hu & Li):
 *   - BGK-Boltzmann equation with a Maxwellian equilibrium, Eq. (1); 2D gas, velocities in
 *     units of sqrt(2kT0/m), so the Maxwellian is rho (lambda/pi) exp(-lambda |c - U|^2)
 *     with lambda = 1/T.  The paper's gas has no internal degrees of freedom; a gas with
 *     internal_dof > 0 (ugks_vgrid) carries a second reduced distribution for their energy.
 *   - Finite volumes over nx*ny uniform Cartesian cells, nu*nv discrete molecular
 *     velocities per cell (Sec. 2).
 *   - Interface fluxes from the integral solution of the BGK equation, Eq. (2), built
 *     through the flux steps S1-S8 (Sec. 2.B); distribution update with a trapezoidal
 *     collision term, Eq. (3); conservative update, Eq. (4).
 *   - The pressure-driven channel of Sec. 3.A: fixed inlet/outlet pressure, diffuse walls.
 *
 * Conventions shared by every call:
 *   - Every function returns int: UGKS_OK (0) or a negative UGKS_E_* code.  Results go
 *     through out-parameters.  ugks_last_error() gives a message for the last failure.
 *   - Host buffers are always owned by the caller.  Device memory is owned by the handle
 *     unless the caller passes a workspace in ugks_opts, which then stays the caller's and
 *     must outlive the handle.
 *   - Host arrays use the canonical layout: cell (i, j) is at index j*nx + i (x fastest);
 *     the velocity index is k*nv + m for (u_k, v_m); f[(j*nx + i)*NF + c*nu*nv + k*nv + m]
 *     with NF = nc*nu*nv values per cell, nc = 1 (c = 0 only) or, with internal degrees of
 *     freedom, nc = 2 (c = 0: G, c = 1: H);
 *     W[(j*nx + i)*4 + q] with W = (rho, rho U, rho V, rho E).
 *   - Work is enqueued on the stream given in ugks_opts (hipStream_t; NULL = the default
 *     stream).  Only ugks_moments, ugks_get_state, ugks_set_state, ugks_get_face_flux,
 *     ugks_get_kernel_timing and ugks_destroy synchronise with it.
 *   - A handle may be used by one host thread at a time.
 */
#ifndef UGKS_H
#define UGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UGKS_OK 0
#define UGKS_E_INVAL (-1)  /* invalid argument (NULL pointer, size, range, inconsistent option) */
#define UGKS_E_NOMEM (-2)  /* device or host allocation failed, or the workspace is too small */
#define UGKS_E_DEVICE (-3) /* a HIP runtime call or kernel launch failed */
#define UGKS_E_STATE (-4)  /* the solution holds NaN, rho <= 0 or T <= 0, or a Maxwellian
                              whose speed ratio |V| / T^(1/2) along v exceeds about 26 */
#define UGKS_E_BUSY (-5)   /* the handle is in use by another call */

typedef struct ugks_handle ugks_handle;

/* Uniform Cartesian mesh of nx*ny cells on [0, lx] x [0, ly] (Sec. 2: I x J cells). */
typedef struct {
  int nx, ny;
  double lx, ly;
} ugks_mesh;

/* Discrete velocity grid (Sec. 2: K x M points (u_k, v_m)): nu uniform points on
   [-umax, umax] and nv on [-vmax, vmax], both ends included, trapezoid weights, built
   exactly mirror-symmetric.  2 <= nu, nv <= 1024; otherwise UGKS_E_INVAL.
   internal_dof (0..16): degrees of freedom of the molecule beyond the two velocities of the
   plane (0: the paper's gas, gamma = 2; 1: a monatomic gas in 3D seen in the plane,
   gamma = 5/3; 3: diatomic, gamma = 7/5).  With internal_dof > 0 each velocity carries
   G = int f dxi and H = int |xi|^2 f dxi over the internal coordinates xi, the energy is
   rho E = sum w (u^2 + v^2)/2 G + sum w H/2 = rho |U|^2/2 + (2 + internal_dof) rho T/4, and
   the equilibrium of H is internal_dof T/2 times that of G.  It doubles the f storage. */
typedef struct {
  int nu, nv;
  double umax, vmax;
  int internal_dof;
} ugks_vgrid;

#define UGKS_BC_PERIODIC 0 /* periodic in x and y */
#define UGKS_BC_CHANNEL 1  /* Sec. 3.A: pressure inlet (x = 0), outlet (x = lx), walls at y = 0, ly */

/* Boundary conditions.  For the channel: p_in / p_out = p_ratio with mean pressure
   p0 = rho0 T0 / 2, so p_in = 2 r p0/(r+1) and p_out = 2 p0/(r+1).  The inlet ghost column
   holds p_in and T_in with (U, V) copied from the first column (inlet_fixed_u = 0) or with
   U = U_in (1 + U_noise xi_j), V = 0 (inlet_fixed_u = 1; xi_j seeded, see ugks_opts.seed).
   The outlet ghost holds p_out with (U, V, T) copied from the last column.  Walls are
   diffuse and isothermal at T_wall with zero net mass flux.  Ignored when periodic. */
typedef struct {
  int kind;
  int inlet_fixed_u;
  double p_ratio;
  double T_in, T_wall;
  double U_in, U_noise;
} ugks_bc;

#define UGKS_FP64 0       /* f stored and computed in FP64 */
#define UGKS_FP32_STORE 1 /* f stored in FP32; moments, W and the scalar flux work in FP64 */

/* Run options.
   precision        UGKS_FP64 or UGKS_FP32_STORE.
   cfl              time step dt = cfl / (umax/dx + vmax/dy) unless dt_override > 0.
   rho0, T0, noise  initial state: rho = rho0 (1 + noise xi_c), U = V = 0, T = T0, and f the
                    discrete Maxwellian of that state (|noise| < 1; H = internal_dof T0/2 G).
   velocity_chunks  Each velocity quadrant of a row segment is split over G workgroups.
                    0: automatic, enough to fill the GPU with this solver alone (at most 16
                    and nu/2); n in 1..16: at most n (the automatic choice capped at n).
                    Solvers that are stepped in large batches gain from a small cap.  Results
                    depend on G only through the order in which velocity sums are added.
                    The same cap bounds the update kernel's v-range chunks (more than one
                    only on meshes too small to fill the GPU otherwise; they change only the
                    rounding of the v-direction Gaussians, started at each chunk's first node).
   seed             xi_c is output c = j*nx + i of the SplitMix64 generator seeded with
                    `seed` (output k = mix(seed + (k+1) * 0x9E3779B97F4A7C15)), mapped to
                    [-1, 1) as 2 (z >> 11) 2^-53 - 1; the inlet noise xi_j uses output
                    nx*ny + j.
   stream           hipStream_t for all work of the handle.
   workspace        optional device buffer of at least ugks_required_bytes() bytes, aligned
                    to 256 bytes; NULL lets the library allocate.
   prandtl          collision model: 0 or 1 selects the paper's BGK operator (Eq. (1));
                    0 < prandtl < 1 the Shakhov model with that Prandtl number (2/3 for a
                    monatomic gas): the equilibrium g becomes g (1 + S) with
                    S = (1 - Pr)(lambda^2/rho)(c . q)(2 lambda |c|^2 - 4), c = u - U and q the
                    heat flux; at an interface S comes from the reconstructed f and is held
                    over the step, in a cell from f^n for both time levels of Eq. (3).
                    Requires internal_dof = 0; other values give UGKS_E_INVAL.
   adaptive_dt      0: every step takes dt (above).  1: each step takes
                    dt^n = cfl / max over cells of [(umax + |U|)/dx + (vmax + |V|)/dy] from
                    the state W^n it starts from (a global max-reduction on the device): the
                    fixed step at rest, smaller where the gas moves.  The paper fixes no time
                    step; this bounds the Courant number of the fastest discrete velocity plus
                    the local flow speed.  Needs dt_override = 0.  ugks_get_time reports the
                    simulated time and the next step. */
typedef struct {
  int precision;
  int velocity_chunks;
  double cfl;
  double rho0, T0, noise;
  uint64_t seed;
  double dt_override;
  void* stream;
  void* workspace;
  size_t workspace_bytes;
  double prandtl;
  int adaptive_dt;
} ugks_opts;

typedef struct {
  int nx, ny, nu, nv;
  int plane_stride; /* values between the velocity planes of f in device memory: f is
                       stored per velocity as (ny+4) x (nx+4) padded planes */
  int precision;
  int internal_dof;  /* as created; f then holds G and H, 2 nu nv values per cell */
  double dx, dy, dt;
  double tau_ref;  /* collision time at rho = T = 1; +inf in the collisionless limit */
  int64_t steps;   /* steps enqueued so far */
  size_t device_bytes;
  double prandtl;  /* 1: BGK; below 1: the Shakhov model with this Prandtl number */
  /* How the solver's steps split its velocities when it runs alone (a serving batch keeps
     the moment chunks and chooses the update chunks for the whole batch): */
  int moment_chunks;  /* u-range chunks per quadrant of the moment kernel (fixed at create) */
  int update_chunks;  /* u-range chunks per quadrant and update workgroup */
  int update_chunks_per_workgroup;  /* 2: FP64 workgroups of eight wavefronts; 1: four */
  int update_v_chunks; /* v-range chunks per half of the update kernel (fixed at create; more
                          than 1 only on meshes too small to fill the GPU otherwise) */
} ugks_info;

/* Device bytes a handle of this shape needs (f twice, twice more with internal degrees of
   freedom; ghosts, moment sums, more of them with the Shakhov model, face records,
   W, velocity tables).  Pure host arithmetic: no HIP call. */
int ugks_required_bytes(const ugks_mesh* mesh, const ugks_vgrid* vgrid, const ugks_opts* opts,
                        size_t* out_bytes);

/* Debug option: with the environment variable UGKS_DEBUG_POISON=1 at ugks_create, every cell
   value of the f and W buffers that the first step writes starts as NaN, and in a channel also
   the inlet and outlet ghost columns of that f (the rest of its halo is left as it is), so a
   step that fails to write a value it later reads leaves a NaN in the state. */

/* Create a solver and initialise its state on the device.  kn is the Knudsen number on the
   y extent of the domain (Sec. 3.A defines Kn on the channel width); kn = +INFINITY selects
   the collisionless limit (tau = inf).  The collision time is tau = mu/p with the hard-sphere
   viscosity mu = (5 sqrt(pi)/16) kn T^(1/2) and p = rho T/2.  On success *out receives the
   handle; on failure *out is NULL and the message is kept for ugks_last_error(NULL). */
int ugks_create(const ugks_mesh* mesh, const ugks_vgrid* vgrid, double kn, const ugks_bc* bc,
                const ugks_opts* opts, ugks_handle** out);

/* Enqueue n >= 0 time steps (Eqs. (2)-(4), steps S1-S8 at every interface) on the handle's
   stream and return without waiting.  Invalid states reached inside a step are flagged on
   the device and reported by the next ugks_moments / ugks_get_state.  If a kernel launch
   fails (UGKS_E_DEVICE), the steps enqueued in full are counted and the handle is marked
   failed: its state is unknown and every later call except ugks_destroy, ugks_last_error and
   ugks_get_info returns UGKS_E_DEVICE. */
int ugks_step(ugks_handle* h, int n);

/* ugks_step for callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid allocation): the same n steps, with the
   transient buffers of each step (per-cell and ghost moment sums, face records) in a
   static device array of UGKS_STATIC_SCRATCH_BYTES that the library holds on every GPU it
   runs on, instead of the handle's workspace.  It calls no allocating routine and records no
   timing events.  The handle's state advances exactly as with ugks_step (bitwise), and the two
   calls may be mixed.  All calls on one GPU share the array: calls on different streams that
   overlap in time race and corrupt each other's results; calls ordered on one stream do not
   interfere (each step rewrites every transient value before reading it).  ugks_get_face_flux
   refuses (UGKS_E_INVAL) until the next ugks_step.  UGKS_E_INVAL also when the handle's
   transient buffers exceed the array (the 400 x 100 x 40^2 channel needs 41 MB) or when the
   array's device address could not be taken at ugks_create; ugks_last_error says which. */
#define UGKS_STATIC_SCRATCH_BYTES ((size_t)48 << 20)
int ugks_step_static(ugks_handle* h, int n);

/* Wait for the stream, then write (rho, U, V, T) for every cell to host_out
   (4*nx*ny doubles, caller-owned).  These are the primitive variables of the conservative
   cell state W = (rho, rho U, rho V, rho E) that Eq. (4) advances; W is the velocity moment
   sum of w psi f with psi = (1, u, v, |c|^2/2) (Sec. 2), and T = 1/lambda follows from
   rho E = rho |U|^2/2 + (2 + internal_dof) rho T/4.  Returns UGKS_E_STATE (after writing)
   if any cell or interface state was invalid since creation. */
int ugks_moments(ugks_handle* h, double* host_out);

/* Release the handle and the device memory it owns; NULL is accepted and ignored. */
int ugks_destroy(ugks_handle* h);

/* Message of the last failure on h (or of the last failed ugks_create when h is NULL).
   The string belongs to the library and stays valid until the next call on h. */
const char* ugks_last_error(const ugks_handle* h);

/* Shape, step and memory of a handle. */
int ugks_get_info(const ugks_handle* h, ugks_info* out);

/* Simulated time (the sum of the steps taken, each the dt of Eq. (2)-(4) it integrated over)
   and the dt the next step takes (fixed, or the adaptive step of the current state).  Waits
   for the stream. */
int ugks_get_time(ugks_handle* h, double* time, double* dt_next);

/* Checkpoint / test hooks.  The state of the method is the distribution f of every cell and
   discrete velocity (Sec. 2, the f of Eq. (3)) together with the conservative variables W
   of Eq. (4).  f: nx*ny*NF doubles, W: 4*nx*ny doubles, canonical layout, caller-owned host
   memory; either may be NULL.  get waits for the stream; set replaces the current state
   (in FP32-store mode f is rounded to FP32).  Errors: UGKS_E_INVAL (NULL handle),
   UGKS_E_BUSY, UGKS_E_DEVICE (a copy failed), UGKS_E_STATE (get: an invalid state was
   flagged; the buffers are still written). */
int ugks_get_state(ugks_handle* h, double* f, double* W);
int ugks_set_state(ugks_handle* h, const double* f, const double* W);

/* Macroscopic face fluxes of the last step (the interface fluxes F of Eq. (4), built by the
   flux steps S1-S7 of Sec. 2.B), integrated over the step and multiplied by the face
   length, global frame: Fx[(j*(nx+1) + i)*4] through the left face of cell i in +x
   (i = nx is the right face of the last column), Fy[(j*nx + i)*4] through the bottom face of
   row j in +y (j = ny is the top face).  Host buffers of 4*(nx+1)*ny and 4*nx*(ny+1)
   doubles; either may be NULL. */
int ugks_get_face_flux(ugks_handle* h, double* Fx, double* Fy);

/* Per-kernel timing with HIP events recorded on the handle's stream around every launch.
   kernel: 0 boundary ghosts, 1 velocity moments, 2 interface scalars, 3 cell update.  Kernel 0
   runs only in a periodic box (a channel's update kernel writes the next step's ghost
   columns), so a channel reports no launches of it.  Enabling resets the totals; get waits
   for the stream and returns the summed milliseconds and the number of launches timed. */
int ugks_set_kernel_timing(ugks_handle* h, int on);
int ugks_get_kernel_timing(ugks_handle* h, int kernel, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------------------------
 * Serving: many independent solvers (any mix of meshes, velocity grids, Knudsen numbers and
 * boundary kinds) advanced together.  Callers: request loops that keep many solves resident on
 * one GPU and want their steps packed into shared launches.
 *
 * A batch owns a device launch plan for up to max_instances handles (the kernels find their
 * instance in it), a pinned staging copy and an event.  ugks_step_batch enqueues n steps of
 * every handle in hs[0..count) with one launch per phase covering all of them and returns
 * without waiting.  Requirements: the handles are distinct and share one precision and one
 * collision model (BGK, or Shakhov with any Prandtl numbers).  A handle
 * created on another stream is adopted: the batch's stream (the stream argument of
 * ugks_batch_create) first waits for the work already enqueued for it, and from then on the
 * handle's work, including ugks_moments and ugks_destroy, runs on the batch's stream.  Each
 * handle's result is bitwise the one ugks_step would give it alone.  The plan is rebuilt and re-sent only when
 * the member list changes or a member was stepped outside the batch; a rebuild first waits for
 * the previous plan upload.  Errors: UGKS_E_INVAL (arguments), UGKS_E_BUSY (a handle in use),
 * UGKS_E_DEVICE (launch failure, or a member that had one; the message is in
 * ugks_batch_last_error).  After a launch failure the steps enqueued in full count for every
 * member and every member is marked failed, as with ugks_step. */
typedef struct ugks_batch ugks_batch;
int ugks_batch_create(void* stream, int max_instances, ugks_batch** out);
int ugks_step_batch(ugks_batch* b, ugks_handle* const* hs, int count, int n);
int ugks_batch_destroy(ugks_batch* b); /* waits for the stream; NULL is accepted */
const char* ugks_batch_last_error(const ugks_batch* b);

#ifdef __cplusplus
}
#endif
#endif
