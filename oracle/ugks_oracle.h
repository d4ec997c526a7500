/*
 * Plain FP64 CPU oracle for one time step of the 2D unified gas-kinetic scheme (UGKS).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or call this
 * library: only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no code, header, table or helper with the HIP implementation.
 *
 * What it computes (paper: "Performance Comparison on Parallel CPU and GPU Algorithms for
 * Unified Gas-Kinetic Scheme", Liu, Hu & Li):
 *   - BGK model with a Maxwellian equilibrium, Eq. (1), 2D gas, velocities in units of
 *     sqrt(2kT0/m) so that lambda = 1/T.  The paper's gas has no internal degrees of
 *     freedom (dof = 0); dof > 0 carries the reduced distributions G and H (the internal
 *     energy), a variant beyond the paper.
 *   - Finite volumes over nx*ny cells, nu*nv discrete velocities per cell (Sec. 2).
 *   - Interface distribution from the integral solution, Eq. (2), assembled through the
 *     flux steps S1-S8 of Sec. 2.B (moments, Maxwellian moments, time weights, micro slopes,
 *     equilibrium flux, interface Maxwellian, free-transport flux, distribution flux).
 *   - Cell update of f with the trapezoidal collision term, Eq. (3), and of W, Eq. (4).
 *   - Variant collision model: Shakhov's, for a Prandtl number below 1.
 * The construction inside S1-S8 that the paper leaves to its references is restated from the
 * mathematics; every reading taken where the paper is silent is listed in the repository's
 * design notes and repeated at the function that implements it.
 *
 * Layout: f[(j*nx + i)*NF + c*NV + k*nv + m], NV = nu*nv, NF = NV (dof = 0) or 2*NV
 * (c = 0: G, c = 1: H), no padding; W[(j*nx + i)*4 + q] with
 * W = (rho, rho U, rho V, rho E).  Face fluxes are in the global frame: Fx[(j*(nx+1) + i)*4]
 * is the flux through the left face of cell i in +x; Fy[(j*nx + i)*4] through the bottom face
 * of row j in +y.
 */
#ifndef UGKS_ORACLE_H
#define UGKS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int nx, ny;
  double lx, ly;
  int nu, nv;
  double umax, vmax;
  double kn;               /* Knudsen number; +INFINITY selects the collisionless limit */
  int bc;                  /* 0: periodic in x and y; 1: channel (pressure inlet/outlet, walls) */
  int inlet_fixed_u;       /* channel: 0 copies (U,V) of the first column into the inlet ghost;
                              1 uses U = U_in*(1 + U_noise*xi_row), V = 0 */
  double p_ratio;          /* channel: p_in / p_out, with mean pressure rho0*T0/2 */
  double T_in, T_wall;
  double U_in, U_noise;
  double cfl;
  double rho0, T0, noise;  /* initial rho = rho0*(1 + noise*xi_cell), U = V = 0, T = T0 */
  uint64_t seed;
  double dt_override;      /* > 0 replaces the CFL step */
  int dof;                 /* internal degrees of freedom, 0..16 (0: the paper's gas) */
  double prandtl;          /* collision model: 1 BGK (the paper's), < 1 Shakhov with this
                              Prandtl number (dof = 0 only) */
  int adaptive_dt;         /* 0: fixed step; 1: each step's dt from the state at its start,
                              dt = cfl / max_cells[(umax + |U|)/dx + (vmax + |V|)/dy]
                              (needs dt_override = 0) */
} ugks_ref_case;

typedef struct ugks_ref ugks_ref;

/* state */
ugks_ref* ugks_ref_create(const ugks_ref_case* c);      /* NULL on invalid input */
int ugks_ref_step(ugks_ref* s, int n);                  /* 0, or -4 on an invalid state */
void ugks_ref_get_state(const ugks_ref* s, double* f, double* W);
void ugks_ref_set_state(ugks_ref* s, const double* f, const double* W);
void ugks_ref_get_face_flux(const ugks_ref* s, double* Fx, double* Fy);
void ugks_ref_get_ghost(const ugks_ref* s, double* Wg, double* fg);  /* [2][ny][4], [2][ny][NF] */
/* per-velocity face fluxes of the last step: [ny][nx+1][NF] and [ny+1][nx][NF] */
void ugks_ref_get_micro_flux(const ugks_ref* s, double* Ffx, double* Ffy);
double ugks_ref_dt(const ugks_ref* s);    /* the step the next ugks_ref_step takes */
double ugks_ref_time(const ugks_ref* s);  /* simulated time: the sum of the steps taken */
/* the adaptive step of a state W (ncell cells): cfl / max over cells of
   (umax + |U|)/dx + (vmax + |V|)/dy; 0 if a cell has rho <= 0 */
double ugks_ref_adaptive_dt(const double* W, int ncell, double cfl, double umax, double vmax,
                            double dx, double dy);
double ugks_ref_tau_ref(const ugks_ref* s);
void ugks_ref_destroy(ugks_ref* s);
void ugks_ref_set_threads(int n);
int ugks_ref_get_threads(void);

/* building blocks, exported so that tests can pin each one on its own */
uint64_t ugks_ref_splitmix64(uint64_t seed, uint64_t k);
double ugks_ref_unit_noise(uint64_t seed, uint64_t k);
void ugks_ref_nodes(int n, double a, double* x, double* w);
double ugks_ref_maxwellian(const double prim[4], double u, double v);
int ugks_ref_prim(const double W[4], double prim[4], int dof);
double ugks_ref_vanleer(double p, double q);
void ugks_ref_moments_1d(double U, double lam, double full[7], double pos[7], double neg[7]);
void ugks_ref_micro_slope(const double prim[4], const double s[4], double a[4], int dof);
void ugks_ref_time_weights(double dt, double tau, double Mt[5]);
void ugks_ref_time_slope(const double prim[4], const double aL[4], const double aR[4],
                         const double b[4], double A[4], int dof);
void ugks_ref_equilibrium_flux(const double prim[4], const double aL[4], const double aR[4],
                               const double b[4], const double A[4], const double Mt[5],
                               double Feq[4], int dof);
/* one interior face in its local frame (normal velocity un, tangential ut);
   returns 0 or -4; Ff may be NULL.  With dof > 0, fhat, sn, st and Ff hold G then H
   (2*nvel values). */
int ugks_ref_face(int nvel, const double* un, const double* ut, const double* w,
                  const double* fhat, const double* sn, const double* st,
                  const double WL[4], const double WR[4], double dn, double len, double dt,
                  double mu_ref, int collisionless, double FW[4], double* Ff, int dof,
                  double prandtl);
/* Shakhov factor S at velocity (u, v): g+ = g (1 + S); q = heat flux, pr = Prandtl number */
double ugks_ref_shakhov(const double prim[4], const double q[2], double pr, double u, double v);

#ifdef __cplusplus
}
#endif
#endif
