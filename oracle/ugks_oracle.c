/*
 * Plain FP64 CPU oracle for the 2D UGKS time step.  TEST INFRASTRUCTURE ONLY: used by the
 * tests, the smoke check and the CPU-baseline leg of the benchmark, never by the product.
 * Built with -O2 -ffp-contract=off (no fused multiply-add, no fast math).
 *
 * Internal degrees of freedom (dof > 0, a variant beyond the paper's monatomic 2D gas): the
 * distribution is carried as the two reduced functions G = int f dxi and H = int |xi|^2 f dxi
 * over the dof internal coordinates xi, stored one after the other per cell (G then H).  The
 * equilibrium of H is dof/(2 lambda) times that of G and the energy variable is
 * psi_4 = (u^2 + v^2 + |xi|^2)/2, whose Gaussian moments need <|xi|^2> = dof/(2 lambda) and
 * <|xi|^4> = dof (dof + 2)/(4 lambda^2).
 *
 * Shakhov collision model (prandtl < 1, a variant beyond the paper's BGK operator, for the gas
 * without internal degrees of freedom): the equilibrium g is replaced by g (1 + S) with
 * S = (1 - Pr) (lambda^2 / rho) (c . q) (2 lambda |c|^2 - 4), c = u - U, q = sum w c |c|^2 f / 2
 * the heat flux; its heat flux is (1 - Pr) q and it carries no mass, momentum or energy.
 * prandtl = 1 is BGK exactly.
 *
 * Every function cites the part of the paper it follows.  Where the paper is silent (it
 * leaves the interface-flux construction to its references), the step is restated from the
 * integral solution, Eq. (2), and the reading taken is named in the comment ("reading: ...").
 */
#include "ugks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define HS_OMEGA 0.5 /* hard-sphere viscosity exponent, mu ~ T^omega (reading) */

struct ugks_ref {
  ugks_ref_case c;
  int K, M, NV;
  int NC, NF;                   /* reduced functions per velocity (1, or 2 with dof > 0); NC*NV */
  double pr;                    /* Prandtl number of the collision model (1: BGK) */
  double dx, dy, dt, mu_ref;     /* dt: the step the next ugks_ref_step takes */
  double time;                  /* simulated time: the sum of the steps taken */
  int collisionless;
  double *uk, *vm, *wk, *wm;    /* 1D nodes and trapezoid weights */
  double *fu, *fv, *fw;         /* the same per velocity k*M + m: u_k, v_m, w_k w_m */
  double *f, *fnew, *W, *Wnew;
  double *sx, *sy;              /* limited slopes of f, per cell and velocity */
  double *Fx, *Fy;              /* macroscopic face fluxes, global frame */
  double *Ffx, *Ffy;            /* distribution fluxes, per face and velocity */
  double *Wg, *fg;              /* channel ghost columns: [2][ny][4], [2][ny][NV] */
  double *xi_in;                /* seeded inlet noise per row */
};

/* ---------------------------------------------------------------------------------------
 * Seeded noise.  SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) written as a counter-based
 * generator: output k of the generator seeded with s is mix(s + (k+1)*gamma).
 * ------------------------------------------------------------------------------------- */
uint64_t ugks_ref_splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* uniform in [-1, 1): the top 53 bits as a fraction, mapped affinely */
double ugks_ref_unit_noise(uint64_t seed, uint64_t k) {
  uint64_t z = ugks_ref_splitmix64(seed, k);
  return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

/* ---------------------------------------------------------------------------------------
 * Discrete velocity space, Sec. 2: K x M points (u_k, v_m).  Reading: uniform nodes on
 * [-a, a] including both ends, trapezoid weights; the grid is made exactly mirror-symmetric.
 * ------------------------------------------------------------------------------------- */
void ugks_ref_nodes(int n, double a, double* x, double* w) {
  double h = 2.0 * a / (double)(n - 1);
  for (int k = 0; k < n; ++k) x[k] = -a + (double)k * h;
  for (int k = 0; k < n / 2; ++k) x[n - 1 - k] = -x[k];
  if (n % 2) x[n / 2] = 0.0;
  for (int k = 0; k < n; ++k) w[k] = h;
  w[0] = 0.5 * h;
  w[n - 1] = 0.5 * h;
}

/* ---------------------------------------------------------------------------------------
 * Maxwellian of Eq. (1) in 2D: g = rho (lambda/pi) exp(-lambda((u-U)^2 + (v-V)^2)),
 * lambda = m/(2kT) = 1/T in the units used.  prim = (rho, U, V, lambda).
 * ------------------------------------------------------------------------------------- */
double ugks_ref_maxwellian(const double p[4], double u, double v) {
  double du = u - p[1];
  double dv = v - p[2];
  return p[0] * (p[3] / M_PI) * exp(-p[3] * (du * du + dv * dv));
}

/* Conservative W = (rho, rho U, rho V, rho E) <-> prim.  Two translational and dof internal
   degrees of freedom, each holding 1/(4 lambda) per unit mass:
   rho E = rho (U^2 + V^2)/2 + (dof + 2) rho/(4 lambda) (reading; dof = 0 is the paper's gas). */
int ugks_ref_prim(const double W[4], double p[4], int dof) {
  double rho = W[0];
  if (!(rho > 0.0) || !isfinite(rho)) return -4;
  double U = W[1] / rho;
  double V = W[2] / rho;
  double e = W[3] - 0.5 * rho * (U * U + V * V); /* = (dof + 2) rho / (4 lambda) */
  if (!(e > 0.0) || !isfinite(e)) return -4;
  p[0] = rho;
  p[1] = U;
  p[2] = V;
  p[3] = 0.25 * (double)(dof + 2) * rho / e;
  if (!isfinite(p[1]) || !isfinite(p[2]) || !isfinite(p[3])) return -4;
  return 0;
}

static void cons_from_prim(const double p[4], int dof, double W[4]) {
  W[0] = p[0];
  W[1] = p[0] * p[1];
  W[2] = p[0] * p[2];
  W[3] = 0.5 * p[0] * (p[1] * p[1] + p[2] * p[2]) + 0.25 * (double)(dof + 2) * p[0] / p[3];
}

/* Gaussian moments of the internal coordinates at lambda: <|xi|^2> and <|xi|^4> */
static void xi_moments(double lam, int dof, double* x2, double* x4) {
  *x2 = (double)dof / (2.0 * lam);
  *x4 = (double)(dof * (dof + 2)) / (4.0 * lam * lam);
}

/* Collision time of the BGK operator, Eq. (1).  Reading: tau = mu/p with a hard-sphere
   viscosity mu = mu_ref T^omega, omega = 1/2, and p = rho T/2. */
static double collision_time(double mu_ref, const double p[4]) {
  double T = 1.0 / p[3];
  double mu = mu_ref * pow(T, HS_OMEGA);
  return mu / (0.5 * p[0] * T);
}

/* Reading: mu_ref from the hard-sphere mean free path, Kn = mfp / channel width at
   rho = T = 1, which gives mu_ref = 5 sqrt(pi) Kn / 16. */
static double viscosity_ref(double kn) { return 5.0 * sqrt(M_PI) * kn / 16.0; }

/* ---------------------------------------------------------------------------------------
 * Second-order reconstruction of f in physical space (Sec. 2.A, "second order
 * interpolation").  Reading: van Leer limiter on the two one-sided differences.
 * ------------------------------------------------------------------------------------- */
double ugks_ref_vanleer(double p, double q) {
  if (p * q > 0.0) return 2.0 * p * q / (p + q);
  return 0.0;
}

/* ---------------------------------------------------------------------------------------
 * S2: moments of the normalised Maxwellian along one velocity axis, for the whole line and
 * for the half lines u > 0 ("from the left") and u < 0 ("from the right").
 * <u^0> over the half lines is erfc/2; <u^1> adds the boundary term of the Gaussian; for
 * n >= 2 all three follow <u^n> = U <u^(n-1)> + (n-1)/(2 lambda) <u^(n-2)>, which is
 * integration by parts of u^(n-1) (u - U) exp(-lambda (u-U)^2).
 * ------------------------------------------------------------------------------------- */
void ugks_ref_moments_1d(double U, double lam, double full[7], double pos[7], double neg[7]) {
  double edge = exp(-lam * U * U) / (2.0 * sqrt(M_PI * lam));
  full[0] = 1.0;
  full[1] = U;
  pos[0] = 0.5 * erfc(-sqrt(lam) * U);
  pos[1] = U * pos[0] + edge;
  neg[0] = 0.5 * erfc(sqrt(lam) * U);
  neg[1] = U * neg[0] - edge;
  for (int n = 2; n < 7; ++n) {
    double c = (double)(n - 1) / (2.0 * lam);
    full[n] = U * full[n - 1] + c * full[n - 2];
    pos[n] = U * pos[n - 1] + c * pos[n - 2];
    neg[n] = U * neg[n - 1] + c * neg[n - 2];
  }
}

/* <u^a v^b psi>, psi = (1, u, v, (u^2 + v^2 + |xi|^2)/2), with normal moments Mu, tangential
   Mv and x2 = <|xi|^2> (xi independent of u and v) */
static void mom_psi(const double* Mu, const double* Mv, int a, int b, double x2, double out[4]) {
  out[0] = Mu[a] * Mv[b];
  out[1] = Mu[a + 1] * Mv[b];
  out[2] = Mu[a] * Mv[b + 1];
  out[3] = 0.5 * (Mu[a + 2] * Mv[b] + Mu[a] * Mv[b + 2] + x2 * Mu[a] * Mv[b]);
}

/* <u^a v^b psi (c . psi)>; the |xi|^2 part of c_4 psi_4 brings <|xi|^2 u^a v^b psi> */
static void mom_psi_c(const double* Mu, const double* Mv, int a, int b, double x2, double x4,
                      const double c[4], double out[4]) {
  double t0[4], t1[4], t2[4], t3[4], t4[4], tx[4];
  mom_psi(Mu, Mv, a, b, x2, t0);
  mom_psi(Mu, Mv, a + 1, b, x2, t1);
  mom_psi(Mu, Mv, a, b + 1, x2, t2);
  mom_psi(Mu, Mv, a + 2, b, x2, t3);
  mom_psi(Mu, Mv, a, b + 2, x2, t4);
  tx[0] = x2 * Mu[a] * Mv[b];
  tx[1] = x2 * Mu[a + 1] * Mv[b];
  tx[2] = x2 * Mu[a] * Mv[b + 1];
  tx[3] = 0.5 * (x2 * (Mu[a + 2] * Mv[b] + Mu[a] * Mv[b + 2]) + x4 * Mu[a] * Mv[b]);
  for (int q = 0; q < 4; ++q)
    out[q] = c[0] * t0[q] + c[1] * t1[q] + c[2] * t2[q] +
             0.5 * c[3] * (t3[q] + t4[q] + tx[q]);
}

/* ---------------------------------------------------------------------------------------
 * S4: micro slope.  Given prim and a moment vector s, find a = (a1..a4) such that the
 * moments of rho g (a . psi) equal s.  The 4x4 system has the closed-form solution below
 * (2D gas with dof internal degrees of freedom; the energy row carries (dof + 2)).
 * ------------------------------------------------------------------------------------- */
void ugks_ref_micro_slope(const double p[4], const double s[4], double a[4], int dof) {
  double rho = p[0], U = p[1], V = p[2], lam = p[3];
  double q2 = U * U + V * V + (double)(dof + 2) / (2.0 * lam);
  double R2 = s[1] - U * s[0];
  double R3 = s[2] - V * s[0];
  double R4 = 2.0 * s[3] - q2 * s[0];
  a[3] = 4.0 * lam * lam / ((double)(dof + 2) * rho) * (R4 - 2.0 * U * R2 - 2.0 * V * R3);
  a[2] = 2.0 * lam * R3 / rho - V * a[3];
  a[1] = 2.0 * lam * R2 / rho - U * a[3];
  a[0] = s[0] / rho - U * a[1] - V * a[2] - 0.5 * a[3] * q2;
}

/* ---------------------------------------------------------------------------------------
 * S3: time weights.  Integrating Eq. (2) over one step [0, dt] with a linear-in-time
 * equilibrium and a linear initial f gives five weights:
 *   Mt1 = int (1 - e^{-t/tau})                     (equilibrium)
 *   Mt2 = -int (tau(1 - e^{-t/tau}) - t e^{-t/tau}) (equilibrium space slopes)
 *   Mt3 = int (t - tau(1 - e^{-t/tau}))             (equilibrium time slope)
 *   Mt4 = int e^{-t/tau}                            (free transport of f)
 *   Mt5 = int t e^{-t/tau}                          (free transport of the f slopes)
 * evaluated through expm1.  tau = +inf gives (0, 0, 0, dt, dt^2/2).
 * ------------------------------------------------------------------------------------- */
void ugks_ref_time_weights(double dt, double tau, double Mt[5]) {
  if (isinf(tau)) {
    Mt[0] = 0.0;
    Mt[1] = 0.0;
    Mt[2] = 0.0;
    Mt[3] = dt;
    Mt[4] = 0.5 * dt * dt;
    return;
  }
  double e = exp(-dt / tau);
  Mt[3] = -tau * expm1(-dt / tau);
  Mt[4] = tau * Mt[3] - tau * dt * e;
  Mt[0] = dt - Mt[3];
  Mt[1] = -tau * Mt[0] + Mt[4];
  Mt[2] = 0.5 * dt * dt - tau * Mt[0];
}

/* S4, time slope A.  Reading: compatibility of the linearised equilibrium with the BGK
   equation, int psi (A + u (a . psi) + v (b . psi)) g = 0, where the normal slope is aL for
   u > 0 and aR for u < 0. */
void ugks_ref_time_slope(const double p[4], const double aL[4], const double aR[4],
                         const double b[4], double A[4], int dof) {
  double full[7], pos[7], neg[7], tf[7], tp[7], tn[7], x2, x4;
  ugks_ref_moments_1d(p[1], p[3], full, pos, neg);
  ugks_ref_moments_1d(p[2], p[3], tf, tp, tn);
  xi_moments(p[3], dof, &x2, &x4);
  double m1[4], m2[4], m3[4], s[4];
  mom_psi_c(pos, tf, 1, 0, x2, x4, aL, m1);
  mom_psi_c(neg, tf, 1, 0, x2, x4, aR, m2);
  mom_psi_c(full, tf, 0, 1, x2, x4, b, m3);
  for (int q = 0; q < 4; ++q) s[q] = -p[0] * (m1[q] + m2[q] + m3[q]);
  ugks_ref_micro_slope(p, s, A, dof);
}

/* S5: equilibrium part of the macroscopic flux, from the analytic Maxwellian moments:
   rho [Mt1 <u psi> + Mt2 (<u^2 psi (aL.psi)>_{u>0} + <u^2 psi (aR.psi)>_{u<0}
        + <u v psi (b.psi)>) + Mt3 <u psi (A.psi)>] */
void ugks_ref_equilibrium_flux(const double p[4], const double aL[4], const double aR[4],
                               const double b[4], const double A[4], const double Mt[5],
                               double Feq[4], int dof) {
  double full[7], pos[7], neg[7], tf[7], tp[7], tn[7], x2, x4;
  ugks_ref_moments_1d(p[1], p[3], full, pos, neg);
  ugks_ref_moments_1d(p[2], p[3], tf, tp, tn);
  xi_moments(p[3], dof, &x2, &x4);
  double m0[4], mL[4], mR[4], mb[4], mA[4];
  mom_psi(full, tf, 1, 0, x2, m0);
  mom_psi_c(pos, tf, 2, 0, x2, x4, aL, mL);
  mom_psi_c(neg, tf, 2, 0, x2, x4, aR, mR);
  mom_psi_c(full, tf, 1, 1, x2, x4, b, mb);
  mom_psi_c(full, tf, 1, 0, x2, x4, A, mA);
  for (int q = 0; q < 4; ++q)
    Feq[q] = p[0] * (Mt[0] * m0[q] + Mt[1] * (mL[q] + mR[q] + mb[q]) + Mt[2] * mA[q]);
}

/* c . psi averaged over the internal coordinates with weight 1 (G, shift x2 = <|xi|^2>) or
   with weight |xi|^2 / <|xi|^2> (H, shift <|xi|^4>/<|xi|^2> = (dof + 2)/(2 lambda)) */
static double dot_psi(const double c[4], double un, double ut, double shift) {
  return c[0] + c[1] * un + c[2] * ut + c[3] * 0.5 * (un * un + ut * ut + shift);
}

/* ---------------------------------------------------------------------------------------
 * Shakhov correction (variant): g+ = g (1 + S) with
 *   S = (1 - Pr) (lambda^2/rho) (c . q) (2 lambda |c|^2 - 4),  c = (u - U, v - V),
 * the 2D form of the S-model written with p = rho/(2 lambda) and RT = 1/(2 lambda), so that
 * sum over the Gaussian of c |c|^2/2 g S = (1 - Pr) q and of psi g S = 0.
 * ------------------------------------------------------------------------------------- */
double ugks_ref_shakhov(const double p[4], const double q[2], double pr, double u, double v) {
  double cx = u - p[1], cy = v - p[2], lam = p[3];
  double cq = cx * q[0] + cy * q[1];
  return (1.0 - pr) * (lam * lam / p[0]) * cq * (2.0 * lam * (cx * cx + cy * cy) - 4.0);
}

/* Heat flux q = sum w c |c|^2 f / 2 about the velocity (U, V) of p (discrete, plain sum) */
static void heat_flux(int nvel, const double* un, const double* ut, const double* w,
                      const double* f, const double p[4], double q[2]) {
  q[0] = q[1] = 0.0;
  for (int v = 0; v < nvel; ++v) {
    double cx = un[v] - p[1], cy = ut[v] - p[2];
    double c2 = cx * cx + cy * cy;
    q[0] += 0.5 * w[v] * cx * c2 * f[v];
    q[1] += 0.5 * w[v] * cy * c2 * f[v];
  }
}

/* ---------------------------------------------------------------------------------------
 * One interior interface in its local frame (S1-S8).  Inputs per velocity: normal and
 * tangential velocity, quadrature weight, the upwinded reconstruction of f at the face
 * (fhat) and the upwinded normal and tangential slopes of f (sn, st).
 *   S1  W0 = sum w psi fhat and the tangential moment slope Wt = sum w psi st
 *       (reading: these are the eight sums of S1).
 *   S2  Maxwellian moments at prim0 = prim(W0).
 *   S3  tau0 from prim0 and the five time weights.
 *   S4  aL, aR from the one-sided differences of the conservative variables across the
 *       half cells (reading), b from Wt, A from compatibility.
 *   S5  equilibrium flux from analytic moments.
 *   S6  interface Maxwellian G at each discrete velocity.
 *   S7  free-transport flux: Mt4 sum w u psi fhat - Mt5 sum w u psi (u sn + v st)
 *       (the four sums of S7).
 *   S8  distribution flux per velocity.
 * Fluxes are integrated over the step and multiplied by the face length.
 * With dof > 0 the arrays fhat, sn, st and Ff hold 2*nvel values: G, then H, whose psi is
 * (0, 0, 0, 1/2) in the sums and whose equilibrium is dof/(2 lambda0) times that of G.
 * ------------------------------------------------------------------------------------- */
int ugks_ref_face(int nvel, const double* un, const double* ut, const double* w,
                  const double* fhat, const double* sn, const double* st, const double WL[4],
                  const double WR[4], double dn, double len, double dt, double mu_ref,
                  int collisionless, double FW[4], double* Ff, int dof, double pr) {
  int nc = dof > 0 ? 2 : 1;
  double W0[4] = {0, 0, 0, 0}, Wt[4] = {0, 0, 0, 0}, Q1[4] = {0, 0, 0, 0},
         Q2[4] = {0, 0, 0, 0};
  for (int v = 0; v < nvel; ++v) {
    double psi[4] = {1.0, un[v], ut[v], 0.5 * (un[v] * un[v] + ut[v] * ut[v])};
    double tr = un[v] * sn[v] + ut[v] * st[v];
    for (int q = 0; q < 4; ++q) {
      W0[q] += w[v] * psi[q] * fhat[v];
      Wt[q] += w[v] * psi[q] * st[v];
      Q1[q] += w[v] * un[v] * psi[q] * fhat[v];
      Q2[q] += w[v] * un[v] * psi[q] * tr;
    }
  }
  for (int v = nvel; v < nc * nvel; ++v) {
    int x = v - nvel;
    double tr = un[x] * sn[v] + ut[x] * st[v];
    W0[3] += w[x] * 0.5 * fhat[v];
    Wt[3] += w[x] * 0.5 * st[v];
    Q1[3] += w[x] * un[x] * 0.5 * fhat[v];
    Q2[3] += w[x] * un[x] * 0.5 * tr;
  }
  double Mt[5];
  if (collisionless) {
    ugks_ref_time_weights(dt, INFINITY, Mt);
    for (int q = 0; q < 4; ++q) FW[q] = len * (Mt[3] * Q1[q] - Mt[4] * Q2[q]);
    if (Ff)
      for (int v = 0; v < nc * nvel; ++v) {
        int x = v % nvel;
        Ff[v] = len * un[x] * (Mt[3] * fhat[v] - Mt[4] * (un[x] * sn[v] + ut[x] * st[v]));
      }
    return 0;
  }
  double p0[4];
  if (ugks_ref_prim(W0, p0, dof)) return -4;
  double tau0 = collision_time(mu_ref, p0);
  ugks_ref_time_weights(dt, tau0, Mt);
  double swL[4], swR[4], Wt_[4];
  for (int q = 0; q < 4; ++q) {
    swL[q] = (W0[q] - WL[q]) / (0.5 * dn);
    swR[q] = (WR[q] - W0[q]) / (0.5 * dn);
    Wt_[q] = Wt[q];
  }
  double aL[4], aR[4], b[4], A[4], Feq[4];
  ugks_ref_micro_slope(p0, swL, aL, dof);
  ugks_ref_micro_slope(p0, swR, aR, dof);
  ugks_ref_micro_slope(p0, Wt_, b, dof);
  ugks_ref_time_slope(p0, aL, aR, b, A, dof);
  ugks_ref_equilibrium_flux(p0, aL, aR, b, A, Mt, Feq, dof);
  /* Shakhov (variant): the correction of the initial interface equilibrium, g0 S0 with the
     heat flux q0 of the reconstructed f, is held over the step like the Mt1 part; its only
     macroscopic flux is the energy flux (1 - Pr) q0_n */
  double q0[2] = {0.0, 0.0};
  if (pr != 1.0) {
    heat_flux(nvel, un, ut, w, fhat, p0, q0);
    Feq[3] += Mt[0] * (1.0 - pr) * q0[0];
  }
  for (int q = 0; q < 4; ++q) FW[q] = len * (Feq[q] + Mt[3] * Q1[q] - Mt[4] * Q2[q]);
  if (Ff) {
    double x2, x4;
    xi_moments(p0[3], dof, &x2, &x4);
    for (int v = 0; v < nc * nvel; ++v) {
      int x = v % nvel, h = v >= nvel;
      double H = un[x] > 0.0 ? 1.0 : (un[x] < 0.0 ? 0.0 : 0.5);
      double a[4];
      for (int q = 0; q < 4; ++q) a[q] = H * aL[q] + (1.0 - H) * aR[q];
      /* H: weight |xi|^2 gives the factor x2 and the shift x4/x2 */
      double G = ugks_ref_maxwellian(p0, un[x], ut[x]) * (h ? x2 : 1.0);
      double shift = h ? x4 / x2 : x2;
      double poly = Mt[0] + Mt[1] * (un[x] * dot_psi(a, un[x], ut[x], shift) +
                                     ut[x] * dot_psi(b, un[x], ut[x], shift)) +
                    Mt[2] * dot_psi(A, un[x], ut[x], shift);
      if (pr != 1.0) poly += Mt[0] * ugks_ref_shakhov(p0, q0, pr, un[x], ut[x]);
      Ff[v] = len * un[x] *
              (G * poly + Mt[3] * fhat[v] - Mt[4] * (un[x] * sn[v] + ut[x] * st[v]));
    }
  }
  return 0;
}

/* ---------------------------------------------------------------------------------------
 * State
 * ------------------------------------------------------------------------------------- */
static size_t cidx(const ugks_ref* s, int i, int j) { return (size_t)j * s->c.nx + i; }

ugks_ref* ugks_ref_create(const ugks_ref_case* c) {
  if (!c || c->nx < 1 || c->ny < 1 || c->nu < 2 || c->nv < 2) return NULL;
  if (!(c->lx > 0) || !(c->ly > 0) || !(c->umax > 0) || !(c->vmax > 0)) return NULL;
  if (!(c->kn > 0) || !(c->rho0 > 0) || !(c->T0 > 0)) return NULL;
  if (c->bc != 0 && c->bc != 1) return NULL;
  if (c->dof < 0 || c->dof > 16) return NULL;
  if (!(c->prandtl > 0.0) || c->prandtl > 1.0) return NULL;
  if (c->prandtl != 1.0 && c->dof != 0) return NULL;  /* Shakhov: gas without internal dof */
  if (c->bc == 1 && (!(c->p_ratio > 0) || !(c->T_in > 0) || !(c->T_wall > 0))) return NULL;
  if (c->adaptive_dt != 0 && (c->adaptive_dt != 1 || c->dt_override > 0)) return NULL;
  ugks_ref* s = (ugks_ref*)calloc(1, sizeof(ugks_ref));
  s->c = *c;
  s->K = c->nu;
  s->M = c->nv;
  s->NV = c->nu * c->nv;
  s->NC = c->dof > 0 ? 2 : 1;
  s->NF = s->NC * s->NV;
  s->pr = c->prandtl;
  s->dx = c->lx / c->nx;
  s->dy = c->ly / c->ny;
  s->collisionless = isinf(c->kn) ? 1 : 0;
  s->mu_ref = viscosity_ref(c->kn);
  /* reading: fixed step from the CFL number and the largest discrete speeds */
  s->dt = c->dt_override > 0 ? c->dt_override
                             : c->cfl / (c->umax / s->dx + c->vmax / s->dy);
  size_t nc = (size_t)c->nx * c->ny, NV = (size_t)s->NF;
  s->uk = malloc(sizeof(double) * s->K);
  s->wk = malloc(sizeof(double) * s->K);
  s->vm = malloc(sizeof(double) * s->M);
  s->wm = malloc(sizeof(double) * s->M);
  ugks_ref_nodes(s->K, c->umax, s->uk, s->wk);
  ugks_ref_nodes(s->M, c->vmax, s->vm, s->wm);
  s->fu = malloc(sizeof(double) * s->NV);
  s->fv = malloc(sizeof(double) * s->NV);
  s->fw = malloc(sizeof(double) * s->NV);
  for (int k = 0; k < s->K; ++k)
    for (int m = 0; m < s->M; ++m) {
      s->fu[k * s->M + m] = s->uk[k];
      s->fv[k * s->M + m] = s->vm[m];
      s->fw[k * s->M + m] = s->wk[k] * s->wm[m];
    }
  s->f = malloc(sizeof(double) * nc * NV);
  s->fnew = malloc(sizeof(double) * nc * NV);
  s->sx = malloc(sizeof(double) * nc * NV);
  s->sy = malloc(sizeof(double) * nc * NV);
  s->W = malloc(sizeof(double) * nc * 4);
  s->Wnew = malloc(sizeof(double) * nc * 4);
  s->Fx = calloc((size_t)(c->nx + 1) * c->ny * 4, sizeof(double));
  s->Fy = calloc((size_t)c->nx * (c->ny + 1) * 4, sizeof(double));
  s->Ffx = malloc(sizeof(double) * (size_t)(c->nx + 1) * c->ny * NV);
  s->Ffy = malloc(sizeof(double) * (size_t)c->nx * (c->ny + 1) * NV);
  s->Wg = calloc((size_t)2 * c->ny * 4, sizeof(double));
  s->fg = calloc((size_t)2 * c->ny * NV, sizeof(double));
  s->xi_in = malloc(sizeof(double) * c->ny);
  if (!s->f || !s->fnew || !s->sx || !s->sy || !s->Ffx || !s->Ffy) {
    ugks_ref_destroy(s);
    return NULL;
  }
  /* initial state: rho = rho0 (1 + noise xi_cell), U = V = 0, T = T0; f = discrete
     Maxwellian of that state.  Cell c draws generator output c; inlet row j draws output
     nx*ny + j. */
  for (int j = 0; j < c->ny; ++j) {
    s->xi_in[j] = ugks_ref_unit_noise(c->seed, nc + (size_t)j);
    for (int i = 0; i < c->nx; ++i) {
      size_t ci = cidx(s, i, j);
      double p[4] = {c->rho0 * (1.0 + c->noise * ugks_ref_unit_noise(c->seed, ci)), 0.0, 0.0,
                     1.0 / c->T0};
      cons_from_prim(p, c->dof, s->W + 4 * ci);
      double kap = (double)c->dof / (2.0 * p[3]);  /* H = dof/(2 lambda) G at equilibrium */
      for (int k = 0; k < s->K; ++k)
        for (int m = 0; m < s->M; ++m) {
          size_t v = ci * NV + (size_t)k * s->M + m;
          s->f[v] = ugks_ref_maxwellian(p, s->uk[k], s->vm[m]);
          if (s->NC > 1) s->f[v + s->NV] = kap * s->f[v];
        }
    }
  }
  if (c->adaptive_dt) s->dt = ugks_ref_adaptive_dt(s->W, (int)nc, c->cfl, c->umax, c->vmax,
                                                   s->dx, s->dy);
  return s;
}

/* Reading (the paper fixes no time step): the adaptive step bounds the Courant number of the
   fastest discrete velocity on each axis plus the local flow speed of the cell, so that the
   grid of discrete velocities, centred on zero, still covers the flow's equilibrium; the
   largest such rate over all cells (a global max-reduction over the state at the start of
   the step) sets dt.  At rest it equals the fixed CFL step. */
double ugks_ref_adaptive_dt(const double* W, int ncell, double cfl, double umax, double vmax,
                            double dx, double dy) {
  double rmax = 0.0;
  for (int c = 0; c < ncell; ++c) {
    const double rho = W[4 * c];
    if (!(rho > 0.0)) return 0.0;
    const double U = W[4 * c + 1] / rho, V = W[4 * c + 2] / rho;
    const double r = (umax + fabs(U)) / dx + (vmax + fabs(V)) / dy;
    if (r > rmax) rmax = r;
  }
  return cfl / rmax;
}

void ugks_ref_destroy(ugks_ref* s) {
  if (!s) return;
  free(s->uk); free(s->wk); free(s->vm); free(s->wm);
  free(s->fu); free(s->fv); free(s->fw);
  free(s->f); free(s->fnew); free(s->sx); free(s->sy); free(s->W); free(s->Wnew);
  free(s->Fx); free(s->Fy); free(s->Ffx); free(s->Ffy); free(s->Wg); free(s->fg);
  free(s->xi_in);
  free(s);
}

double ugks_ref_dt(const ugks_ref* s) { return s->dt; }
double ugks_ref_time(const ugks_ref* s) { return s->time; }
double ugks_ref_tau_ref(const ugks_ref* s) {
  double p[4] = {1.0, 0.0, 0.0, 1.0};
  return s->collisionless ? INFINITY : collision_time(s->mu_ref, p);
}

void ugks_ref_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int ugks_ref_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void ugks_ref_get_state(const ugks_ref* s, double* f, double* W) {
  size_t nc = (size_t)s->c.nx * s->c.ny;
  if (f) memcpy(f, s->f, sizeof(double) * nc * s->NF);
  if (W) memcpy(W, s->W, sizeof(double) * nc * 4);
}
void ugks_ref_set_state(ugks_ref* s, const double* f, const double* W) {
  size_t nc = (size_t)s->c.nx * s->c.ny;
  if (f) memcpy(s->f, f, sizeof(double) * nc * s->NF);
  if (W) memcpy(s->W, W, sizeof(double) * nc * 4);
  if (W && s->c.adaptive_dt)
    s->dt = ugks_ref_adaptive_dt(s->W, (int)nc, s->c.cfl, s->c.umax, s->c.vmax, s->dx, s->dy);
}
void ugks_ref_get_face_flux(const ugks_ref* s, double* Fx, double* Fy) {
  if (Fx) memcpy(Fx, s->Fx, sizeof(double) * (size_t)(s->c.nx + 1) * s->c.ny * 4);
  if (Fy) memcpy(Fy, s->Fy, sizeof(double) * (size_t)s->c.nx * (s->c.ny + 1) * 4);
}
void ugks_ref_get_micro_flux(const ugks_ref* s, double* Ffx, double* Ffy) {
  size_t NV = (size_t)s->NF;
  if (Ffx) memcpy(Ffx, s->Ffx, sizeof(double) * (size_t)(s->c.nx + 1) * s->c.ny * NV);
  if (Ffy) memcpy(Ffy, s->Ffy, sizeof(double) * (size_t)s->c.nx * (s->c.ny + 1) * NV);
}
void ugks_ref_get_ghost(const ugks_ref* s, double* Wg, double* fg) {
  if (Wg) memcpy(Wg, s->Wg, sizeof(double) * 2 * (size_t)s->c.ny * 4);
  if (fg) memcpy(fg, s->fg, sizeof(double) * 2 * (size_t)s->c.ny * s->NF);
}

/* ---------------------------------------------------------------------------------------
 * O1, channel ghosts (Sec. 3.A: flow driven by a fixed inlet and outlet pressure).
 * Reading: the mean of p_in and p_out is p0 = rho0 T0 / 2 and their ratio is p_ratio.
 * Inlet: p_in and T_in fixed, (U, V) taken from the first column (or a fixed, seeded U).
 * Outlet: p_out fixed, (U, V, T) taken from the last column.  Ghost rho = 2 p / T, ghost
 * f = discrete Maxwellian of the ghost state (H: dof/(2 lambda) times it); ghost slopes are
 * zero.
 * ------------------------------------------------------------------------------------- */
static int channel_ghosts(ugks_ref* s) {
  const ugks_ref_case* c = &s->c;
  double p0 = 0.5 * c->rho0 * c->T0;
  double p_in = 2.0 * c->p_ratio * p0 / (c->p_ratio + 1.0);
  double p_out = 2.0 * p0 / (c->p_ratio + 1.0);
  for (int j = 0; j < c->ny; ++j) {
    double pin[4], pout[4], pr[4];
    if (ugks_ref_prim(s->W + 4 * cidx(s, 0, j), pr, c->dof)) return -4;
    if (c->inlet_fixed_u) {
      pin[1] = c->U_in * (1.0 + c->U_noise * s->xi_in[j]);
      pin[2] = 0.0;
    } else {
      pin[1] = pr[1];
      pin[2] = pr[2];
    }
    pin[3] = 1.0 / c->T_in;
    pin[0] = 2.0 * p_in / c->T_in;
    if (ugks_ref_prim(s->W + 4 * cidx(s, c->nx - 1, j), pr, c->dof)) return -4;
    double Tout = 1.0 / pr[3];
    pout[0] = 2.0 * p_out / Tout;
    pout[1] = pr[1];
    pout[2] = pr[2];
    pout[3] = pr[3];
    cons_from_prim(pin, c->dof, s->Wg + 4 * (size_t)j);
    cons_from_prim(pout, c->dof, s->Wg + 4 * ((size_t)c->ny + j));
    double kin = (double)c->dof / (2.0 * pin[3]), kout = (double)c->dof / (2.0 * pout[3]);
    double* gin = s->fg + (size_t)j * s->NF;
    double* gout = s->fg + ((size_t)c->ny + j) * s->NF;
    for (int k = 0; k < s->K; ++k)
      for (int m = 0; m < s->M; ++m) {
        size_t v = (size_t)k * s->M + m;
        gin[v] = ugks_ref_maxwellian(pin, s->uk[k], s->vm[m]);
        gout[v] = ugks_ref_maxwellian(pout, s->uk[k], s->vm[m]);
        if (s->NC > 1) {
          gin[v + s->NV] = kin * gin[v];
          gout[v + s->NV] = kout * gout[v];
        }
      }
  }
  return 0;
}

/* f of the x-neighbour (i + di, j): a cell, a wrapped cell, or a channel ghost */
static const double* fx_nb(const ugks_ref* s, int i, int j) {
  int nx = s->c.nx;
  if (i >= 0 && i < nx) return s->f + cidx(s, i, j) * s->NF;
  if (s->c.bc == 0) return s->f + cidx(s, (i + nx) % nx, j) * s->NF;
  return s->fg + ((size_t)(i < 0 ? 0 : s->c.ny) + j) * s->NF;
}

/* ---------------------------------------------------------------------------------------
 * O2, slopes.  sigma_x = VL(f_{i+1} - f_i, f_i - f_{i-1}) / dx, likewise in y.
 * Reading: in the first and last rows of a channel (next to the walls) sigma_y = 0; the
 * columns next to the inlet and outlet use the ghost value.
 * ------------------------------------------------------------------------------------- */
static void slopes(ugks_ref* s) {
  int nx = s->c.nx, ny = s->c.ny, NV = s->NF;  /* G and H alike */
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const double* f0 = s->f + cidx(s, i, j) * NV;
      const double* fw = fx_nb(s, i - 1, j);
      const double* fe = fx_nb(s, i + 1, j);
      double* sx = s->sx + cidx(s, i, j) * NV;
      double* sy = s->sy + cidx(s, i, j) * NV;
      int wall_row = s->c.bc == 1 && (j == 0 || j == ny - 1);
      const double* fs = s->f + cidx(s, i, (j - 1 + ny) % ny) * NV;
      const double* fn = s->f + cidx(s, i, (j + 1) % ny) * NV;
      for (int v = 0; v < NV; ++v) {
        sx[v] = ugks_ref_vanleer(fe[v] - f0[v], f0[v] - fw[v]) / s->dx;
        sy[v] = wall_row ? 0.0 : ugks_ref_vanleer(fn[v] - f0[v], f0[v] - fs[v]) / s->dy;
      }
    }
}

/* ---------------------------------------------------------------------------------------
 * Diffuse isothermal wall (not described in the paper; reading).  Particles leaving the
 * wall follow rho_w g(1, 0, 0, T_wall) with rho_w set by zero net discrete mass flux;
 * particles reaching it carry the wall-row cell value (first order in space and time).
 * F_f = dx dt v f_wall, F_W = sum w psi F_f.  top != 0: wall above the cell.  With dof > 0
 * the reflected H is dof/(2 lambda_w) times the reflected G and adds its energy to F_W.
 * ------------------------------------------------------------------------------------- */
static void wall_face(const ugks_ref* s, const double* fc, int top, double FW[4], double* Ff) {
  double pw[4] = {1.0, 0.0, 0.0, 1.0 / s->c.T_wall};
  double kw = (double)s->c.dof * s->c.T_wall / 2.0;
  double num = 0.0, den = 0.0;
  for (int k = 0; k < s->K; ++k)
    for (int m = 0; m < s->M; ++m) {
      double vv = s->vm[m], w = s->wk[k] * s->wm[m];
      size_t v = (size_t)k * s->M + m;
      int into = top ? vv > 0.0 : vv < 0.0;
      int from = top ? vv < 0.0 : vv > 0.0;
      if (into) num += w * vv * fc[v];
      if (from) den += w * vv * ugks_ref_maxwellian(pw, s->uk[k], vv);
    }
  double rho_w = -num / den;
  for (int q = 0; q < 4; ++q) FW[q] = 0.0;
  for (int k = 0; k < s->K; ++k)
    for (int m = 0; m < s->M; ++m) {
      double uu = s->uk[k], vv = s->vm[m], w = s->wk[k] * s->wm[m];
      size_t v = (size_t)k * s->M + m;
      int from = top ? vv < 0.0 : vv > 0.0;
      double fw = from ? rho_w * ugks_ref_maxwellian(pw, uu, vv) : fc[v];
      Ff[v] = s->dx * s->dt * vv * fw;
      double psi[4] = {1.0, uu, vv, 0.5 * (uu * uu + vv * vv)};
      for (int q = 0; q < 4; ++q) FW[q] += w * psi[q] * Ff[v];
      if (s->NC > 1) {
        size_t h = v + (size_t)s->NV;
        double hw = from ? kw * rho_w * ugks_ref_maxwellian(pw, uu, vv) : fc[h];
        Ff[h] = s->dx * s->dt * vv * hw;
        FW[3] += w * 0.5 * Ff[h];
      }
    }
}

/* O3-O5: all faces of the mesh.  x-face i of row j lies between cells i-1 and i. */
static int faces(ugks_ref* s) {
  int nx = s->c.nx, ny = s->c.ny, NV = s->NV, NF = s->NF, K = s->K, M = s->M;
  int dof = s->c.dof;
  int per = s->c.bc == 0;
  int err = 0;
#pragma omp parallel reduction(| : err)
  {
    double* un = malloc(sizeof(double) * NV);
    double* ut = malloc(sizeof(double) * NV);
    double* w = malloc(sizeof(double) * NV);
    double* fh = malloc(sizeof(double) * NF);
    double* sn = malloc(sizeof(double) * NF);
    double* st = malloc(sizeof(double) * NF);
    /* x-faces: normal u, tangential v, local W = W */
#pragma omp for schedule(static)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < (per ? nx : nx + 1); ++i) {
        int il = i - 1, ir = i;
        const double *fL, *fR, *sxL = NULL, *syL = NULL, *sxR = NULL, *syR = NULL;
        const double *WL, *WR;
        if (per) il = (il + nx) % nx;
        if (il >= 0) {
          fL = s->f + cidx(s, il, j) * NF;
          sxL = s->sx + cidx(s, il, j) * NF;
          syL = s->sy + cidx(s, il, j) * NF;
          WL = s->W + 4 * cidx(s, il, j);
        } else {
          fL = s->fg + (size_t)j * NF;
          WL = s->Wg + 4 * (size_t)j;
        }
        if (ir < nx) {
          fR = s->f + cidx(s, ir, j) * NF;
          sxR = s->sx + cidx(s, ir, j) * NF;
          syR = s->sy + cidx(s, ir, j) * NF;
          WR = s->W + 4 * cidx(s, ir, j);
        } else {
          fR = s->fg + ((size_t)ny + j) * NF;
          WR = s->Wg + 4 * ((size_t)ny + j);
        }
        for (int k = 0; k < K; ++k)
          for (int m = 0; m < M; ++m) {
            int v = k * M + m;
            un[v] = s->uk[k];
            ut[v] = s->vm[m];
            w[v] = s->wk[k] * s->wm[m];
            /* reading: H(0) = 1/2 */
            double H = un[v] > 0.0 ? 1.0 : (un[v] < 0.0 ? 0.0 : 0.5);
            for (int x = v; x < NF; x += NV) {  /* G, then H */
              double sxl = sxL ? sxL[x] : 0.0, syl = syL ? syL[x] : 0.0;
              double sxr = sxR ? sxR[x] : 0.0, syr = syR ? syR[x] : 0.0;
              fh[x] = H * (fL[x] + 0.5 * s->dx * sxl) + (1.0 - H) * (fR[x] - 0.5 * s->dx * sxr);
              sn[x] = H * sxl + (1.0 - H) * sxr;
              st[x] = H * syl + (1.0 - H) * syr;
            }
          }
        size_t fi = (size_t)j * (nx + 1) + i;
        if (ugks_ref_face(NV, un, ut, w, fh, sn, st, WL, WR, s->dx, s->dy, s->dt, s->mu_ref,
                          s->collisionless, s->Fx + 4 * fi, s->Ffx + fi * NF, dof, s->pr))
          err |= 1;
      }
    /* y-faces: normal v, tangential u, local W = (rho, rho V, rho U, rho E) */
#pragma omp for schedule(static)
    for (int j = 0; j < (per ? ny : ny + 1); ++j)
      for (int i = 0; i < nx; ++i) {
        size_t fi = (size_t)j * nx + i;
        if (!per && (j == 0 || j == ny)) {
          wall_face(s, s->f + cidx(s, i, j == 0 ? 0 : ny - 1) * NF, j == ny, s->Fy + 4 * fi,
                    s->Ffy + fi * NF);
          continue;
        }
        int jl = per ? (j - 1 + ny) % ny : j - 1, jr = j;
        size_t cl = cidx(s, i, jl), cr = cidx(s, i, jr);
        const double *fL = s->f + cl * NF, *fR = s->f + cr * NF;
        const double *sxL = s->sx + cl * NF, *syL = s->sy + cl * NF;
        const double *sxR = s->sx + cr * NF, *syR = s->sy + cr * NF;
        const double* WLg = s->W + 4 * cl;
        const double* WRg = s->W + 4 * cr;
        double WL[4] = {WLg[0], WLg[2], WLg[1], WLg[3]};
        double WR[4] = {WRg[0], WRg[2], WRg[1], WRg[3]};
        for (int k = 0; k < K; ++k)
          for (int m = 0; m < M; ++m) {
            int v = k * M + m;
            un[v] = s->vm[m];
            ut[v] = s->uk[k];
            w[v] = s->wk[k] * s->wm[m];
            double H = un[v] > 0.0 ? 1.0 : (un[v] < 0.0 ? 0.0 : 0.5);
            for (int x = v; x < NF; x += NV) {
              fh[x] = H * (fL[x] + 0.5 * s->dy * syL[x]) + (1.0 - H) * (fR[x] - 0.5 * s->dy * syR[x]);
              sn[x] = H * syL[x] + (1.0 - H) * syR[x];
              st[x] = H * sxL[x] + (1.0 - H) * sxR[x];
            }
          }
        double FWl[4];
        if (ugks_ref_face(NV, un, ut, w, fh, sn, st, WL, WR, s->dy, s->dx, s->dt, s->mu_ref,
                          s->collisionless, FWl, s->Ffy + fi * NF, dof, s->pr))
          err |= 1;
        double* F = s->Fy + 4 * fi;
        F[0] = FWl[0];
        F[1] = FWl[2];
        F[2] = FWl[1];
        F[3] = FWl[3];
      }
    free(un); free(ut); free(w); free(fh); free(sn); free(st);
  }
  if (per) {
    /* the last face of a periodic row or column is the first one */
    for (int j = 0; j < ny; ++j) {
      memcpy(s->Fx + 4 * ((size_t)j * (nx + 1) + nx), s->Fx + 4 * ((size_t)j * (nx + 1)),
             sizeof(double) * 4);
      memcpy(s->Ffx + ((size_t)j * (nx + 1) + nx) * NF, s->Ffx + ((size_t)j * (nx + 1)) * NF,
             sizeof(double) * NF);
    }
    memcpy(s->Fy + 4 * (size_t)ny * nx, s->Fy, sizeof(double) * 4 * nx);
    memcpy(s->Ffy + (size_t)ny * nx * NF, s->Ffy, sizeof(double) * (size_t)nx * NF);
  }
  return err ? -4 : 0;
}

/* ---------------------------------------------------------------------------------------
 * O6, cell update.  W first, Eq. (4) (fluxes carry the face length, so the divergence is
 * divided by the cell area); then f, Eq. (3), whose trapezoidal collision term is implicit
 * in f^{n+1} through g^{n+1} and tau^{n+1} built from W^{n+1}:
 *   f^{n+1} = [f^n + dF/(dx dy) + dt/2 (g^{n+1}/tau^{n+1} + (g^n - f^n)/tau^n)]
 *             / (1 + dt/(2 tau^{n+1})).
 * The collisionless limit drops the collision term.  H takes the same update with the
 * equilibria dof/(2 lambda^n) g^n and dof/(2 lambda^{n+1}) g^{n+1}.  Shakhov (variant): g^n
 * and g^{n+1} become g (1 + S) with the heat flux q^n of f^n at both levels (reading).
 * ------------------------------------------------------------------------------------- */
static int update(ugks_ref* s) {
  int nx = s->c.nx, ny = s->c.ny, NV = s->NF, NG = s->NV, K = s->K, M = s->M;
  int dof = s->c.dof;
  double area = s->dx * s->dy, dt = s->dt;
  int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t c = cidx(s, i, j);
      const double* Fl = s->Fx + 4 * ((size_t)j * (nx + 1) + i);
      const double* Fr = s->Fx + 4 * ((size_t)j * (nx + 1) + i + 1);
      const double* Fb = s->Fy + 4 * ((size_t)j * nx + i);
      const double* Ft = s->Fy + 4 * ((size_t)(j + 1) * nx + i);
      const double* Ffl = s->Ffx + ((size_t)j * (nx + 1) + i) * NV;
      const double* Ffr = s->Ffx + ((size_t)j * (nx + 1) + i + 1) * NV;
      const double* Ffb = s->Ffy + ((size_t)j * nx + i) * NV;
      const double* Fft = s->Ffy + ((size_t)(j + 1) * nx + i) * NV;
      double* W = s->W + 4 * c;
      double* Wn = s->Wnew + 4 * c;
      for (int q = 0; q < 4; ++q) Wn[q] = W[q] + (Fl[q] - Fr[q] + Fb[q] - Ft[q]) / area;
      const double* f = s->f + c * NV;
      double* fn = s->fnew + c * NV;
      if (s->collisionless) {
        for (int v = 0; v < NV; ++v) fn[v] = f[v] + (Ffl[v] - Ffr[v] + Ffb[v] - Fft[v]) / area;
        continue;
      }
      double pn[4], pn1[4];
      if (ugks_ref_prim(W, pn, dof) || ugks_ref_prim(Wn, pn1, dof)) {
        err |= 1;
        continue;
      }
      double tn = collision_time(s->mu_ref, pn), tn1 = collision_time(s->mu_ref, pn1);
      double kn = (double)dof / (2.0 * pn[3]), kn1 = (double)dof / (2.0 * pn1[3]);
      double qn[2] = {0.0, 0.0};
      if (s->pr != 1.0) heat_flux(NG, s->fu, s->fv, s->fw, f, pn, qn);
      for (int k = 0; k < K; ++k)
        for (int m = 0; m < M; ++m)
          for (int v = k * M + m; v < NV; v += NG) {  /* G, then H */
            double gn = ugks_ref_maxwellian(pn, s->uk[k], s->vm[m]);
            double gn1 = ugks_ref_maxwellian(pn1, s->uk[k], s->vm[m]);
            if (v >= NG) {
              gn *= kn;
              gn1 *= kn1;
            }
            if (s->pr != 1.0) {
              gn *= 1.0 + ugks_ref_shakhov(pn, qn, s->pr, s->uk[k], s->vm[m]);
              gn1 *= 1.0 + ugks_ref_shakhov(pn1, qn, s->pr, s->uk[k], s->vm[m]);
            }
            double dF = (Ffl[v] - Ffr[v] + Ffb[v] - Fft[v]) / area;
            fn[v] = (f[v] + dF + 0.5 * dt * (gn1 / tn1 + (gn - f[v]) / tn)) /
                    (1.0 + 0.5 * dt / tn1);
          }
    }
  return err ? -4 : 0;
}

int ugks_ref_step(ugks_ref* s, int n) {
  size_t nc = (size_t)s->c.nx * s->c.ny;
  for (int it = 0; it < n; ++it) {
    if (s->c.bc == 1 && channel_ghosts(s)) return -4;
    slopes(s);
    if (faces(s)) return -4;
    if (update(s)) return -4;
    double* t = s->f;
    s->f = s->fnew;
    s->fnew = t;
    t = s->W;
    s->W = s->Wnew;
    s->Wnew = t;
    for (size_t c = 0; c < nc; ++c) {
      double p[4];
      if (ugks_ref_prim(s->W + 4 * c, p, s->c.dof)) return -4;
    }
    s->time += s->dt;
    /* adaptive step: the next step's dt from the state it starts from */
    if (s->c.adaptive_dt)
      s->dt = ugks_ref_adaptive_dt(s->W, (int)nc, s->c.cfl, s->c.umax, s->c.vmax, s->dx, s->dy);
  }
  return 0;
}
