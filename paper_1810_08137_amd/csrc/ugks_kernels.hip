// gfx950 kernels of the 2D UGKS time step.
//
// One step is four launches on one stream:
//   ghost   pressure inlet/outlet ghost columns of a channel (Sec. 3.A)
//   sums    per cell and velocity: limited slopes of f, the upwind reconstruction at each of
//           the cell's four faces and their velocity moments (S1 and the sums of S7); one
//           wavefront per cell, velocities across lanes, a 64-wide reduce-scatter at the end
//   faces   per interface: add the two sides' sums, then the scalar part of the flux
//           (S2-S5: Maxwellian moments, time weights, micro slopes, equilibrium flux) into a
//           32-double record
//   update  per cell and velocity: rebuild the upwind f at the four faces, the interface
//           Maxwellian from separable exp tables (S6), the distribution flux (S8), then
//           Eq. (4) for W and Eq. (3) for f
// f is laid out [cell][velocity] with the velocity index contiguous and padded to a multiple
// of 64, so every wavefront load is coalesced along velocity.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ugks_internal.hpp"

namespace ugks {
namespace {

constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------ storage
template <typename S>
__device__ __forceinline__ double ld(const S* __restrict__ p, size_t i) {
  return static_cast<double>(p[i]);
}
template <typename S>
__device__ __forceinline__ void st(S* __restrict__ p, size_t i, double x) {
  p[i] = static_cast<S>(x);
}

// ------------------------------------------------------------------ pointwise physics
// Van Leer limited slope of two one-sided differences (second-order reconstruction, Sec. 2.A).
__device__ __forceinline__ double limited(double p, double q) {
  const double pq = p * q;
  return pq > 0.0 ? 2.0 * pq / (p + q) : 0.0;
}

// Upwind weight of the left state for normal velocity un (1/2 when un = 0).
__device__ __forceinline__ double upwind_left(double un) {
  return un > 0.0 ? 1.0 : (un < 0.0 ? 0.0 : 0.5);
}

struct Prim {
  double rho, U, V, lam;  // lambda = 1/T
};

// Primitive variables of W = (rho, rho U, rho V, rho E), 2D gas without internal energy
// modes: rho E = rho (U^2 + V^2)/2 + rho/(2 lambda).  false on an invalid state.
__device__ __forceinline__ bool prim_of(const double* W, Prim& p) {
  const double rho = W[0];
  const double U = W[1] / rho;
  const double V = W[2] / rho;
  const double e = W[3] - 0.5 * rho * (U * U + V * V);
  p.rho = rho;
  p.U = U;
  p.V = V;
  p.lam = 0.5 * rho / e;
  return rho > 0.0 && e > 0.0 && isfinite(rho) && isfinite(e) && isfinite(U) && isfinite(V) &&
         isfinite(p.lam);
}

// BGK collision time tau = mu/p, mu = mu_ref T^(1/2), p = rho T/2.
__device__ __forceinline__ double collision_time(const Prim& p, double mu_ref) {
  return 2.0 * mu_ref * sqrt(p.lam) / p.rho;
}

// Moments of the normalised 1D Maxwellian along one axis: full line, u > 0, u < 0.
__device__ void axis_moments(double U, double lam, double* full, double* pos, double* neg) {
  const double edge = exp(-lam * U * U) / (2.0 * sqrt(kPi * lam));
  const double sl = sqrt(lam);
  full[0] = 1.0;
  full[1] = U;
  pos[0] = 0.5 * erfc(-sl * U);
  neg[0] = 0.5 * erfc(sl * U);
  pos[1] = U * pos[0] + edge;
  neg[1] = U * neg[0] - edge;
#pragma unroll
  for (int n = 2; n < 7; ++n) {
    const double c = (double)(n - 1) / (2.0 * lam);
    full[n] = U * full[n - 1] + c * full[n - 2];
    pos[n] = U * pos[n - 1] + c * pos[n - 2];
    neg[n] = U * neg[n - 1] + c * neg[n - 2];
  }
}

// <un^a ut^b psi>, psi = (1, un, ut, (un^2 + ut^2)/2)
__device__ __forceinline__ void mpsi(const double* mu, const double* mv, int a, int b, double* o) {
  o[0] = mu[a] * mv[b];
  o[1] = mu[a + 1] * mv[b];
  o[2] = mu[a] * mv[b + 1];
  o[3] = 0.5 * (mu[a + 2] * mv[b] + mu[a] * mv[b + 2]);
}

// <un^a ut^b psi (c . psi)>
__device__ __forceinline__ void mpsi_c(const double* mu, const double* mv, int a, int b,
                                       const double* c, double* o) {
  double t0[4], t1[4], t2[4], t3[4], t4[4];
  mpsi(mu, mv, a, b, t0);
  mpsi(mu, mv, a + 1, b, t1);
  mpsi(mu, mv, a, b + 1, t2);
  mpsi(mu, mv, a + 2, b, t3);
  mpsi(mu, mv, a, b + 2, t4);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    o[q] = c[0] * t0[q] + c[1] * t1[q] + c[2] * t2[q] + 0.5 * c[3] * (t3[q] + t4[q]);
}

// S4 micro slope: a such that the moments of rho g (a . psi) equal s (closed form, 2D gas).
__device__ __forceinline__ void micro_slope(const Prim& p, const double* s, double* a) {
  const double q2 = p.U * p.U + p.V * p.V + 1.0 / p.lam;
  const double R2 = s[1] - p.U * s[0];
  const double R3 = s[2] - p.V * s[0];
  const double R4 = 2.0 * s[3] - q2 * s[0];
  a[3] = 2.0 * p.lam * p.lam / p.rho * (R4 - 2.0 * p.U * R2 - 2.0 * p.V * R3);
  a[2] = 2.0 * p.lam * R3 / p.rho - p.V * a[3];
  a[1] = 2.0 * p.lam * R2 / p.rho - p.U * a[3];
  a[0] = s[0] / p.rho - p.U * a[1] - p.V * a[2] - 0.5 * a[3] * q2;
}

// S3 time weights of Eq. (2) integrated over [0, dt] (see the record layout for their use).
__device__ __forceinline__ void time_weights(double dt, double tau, double* Mt) {
  const double e = exp(-dt / tau);
  Mt[3] = -tau * expm1(-dt / tau);
  Mt[4] = tau * Mt[3] - tau * dt * e;
  Mt[0] = dt - Mt[3];
  Mt[1] = -tau * Mt[0] + Mt[4];
  Mt[2] = 0.5 * dt * dt - tau * Mt[0];
}

// ------------------------------------------------------------------ addressing
__device__ __forceinline__ int wrap(int i, int n) { return ((i % n) + n) % n; }

// f slab of column i of row j, i in [-2, nx+1]: a cell, a wrapped cell (periodic) or the
// inlet/outlet ghost column (channel).
template <typename S>
__device__ __forceinline__ const S* xslab(const KParams& P, const S* f, const S* fg, int i, int j) {
  if (i >= 0 && i < P.nx) return f + ((size_t)j * P.nx + i) * P.NVP;
  if (P.bc == UGKS_BC_PERIODIC) return f + ((size_t)j * P.nx + wrap(i, P.nx)) * P.NVP;
  return fg + ((size_t)(i < 0 ? 0 : P.ny) + j) * P.NVP;
}

// ------------------------------------------------------------------ wave reductions
// Reduce-scatter of 64 per-lane partial sums: afterwards lane l holds the wave total of
// slot l.  Recursive halving: 32 + 16 + ... + 1 = 63 exchanges, fixed order.
template <int H>
__device__ __forceinline__ void reduce_scatter(double* a, int lane) {
  const bool upper = (lane & H) != 0;
#pragma unroll
  for (int q = 0; q < H; ++q) {
    const double send = upper ? a[q] : a[q + H];
    const double keep = upper ? a[q + H] : a[q];
    a[q] = keep + __shfl_xor(send, H, kWave);
  }
  if constexpr (H > 1) reduce_scatter<H / 2>(a, lane);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) x += __shfl_xor(x, h, kWave);
  return x;
}

// 16 moment sums of one face side (S1 and S7): weight wt, normal/tangential velocity
// (un, ut), reconstructed f and its normal/tangential slopes.
__device__ __forceinline__ void add_side(double* a, double wt, double un, double ut, double c2h,
                                         double fh, double sn, double st) {
  const double psi[4] = {1.0, un, ut, c2h};
  const double x0 = wt * fh;
  const double x1 = wt * st;
  const double x2 = x0 * un;
  const double x3 = wt * un * (un * sn + ut * st);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    a[q] += x0 * psi[q];
    a[4 + q] += x1 * psi[q];
    a[8 + q] += x2 * psi[q];
    a[12 + q] += x3 * psi[q];
  }
}

// ================================================================== kernels
// Discrete Maxwellian of each cell's W (initial state).
template <typename S>
__global__ __launch_bounds__(kWave) void init_kernel(KParams P, S* __restrict__ f,
                                                     const double* __restrict__ W) {
  const int c = blockIdx.x;
  Prim p;
  if (!prim_of(W + 4 * (size_t)c, p) && threadIdx.x == 0) *P.flag = 1;
  const double coef = p.rho * p.lam / kPi;
  S* fc = f + (size_t)c * P.NVP;
  for (int v = threadIdx.x; v < P.NVP; v += kWave) {
    double g = 0.0;
    if (v < P.NV) {
      const double du = P.U[v] - p.U, dv = P.V[v] - p.V;
      g = coef * exp(-p.lam * (du * du + dv * dv));
    }
    st(fc, v, g);
  }
}

// Inlet/outlet ghost of one row: state, discrete Maxwellian, and the ghost's moment sums
// towards the domain (its slopes are zero).  grid (ny, 2), one wavefront each.
template <typename S>
__global__ __launch_bounds__(kWave) void ghost_kernel(KParams P, const double* __restrict__ W,
                                                      double* __restrict__ Wg, S* __restrict__ fg,
                                                      double* __restrict__ hsg) {
  const int j = blockIdx.x, side = blockIdx.y, lane = threadIdx.x;
  const int col = side == 0 ? 0 : P.nx - 1;
  Prim pc, pg;
  bool ok = prim_of(W + 4 * ((size_t)j * P.nx + col), pc);
  if (side == 0) {
    const double T = P.T_in;
    pg.lam = 1.0 / T;
    pg.rho = 2.0 * P.p_in / T;
    if (P.inlet_fixed_u) {
      pg.U = P.U_in * (1.0 + P.U_noise * P.xi_in[j]);
      pg.V = 0.0;
    } else {
      pg.U = pc.U;
      pg.V = pc.V;
    }
  } else {
    const double T = 1.0 / pc.lam;
    pg.rho = 2.0 * P.p_out / T;
    pg.U = pc.U;
    pg.V = pc.V;
    pg.lam = pc.lam;
  }
  if (!ok && lane == 0) *P.flag = 1;
  double* wg = Wg + 4 * ((size_t)side * P.ny + j);
  if (lane == 0) {
    wg[0] = pg.rho;
    wg[1] = pg.rho * pg.U;
    wg[2] = pg.rho * pg.V;
    wg[3] = 0.5 * pg.rho * (pg.U * pg.U + pg.V * pg.V) + 0.5 * pg.rho / pg.lam;
  }
  const double coef = pg.rho * pg.lam / kPi;
  S* row = fg + ((size_t)side * P.ny + j) * P.NVP;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int v = lane; v < P.NVP; v += kWave) {
    const double u = P.U[v], vv = P.V[v];
    double g = 0.0;
    if (v < P.NV) {
      const double du = u - pg.U, dv = vv - pg.V;
      g = coef * exp(-pg.lam * (du * du + dv * dv));
    }
    st(row, v, g);
    const double gs = ld(row, v);  // the value the cells will read
    const double h = side == 0 ? upwind_left(u) : 1.0 - upwind_left(u);
    add_side(acc, P.Wq[v] * h, u, vv, 0.5 * (u * u + vv * vv), gs, 0.0, 0.0);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == q) hsg[((size_t)side * P.ny + j) * 16 + q] = t;
  }
}

// Per cell: slopes and the outgoing moment sums of all four faces.  One wavefront per cell.
template <typename S>
__global__ __launch_bounds__(kWave) void sums_kernel(KParams P, const S* __restrict__ f,
                                                     const S* __restrict__ fg,
                                                     double* __restrict__ hs) {
  const int c = blockIdx.x, lane = threadIdx.x;
  const int i = c % P.nx, j = c / P.nx;
  const bool chan = P.bc == UGKS_BC_CHANNEL;
  const bool wall_row = chan && (j == 0 || j == P.ny - 1);
  const S* f0 = f + (size_t)c * P.NVP;
  const S* fw = xslab(P, f, fg, i - 1, j);
  const S* fe = xslab(P, f, fg, i + 1, j);
  const S* fs = f + ((size_t)wrap(j - 1, P.ny) * P.nx + i) * P.NVP;
  const S* fn = f + ((size_t)wrap(j + 1, P.ny) * P.nx + i) * P.NVP;
  const double hdx = 0.5 * P.dx, hdy = 0.5 * P.dy;
  double acc[kSlots];
#pragma unroll
  for (int q = 0; q < kSlots; ++q) acc[q] = 0.0;
  for (int v = lane; v < P.NVP; v += kWave) {
    const double fc = ld(f0, v);
    const double sx = limited(ld(fe, v) - fc, fc - ld(fw, v)) * P.inv_dx;
    const double sy = wall_row ? 0.0 : limited(ld(fn, v) - fc, fc - ld(fs, v)) * P.inv_dy;
    const double u = P.U[v], vv = P.V[v], w = P.Wq[v];
    const double c2h = 0.5 * (u * u + vv * vv);
    const double hx = upwind_left(u), hy = upwind_left(vv);
    add_side(acc + 16 * S_XP, w * hx, u, vv, c2h, fc + hdx * sx, sx, sy);
    add_side(acc + 16 * S_XM, w * (1.0 - hx), u, vv, c2h, fc - hdx * sx, sx, sy);
    add_side(acc + 16 * S_YP, w * hy, vv, u, c2h, fc + hdy * sy, sy, sx);
    add_side(acc + 16 * S_YM, w * (1.0 - hy), vv, u, c2h, fc - hdy * sy, sy, sx);
  }
  reduce_scatter<32>(acc, lane);
  hs[(size_t)c * kSlots + lane] = acc[0];
}

// S2-S5 at one interior interface, local frame.  S = [W0, Wt, Q1, Q2].  Writes the local
// macroscopic flux to F and every coefficient the cell update needs to rec.
__device__ void interface_scalars(const KParams& P, const double* S, const double* WL,
                                  const double* WR, double dn, double len, double* F,
                                  double* rec) {
  const double* W0 = S;
  const double* Wt = S + 4;
  const double* Q1 = S + 8;
  const double* Q2 = S + 12;
  rec[R_LEN] = len;
  if (P.collisionless) {
    const double Mt4 = P.dt, Mt5 = 0.5 * P.dt * P.dt;
#pragma unroll
    for (int q = 0; q < 4; ++q) F[q] = len * (Mt4 * Q1[q] - Mt5 * Q2[q]);
    rec[R_MT + 0] = 0.0;
    rec[R_MT + 1] = 0.0;
    rec[R_MT + 2] = 0.0;
    rec[R_MT + 3] = Mt4;
    rec[R_MT + 4] = Mt5;
    rec[R_KIND] = K_FREE;
    rec[R_GCOEF] = 0.0;
    rec[R_LAM] = 0.0;
    return;
  }
  Prim p0;
  if (!prim_of(W0, p0)) *P.flag = 1;
  const double tau0 = collision_time(p0, P.mu_ref);
  double Mt[5];
  time_weights(P.dt, tau0, Mt);
  double swL[4], swR[4], aL[4], aR[4], b[4], A[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    swL[q] = (W0[q] - WL[q]) / (0.5 * dn);
    swR[q] = (WR[q] - W0[q]) / (0.5 * dn);
  }
  micro_slope(p0, swL, aL);
  micro_slope(p0, swR, aR);
  micro_slope(p0, Wt, b);
  double mu[7], mp[7], mn[7], mv[7], tp[7], tn[7];
  axis_moments(p0.U, p0.lam, mu, mp, mn);
  axis_moments(p0.V, p0.lam, mv, tp, tn);
  double m1[4], m2[4], m3[4], sA[4];
  mpsi_c(mp, mv, 1, 0, aL, m1);
  mpsi_c(mn, mv, 1, 0, aR, m2);
  mpsi_c(mu, mv, 0, 1, b, m3);
#pragma unroll
  for (int q = 0; q < 4; ++q) sA[q] = -p0.rho * (m1[q] + m2[q] + m3[q]);
  micro_slope(p0, sA, A);
  double e0[4], eL[4], eR[4], eb[4], eA[4];
  mpsi(mu, mv, 1, 0, e0);
  mpsi_c(mp, mv, 2, 0, aL, eL);
  mpsi_c(mn, mv, 2, 0, aR, eR);
  mpsi_c(mu, mv, 1, 1, b, eb);
  mpsi_c(mu, mv, 1, 0, A, eA);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double feq = p0.rho * (Mt[0] * e0[q] + Mt[1] * (eL[q] + eR[q] + eb[q]) + Mt[2] * eA[q]);
    F[q] = len * (feq + Mt[3] * Q1[q] - Mt[4] * Q2[q]);
  }
  rec[R_GCOEF] = p0.rho * p0.lam / kPi;
  rec[R_LAM] = p0.lam;
#pragma unroll
  for (int q = 0; q < 5; ++q) rec[R_MT + q] = Mt[q];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    rec[R_AL + q] = aL[q];
    rec[R_AR + q] = aR[q];
    rec[R_B + q] = b[q];
    rec[R_A + q] = A[q];
  }
  rec[R_KIND] = K_INTERIOR;
  rec[6] = p0.U;  // local normal / tangential; the caller maps them to the global frame
  rec[7] = p0.V;
}

// One thread per interface: x-faces first (ny rows of nx+1), then y-faces (ny+1 rows of nx).
__global__ __launch_bounds__(256) void faces_kernel(KParams P, const double* __restrict__ hs,
                                                    const double* __restrict__ hsg,
                                                    const double* __restrict__ W,
                                                    const double* __restrict__ Wg,
                                                    double* __restrict__ recx,
                                                    double* __restrict__ recy) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nfx = (long)P.ny * (P.nx + 1);
  const long nfy = (long)(P.ny + 1) * P.nx;
  const bool chan = P.bc == UGKS_BC_CHANNEL;
  double S[16], F[4];
  if (e < nfx) {
    const int j = (int)(e / (P.nx + 1)), i = (int)(e % (P.nx + 1));
    const double *sL, *sR, *WL, *WR;
    if (i > 0 || !chan) {
      const size_t cl = (size_t)j * P.nx + wrap(i - 1, P.nx);
      sL = hs + cl * kSlots + 16 * S_XP;
      WL = W + 4 * cl;
    } else {
      sL = hsg + (size_t)j * 16;
      WL = Wg + 4 * (size_t)j;
    }
    if (i < P.nx || !chan) {
      const size_t cr = (size_t)j * P.nx + wrap(i, P.nx);
      sR = hs + cr * kSlots + 16 * S_XM;
      WR = W + 4 * cr;
    } else {
      sR = hsg + ((size_t)P.ny + j) * 16;
      WR = Wg + 4 * ((size_t)P.ny + j);
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) S[q] = sL[q] + sR[q];
    double wl[4], wr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wl[q] = WL[q];
      wr[q] = WR[q];
    }
    double* rec = recx + (size_t)e * kRec;
    interface_scalars(P, S, wl, wr, P.dx, P.dy, F, rec);
#pragma unroll
    for (int q = 0; q < 4; ++q) rec[R_FX + q] = F[q];
    // local frame = global frame for x-faces (rec[6], rec[7] already hold U, V)
    return;
  }
  if (e >= nfx + nfy) return;
  const long e2 = e - nfx;
  const int j = (int)(e2 / P.nx), i = (int)(e2 % P.nx);
  double* rec = recy + (size_t)e2 * kRec;
  if (chan && (j == 0 || j == P.ny)) {
    // diffuse wall: sums of the wall-row cell towards the wall; local frame (v, u)
    const bool top = j == P.ny;
    const size_t c = (size_t)(top ? P.ny - 1 : 0) * P.nx + i;
    const double* Q1 = hs + c * kSlots + 16 * (top ? S_YP : S_YM) + 8;
    const double den = top ? P.wall_den_top : P.wall_den_bot;
    const double* Gw = top ? P.wall_G_top : P.wall_G_bot;
    const double rho_w = -Q1[0] / den;
    const double s = P.dx * P.dt;
    double Fl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) Fl[q] = s * (Q1[q] + rho_w * Gw[q]);
    rec[R_FX + 0] = Fl[0];
    rec[R_FX + 1] = Fl[2];
    rec[R_FX + 2] = Fl[1];
    rec[R_FX + 3] = Fl[3];
    rec[R_GCOEF] = rho_w * P.lam_w / kPi;
    rec[R_LAM] = P.lam_w;
    rec[R_UX] = 0.0;
    rec[R_VY] = 0.0;
    rec[R_KIND] = K_WALL;
    rec[R_LEN] = P.dx;
    if (!(rho_w > 0.0) || !isfinite(rho_w)) *P.flag = 1;
    return;
  }
  const size_t cl = (size_t)wrap(j - 1, P.ny) * P.nx + i;
  const size_t cr = (size_t)wrap(j, P.ny) * P.nx + i;
  const double* sL = hs + cl * kSlots + 16 * S_YP;
  const double* sR = hs + cr * kSlots + 16 * S_YM;
#pragma unroll
  for (int q = 0; q < 16; ++q) S[q] = sL[q] + sR[q];
  const double wl[4] = {W[4 * cl], W[4 * cl + 2], W[4 * cl + 1], W[4 * cl + 3]};
  const double wr[4] = {W[4 * cr], W[4 * cr + 2], W[4 * cr + 1], W[4 * cr + 3]};
  interface_scalars(P, S, wl, wr, P.dy, P.dx, F, rec);
  rec[R_FX + 0] = F[0];
  rec[R_FX + 1] = F[2];
  rec[R_FX + 2] = F[1];
  rec[R_FX + 3] = F[3];
  const double un0 = rec[6], ut0 = rec[7];
  rec[R_UX] = ut0;
  rec[R_VY] = un0;
}

// S6 + S8: time-integrated flux of f through one face for one velocity.  tk/tm: separable
// exp tables of the face's Maxwellian along u and v; (un, ut) the face-frame velocity.
__device__ __forceinline__ double face_flux(const double* __restrict__ r,
                                            const double* __restrict__ tk,
                                            const double* __restrict__ tm, int k, int m,
                                            double un, double ut, double fh, double sn,
                                            double st) {
  const double free_part = r[R_MT + 3] * fh - r[R_MT + 4] * (un * sn + ut * st);
  if (r[R_KIND] == (double)K_FREE) return r[R_LEN] * un * free_part;
  const double c2h = 0.5 * (un * un + ut * ut);
  const bool pos = un > 0.0;
  const double a0 = pos ? r[R_AL + 0] : r[R_AR + 0];
  const double a1 = pos ? r[R_AL + 1] : r[R_AR + 1];
  const double a2 = pos ? r[R_AL + 2] : r[R_AR + 2];
  const double a3 = pos ? r[R_AL + 3] : r[R_AR + 3];
  const double pa = a0 + a1 * un + a2 * ut + a3 * c2h;
  const double pb = r[R_B] + r[R_B + 1] * un + r[R_B + 2] * ut + r[R_B + 3] * c2h;
  const double pA = r[R_A] + r[R_A + 1] * un + r[R_A + 2] * ut + r[R_A + 3] * c2h;
  const double G = r[R_GCOEF] * tk[k] * tm[m];
  const double poly = r[R_MT] + r[R_MT + 1] * (un * pa + ut * pb) + r[R_MT + 2] * pA;
  return r[R_LEN] * un * (G * poly + free_part);
}

// Per cell: Eq. (4) for W, then Eq. (3) for every velocity.  One wavefront per cell; six
// separable exp tables (four faces, g^n, g^{n+1}) of nu + nv doubles each in LDS.
template <typename S>
__global__ __launch_bounds__(kWave) void update_kernel(KParams P, const S* __restrict__ fin,
                                                       S* __restrict__ fout,
                                                       const S* __restrict__ fg,
                                                       const double* __restrict__ recx,
                                                       const double* __restrict__ recy,
                                                       double* __restrict__ W) {
  extern __shared__ double tab[];
  const int c = blockIdx.x, lane = threadIdx.x;
  const int i = c % P.nx, j = c / P.nx;
  const int KM = P.K + P.M;
  const bool chan = P.bc == UGKS_BC_CHANNEL;
  const double* rl = recx + ((size_t)j * (P.nx + 1) + i) * kRec;
  const double* rr = recx + ((size_t)j * (P.nx + 1) + i + 1) * kRec;
  const double* rb = recy + ((size_t)j * P.nx + i) * kRec;
  const double* rt = recy + ((size_t)(j + 1) * P.nx + i) * kRec;
  // Eq. (4)
  double Wn[4], W1[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    Wn[q] = W[4 * (size_t)c + q];
    W1[q] = Wn[q] + (rl[q] - rr[q] + rb[q] - rt[q]) / P.area;
  }
  Prim pn{}, p1{};
  double tn = 0.0, t1 = 0.0;
  if (!P.collisionless) {
    const bool ok = prim_of(Wn, pn) && prim_of(W1, p1);
    if (!ok && lane == 0) *P.flag = 1;
    tn = collision_time(pn, P.mu_ref);
    t1 = collision_time(p1, P.mu_ref);
  }
  // tables: 0 left, 1 right, 2 bottom, 3 top face; 4 g^n; 5 g^{n+1}
  for (int e = lane; e < 6 * KM; e += kWave) {
    const int s = e / KM, r = e - s * KM;
    double lam = 0.0, ux = 0.0, vy = 0.0;
    bool use = true;
    if (s < 4) {
      const double* rs = s == 0 ? rl : (s == 1 ? rr : (s == 2 ? rb : rt));
      use = rs[R_KIND] != (double)K_FREE;
      lam = rs[R_LAM];
      ux = rs[R_UX];
      vy = rs[R_VY];
    } else {
      use = !P.collisionless;
      const Prim& p = s == 4 ? pn : p1;
      lam = p.lam;
      ux = p.U;
      vy = p.V;
    }
    const double d = r < P.K ? P.uk[r] - ux : P.vm[r - P.K] - vy;
    tab[e] = use ? exp(-lam * d * d) : 0.0;
  }
  __syncthreads();
  const double cn = pn.rho * pn.lam / kPi, c1 = p1.rho * p1.lam / kPi;
  const bool wall_b = chan && j == 0, wall_t = chan && j == P.ny - 1;
  const bool wall_row = wall_b || wall_t;
  const S* f0 = fin + (size_t)c * P.NVP;
  const S* xw = xslab(P, fin, fg, i - 1, j);
  const S* xe = xslab(P, fin, fg, i + 1, j);
  const S* xww = xslab(P, fin, fg, i - 2, j);
  const S* xee = xslab(P, fin, fg, i + 2, j);
  const bool ghost_w = chan && i == 0, ghost_e = chan && i == P.nx - 1;
  // rows j-1 and j+1 (absent beyond a wall) at columns i-1, i, i+1; rows j-2, j+2 at i
  const bool has_s = !wall_b, has_n = !wall_t;
  const int js = wrap(j - 1, P.ny), jn = wrap(j + 1, P.ny);
  const S* sw = xslab(P, fin, fg, i - 1, js);
  const S* sc = xslab(P, fin, fg, i, js);
  const S* se = xslab(P, fin, fg, i + 1, js);
  const S* nw = xslab(P, fin, fg, i - 1, jn);
  const S* nc = xslab(P, fin, fg, i, jn);
  const S* ne = xslab(P, fin, fg, i + 1, jn);
  const int jss = wrap(j - 2, P.ny), jnn = wrap(j + 2, P.ny);
  const S* scc = fin + ((size_t)jss * P.nx + i) * P.NVP;
  const S* ncc = fin + ((size_t)jnn * P.nx + i) * P.NVP;
  // y-neighbour rows that sit next to a wall carry no y-slope
  const bool s_wallrow = chan && (j - 1 == 0);
  const bool n_wallrow = chan && (j + 1 == P.ny - 1);
  const double hdx = 0.5 * P.dx, hdy = 0.5 * P.dy;
  const double* tl = tab + 0 * KM;
  const double* trr = tab + 1 * KM;
  const double* tb = tab + 2 * KM;
  const double* tt = tab + 3 * KM;
  const double* tgn = tab + 4 * KM;
  const double* tg1 = tab + 5 * KM;
  S* fo = fout + (size_t)c * P.NVP;
  for (int v = lane; v < P.NVP; v += kWave) {
    if (v >= P.NV) {
      st(fo, v, 0.0);
      continue;
    }
    const int k = P.kidx[v], m = P.midx[v];
    const double u = P.U[v], vv = P.V[v];
    const double fc = ld(f0, v);
    const double fW = ld(xw, v), fE = ld(xe, v);
    const double fS = has_s ? ld(sc, v) : 0.0;
    const double fN = has_n ? ld(nc, v) : 0.0;
    const double sx0 = limited(fE - fc, fc - fW) * P.inv_dx;
    const double sy0 = wall_row ? 0.0 : limited(fN - fc, fc - fS) * P.inv_dy;
    double dF = 0.0;
    if (u != 0.0) {
      const bool right = u > 0.0;  // particles move in +x: the left face is the inflow face
      const double sgn = right ? 1.0 : -1.0;
      const bool ghostX = right ? ghost_w : ghost_e;
      const double fX = right ? fW : fE;
      double sxX = 0.0, syX = 0.0;
      if (!ghostX) {
        const double fXX = ld(right ? xww : xee, v);
        sxX = (right ? limited(fc - fX, fX - fXX) : limited(fXX - fX, fX - fc)) * P.inv_dx;
        if (!wall_row) {
          const double fXn = ld(right ? nw : ne, v), fXs = ld(right ? sw : se, v);
          syX = limited(fXn - fX, fX - fXs) * P.inv_dy;
        }
      }
      const double fin_h = fX + sgn * hdx * sxX;
      const double fout_h = fc + sgn * hdx * sx0;
      const double* rin = right ? rl : rr;
      const double* rout = right ? rr : rl;
      const double* tin = right ? tl : trr;
      const double* tout = right ? trr : tl;
      const double Fin = face_flux(rin, tin, tin + P.K, k, m, u, vv, fin_h, sxX, syX);
      const double Fout = face_flux(rout, tout, tout + P.K, k, m, u, vv, fout_h, sx0, sy0);
      dF += sgn * (Fin - Fout);
    }
    if (vv != 0.0) {
      const bool up = vv > 0.0;  // particles move in +y: the bottom face is the inflow face
      const double sgn = up ? 1.0 : -1.0;
      const double* rin = up ? rb : rt;
      const double* rout = up ? rt : rb;
      const double* tin = up ? tb : tt;
      const double* tout = up ? tt : tb;
      double Fin, Fout;
      if (up ? wall_b : wall_t) {
        // particles leaving the wall: rho_w times the wall Maxwellian
        Fin = rin[R_LEN] * P.dt * vv * (rin[R_GCOEF] * tin[k] * tin[P.K + m]);
      } else {
        const double fY = up ? fS : fN;
        const bool Y_wallrow = up ? s_wallrow : n_wallrow;
        double syY = 0.0;
        if (!Y_wallrow) {
          const double fYY = ld(up ? scc : ncc, v);
          syY = (up ? limited(fc - fY, fY - fYY) : limited(fYY - fY, fY - fc)) * P.inv_dy;
        }
        const double fYe = ld(up ? se : ne, v), fYw = ld(up ? sw : nw, v);
        const double sxY = limited(fYe - fY, fY - fYw) * P.inv_dx;
        Fin = face_flux(rin, tin, tin + P.K, k, m, vv, u, fY + sgn * hdy * syY, syY, sxY);
      }
      if (up ? wall_t : wall_b) {
        // particles reaching the wall carry the wall-row value
        Fout = rout[R_LEN] * P.dt * vv * fc;
      } else {
        Fout = face_flux(rout, tout, tout + P.K, k, m, vv, u, fc + sgn * hdy * sy0, sy0, sx0);
      }
      dF += sgn * (Fin - Fout);
    }
    double f1;
    if (P.collisionless) {
      f1 = fc + dF / P.area;
    } else {
      const double gn = cn * tgn[k] * tgn[P.K + m];
      const double g1 = c1 * tg1[k] * tg1[P.K + m];
      f1 = (fc + dF / P.area + 0.5 * P.dt * (g1 / t1 + (gn - fc) / tn)) /
           (1.0 + 0.5 * P.dt / t1);
    }
    st(fo, v, f1);
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) W[4 * (size_t)c + q] = W1[q];
  }
}

}  // namespace

// ================================================================== launchers
hipError_t launch_init(const KParams& P, int fp32, void* f, const double* W, hipStream_t s) {
  const unsigned nc = (unsigned)((size_t)P.nx * P.ny);
  if (fp32)
    init_kernel<float><<<nc, kWave, 0, s>>>(P, static_cast<float*>(f), W);
  else
    init_kernel<double><<<nc, kWave, 0, s>>>(P, static_cast<double*>(f), W);
  return hipGetLastError();
}

hipError_t launch_ghost(const KParams& P, int fp32, const double* W, double* Wg, void* fg,
                        double* hsg, hipStream_t s) {
  const dim3 grid((unsigned)P.ny, 2);
  if (fp32)
    ghost_kernel<float><<<grid, kWave, 0, s>>>(P, W, Wg, static_cast<float*>(fg), hsg);
  else
    ghost_kernel<double><<<grid, kWave, 0, s>>>(P, W, Wg, static_cast<double*>(fg), hsg);
  return hipGetLastError();
}

hipError_t launch_sums(const KParams& P, int fp32, const void* f, const void* fg, double* hs,
                       hipStream_t s) {
  const unsigned nc = (unsigned)((size_t)P.nx * P.ny);
  if (fp32)
    sums_kernel<float><<<nc, kWave, 0, s>>>(P, static_cast<const float*>(f),
                                            static_cast<const float*>(fg), hs);
  else
    sums_kernel<double><<<nc, kWave, 0, s>>>(P, static_cast<const double*>(f),
                                             static_cast<const double*>(fg), hs);
  return hipGetLastError();
}

hipError_t launch_faces(const KParams& P, const double* hs, const double* hsg, const double* W,
                        const double* Wg, double* recx, double* recy, hipStream_t s) {
  const long n = (long)P.ny * (P.nx + 1) + (long)(P.ny + 1) * P.nx;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  faces_kernel<<<blocks, 256, 0, s>>>(P, hs, hsg, W, Wg, recx, recy);
  return hipGetLastError();
}

hipError_t launch_update(const KParams& P, int fp32, const void* fin, void* fout, const void* fg,
                         const double* recx, const double* recy, double* W, hipStream_t s) {
  const unsigned nc = (unsigned)((size_t)P.nx * P.ny);
  const size_t lds = sizeof(double) * 6 * (size_t)(P.K + P.M);
  if (fp32)
    update_kernel<float><<<nc, kWave, lds, s>>>(P, static_cast<const float*>(fin),
                                                static_cast<float*>(fout),
                                                static_cast<const float*>(fg), recx, recy, W);
  else
    update_kernel<double><<<nc, kWave, lds, s>>>(P, static_cast<const double*>(fin),
                                                 static_cast<double*>(fout),
                                                 static_cast<const double*>(fg), recx, recy, W);
  return hipGetLastError();
}

}  // namespace ugks
