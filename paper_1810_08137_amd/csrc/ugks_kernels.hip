// gfx950 kernels of the 2D UGKS time step.
//
// One step is four launches on one stream:
//   ghost   pressure inlet/outlet ghost columns of a channel (Sec. 3.A)
//   sums    per cell and velocity: limited slopes of f, the upwind reconstruction at each of
//           the cell's four faces and their velocity moments (S1 and the sums of S7); one
//           wavefront per cell, velocities across lanes, running sums reduced through LDS
//   faces   per interface: add the two sides' sums, then the scalar part of the flux
//           (S2-S5: Maxwellian moments, time weights, micro slopes, equilibrium flux) into a
//           record of folded coefficients
//   update  per cell and velocity: rebuild the upwind f at the four faces, the interface
//           Maxwellian from separable exp tables (S6), the distribution flux (S8), then
//           Eq. (4) for W and Eq. (3) for f
// f is laid out [cell][velocity slot] with the slot index contiguous and padded to a multiple
// of 64, so every wavefront load is coalesced.  Slots are ordered by velocity quadrant, so
// most 64-slot chunks have one sign of u and one of v: their upwind choices and moment slots
// are then uniform across the wavefront.  The cell kernels visit cells in band order (columns
// of 16-row bands) so that stencil neighbours are read from L2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>

#include "ugks_internal.hpp"

namespace ugks {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kCellsPerBlock = 4;  // one wavefront per cell

// ------------------------------------------------------------------ storage
template <typename S>
__device__ __forceinline__ double ld(const UGKS_GLOBAL S* p, unsigned i) {
  return static_cast<double>(p[i]);
}
// Load at a 32-bit byte offset from a uniform base: one instruction with a scalar base.
template <typename T>
__device__ __forceinline__ T ldb(const UGKS_GLOBAL T* p, unsigned byte_off) {
  return *reinterpret_cast<const UGKS_GLOBAL T*>(reinterpret_cast<const UGKS_GLOBAL char*>(p) +
                                                 byte_off);
}
template <typename S>
__device__ __forceinline__ void st(UGKS_GLOBAL S* p, unsigned i, double x) {
  p[i] = static_cast<S>(x);
}

// ------------------------------------------------------------------ pointwise physics
// Reciprocal: the hardware estimate (relative error below 5e-8 on gfx950) refined by one
// Newton step (below 3e-15).
__device__ __forceinline__ double recip(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// Van Leer limited slope of two one-sided differences p, q (second-order reconstruction,
// Sec. 2.A), 2 p q / ((p + q) dx) when p and q agree in sign, else 0, times half a cell: the
// change of the reconstruction from the cell centre to a face, p q / (p + q).
__device__ __forceinline__ double half_limited(double p, double q) {
  const double pq = p * q;
  const double r = pq * recip(p + q);
  return pq > 0.0 ? r : 0.0;
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
template <typename Ptr>
__device__ __forceinline__ bool prim_of(Ptr W, Prim& p) {
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

// S3 time weights of Eq. (2) integrated over [0, dt]:
// Mt1 int(1 - e^{-t/tau}), Mt2 -int(tau(1 - e^{-t/tau}) - t e^{-t/tau}),
// Mt3 int(t - tau(1 - e^{-t/tau})), Mt4 int e^{-t/tau}, Mt5 int t e^{-t/tau}.
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

// Workgroups are handed to the 8 XCDs round-robin; renumber them so that each XCD works
// through one contiguous range of cells (its own L2 then serves the stencil neighbours).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}


// Cell (or tile) order of a launch: bands of kBand rows, column by column inside a band.  The
// workgroups an XCD runs at one time then cover a compact patch of the mesh, so the stencil
// neighbours a wavefront reads were read by its neighbours at about the same time and come
// from that XCD's L2.
constexpr int kBand = 16;
__device__ __forceinline__ void band_order(int L, int nx, int ny, int band, int& i, int& j) {
  const int per = band * nx;
  const int bnd = L / per;
  const int r = L - bnd * per;
  const int rows = ny - bnd * band < band ? ny - bnd * band : band;
  i = r / rows;
  j = bnd * band + (r - i * rows);
}

// f slab of column i of row j, i in [-2, nx+1]: a cell, a wrapped cell (periodic) or the
// inlet/outlet ghost column (channel).
template <typename S>
__device__ __forceinline__ const UGKS_GLOBAL S* xslab(const KParams& P, const UGKS_GLOBAL S* f,
                                                     const UGKS_GLOBAL S* fg, int i, int j) {
  if (i >= 0 && i < P.nx) return f + ((size_t)j * P.nx + i) * P.NVP;
  if (P.bc == UGKS_BC_PERIODIC) return f + ((size_t)j * P.nx + wrap(i, P.nx)) * P.NVP;
  return fg + ((size_t)(i < 0 ? 0 : P.ny) + j) * P.NVP;
}

// ------------------------------------------------------------------ wave reductions
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) x += __shfl_xor(x, h, kWave);
  return x;
}

// Reduce 16 per-lane partial sums over the wavefront through the wave's LDS block (16 rows
// of 65 doubles, the pad keeping the transposed reads on distinct banks) and add the totals
// to `fin`, whose lane 16 face + q holds sum q of that face.  Lane l adds the values of
// element l & 15 held by lanes 16 (l >> 4) .. 16 (l >> 4) + 15, then two exchanges combine
// the quarters.  Sums 4..7 (the tangential-slope moments) were accumulated from half-cell
// changes and take the factor `tscale` (2 / tangential spacing) here.  LDS operations of one
// wavefront complete in program order.
constexpr int kRedRow = kWave + 1;
__device__ __forceinline__ void flush_face(const double* a, int face, double& fin, int lane,
                                           double* red, double tscale) {
#pragma unroll
  for (int q = 0; q < 16; ++q) red[q * kRedRow + lane] = a[q];
  __builtin_amdgcn_wave_barrier();
  const int e = lane & 15, r = lane >> 4;
  const double* row = red + e * kRedRow + r * 16;
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) t += row[k];
  t += __shfl_xor(t, 16, kWave);
  t += __shfl_xor(t, 32, kWave);
  if (e >= 4 && e < 8) t *= tscale;
  if (r == face) fin += t;
  __builtin_amdgcn_wave_barrier();
}

// 16 moment sums of one face side (S1 and S7): weight wt, normal/tangential velocity
// (un, ut), reconstructed f, the tangential half-cell change ht (the tangential slope times
// half the tangential spacing; its sums are scaled when flushed) and the slope term
// D = u sigma_x + v sigma_y.
__device__ __forceinline__ void add_side(double* a, double wt, double un, double ut, double c2h,
                                         double fh, double ht, double D) {
  const double x0 = wt * fh;
  const double x1 = wt * ht;
  const double x2 = x0 * un;
  const double x3 = (wt * un) * D;
  a[0] += x0;
  a[1] = fma(x0, un, a[1]);
  a[2] = fma(x0, ut, a[2]);
  a[3] = fma(x0, c2h, a[3]);
  a[4] += x1;
  a[5] = fma(x1, un, a[5]);
  a[6] = fma(x1, ut, a[6]);
  a[7] = fma(x1, c2h, a[7]);
  a[8] += x2;
  a[9] = fma(x2, un, a[9]);
  a[10] = fma(x2, ut, a[10]);
  a[11] = fma(x2, c2h, a[11]);
  a[12] += x3;
  a[13] = fma(x3, un, a[13]);
  a[14] = fma(x3, ut, a[14]);
  a[15] = fma(x3, c2h, a[15]);
}

// Per-chunk sign code of the velocity slots: +1 / -1 when every real slot of the chunk has
// that sign of the component, 0 when mixed (or zero).
__device__ __forceinline__ int chunk_sign_u(int code) {
  return (code & 1) ? 1 : ((code & 2) ? -1 : 0);
}
__device__ __forceinline__ int chunk_sign_v(int code) {
  return (code & 4) ? 1 : ((code & 8) ? -1 : 0);
}

// ------------------------------------------------------------------ launch plans
typedef const Inst* __restrict__ inst_cptr;
typedef const int* __restrict__ int_cptr;

// Instance owning workgroup b: the last instance whose first workgroup is <= b (uniform).
__device__ __forceinline__ int find_inst(const int* off_generic, int n, int b) {
  const int_cptr off = (int_cptr)off_generic;
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int first_block(const int* off_generic, int ii) {
  return ((int_cptr)off_generic)[ii];
}

// The plan is read-only for the whole launch.
__device__ __forceinline__ const Inst* inst_at(const PlanView& pv, int ii) {
  return pv.inst + ii;
}


// ================================================================== kernels
// Discrete Maxwellian of each cell's W (initial state).
template <typename S>
__global__ __launch_bounds__(kWave) void init_kernel(PlanView pv) {
  const Inst* __restrict__ I = inst_at(pv, 0);
  const KParams P = I->P;
  UGKS_GLOBAL S* f = static_cast<UGKS_GLOBAL S*>(I->f[I->cur]);
  const UGKS_GLOBAL double* W = I->W;
  const int c = blockIdx.x;
  Prim p;
  if (!prim_of(W + 4 * (size_t)c, p) && threadIdx.x == 0) *P.flag = 1;
  const double coef = p.rho * p.lam / kPi;
  UGKS_GLOBAL S* fc = f + (size_t)c * P.NVP;
  for (int v = threadIdx.x; v < P.NVP; v += kWave) {
    double g = 0.0;
    if (v < P.NV) {
      const double du = P.U[v] - p.U, dv = P.V[v] - p.V;
      g = P.Wq[v] > 0.0 ? coef * exp(-p.lam * (du * du + dv * dv)) : 0.0;
    }
    st(fc, v, g);
  }
}

// Inlet/outlet ghost of one row: state, discrete Maxwellian, and the ghost's moment sums
// towards the domain (its slopes are zero).  2 ny workgroups per channel instance, one
// wavefront each.
template <typename S>
__global__ __launch_bounds__(kWave) void ghost_kernel(PlanView pv) {
  const int b = blockIdx.x;
  const int ii = find_inst(pv.off_ghost, pv.ninst, b);
  const Inst* __restrict__ I = inst_at(pv, ii);
  const KParams P = I->P;
  const UGKS_GLOBAL double* W = I->W;
  UGKS_GLOBAL double* Wg = I->Wg;
  UGKS_GLOBAL S* fg = static_cast<UGKS_GLOBAL S*>(I->fg);
  UGKS_GLOBAL double* hsg = I->hsg;
  const int local = b - first_block(pv.off_ghost, ii);
  const int side = local / P.ny, j = local - side * P.ny, lane = threadIdx.x;
  const int col = side == 0 ? 0 : P.nx - 1;
  Prim pc, pg;
  const bool ok = prim_of(W + 4 * ((size_t)j * P.nx + col), pc);
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
  UGKS_GLOBAL double* wg = Wg + 4 * ((size_t)side * P.ny + j);
  if (lane == 0) {
    wg[0] = pg.rho;
    wg[1] = pg.rho * pg.U;
    wg[2] = pg.rho * pg.V;
    wg[3] = 0.5 * pg.rho * (pg.U * pg.U + pg.V * pg.V) + 0.5 * pg.rho / pg.lam;
  }
  const double coef = pg.rho * pg.lam / kPi;
  UGKS_GLOBAL S* row = fg + ((size_t)side * P.ny + j) * P.NVP;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int v = lane; v < P.NVP; v += kWave) {
    const double u = P.U[v], vv = P.V[v], w = P.Wq[v];
    double g = 0.0;
    if (w > 0.0) {
      const double du = u - pg.U, dv = vv - pg.V;
      g = coef * exp(-pg.lam * (du * du + dv * dv));
    }
    st(row, v, g);
    const double gs = ld(row, v);  // the value the cells will read
    const double h = side == 0 ? upwind_left(u) : 1.0 - upwind_left(u);
    add_side(acc, w * h, u, vv, 0.5 * (u * u + vv * vv), gs, 0.0, 0.0);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double t = wave_sum(acc[q]);
    if (lane == q) hsg[((size_t)side * P.ny + j) * 16 + q] = t;
  }
}

// Per cell: slopes and the outgoing moment sums of all four faces.  One wavefront per cell,
// four cells per block.  Chunks come in velocity-quadrant order: a run of chunks with one
// sign of u and one of v feeds one x-face and one y-face, whose 16 running sums are flushed
// into `fin` (lane 16 face + q) at the end of the run; a chunk of mixed signs feeds each
// face in turn with per-lane upwind weights.
template <typename S>
__global__ __launch_bounds__(kWave* kCellsPerBlock) __attribute__((amdgpu_waves_per_eu(4)))
void sums_kernel(PlanView pv) {
  // LDS: per wavefront the 16 x 65 flush block, then the node tables u_k, v_m, w_k, w_m
  extern __shared__ double lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int ii = find_inst(pv.off_sums, pv.ninst, b);
  const Inst* __restrict__ I = inst_at(pv, ii);
  const KParams P = I->P;
  const UGKS_GLOBAL S* f = static_cast<const UGKS_GLOBAL S*>(I->f[(I->cur + pv.step) & 1]);
  const UGKS_GLOBAL S* fg = static_cast<const UGKS_GLOBAL S*>(I->fg);
  UGKS_GLOBAL double* hs = I->hs;
  double* tu = lds + kCellsPerBlock * 16 * kRedRow;
  double* tv = tu + (P.K + 1);
  double* twu = tv + (P.M + 1);
  double* twv = twu + (P.K + 1);
  for (int e = threadIdx.x; e < 2 * (P.K + 1) + 2 * (P.M + 1); e += blockDim.x) {
    double x = 0.0;  // entries K and M (padding slots) stay zero
    if (e < P.K) x = P.uk[e];
    else if (e >= P.K + 1 && e < P.K + 1 + P.M) x = P.vm[e - (P.K + 1)];
    else if (e >= P.K + P.M + 2 && e < 2 * P.K + P.M + 2) x = P.wk[e - (P.K + P.M + 2)];
    else if (e >= 2 * P.K + P.M + 3 && e < 2 * P.K + 2 * P.M + 3) x = P.wm[e - (2 * P.K + P.M + 3)];
    tu[e] = x;
  }
  __syncthreads();
  // the wavefront index is uniform: keep everything derived from it in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = (b - first_block(pv.off_sums, ii)) * kCellsPerBlock + wv;
  if (c >= P.nx * P.ny) return;
  double* red = lds + wv * 16 * kRedRow;
  int i, j;
  band_order(c, P.nx, P.ny, kBand, i, j);
  const bool wall_row = P.bc == UGKS_BC_CHANNEL && (j == 0 || j == P.ny - 1);
  const size_t cell = (size_t)j * P.nx + i;
  const UGKS_GLOBAL S* f0 = f + cell * P.NVP;
  const UGKS_GLOBAL S* fw = xslab(P, f, fg, i - 1, j);
  const UGKS_GLOBAL S* fe = xslab(P, f, fg, i + 1, j);
  const UGKS_GLOBAL S* fs = f + ((size_t)wrap(j - 1, P.ny) * P.nx + i) * P.NVP;
  const UGKS_GLOBAL S* fn = f + ((size_t)wrap(j + 1, P.ny) * P.nx + i) * P.NVP;
  double fin = 0.0;
  const int nch = P.NVP / kWave;
  // the five stencil values and the node index of chunk ch, loaded while chunk ch - 1 is
  // summed
  double buf[5];
  int kmb;
  {
    const unsigned o0 = (unsigned)lane * (unsigned)sizeof(S);
    buf[0] = (double)ldb(f0, o0);
    buf[1] = (double)ldb(fw, o0);
    buf[2] = (double)ldb(fe, o0);
    buf[3] = (double)ldb(fs, o0);
    buf[4] = (double)ldb(fn, o0);
    kmb = ldb(P.km, (unsigned)lane * 4u);
  }
  struct Point {
    double fc, hx, hy, D, u, vv, w, c2h;
  };
  const double two_idx = 2.0 * P.inv_dx, two_idy = 2.0 * P.inv_dy;
  // take chunk ch out of the buffer, start loading chunk ch + 1, and form the half-cell
  // changes hx = sigma_x dx / 2, hy = sigma_y dy / 2 and D = u sigma_x + v sigma_y
  auto point = [&](int ch) {
    Point q;
    const int v = ch * kWave + lane;
    const double fwv = buf[1], fev = buf[2], fsv = buf[3], fnv = buf[4];
    q.fc = buf[0];
    const int k = kmb & 0xffff, m = kmb >> 16;
    const unsigned vn = (unsigned)(ch + 1 < nch ? v + kWave : v);
    const unsigned on = vn * (unsigned)sizeof(S);
    buf[0] = (double)ldb(f0, on);
    buf[1] = (double)ldb(fw, on);
    buf[2] = (double)ldb(fe, on);
    buf[3] = (double)ldb(fs, on);
    buf[4] = (double)ldb(fn, on);
    kmb = ldb(P.km, vn * 4u);
    q.hx = half_limited(fev - q.fc, q.fc - fwv);
    const double hyl = half_limited(fnv - q.fc, q.fc - fsv);
    q.hy = wall_row ? 0.0 : hyl;
    q.u = tu[k];
    q.vv = tv[m];
    q.w = twu[k] * twv[m];
    q.c2h = 0.5 * fma(q.u, q.u, q.vv * q.vv);
    q.D = fma(q.u * two_idx, q.hx, (q.vv * two_idy) * q.hy);
    return q;
  };
  int ch = 0;
  while (ch < nch) {
    const int code = P.chunk_sign[ch];
    const int su = chunk_sign_u(code), sv = chunk_sign_v(code);
    if (su != 0 && sv != 0) {
      double ax[16], ay[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) ax[q] = ay[q] = 0.0;
      do {
        const Point q = point(ch);
        add_side(ax, q.w, q.u, q.vv, q.c2h, su > 0 ? q.fc + q.hx : q.fc - q.hx, q.hy, q.D);
        add_side(ay, q.w, q.vv, q.u, q.c2h, sv > 0 ? q.fc + q.hy : q.fc - q.hy, q.hx, q.D);
        ++ch;
      } while (ch < nch && P.chunk_sign[ch] == code);
      flush_face(ax, su > 0 ? S_XP : S_XM, fin, lane, red, two_idy);
      flush_face(ay, sv > 0 ? S_YP : S_YM, fin, lane, red, two_idx);
    } else {
      const Point q = point(ch);
      const double hx = upwind_left(q.u), hy = upwind_left(q.vv);
      for (int face = 0; face < 4; ++face) {
        double a[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) a[k] = 0.0;
        if (face == S_XP)
          add_side(a, q.w * hx, q.u, q.vv, q.c2h, q.fc + q.hx, q.hy, q.D);
        else if (face == S_XM)
          add_side(a, q.w * (1.0 - hx), q.u, q.vv, q.c2h, q.fc - q.hx, q.hy, q.D);
        else if (face == S_YP)
          add_side(a, q.w * hy, q.vv, q.u, q.c2h, q.fc + q.hy, q.hx, q.D);
        else
          add_side(a, q.w * (1.0 - hy), q.vv, q.u, q.c2h, q.fc - q.hy, q.hx, q.D);
        flush_face(a, face, fin, lane, red, face < 2 ? two_idy : two_idx);
      }
      ++ch;
    }
  }
  hs[cell * kSlots + lane] = fin;
}

// S2-S5 at one interior interface, local frame.  S = [W0, Wt, Q1, Q2].  Writes the local
// macroscopic flux to F and the folded coefficients of the distribution flux to rec.
__device__ void interface_scalars(const KParams& P, const double* S, const double* WL,
                                  const double* WR, double dn, double len, double* F,
                                  UGKS_GLOBAL double* rec, double& U0, double& V0) {
  const double* W0 = S;
  const double* Wt = S + 4;
  const double* Q1 = S + 8;
  const double* Q2 = S + 12;
  if (P.collisionless) {
    const double Mt4 = P.dt, Mt5 = 0.5 * P.dt * P.dt;
#pragma unroll
    for (int q = 0; q < 4; ++q) F[q] = len * (Mt4 * Q1[q] - Mt5 * Q2[q]);
#pragma unroll
    for (int q = 0; q < 13; ++q) rec[R_E + q] = 0.0;
    rec[R_GC] = 0.0;
    rec[R_LAM] = 0.0;
    rec[R_M4] = len * Mt4;
    rec[R_M5] = len * Mt5;
    rec[R_KIND] = K_FREE;
    U0 = V0 = 0.0;
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
  // folded polynomial of the equilibrium part of the distribution flux
  rec[R_E + 0] = Mt[0] + Mt[2] * A[0];
  rec[R_E + 1] = Mt[1] * aL[0] + Mt[2] * A[1];
  rec[R_E + 2] = Mt[1] * b[0] + Mt[2] * A[2];
  rec[R_E + 3] = Mt[2] * A[3];
  rec[R_E + 4] = Mt[1] * aL[1];
  rec[R_E + 5] = Mt[1] * (aL[2] + b[1]);
  rec[R_E + 6] = Mt[1] * b[2];
  rec[R_E + 7] = Mt[1] * aL[3];
  rec[R_E + 8] = Mt[1] * b[3];
  rec[R_ER + 0] = Mt[1] * aR[0] + Mt[2] * A[1];
  rec[R_ER + 1] = Mt[1] * aR[1];
  rec[R_ER + 2] = Mt[1] * (aR[2] + b[1]);
  rec[R_ER + 3] = Mt[1] * aR[3];
  rec[R_GC] = len * p0.rho * p0.lam / kPi;
  rec[R_LAM] = p0.lam;
  rec[R_M4] = len * Mt[3];
  rec[R_M5] = len * Mt[4];
  rec[R_KIND] = K_INTERIOR;
  U0 = p0.U;
  V0 = p0.V;
}

// One thread per interface: x-faces first (ny rows of nx+1), then y-faces (ny+1 rows of nx).
__global__ __launch_bounds__(256) void faces_kernel(PlanView pv) {
  const int b = blockIdx.x;
  const int ii = find_inst(pv.off_face, pv.ninst, b);
  const Inst* __restrict__ I = inst_at(pv, ii);
  const KParams P = I->P;
  const UGKS_GLOBAL double* hs = I->hs;
  const UGKS_GLOBAL double* hsg = I->hsg;
  const UGKS_GLOBAL double* W = I->W;
  const UGKS_GLOBAL double* Wg = I->Wg;
  UGKS_GLOBAL double* recx = I->recx;
  UGKS_GLOBAL double* recy = I->recy;
  const long e = (long)(b - first_block(pv.off_face, ii)) * blockDim.x + threadIdx.x;
  const long nfx = (long)P.ny * (P.nx + 1);
  const long nfy = (long)(P.ny + 1) * P.nx;
  const bool chan = P.bc == UGKS_BC_CHANNEL;
  double S[16], F[4];
  double U0, V0;
  if (e < nfx) {
    const int j = (int)(e / (P.nx + 1)), i = (int)(e % (P.nx + 1));
    const UGKS_GLOBAL double *sL, *sR, *WL, *WR;
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
    UGKS_GLOBAL double* rec = recx + (size_t)e * kRec;
    interface_scalars(P, S, wl, wr, P.dx, P.dy, F, rec, U0, V0);
#pragma unroll
    for (int q = 0; q < 4; ++q) rec[R_FX + q] = F[q];
    rec[R_UX] = U0;
    rec[R_VY] = V0;
    return;
  }
  if (e >= nfx + nfy) return;
  const long e2 = e - nfx;
  const int j = (int)(e2 / P.nx), i = (int)(e2 % P.nx);
  UGKS_GLOBAL double* rec = recy + (size_t)e2 * kRec;
  if (chan && (j == 0 || j == P.ny)) {
    // diffuse wall: sums of the wall-row cell towards the wall; local frame (v, u)
    const bool top = j == P.ny;
    const size_t c = (size_t)(top ? P.ny - 1 : 0) * P.nx + i;
    const UGKS_GLOBAL double* Q1 = hs + c * kSlots + 16 * (top ? S_YP : S_YM) + 8;
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
    rec[R_GC] = s * rho_w * P.lam_w / kPi;
    rec[R_LAM] = P.lam_w;
    rec[R_UX] = 0.0;
    rec[R_VY] = 0.0;
    rec[R_M4] = s;
    rec[R_M5] = 0.0;
    rec[R_KIND] = K_WALL;
    if (!(rho_w > 0.0) || !isfinite(rho_w)) *P.flag = 1;
    return;
  }
  const size_t cl = (size_t)wrap(j - 1, P.ny) * P.nx + i;
  const size_t cr = (size_t)wrap(j, P.ny) * P.nx + i;
  const UGKS_GLOBAL double* sL = hs + cl * kSlots + 16 * S_YP;
  const UGKS_GLOBAL double* sR = hs + cr * kSlots + 16 * S_YM;
#pragma unroll
  for (int q = 0; q < 16; ++q) S[q] = sL[q] + sR[q];
  const double wl[4] = {W[4 * cl], W[4 * cl + 2], W[4 * cl + 1], W[4 * cl + 3]};
  const double wr[4] = {W[4 * cr], W[4 * cr + 2], W[4 * cr + 1], W[4 * cr + 3]};
  interface_scalars(P, S, wl, wr, P.dy, P.dx, F, rec, U0, V0);
  rec[R_FX + 0] = F[0];
  rec[R_FX + 1] = F[2];
  rec[R_FX + 2] = F[1];
  rec[R_FX + 3] = F[3];
  rec[R_UX] = V0;  // local (normal, tangential) = global (y, x)
  rec[R_VY] = U0;
}

// ------------------------------------------------------------------ update kernel
// Each wavefront (one cell) builds in LDS, for each of its four faces, the equilibrium part of
// the distribution flux in separable form: with un the normal and ut the tangential velocity,
//   GC En(un) Et(ut) P(un, ut) = TE[t] (TA[n] + ut (TB[n] + ut (TC[n] + ut TD[n])))
// where P is the folded cubic of the record, n / t index the normal / tangential velocity node
// and the normal-slope choice (aL for un > 0, aR for un < 0) is made per node n.  The cell's
// g^n and g^{n+1} are kept as products of two 1D tables with the Eq. (3) weights folded in.
// Everything indexed by the u node k sits in one row of 12 doubles, everything indexed by the
// v node m in another, so a lane reads all its table entries from two rows:
//   u row k: left and right face polys (4 + 4), bottom and top face exps, g^n and g^{n+1}
//            u factors;
//   v row m: bottom and top face polys (4 + 4), left and right face exps, g^n and g^{n+1}
//            v factors.
// Row K and row M stay zero: padding slots point there, so their update is exactly zero.
// Rows are 13 doubles apart (one unused): with an odd stride up to 16 different rows a chunk
// touches sit on distinct LDS banks for 8-byte reads.
constexpr int kRow = 13;
enum RowEntry { RP_LO = 0, RP_HI = 4, RE_LO = 8, RE_HI = 9, RG_N = 10, RG_1 = 11 };

__host__ __device__ __forceinline__ int tab_doubles(int K, int M) {
  return kRow * (K + 1) + kRow * (M + 1);
}

// Doubles of the block-shared node tables.
__host__ __device__ __forceinline__ int node_doubles(int K, int M) { return K + M + 2; }

// Fill the four-entry polynomial table of one face at normal node with velocity un.
__device__ __forceinline__ void face_poly(const UGKS_GLOBAL double* r, double un, double lam,
                                          double U0, double* out) {
  const double d = un - U0;
  const double En = exp(-lam * d * d) * r[R_GC];
  const bool pos = un > 0.0;
  const double e1 = pos ? r[R_E + 1] : r[R_ER + 0];
  const double e4 = pos ? r[R_E + 4] : r[R_ER + 1];
  const double e5 = pos ? r[R_E + 5] : r[R_ER + 2];
  const double e7 = pos ? r[R_E + 7] : r[R_ER + 3];
  const double e0 = r[R_E + 0], e2 = r[R_E + 2], e3 = r[R_E + 3], e6 = r[R_E + 6],
               e8 = r[R_E + 8];
  // P(un, ut) = A + ut (B + ut (C + ut D)) with
  // A = e0 + un (e1 + un (e4 + e3/2 + un e7/2)), B = e2 + un (e5 + un e8/2),
  // C = e6 + e3/2 + un e7/2, D = e8/2
  out[0] = En * fma(un, fma(un, fma(un, 0.5 * e7, e4 + 0.5 * e3), e1), e0);
  out[1] = En * fma(un, fma(un, 0.5 * e8, e5), e2);
  out[2] = En * fma(un, 0.5 * e7, e6 + 0.5 * e3);
  out[3] = En * (0.5 * e8);
}

// Equilibrium part at one velocity from a face's tables (poly at the normal node, E at the
// tangential node) and the time-integrated flux of the face.
// D = u sigma_x + v sigma_y is the slope term of the upwind cell (the same for its x- and
// y-faces).
__device__ __forceinline__ double face_flux(double2 pab, double2 pcd, double E, double un,
                                            double ut, double fh, double D, double m4,
                                            double m5) {
  const double G = E * fma(ut, fma(ut, fma(ut, pcd.y, pcd.x), pab.y), pab.x);
  const double free_part = fma(m4, fh, -m5 * D);
  return un * (G + free_part);
}

template <typename S>
struct UpdateCtx {
  const UGKS_GLOBAL S* f0;
  const UGKS_GLOBAL S* xw;
  const UGKS_GLOBAL S* xe;
  const UGKS_GLOBAL S* xww;
  const UGKS_GLOBAL S* xee;
  const UGKS_GLOBAL S* sw;
  const UGKS_GLOBAL S* sc;
  const UGKS_GLOBAL S* se;
  const UGKS_GLOBAL S* nw;
  const UGKS_GLOBAL S* nc;
  const UGKS_GLOBAL S* ne;
  const UGKS_GLOBAL S* scc;
  const UGKS_GLOBAL S* ncc;
};

// Left-minus-right flux difference for one velocity.  SX = +1 / -1: u has that sign across
// the wavefront; 0: per lane.  Every stencil value is loaded (every slab pointer is valid);
// boundaries only switch results.  Slopes are carried as half-cell changes h = sigma dx / 2
// (or dy / 2); ucx = 2 u / dx and vcy = 2 v / dy turn them into u sigma_x + v sigma_y.
template <int SX>
__device__ __forceinline__ double x_part(double u, double vv, double ucx, double vcy, double fc,
                                         double fW, double fE, double fXX, double fXn,
                                         double fXs, double hx0, double D0, bool ghost_w,
                                         bool ghost_e, bool wall_row, const double* lp,
                                         const double* rp, double le, double re, double m4l,
                                         double m5l, double m4r, double m5r) {
  // particles with u > 0 enter through the left face from cell i-1 (the upwind cell X); fXX
  // is X's far x-neighbour (i -+ 2), fXn and fXs its y-neighbours
  const bool right = SX > 0 ? true : (SX < 0 ? false : (u > 0.0));
  const double fX = right ? fW : fE;
  const bool ghostX = right ? ghost_w : ghost_e;
  const double hxl = right ? half_limited(fc - fX, fX - fXX) : half_limited(fXX - fX, fX - fc);
  const double hyl = half_limited(fXn - fX, fX - fXs);
  const double hxX = ghostX ? 0.0 : hxl;
  const double hyX = (ghostX || wall_row) ? 0.0 : hyl;
  const double DX = fma(ucx, hxX, vcy * hyX);
  const double fh_in = right ? fX + hxX : fX - hxX;
  const double fh_own = right ? fc + hx0 : fc - hx0;
  // left face: upwind is X when moving right, the cell itself when moving left
  const double fl = right ? fh_in : fh_own, Dl = right ? DX : D0;
  const double fr = right ? fh_own : fh_in, Dr = right ? D0 : DX;
  const double2 lab = make_double2(lp[0], lp[1]);
  const double2 lcd = make_double2(lp[2], lp[3]);
  const double2 rab = make_double2(rp[0], rp[1]);
  const double2 rcd = make_double2(rp[2], rp[3]);
  const double Fl = face_flux(lab, lcd, le, u, vv, fl, Dl, m4l, m5l);
  const double Fr = face_flux(rab, rcd, re, u, vv, fr, Dr, m4r, m5r);
  return Fl - Fr;
}

// Bottom-minus-top flux difference.  Walls: particles leaving a wall follow rho_w times the
// wall Maxwellian (its tables hold dx dt rho_w g_w), those reaching it carry the wall-row value.
template <int SY>
__device__ __forceinline__ double y_part(double u, double vv, double ucx, double vcy, double fc,
                                         double fS, double fN, double fYY, double fYe,
                                         double fYw, double hy0, double D0, bool wall_b,
                                         bool wall_t, bool s_wallrow, bool n_wallrow,
                                         const double* bp, const double* tp, double be,
                                         double te, double m4b, double m5b, double m4t,
                                         double m5t) {
  // the upwind cell Y is (i, j -+ 1); fYY is its far y-neighbour, fYe and fYw its x-neighbours
  const bool up = SY > 0 ? true : (SY < 0 ? false : (vv > 0.0));
  const double fY = up ? fS : fN;
  const bool Y_wallrow = up ? s_wallrow : n_wallrow;
  const double hyl = up ? half_limited(fc - fY, fY - fYY) : half_limited(fYY - fY, fY - fc);
  const double hyY = Y_wallrow ? 0.0 : hyl;
  const double hxY = half_limited(fYe - fY, fY - fYw);
  const double DY = fma(ucx, hxY, vcy * hyY);
  const double fh_in = up ? fY + hyY : fY - hyY;
  const double fh_own = up ? fc + hy0 : fc - hy0;
  // bottom face: upwind is Y when moving up, the cell itself when moving down
  const double fb = up ? fh_in : fh_own, Db = up ? DY : D0;
  const double ft = up ? fh_own : fh_in, Dt = up ? D0 : DY;
  const double2 bab = make_double2(bp[0], bp[1]);
  const double2 bcd = make_double2(bp[2], bp[3]);
  const double2 tab2 = make_double2(tp[0], tp[1]);
  const double2 tcd = make_double2(tp[2], tp[3]);
  const double Fb_face = face_flux(bab, bcd, be, vv, u, fb, Db, m4b, m5b);
  const double Ft_face = face_flux(tab2, tcd, te, vv, u, ft, Dt, m4t, m5t);
  const double Fb_wall = up ? vv * (be * bab.x) : vv * (m4b * fc);
  const double Ft_wall = up ? vv * (m4t * fc) : vv * (te * tab2.x);
  const double Fb = wall_b ? Fb_wall : Fb_face;
  const double Ft = wall_t ? Ft_wall : Ft_face;
  return Fb - Ft;
}

// Per cell: Eq. (4) for W, then Eq. (3) for every velocity.  One wavefront per cell.
template <typename S>
__global__ __launch_bounds__(kWave* kCellsPerBlock) __attribute__((amdgpu_waves_per_eu(4)))
void update_kernel(PlanView pv) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int cpb = (int)(blockDim.x >> 6);
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int ii = find_inst(pv.off_upd, pv.ninst, b);
  const Inst* __restrict__ I = inst_at(pv, ii);
  const KParams P = I->P;
  const int parity = (I->cur + pv.step) & 1;
  const UGKS_GLOBAL S* fin = static_cast<const UGKS_GLOBAL S*>(I->f[parity]);
  UGKS_GLOBAL S* fout = static_cast<UGKS_GLOBAL S*>(I->f[parity ^ 1]);
  const UGKS_GLOBAL S* fg = static_cast<const UGKS_GLOBAL S*>(I->fg);
  const UGKS_GLOBAL double* recx = I->recx;
  const UGKS_GLOBAL double* recy = I->recy;
  UGKS_GLOBAL double* W = I->W;
  // LDS: the block's node tables u_k (K + 1 entries) and v_m (M + 1), zero in the padding
  // entries, then the per-cell tables (8-byte aligned)
  double* tuu = lds;
  double* tvv = lds + (P.K + 1);
  double* tb = lds + node_doubles(P.K, P.M) + (size_t)wv * (size_t)(pv.lds_per_cell / 8);
  double* urow = tb;                        // rows k = 0..K
  double* vrow = tb + kRow * (P.K + 1);     // rows m = 0..M
  for (int e = threadIdx.x; e < P.K + P.M + 2; e += blockDim.x)
    tuu[e] = e < P.K ? P.uk[e] : ((e > P.K && e < P.K + 1 + P.M) ? P.vm[e - P.K - 1] : 0.0);
  const int c = (b - first_block(pv.off_upd, ii)) * cpb + wv;
  const bool active = c < P.nx * P.ny;
  int i, j;
  band_order(active ? c : 0, P.nx, P.ny, kBand, i, j);
  const int cc = j * P.nx + i;
  const bool chan = P.bc == UGKS_BC_CHANNEL;
  const UGKS_GLOBAL double* rl = recx + ((size_t)j * (P.nx + 1) + i) * kRec;
  const UGKS_GLOBAL double* rr = recx + ((size_t)j * (P.nx + 1) + i + 1) * kRec;
  const UGKS_GLOBAL double* rb = recy + ((size_t)j * P.nx + i) * kRec;
  const UGKS_GLOBAL double* rt = recy + ((size_t)(j + 1) * P.nx + i) * kRec;
  // Eq. (4)
  double Wn[4], W1[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    Wn[q] = W[4 * (size_t)cc + q];
    W1[q] = Wn[q] + (rl[q] - rr[q] + rb[q] - rt[q]) / P.area;
  }
  Prim pn{}, p1{};
  // Eq. (3) solved for f^{n+1}: f1 = Af f + AdF dF + (A1 g^{n+1} + An g^n), the weights of
  // g folded into its tables
  double Af = 1.0, AdF = 1.0 / P.area, A1 = 0.0, An = 0.0;
  if (!P.collisionless) {
    const bool ok = prim_of(Wn, pn) && prim_of(W1, p1);
    if (!ok && lane == 0 && active) *P.flag = 1;
    const double tn = collision_time(pn, P.mu_ref), t1 = collision_time(p1, P.mu_ref);
    const double hdt = 0.5 * P.dt;
    const double den = 1.0 / (1.0 + hdt / t1);
    Af = (1.0 - hdt / tn) * den;
    AdF = den / P.area;
    A1 = (p1.rho * p1.lam / kPi) * (hdt / t1) * den;
    An = (pn.rho * pn.lam / kPi) * (hdt / tn) * den;
  }
  // poly tables of the two x-faces (normal node k) and the two y-faces (normal node m)
  for (int e = lane; e < 2 * P.K + 2 * P.M; e += kWave) {
    double* out;
    const UGKS_GLOBAL double* rs;
    double un, lamf, U0;
    if (e < 2 * P.K) {
      const int side = e / P.K, k = e - side * P.K;
      rs = side ? rr : rl;
      un = P.uk[k];
      U0 = rs[R_UX];
      out = urow + kRow * k + (side ? RP_HI : RP_LO);
    } else {
      const int e2 = e - 2 * P.K;
      const int side = e2 / P.M, m = e2 - side * P.M;
      rs = side ? rt : rb;
      un = P.vm[m];
      U0 = rs[R_VY];
      out = vrow + kRow * m + (side ? RP_HI : RP_LO);
    }
    lamf = rs[R_LAM];
    if (rs[R_KIND] == (double)K_WALL) {
      // wall: only the Maxwellian itself (P = 1), scaled by dx dt rho_w lambda_w / pi
      const double d = un - U0;
      out[0] = exp(-lamf * d * d) * rs[R_GC];
      out[1] = out[2] = out[3] = 0.0;
    } else {
      double tmp[4];
      face_poly(rs, un, lamf, U0, tmp);
      out[0] = tmp[0];
      out[1] = tmp[1];
      out[2] = tmp[2];
      out[3] = tmp[3];
    }
  }
  // tangential tables of the faces and the two factors of g^n and g^{n+1}
  for (int e = lane; e < 4 * (P.K + P.M); e += kWave) {
    double lam, vel, c0, coef = 1.0;
    double* dst;
    if (e < 2 * P.M) {  // x-faces: tangential v
      const int side = e / P.M, m = e - side * P.M;
      const UGKS_GLOBAL double* rs = side ? rr : rl;
      lam = rs[R_LAM];
      vel = P.vm[m];
      c0 = rs[R_VY];
      dst = vrow + kRow * m + (side ? RE_HI : RE_LO);
    } else if (e < 2 * P.M + 2 * P.K) {  // y-faces: tangential u
      const int e2 = e - 2 * P.M;
      const int side = e2 / P.K, k = e2 - side * P.K;
      const UGKS_GLOBAL double* rs = side ? rt : rb;
      lam = rs[R_LAM];
      vel = P.uk[k];
      c0 = rs[R_UX];
      dst = urow + kRow * k + (side ? RE_HI : RE_LO);
    } else {  // g^n, g^{n+1}: u factor carries the Eq. (3) weight
      const int e3 = e - 2 * P.M - 2 * P.K;
      const int which = e3 / (P.K + P.M), r = e3 - which * (P.K + P.M);
      lam = which ? p1.lam : pn.lam;
      if (r < P.K) {
        vel = P.uk[r];
        c0 = which ? p1.U : pn.U;
        coef = which ? A1 : An;
        dst = urow + kRow * r + (which ? RG_1 : RG_N);
      } else {
        vel = P.vm[r - P.K];
        c0 = which ? p1.V : pn.V;
        dst = vrow + kRow * (r - P.K) + (which ? RG_1 : RG_N);
      }
    }
    const double d = vel - c0;
    *dst = coef * exp(-lam * d * d);
  }
  // the zero rows of the padding slots
  for (int e = lane; e < 2 * kRow; e += kWave)
    (e < kRow ? urow + kRow * P.K : vrow + kRow * P.M)[e % kRow] = 0.0;
  __syncthreads();
  if (!active) return;
  const double m4l = rl[R_M4], m5l = rl[R_M5], m4r = rr[R_M4], m5r = rr[R_M5];
  const double m4b = rb[R_M4], m5b = rb[R_M5], m4t = rt[R_M4], m5t = rt[R_M5];
  const bool wall_b = chan && j == 0, wall_t = chan && j == P.ny - 1;
  const bool wall_row = wall_b || wall_t;
  const bool ghost_w = chan && i == 0, ghost_e = chan && i == P.nx - 1;
  const bool s_wallrow = chan && (j - 1 == 0);
  const bool n_wallrow = chan && (j + 1 == P.ny - 1);
  const int js = wrap(j - 1, P.ny), jn = wrap(j + 1, P.ny);
  UpdateCtx<S> X;
  X.f0 = fin + (size_t)cc * P.NVP;
  X.xw = xslab(P, fin, fg, i - 1, j);
  X.xe = xslab(P, fin, fg, i + 1, j);
  X.xww = xslab(P, fin, fg, i - 2, j);
  X.xee = xslab(P, fin, fg, i + 2, j);
  X.sw = xslab(P, fin, fg, i - 1, js);
  X.sc = xslab(P, fin, fg, i, js);
  X.se = xslab(P, fin, fg, i + 1, js);
  X.nw = xslab(P, fin, fg, i - 1, jn);
  X.nc = xslab(P, fin, fg, i, jn);
  X.ne = xslab(P, fin, fg, i + 1, jn);
  X.scc = fin + ((size_t)wrap(j - 2, P.ny) * P.nx + i) * P.NVP;
  X.ncc = fin + ((size_t)wrap(j + 2, P.ny) * P.nx + i) * P.NVP;
  UGKS_GLOBAL S* fo = fout + (size_t)cc * P.NVP;
  const double two_idx = 2.0 * P.inv_dx, two_idy = 2.0 * P.inv_dy;
  const int nch = P.NVP / kWave;
  // The chunk loop, compiled twice: for cells next to a ghost column or a wall (EDGE) and for
  // the interior, where every boundary switch is constant false.
  auto chunks = [&](auto edge_c) {
    constexpr bool EDGE = decltype(edge_c)::value;
    const bool gw = EDGE && ghost_w, ge = EDGE && ghost_e, wr = EDGE && wall_row;
    const bool wb = EDGE && wall_b, wt = EDGE && wall_t;
    const bool swr = EDGE && s_wallrow, nwr = EDGE && n_wallrow;
    // one chunk; MIXED: its lanes have both signs of u or of v, so the upwind neighbours'
    // far slabs are chosen per lane (otherwise per chunk, in scalar registers)
    auto chunk = [&](auto mixed_c, int ch, int su, int sv) {
      constexpr bool MIXED = decltype(mixed_c)::value;
      const unsigned v = (unsigned)(ch * kWave + lane);
      const unsigned vb = v * (unsigned)sizeof(S);
      // all stencil values of the chunk are requested before any is used
      const int kmv = ldb(P.km, v * 4u);
      const double fc = (double)ldb(X.f0, vb);
      const double fW = (double)ldb(X.xw, vb), fE = (double)ldb(X.xe, vb);
      const double fS = (double)ldb(X.sc, vb), fN = (double)ldb(X.nc, vb);
      double xxx, xxn, xxs, yyy, yye, yyw;
      if (!MIXED) {
        const UGKS_GLOBAL S* pxx = su > 0 ? X.xww : X.xee;
        const UGKS_GLOBAL S* pxn = su > 0 ? X.nw : X.ne;
        const UGKS_GLOBAL S* pxs = su > 0 ? X.sw : X.se;
        const UGKS_GLOBAL S* pyy = sv > 0 ? X.scc : X.ncc;
        const UGKS_GLOBAL S* pye = sv > 0 ? X.se : X.ne;
        const UGKS_GLOBAL S* pyw = sv > 0 ? X.sw : X.nw;
        xxx = (double)ldb(pxx, vb);
        xxn = (double)ldb(pxn, vb);
        xxs = (double)ldb(pxs, vb);
        yyy = (double)ldb(pyy, vb);
        yye = (double)ldb(pye, vb);
        yyw = (double)ldb(pyw, vb);
      }
      const int k = kmv & 0xffff, m = kmv >> 16;
      const double u = tuu[k], vv = tvv[m];
      if (MIXED) {
        const bool r = su > 0 || (su == 0 && u > 0.0);
        const bool t = sv > 0 || (sv == 0 && vv > 0.0);
        xxx = (double)ldb(r ? X.xww : X.xee, vb);
        xxn = (double)ldb(r ? X.nw : X.ne, vb);
        xxs = (double)ldb(r ? X.sw : X.se, vb);
        yyy = (double)ldb(t ? X.scc : X.ncc, vb);
        yye = (double)ldb(t ? X.se : X.ne, vb);
        yyw = (double)ldb(t ? X.sw : X.nw, vb);
      }
      const double hx0 = half_limited(fE - fc, fc - fW);
      const double hyl = half_limited(fN - fc, fc - fS);
      const double hy0 = wr ? 0.0 : hyl;
      const double ucx = u * two_idx, vcy = vv * two_idy;
      const double D0 = fma(ucx, hx0, vcy * hy0);
      const double* ur = urow + kRow * k;
      const double* vr = vrow + kRow * m;
      const double* lp = ur + RP_LO;
      const double* rp = ur + RP_HI;
      const double* bp = vr + RP_LO;
      const double* tp = vr + RP_HI;
      const double le = vr[RE_LO], re = vr[RE_HI];
      const double be = ur[RE_LO], te = ur[RE_HI];
      double dFx, dFy;
      if (su > 0)
        dFx = x_part<1>(u, vv, ucx, vcy, fc, fW, fE, xxx, xxn, xxs, hx0, D0, gw, ge, wr, lp, rp,
                        le, re, m4l, m5l, m4r, m5r);
      else if (su < 0)
        dFx = x_part<-1>(u, vv, ucx, vcy, fc, fW, fE, xxx, xxn, xxs, hx0, D0, gw, ge, wr, lp, rp,
                         le, re, m4l, m5l, m4r, m5r);
      else
        dFx = x_part<0>(u, vv, ucx, vcy, fc, fW, fE, xxx, xxn, xxs, hx0, D0, gw, ge, wr, lp, rp,
                        le, re, m4l, m5l, m4r, m5r);
      if (sv > 0)
        dFy = y_part<1>(u, vv, ucx, vcy, fc, fS, fN, yyy, yye, yyw, hy0, D0, wb, wt, swr, nwr,
                        bp, tp, be, te, m4b, m5b, m4t, m5t);
      else if (sv < 0)
        dFy = y_part<-1>(u, vv, ucx, vcy, fc, fS, fN, yyy, yye, yyw, hy0, D0, wb, wt, swr, nwr,
                         bp, tp, be, te, m4b, m5b, m4t, m5t);
      else
        dFy = y_part<0>(u, vv, ucx, vcy, fc, fS, fN, yyy, yye, yyw, hy0, D0, wb, wt, swr, nwr,
                        bp, tp, be, te, m4b, m5b, m4t, m5t);
      const double g = fma(ur[RG_1], vr[RG_1], ur[RG_N] * vr[RG_N]);
      const double f1 = fma(Af, fc, fma(AdF, dFx + dFy, g));
      *reinterpret_cast<UGKS_GLOBAL S*>(reinterpret_cast<UGKS_GLOBAL char*>(fo) + vb) =
          static_cast<S>(f1);
    };
    for (int ch = 0; ch < nch; ++ch) {
      const int code = P.chunk_sign[ch];
      const int su = chunk_sign_u(code), sv = chunk_sign_v(code);
      if (su != 0 && sv != 0)
        chunk(std::false_type{}, ch, su, sv);
      else
        chunk(std::true_type{}, ch, su, sv);
    }
  };
  if (ghost_w || ghost_e || wall_row || s_wallrow || n_wallrow)
    chunks(std::true_type{});
  else
    chunks(std::false_type{});
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) W[4 * (size_t)cc + q] = W1[q];
  }
}

}  // namespace

// ================================================================== launchers
size_t plan_bytes(int n) {
  const size_t inst = ((sizeof(Inst) * (size_t)n + 255) / 256) * 256;
  return inst + 5 * (((size_t)(n + 1) * sizeof(int) + 255) / 256) * 256;
}

PlanTotals build_plan(const Inst* insts, int n, void* buf, const void* dev, PlanView* view) {
  char* h = static_cast<char*>(buf);
  const char* d = static_cast<const char*>(dev);
  const size_t inst_bytes = ((sizeof(Inst) * (size_t)n + 255) / 256) * 256;
  const size_t off_bytes = (((size_t)(n + 1) * sizeof(int) + 255) / 256) * 256;
  std::memcpy(h, insts, sizeof(Inst) * (size_t)n);
  int* off[5];
  for (int a = 0; a < 5; ++a) off[a] = reinterpret_cast<int*>(h + inst_bytes + a * off_bytes);
  PlanTotals t{};
  // update kernel: cells per workgroup limited by the (nu + 1) + (nv + 1) table rows per cell
  int max_cell = 0, max_nodes = 0, max_sums = 0;
  for (int q = 0; q < n; ++q) {
    const int K = insts[q].P.K, M = insts[q].P.M;
    const int bytes = tab_doubles(K, M) * 8;
    max_cell = bytes > max_cell ? bytes : max_cell;
    max_nodes = node_doubles(K, M) * 8 > max_nodes ? node_doubles(K, M) * 8 : max_nodes;
    const int sums = (kCellsPerBlock * 16 * kRedRow + 2 * (K + 1) + 2 * (M + 1)) * 8;
    max_sums = sums > max_sums ? sums : max_sums;
  }
  int cpb = kCellsPerBlock;
  while (cpb > 1 && (size_t)max_nodes + (size_t)max_cell * cpb > 64 * 1024) cpb /= 2;
  t.cpb_upd = cpb;
  t.lds_per_cell = max_cell;
  t.lds_upd = max_nodes + max_cell * cpb;
  t.lds_sums = max_sums;
  for (int q = 0; q < n; ++q) {
    const KParams& P = insts[q].P;
    const int nc = P.nx * P.ny;
    const int nf = P.ny * (P.nx + 1) + (P.ny + 1) * P.nx;
    off[0][q] = t.sums;
    off[1][q] = t.upd;
    off[2][q] = t.face;
    off[3][q] = t.ghost;
    off[4][q] = 0;
    t.sums += (nc + kCellsPerBlock - 1) / kCellsPerBlock;
    t.upd += (nc + cpb - 1) / cpb;
    t.face += (nf + 255) / 256;
    t.ghost += P.bc == UGKS_BC_CHANNEL ? 2 * P.ny : 0;
  }
  off[0][n] = t.sums;
  off[1][n] = t.upd;
  off[2][n] = t.face;
  off[3][n] = t.ghost;
  off[4][n] = 0;
  view->inst = reinterpret_cast<const Inst*>(d);
  view->off_sums = reinterpret_cast<const int*>(d + inst_bytes + 0 * off_bytes);
  view->off_upd = reinterpret_cast<const int*>(d + inst_bytes + 1 * off_bytes);
  view->off_face = reinterpret_cast<const int*>(d + inst_bytes + 2 * off_bytes);
  view->off_ghost = reinterpret_cast<const int*>(d + inst_bytes + 3 * off_bytes);
  view->ninst = n;
  view->step = 0;
  view->cpb_upd = cpb;
  view->lds_per_cell = max_cell;
  return t;
}

hipError_t launch_init(const PlanView& pv, int fp32, int ncells, hipStream_t s) {
  if (fp32)
    init_kernel<float><<<(unsigned)ncells, kWave, 0, s>>>(pv);
  else
    init_kernel<double><<<(unsigned)ncells, kWave, 0, s>>>(pv);
  return hipGetLastError();
}

// phase 0 ghosts, 1 moment sums, 2 interface scalars, 3 cell update
hipError_t launch_phase(const PlanView& pv, const PlanTotals& t, int fp32, int phase,
                        hipStream_t s) {
  switch (phase) {
    case 0:
      if (t.ghost == 0) return hipSuccess;
      if (fp32)
        ghost_kernel<float><<<(unsigned)t.ghost, kWave, 0, s>>>(pv);
      else
        ghost_kernel<double><<<(unsigned)t.ghost, kWave, 0, s>>>(pv);
      break;
    case 1:
      if (fp32)
        sums_kernel<float><<<(unsigned)t.sums, kWave * kCellsPerBlock, t.lds_sums, s>>>(pv);
      else
        sums_kernel<double><<<(unsigned)t.sums, kWave * kCellsPerBlock, t.lds_sums, s>>>(pv);
      break;
    case 2:
      faces_kernel<<<(unsigned)t.face, 256, 0, s>>>(pv);
      break;
    default: {
      const size_t lds = (size_t)t.lds_upd;
      const unsigned threads = kWave * (unsigned)t.cpb_upd;
      if (fp32)
        update_kernel<float><<<(unsigned)t.upd, threads, lds, s>>>(pv);
      else
        update_kernel<double><<<(unsigned)t.upd, threads, lds, s>>>(pv);
    }
  }
  return hipGetLastError();
}

hipError_t launch_step(const PlanView& pv, const PlanTotals& t, int fp32, hipStream_t s,
                       hipEvent_t* ev) {
  for (int phase = 0; phase < 4; ++phase) {
    if (ev) (void)hipEventRecord(ev[2 * phase], s);
    const hipError_t e = launch_phase(pv, t, fp32, phase, s);
    if (ev) (void)hipEventRecord(ev[2 * phase + 1], s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ugks
