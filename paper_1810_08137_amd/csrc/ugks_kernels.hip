// gfx950 kernels of the 2D UGKS time step.
//
// One step is three launches on one stream (four in a periodic box):
//   ghost   periodic box only: the periodic images into the halo of every velocity plane
//   sums    per cell and velocity: limited slopes of f, the upwind reconstruction at the
//           cell's outgoing faces and their velocity moments (S1 and the sums of S7); in a
//           channel also the sums of the inlet and outlet ghost columns (Sec. 3.A); a solver
//           that splits its velocities into chunks adds the chunks' partial sums in a second,
//           small launch
//   faces   per interface: add the two sides' sums, then the scalar part of the flux
//           (S2-S5: Maxwellian moments, time weights, micro slopes, equilibrium flux) into a
//           record of folded coefficients
//   update  per cell and velocity: the distribution flux at the faces (S6, S8), then Eq. (4)
//           for W and Eq. (3) for f; in a channel also the ghost states of the next step
//           (from W^{n+1}) and their Maxwellians in the ghost columns of f^{n+1}
// After the initial state and after a state is set, the update kernel's fill mode writes a
// channel's ghost columns from the current W.
// f is stored velocity-major: one plane per discrete velocity, a padded nx x ny array with
// two halo columns and rows on each side (KParams).  A wavefront takes 64 consecutive cells
// of one row at one velocity, so every load is one coalesced row segment and the x
// neighbours of a cell come from the neighbouring lanes.  The wavefronts of a workgroup share
// one row segment (the update kernel: the same segment of two rows) and take one velocity
// quadrant each (the FP64 update kernel: two wavefronts per quadrant, one per velocity
// chunk): within a quadrant the upwind direction of both axes is uniform, so an x-face flux
// is evaluated once, by the lane of its upwind cell, and handed to the downwind lane.
// Two variants run through the same kernels: a gas with internal degrees of freedom, whose
// second reduced distribution H takes velocity chunks of its own (its planes follow those of
// G), and the Shakhov collision model, a separate instantiation of the moment and update
// kernels (heat sums; equilibria times (1 + S)).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>

#include "ugks_internal.hpp"

namespace ugks {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kQuads = 4;                     // wavefronts per workgroup, one per quadrant
constexpr int kTileS = kWave - 2;             // cells per moment-kernel wavefront
constexpr int kTileU = kWave - 2 * kHalo;     // cells per update-kernel wavefront
constexpr unsigned kDropOffset = 0xFFFFFFF0u;  // beyond any plane (at most 2^31 bytes)

// Quadrant q of a workgroup: sign of u and of v.  Around the cycle (+,+) (-,+) (-,-) (+,-)
// neighbours share one sign, so each face side collects its sums from two adjacent waves.
__device__ __forceinline__ int quad_su(int q) { return (q == 0 || q == 3) ? 1 : -1; }
__device__ __forceinline__ int quad_sv(int q) { return q < 2 ? 1 : -1; }

// ------------------------------------------------------------------ storage
template <typename T>
__device__ __forceinline__ T ldb(const UGKS_GLOBAL T* p, unsigned byte_off) {
  return *reinterpret_cast<const UGKS_GLOBAL T*>(reinterpret_cast<const UGKS_GLOBAL char*>(p) +
                                                 byte_off);
}
template <typename S>
__device__ __forceinline__ double ldv(const UGKS_GLOBAL S* plane, int idx) {
  return (double)ldb(plane, (unsigned)idx * (unsigned)sizeof(S));
}
template <typename S>
__device__ __forceinline__ void stv(UGKS_GLOBAL S* plane, int idx, double x) {
  *reinterpret_cast<UGKS_GLOBAL S*>(reinterpret_cast<UGKS_GLOBAL char*>(plane) +
                                    (unsigned)idx * (unsigned)sizeof(S)) = static_cast<S>(x);
}
template <typename S>
__device__ __forceinline__ const UGKS_GLOBAL S* plane_of(const UGKS_GLOBAL S* f, const KParams& P,
                                                         int p) {
  return f + (long long)p * P.PS;
}
template <typename S>
__device__ __forceinline__ UGKS_GLOBAL S* plane_of(UGKS_GLOBAL S* f, const KParams& P, int p) {
  return f + (long long)p * P.PS;
}
// Buffer resource of one plane (base, size in bytes): loads at a per-lane 32-bit byte offset
// from a scalar base, range-checked by the hardware.  The size field is an unsigned 32-bit
// count (a plane holds at most 2^28 values, so at most 2^31 bytes).  Word 3 selects 32-bit
// data for the untyped buffer instructions.
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const UGKS_GLOBAL S* plane,
                                                             const KParams& P) {
  const unsigned bytes = (unsigned)((unsigned long long)P.PS * sizeof(S));
  return __builtin_amdgcn_make_buffer_rsrc((void*)plane, (short)0, __builtin_bit_cast(int, bytes),
                                           0x00020000);
}
// Stores through the same resources; an offset past the plane's range is dropped by the
// hardware range check, so lanes without a cell to write need no branch.
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, double x, double) {
  typedef unsigned u2v __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, x), r, off, 0, 0);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, double x, float) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, (float)x), r, off, 0, 0);
}
// Loads through the same resources, in the storage type (converted where they are used).
__device__ __forceinline__ double bload_raw(__amdgpu_buffer_rsrc_t r, unsigned off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float bload_raw(__amdgpu_buffer_rsrc_t r, unsigned off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// index of cell (i, j) in a plane; i and j may lie in the halo
__device__ __forceinline__ int pidx(const KParams& P, int i, int j) {
  return (j + kHalo) * P.Lx + i + kHalo;
}

// ------------------------------------------------------------------ lane exchange
// Whole-wavefront DPP shifts by one lane: lane l receives the value lane l - 1 holds
// (from_lower) or lane l + 1 holds (from_upper); the edge lane, which has no source, reads 0
// (bound control), so no copy of an "old" value is needed.
__device__ __forceinline__ double dpp_shift(double x, int ctrl_lower) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)(unsigned)(b & 0xffffffffll), hi = (int)(b >> 32);
  int rlo, rhi;
  if (ctrl_lower) {
    rlo = __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true);  // wave_shr:1
    rhi = __builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true);
  } else {
    rlo = __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true);  // wave_shl:1
    rhi = __builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true);
  }
  return __longlong_as_double(((long long)rhi << 32) | (long long)(unsigned)rlo);
}
__device__ __forceinline__ double from_lower(double x) { return dpp_shift(x, 1); }
__device__ __forceinline__ double from_upper(double x) { return dpp_shift(x, 0); }
__device__ __forceinline__ float from_lower(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_upper(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x130, 0xf, 0xf, true));
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
// The same, forced to zero where `keep` is false (ghost columns, rows next to a wall): in the
// update kernel the mask joins the sign test instead of multiplying the result (one FP64
// multiply less per limiter; in the moment kernel the multiply measured faster).
__device__ __forceinline__ double half_limited(double p, double q, bool keep) {
  const double pq = p * q;
  const double r = pq * recip(p + q);
  return (pq > 0.0 && keep) ? r : 0.0;
}
// FP32 forms (the FP32-storage update): the hardware reciprocal is accurate to 1 ulp.
__device__ __forceinline__ float half_limited(float p, float q) {
  const float pq = p * q;
  const float r = pq * __builtin_amdgcn_rcpf(p + q);
  return pq > 0.0f ? r : 0.0f;
}
__device__ __forceinline__ float half_limited(float p, float q, bool keep) {
  const float pq = p * q;
  const float r = pq * __builtin_amdgcn_rcpf(p + q);
  return (pq > 0.0f && keep) ? r : 0.0f;
}
__device__ __forceinline__ float exp_of(float x) { return expf(x); }
__device__ __forceinline__ double exp_of(double x) { return exp(x); }
__device__ __forceinline__ float expm1_of(float x) { return expm1f(x); }
__device__ __forceinline__ double expm1_of(double x) { return expm1(x); }


struct Prim {
  double rho, U, V, lam;  // lambda = 1/T
};

// Primitive variables of W = (rho, rho U, rho V, rho E) of a 2D gas with dof internal degrees
// of freedom: rho E = rho (U^2 + V^2)/2 + (2 + dof) rho/(4 lambda), lam_c = (2 + dof)/4 (the
// paper's gas: dof = 0).  false on an invalid state.
template <typename Ptr>
__device__ __forceinline__ bool prim_of(Ptr W, Prim& p, double lam_c) {
  const double rho = W[0];
  const double U = W[1] / rho;
  const double V = W[2] / rho;
  const double e = W[3] - 0.5 * rho * (U * U + V * V);
  p.rho = rho;
  p.U = U;
  p.V = V;
  p.lam = lam_c * rho / e;
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

// Gaussian moments of the internal coordinates xi at lambda: x2 = <|xi|^2> = dof/(2 lambda),
// x4 = <|xi|^4> = dof (dof + 2)/(4 lambda^2).  They enter through psi_4 = (un^2 + ut^2 + |xi|^2)/2;
// kXi = false is the paper's gas, whose moments carry no xi terms.
struct Xi {
  double x2, x4;
};

// <un^a ut^b psi>, psi = (1, un, ut, psi_4)
template <bool kXi>
__device__ __forceinline__ void mpsi(const double* mu, const double* mv, int a, int b,
                                     const Xi& xi, double* o) {
  o[0] = mu[a] * mv[b];
  o[1] = mu[a + 1] * mv[b];
  o[2] = mu[a] * mv[b + 1];
  if constexpr (kXi)
    o[3] = 0.5 * (mu[a + 2] * mv[b] + mu[a] * mv[b + 2] + xi.x2 * (mu[a] * mv[b]));
  else
    o[3] = 0.5 * (mu[a + 2] * mv[b] + mu[a] * mv[b + 2]);
}

// <un^a ut^b psi (c . psi)>; the |xi|^2 of c_4 psi_4 brings <|xi|^2 un^a ut^b psi>
template <bool kXi>
__device__ __forceinline__ void mpsi_c(const double* mu, const double* mv, int a, int b,
                                       const Xi& xi, const double* c, double* o) {
  double t0[4], t1[4], t2[4], t3[4], t4[4];
  mpsi<kXi>(mu, mv, a, b, xi, t0);
  mpsi<kXi>(mu, mv, a + 1, b, xi, t1);
  mpsi<kXi>(mu, mv, a, b + 1, xi, t2);
  mpsi<kXi>(mu, mv, a + 2, b, xi, t3);
  mpsi<kXi>(mu, mv, a, b + 2, xi, t4);
  if constexpr (kXi) {
    const double m00 = mu[a] * mv[b];
    const double tx[4] = {xi.x2 * m00, xi.x2 * (mu[a + 1] * mv[b]), xi.x2 * (mu[a] * mv[b + 1]),
                          0.5 * (xi.x2 * (mu[a + 2] * mv[b] + mu[a] * mv[b + 2]) + xi.x4 * m00)};
#pragma unroll
    for (int q = 0; q < 4; ++q)
      o[q] = c[0] * t0[q] + c[1] * t1[q] + c[2] * t2[q] + 0.5 * c[3] * (t3[q] + t4[q] + tx[q]);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      o[q] = c[0] * t0[q] + c[1] * t1[q] + c[2] * t2[q] + 0.5 * c[3] * (t3[q] + t4[q]);
  }
}

// S4 micro slope: a such that the moments of rho g (a . psi) equal s (closed form, 2D gas with
// q_c = (2 + dof)/2 and a4_c = 4/(2 + dof); the paper's gas has 1 and 2).
__device__ __forceinline__ void micro_slope(const Prim& p, const double* s, double* a,
                                            double q_c, double a4_c) {
  const double q2 = p.U * p.U + p.V * p.V + q_c / p.lam;
  const double R2 = s[1] - p.U * s[0];
  const double R3 = s[2] - p.V * s[0];
  const double R4 = 2.0 * s[3] - q2 * s[0];
  a[3] = a4_c * p.lam * p.lam / p.rho * (R4 - 2.0 * p.U * R2 - 2.0 * p.V * R3);
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

// The step of the launch's step (parity = the f/W buffer it reads): fixed, or with the
// adaptive step cfl / rmax of the state W^n it starts from.
__device__ __forceinline__ double step_dt(const KParams& P, int parity) {
  if (!P.adaptive) return P.dt;
  return P.cfl / __longlong_as_double((long long)P.rmax[parity]);
}

// ------------------------------------------------------------------ addressing
__device__ __forceinline__ int wrap(int i, int n) { return ((i % n) + n) % n; }
__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Workgroups are handed to the 8 XCDs round-robin; renumber them so that each XCD works
// through one contiguous range (its own L2 then serves the rows its neighbours also read).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ------------------------------------------------------------------ wave reductions
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) x = fmax(x, __shfl_xor(x, h, kWave));
  return x;
}

// Node range of one half of a velocity axis.  Half s = +1 takes the nodes with positive
// velocity, s = -1 the negative ones; a node at exactly zero belongs to both halves when
// `share_zero` (moment sums, each visit with weight 1/2), else only to the positive half.
struct Half {
  int first, count, step;
};
__device__ __forceinline__ Half axis_half(int n, int s, bool share_zero) {
  const int odd = n & 1, mid = n >> 1;  // with n odd, node mid is zero
  Half h;
  if (s > 0) {
    h.first = mid;
    h.count = n - mid;
    h.step = 1;
  } else {
    h.first = mid - 1 + (share_zero ? odd : 0);
    h.count = h.first + 1;
    h.step = -1;
  }
  return h;
}

// Nodes [a0, a1) of a half's node sequence taken by velocity chunk g of G.
__device__ __forceinline__ void chunk_range(int count, int g, int G, int& a0, int& a1) {
  a0 = (int)((long long)g * count / G);
  a1 = (int)((long long)(g + 1) * count / G);
}

// Workgroup L of a cell kernel: row segment t (fastest), row j, velocity chunk g.  The
// workgroups an XCD runs at once then cover whole rows of a band of neighbouring rows, so the
// cache lines a segment shares with the next one, and the rows j +- 1, j +- 2 it reads, come
// from that XCD's L2.
__device__ __forceinline__ void cell_block(int L, int ny, int ntx, int& t, int& g, int& j) {
  t = L % ntx;
  const int r = L / ntx;
  j = r % ny;
  g = r / ny;
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
// Discrete Maxwellian of each cell's W (initial state), one thread per plane value; the
// planes of H hold dof/(2 lambda) times those of G.
template <typename S>
__global__ __launch_bounds__(256) void init_kernel(PlanView pv) {
  const Inst* __restrict__ I = inst_at(pv, 0);
  const KParams P = I->P;
  UGKS_GLOBAL S* f = static_cast<UGKS_GLOBAL S*>(I->f[I->cur]);
  const UGKS_GLOBAL double* W = I->W[I->cur];
  const long long nc = (long long)P.nx * P.ny;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc * P.NV * P.NC) return;
  const int p = (int)(e / nc);
  const int c = (int)(e - (long long)p * nc);
  const int j = c / P.nx, i = c - j * P.nx;
  Prim pr;
  if (!prim_of(W + 4 * (size_t)c, pr, P.lam_c) && p == 0) *P.flag = 1;
  const bool h = p >= P.NV;
  const int pg = h ? p - P.NV : p;
  const int k = pg / P.M, m = pg - k * P.M;
  const double du = P.uk[k] - pr.U, dv = P.vm[m] - pr.V;
  double g = pr.rho * pr.lam / kPi * exp(-pr.lam * (du * du + dv * dv));
  if (h) g *= (double)P.dof / (2.0 * pr.lam);
  stv(plane_of(f, P, p), pidx(P, i, j), g);
}

// Debug: quiet NaN in every cell value of the f and W buffers the next step writes (the
// halo is left as it is: the kernels read it, where a wall or ghost switch discards it).  A
// step that failed to write one of these values would leave a NaN in the state.
template <typename S>
__global__ __launch_bounds__(256) void poison_kernel(PlanView pv) {
  const Inst* __restrict__ I = inst_at(pv, 0);
  const KParams P = I->P;
  const int nxt = (I->cur + pv.step + 1) & 1;
  UGKS_GLOBAL S* f = static_cast<UGKS_GLOBAL S*>(I->f[nxt]);
  UGKS_GLOBAL double* W = I->W[nxt];
  const long long nc = (long long)P.nx * P.ny;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc * P.NV * P.NC) return;
  const int p = (int)(e / nc);
  const int c = (int)(e - (long long)p * nc);
  const int j = c / P.nx, i = c - j * P.nx;
  plane_of(f, P, p)[pidx(P, i, j)] = static_cast<S>(__builtin_nan(""));
  // a channel's ghost columns, which the update kernel writes into f^{n+1}
  if (P.bc == UGKS_BC_CHANNEL && (i == 0 || i == P.nx - 1))
    plane_of(f, P, p)[pidx(P, i == 0 ? -1 : P.nx, j)] = static_cast<S>(__builtin_nan(""));
  if (p == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) W[4 * (size_t)c + q] = __builtin_nan("");
  }
}

// Ghost state of row j of a channel (Sec. 3.A) from the primitive state pc of the cell next
// to it: the inlet (side 0) holds p_in and T_in (its velocity that of the cell, or the fixed
// inlet profile), the outlet (side 1) p_out with the cell's velocity and temperature.
__device__ __forceinline__ Prim ghost_prim(const KParams& P, int side, int j, const Prim& pc) {
  Prim pg;
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
  return pg;
}

// Ghost state W of a channel ghost cell, stored for the interface kernel.
__device__ __forceinline__ void store_wg(UGKS_GLOBAL double* wg, const Prim& pg, double lam_c) {
  wg[0] = pg.rho;
  wg[1] = pg.rho * pg.U;
  wg[2] = pg.rho * pg.V;
  wg[3] = 0.5 * pg.rho * (pg.U * pg.U + pg.V * pg.V) + lam_c * pg.rho / pg.lam;
}

// Halo of the current f of a periodic box (a step's first launch): one thread per halo value
// of every plane copies the periodic image.  A channel's halo is written by the update kernel
// (its ghost columns; the rest stays zero).
constexpr int kGhostThreads = 256;
template <typename S>
__global__ __launch_bounds__(kGhostThreads) void ghost_kernel(PlanView pv) {
  const int b = blockIdx.x;
  const int ii = find_inst(pv.off_ghost, pv.ninst, b);
  const Inst* __restrict__ I = inst_at(pv, ii);
  const KParams P = I->P;
  UGKS_GLOBAL S* f = static_cast<UGKS_GLOBAL S*>(I->f[(I->cur + pv.step) & 1]);
  const int local = b - first_block(pv.off_ghost, ii);
  const int tid = threadIdx.x;
  const long long frame = (long long)P.Lx * P.Ly - (long long)P.nx * P.ny;
  const long long e = (long long)local * kGhostThreads + tid;
  if (e >= frame * P.NV * P.NC) return;
  const int p = (int)(e / frame);
  int r = (int)(e - (long long)p * frame);
  // frame order: the 2 halo rows below, then ny rows of 4 halo columns, then 2 rows above
  int i, j;
  const int band = kHalo * P.Lx;
  if (r < band) {
    j = r / P.Lx - kHalo;
    i = r % P.Lx - kHalo;
  } else if (r < band + 2 * kHalo * P.ny) {
    r -= band;
    j = r / (2 * kHalo);
    const int c = r % (2 * kHalo);
    i = c < kHalo ? c - kHalo : P.nx + (c - kHalo);
  } else {
    r -= band + 2 * kHalo * P.ny;
    j = P.ny + r / P.Lx;
    i = r % P.Lx - kHalo;
  }
  UGKS_GLOBAL S* pl = plane_of(f, P, p);
  const double x = ldv(pl, pidx(P, wrap(i, P.nx), wrap(j, P.ny)));
  stv(pl, pidx(P, i, j), x);
}

// Per cell: slopes and the outgoing moment sums of all four faces.  A workgroup takes one
// segment of kTileS cells of one row (lanes hold the segment and one neighbour on each side);
// wavefront q sums velocity quadrant q into the x face and the y face its particles leave
// through.  Along one v line (u fixed) every sum is a combination of the running v moments
//   F^n = sum_m w_m v^n f,  X^n = sum_m w_m v^n hx,  Y^n = sum_m w_m v^n hy
// (hx, hy: half-cell changes; n up to 3, 3 and 4), with f_hat = f + s hx (or s hy) and
// D = (2u/dx) hx + (2v/dy) hy; the 32 face sums take them in once per line.  The two partial
// sums of each face side meet in LDS at the end.  With internal degrees of freedom the
// chunks G..2G-1 of a segment walk the planes of H, whose psi is (0, 0, 0, 1/2): they add to
// the energy sums only.  The Shakhov instantiation (kShak) also sums, per face side, ut c2h
// of the reconstruction (c2h = (un^2 + ut^2)/2) and, per cell, eight raw moments of f for
// the heat fluxes.
template <typename S, bool kShak>
__global__ __launch_bounds__(kWave* kQuads) void sums_kernel(PlanView pv) {
  constexpr int kR = kShak ? 17 : 16;
  __shared__ double red[4][kR][kWave];
  __shared__ double cellred[kShak ? 3 : 1][8][kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int ii = find_inst(pv.off_sums, pv.ninst, b);
  const Inst* __restrict__ I = inst_at(pv, ii);
  const KParams P = I->P;
  const int G = I->gsplit;
  int t, gg, j;
  cell_block(b - first_block(pv.off_sums, ii), P.ny, (P.nx + kTileS - 1) / kTileS, t, gg, j);
  const bool hpart = gg >= G;  // planes of H
  const int g = hpart ? gg - G : gg;
  const UGKS_GLOBAL S* f = static_cast<const UGKS_GLOBAL S*>(I->f[(I->cur + pv.step) & 1]) +
                           (hpart ? (long long)P.NV * P.PS : 0ll);
  UGKS_GLOBAL double* hs = I->hs + (size_t)gg * P.nslot * ((size_t)P.nx * P.ny);
  const int i = t * kTileS - 1 + lane;
  const bool valid = lane >= 1 && lane <= kTileS && i < P.nx;
  // channel ghost columns (i = -1, nx): their sums towards the domain are the ghost sums of
  // the inlet and outlet faces (zero slopes); only the first and last segments hold them
  const bool chan = P.bc == UGKS_BC_CHANNEL;
  const bool ghost = chan && (i == -1 || i == P.nx);
  const bool ghost_wave = chan && (t == 0 || (t + 1) * kTileS >= P.nx);
  const int o = pidx(P, i < P.nx + 1 ? i : P.nx + 1, j);
  const unsigned bs = (unsigned)sizeof(S);
  const unsigned oc = (unsigned)o * bs, oS = (unsigned)(o - P.Lx) * bs;
  const unsigned oN = (unsigned)(o + P.Lx) * bs;
  const double my = (P.bc == UGKS_BC_CHANNEL && (j == 0 || j == P.ny - 1)) ? 0.0 : 1.0;
  const int su = quad_su(q), sv = quad_sv(q);
  // each half is walked inwards, towards v = 0 and u = 0: the update kernel walks it
  // outwards, so each kernel starts on the planes the other touched last
  const Half hu0 = axis_half(P.K, su, true), hv0 = axis_half(P.M, sv, true);
  const Half hu = {hu0.first + (hu0.count - 1) * hu0.step, hu0.count, -hu0.step};
  const Half hv = {hv0.first + (hv0.count - 1) * hv0.step, hv0.count, -hv0.step};
  const double two_idx = 2.0 * P.inv_dx, two_idy = 2.0 * P.inv_dy;
  double ax[kR], ay[kR];
#pragma unroll
  for (int r = 0; r < kR; ++r) ax[r] = ay[r] = 0.0;
  // raw cell moments (kShak): f, u f, v f, u^2 f, u v f, v^2 f, u |c|^2 f, v |c|^2 f
  double cm[kShak ? 8 : 1];
#pragma unroll
  for (int r = 0; r < (kShak ? 8 : 1); ++r) cm[r] = 0.0;
  int a0, a1;
  chunk_range(hu.count, g, G, a0, a1);
  for (int a = a0; a < a1; ++a) {
    const int k = hu.first + a * hu.step;
    const double u = P.uk[k];
    const double wu = P.wk[k] * (u == 0.0 ? 0.5 : 1.0);
    const UGKS_GLOBAL S* line = plane_of(f, P, k * P.M);
    double F0 = 0, F1 = 0, F2 = 0, F3 = 0, X0 = 0, X1 = 0, X2 = 0, X3 = 0;
    double Y0 = 0, Y1 = 0, Y2 = 0, Y3 = 0, Y4 = 0;
    struct Vals {
      S c, s, n;  // in the storage type
    };
    // planes and weight rows are walked with running pointers: one add per node each
    const long long pstep = (long long)hv.step * P.PS;
    const UGKS_GLOBAL S* pcur = line + (long long)hv.first * P.PS;
    const UGKS_CONST double* wp = (const UGKS_CONST double*)(P.vmom + 5 * hv.first);
    // FP64: each node's weights are requested one node ahead, as scalar loads (one node
    // beyond the last node of a half lies in the other half)
    double w0 = wp[0], w1 = wp[1], w2 = wp[2], w3 = wp[3], w4 = wp[4];
    const int wstep = 5 * hv.step;
    auto load_at = [&](const UGKS_GLOBAL S* p) {
      const __amdgpu_buffer_rsrc_t r = plane_rsrc(p, P);
      return Vals{bload_raw(r, oc, S{}), bload_raw(r, oS, S{}), bload_raw(r, oN, S{})};
    };
    auto node = [&](const Vals& x) {
      // w_m v_m^n, n = 0..4, with the weight 1/2 of a node at v = 0 (visited by both halves)
      double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0, n4 = 0.0;
      if constexpr (sizeof(S) == 8) {
        n0 = wp[wstep];
        n1 = wp[wstep + 1];
        n2 = wp[wstep + 2];
        n3 = wp[wstep + 3];
        n4 = wp[wstep + 4];
      } else {  // FP32 storage: read at the node (holding the next node's weights would cost
                // this kernel its fourth wave per SIMD)
        w0 = wp[0];
        w1 = wp[1];
        w2 = wp[2];
        w3 = wp[3];
        w4 = wp[4];
      }
      // slopes in the storage type (FP32 storage: FP32 slopes), sums in FP64
      const S fW = from_lower(x.c), fE = from_upper(x.c);
      const double hx = half_limited(fE - x.c, x.c - fW);
      const double hy = my * (double)half_limited(x.n - x.c, x.c - x.s);
      const double fc = x.c;
      F0 = fma(fc, w0, F0);
      F1 = fma(fc, w1, F1);
      F2 = fma(fc, w2, F2);
      F3 = fma(fc, w3, F3);
      X0 = fma(hx, w0, X0);
      X1 = fma(hx, w1, X1);
      X2 = fma(hx, w2, X2);
      X3 = fma(hx, w3, X3);
      Y0 = fma(hy, w0, Y0);
      Y1 = fma(hy, w1, Y1);
      Y2 = fma(hy, w2, Y2);
      Y3 = fma(hy, w3, Y3);
      Y4 = fma(hy, w4, Y4);
      wp += wstep;
      if constexpr (sizeof(S) == 8) {
        w0 = n0;
        w1 = n1;
        w2 = n2;
        w3 = n3;
        w4 = n4;
      }
    };
    if constexpr (sizeof(S) == 8) {
      // FP64: two value sets, each node's loads issued one node ahead (deeper prefetch costs
      // this kernel its fourth wave per SIMD)
      Vals va = load_at(pcur);
      int c = 0;
      for (; c + 1 < hv.count; c += 2) {
        pcur += pstep;
        const Vals vb = load_at(pcur);
        node(va);
        if (c + 2 < hv.count) pcur += pstep;
        va = load_at(pcur);
        node(vb);
      }
      if (c < hv.count) node(va);
    } else {
      // FP32 storage: a row load brings half the bytes, so each node's loads are issued six
      // nodes ahead (kSA + 1 value sets in a ring; 3 and 4 ahead measured 6% and 2% slower at
      // 400 x 100 x 40^2); past the last node of the half the loads read its plane again
      constexpr int kSA = 6, NB = kSA + 1;
      int nl = 0;
      auto load_next = [&]() {
        const Vals v = load_at(pcur);
        if (++nl < hv.count) pcur += pstep;
        return v;
      };
      Vals ring[NB];
#pragma unroll
      for (int d = 0; d < kSA; ++d) ring[d] = load_next();
      int c = 0;
      for (; c + NB <= hv.count; c += NB) {
#pragma unroll
        for (int s = 0; s < NB; ++s) {
          ring[(s + kSA) % NB] = load_next();
          node(ring[s]);
        }
      }
#pragma unroll
      for (int s = 0; s < NB; ++s) {
        if (c + s < hv.count) {
          ring[(s + kSA) % NB] = load_next();
          node(ring[s]);
        }
      }
    }
    if (ghost_wave && ghost) {  // a ghost cell has zero slopes
      X0 = X1 = X2 = X3 = 0.0;
      Y0 = Y1 = Y2 = Y3 = Y4 = 0.0;
    }
    // moments of the x-face reconstruction (S), the y-face one (R) and of D
    const double ucx = u * two_idx, u2h = 0.5 * u * u, wuu = wu * u;
    if (hpart) {
      const double wh = 0.5 * wu, whu = 0.5 * wuu;
      const double S0 = su > 0 ? F0 + X0 : F0 - X0;
      const double R0 = sv > 0 ? F0 + Y0 : F0 - Y0, R1 = sv > 0 ? F1 + Y1 : F1 - Y1;
      const double D0 = fma(ucx, X0, two_idy * Y1), D1 = fma(ucx, X1, two_idy * Y2);
      ax[3] = fma(wh, S0, ax[3]);
      ax[7] = fma(wh, Y0, ax[7]);
      ax[11] = fma(whu, S0, ax[11]);
      ax[15] = fma(whu, D0, ax[15]);
      ay[3] = fma(wh, R0, ay[3]);
      ay[7] = fma(wh, X0, ay[7]);
      ay[11] = fma(wh, R1, ay[11]);
      ay[15] = fma(wh, D1, ay[15]);
      continue;
    }
    const double S0 = su > 0 ? F0 + X0 : F0 - X0, S1 = su > 0 ? F1 + X1 : F1 - X1;
    const double S2 = su > 0 ? F2 + X2 : F2 - X2;
    const double R0 = sv > 0 ? F0 + Y0 : F0 - Y0, R1 = sv > 0 ? F1 + Y1 : F1 - Y1;
    const double R2 = sv > 0 ? F2 + Y2 : F2 - Y2, R3 = sv > 0 ? F3 + Y3 : F3 - Y3;
    const double D0 = fma(ucx, X0, two_idy * Y1), D1 = fma(ucx, X1, two_idy * Y2);
    const double D2 = fma(ucx, X2, two_idy * Y3), D3 = fma(ucx, X3, two_idy * Y4);
    // x face: psi = (1, u, v, c2h), c2h = (u^2 + v^2)/2
    const double cS = fma(u2h, S0, 0.5 * S2), cT = fma(u2h, Y0, 0.5 * Y2);
    const double cD = fma(u2h, D0, 0.5 * D2);
    ax[0] = fma(wu, S0, ax[0]);
    ax[1] = fma(wuu, S0, ax[1]);
    ax[2] = fma(wu, S1, ax[2]);
    ax[3] = fma(wu, cS, ax[3]);
    ax[4] = fma(wu, Y0, ax[4]);
    ax[5] = fma(wuu, Y0, ax[5]);
    ax[6] = fma(wu, Y1, ax[6]);
    ax[7] = fma(wu, cT, ax[7]);
    ax[8] = fma(wuu, S0, ax[8]);
    ax[9] = fma(wuu * u, S0, ax[9]);
    ax[10] = fma(wuu, S1, ax[10]);
    ax[11] = fma(wuu, cS, ax[11]);
    ax[12] = fma(wuu, D0, ax[12]);
    ax[13] = fma(wuu * u, D0, ax[13]);
    ax[14] = fma(wuu, D1, ax[14]);
    ax[15] = fma(wuu, cD, ax[15]);
    // y face: psi = (1, v, u, c2h)
    const double cR = fma(u2h, R0, 0.5 * R2), cX = fma(u2h, X0, 0.5 * X2);
    const double cR1 = fma(u2h, R1, 0.5 * R3), cD1 = fma(u2h, D1, 0.5 * D3);
    ay[0] = fma(wu, R0, ay[0]);
    ay[1] = fma(wu, R1, ay[1]);
    ay[2] = fma(wuu, R0, ay[2]);
    ay[3] = fma(wu, cR, ay[3]);
    ay[4] = fma(wu, X0, ay[4]);
    ay[5] = fma(wu, X1, ay[5]);
    ay[6] = fma(wuu, X0, ay[6]);
    ay[7] = fma(wu, cX, ay[7]);
    ay[8] = fma(wu, R1, ay[8]);
    ay[9] = fma(wu, R2, ay[9]);
    ay[10] = fma(wuu, R1, ay[10]);
    ay[11] = fma(wu, cR1, ay[11]);
    ay[12] = fma(wu, D1, ay[12]);
    ay[13] = fma(wu, D2, ay[13]);
    ay[14] = fma(wuu, D1, ay[14]);
    ay[15] = fma(wu, cD1, ay[15]);
    if constexpr (kShak) {
      const double S3 = su > 0 ? F3 + X3 : F3 - X3;
      ax[16] = fma(wu, fma(u2h, S1, 0.5 * S3), ax[16]);
      ay[16] = fma(wuu, cR, ay[16]);
      const double wu2 = wuu * u;
      cm[0] = fma(wu, F0, cm[0]);
      cm[1] = fma(wuu, F0, cm[1]);
      cm[2] = fma(wu, F1, cm[2]);
      cm[3] = fma(wu2, F0, cm[3]);
      cm[4] = fma(wuu, F1, cm[4]);
      cm[5] = fma(wu, F2, cm[5]);
      cm[6] = fma(wuu, fma(u * u, F0, F2), cm[6]);
      cm[7] = fma(wu, fma(u * u, F1, F3), cm[7]);
    }
  }
  // x faces: (+) from waves 0 and 3, (-) from 1 and 2; y faces: (+) from 0 and 1, (-) from
  // 2 and 3.  Waves 1 and 3 hand their sums over, waves 0 and 2 add and write.
  if (q == 1 || q == 3) {
    const int s = q == 1 ? 0 : 1;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      red[s][r][lane] = ay[r];
      red[2 + s][r][lane] = ax[r];
    }
  }
  if constexpr (kShak) {
    // every quadrant holds part of each cell's moments; wavefront 0 adds them
    if (q > 0) {
#pragma unroll
      for (int r = 0; r < 8; ++r) cellred[q - 1][r][lane] = cm[r];
    }
  }
  __syncthreads();
  const size_t nc = (size_t)P.nx * P.ny;
  // the inlet ghost's sums towards +x (waves 0 and 3), the outlet ghost's towards -x (waves
  // 1 and 2): this chunk's part, added over the chunks by the interface kernel
  if (ghost_wave && ghost && q == (i < 0 ? 0 : 2)) {
    const int ox = q == 0 ? 3 : 2, side = i < 0 ? 0 : 1;
    UGKS_GLOBAL double* gs = I->hsg + (((size_t)gg * 2 + side) * P.ny + j) * kGhostSums;
#pragma unroll
    for (int r = 0; r < kR; ++r) gs[r] = ax[r] + red[ox][r][lane];
    if constexpr (kR < kGhostSums) gs[kGhostSums - 1] = 0.0;  // no heat sum without Shakhov
  }
  if (valid && (q == 0 || q == 2)) {
    const size_t cell = (size_t)j * P.nx + i;
    const int fy = q == 0 ? S_YP : S_YM, fx = q == 0 ? S_XP : S_XM;
    const int oy = q == 0 ? 0 : 1, ox = q == 0 ? 3 : 2;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const double sx = (ax[r] + red[ox][r][lane]) * (r >= 4 && r < 8 ? two_idy : 1.0);
      const double sy = (ay[r] + red[oy][r][lane]) * (r >= 4 && r < 8 ? two_idx : 1.0);
      hs[(size_t)(16 * fx + r) * nc + cell] = sx;
      hs[(size_t)(16 * fy + r) * nc + cell] = sy;
    }
    if constexpr (kShak) {
      hs[(size_t)(kSlotHeat + fx) * nc + cell] = ax[16] + red[ox][16][lane];
      hs[(size_t)(kSlotHeat + fy) * nc + cell] = ay[16] + red[oy][16][lane];
      if (q == 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
          hs[(size_t)(kSlotCell + r) * nc + cell] =
              ((cm[r] + cellred[0][r][lane]) + cellred[1][r][lane]) + cellred[2][r][lane];
      }
    }
  }
}

// With several velocity chunks per quadrant, or the chunks of H, the moment kernel leaves
// NC G partial sums per value; one thread per (sum, cell) adds them, in chunk order, into the
// first.
__global__ __launch_bounds__(256) void chunk_sum_kernel(PlanView pv) {
  const int b = blockIdx.x;
  const int ii = find_inst(pv.off_red, pv.ninst, b);
  const Inst* __restrict__ I = inst_at(pv, ii);
  const KParams P = I->P;
  const size_t nc = (size_t)P.nx * P.ny;
  size_t e = (size_t)(b - first_block(pv.off_red, ii)) * blockDim.x + threadIdx.x;
  UGKS_GLOBAL double* at;
  size_t gstride;
  if (e < (size_t)P.nslot * nc) {
    at = I->hs + e;
    gstride = (size_t)P.nslot * nc;
  } else {
    // a channel's ghost sums (2 ny rows of kGhostSums per chunk)
    e -= (size_t)P.nslot * nc;
    gstride = 2 * (size_t)P.ny * kGhostSums;
    if (P.bc != UGKS_BC_CHANNEL || e >= gstride) return;
    at = I->hsg + e;
  }
  // the chunks are added in chunk order; their loads go out eight at a time (a load per
  // loop trip would wait out one memory latency per chunk)
  const int n = I->gsplit * P.NC;
  double x = at[0];
  for (int g0 = 1; g0 < n; g0 += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = g0 + k < n ? at[(size_t)(g0 + k) * gstride] : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (g0 + k < n) x += v[k];
  }
  at[0] = x;
}

// S2-S5 at one interior interface, local frame.  S = [W0, Wt, Q1, Q2].  Writes the local
// macroscopic flux to F and the folded coefficients of the distribution flux to rec; with
// internal degrees of freedom (kXi) also those of H to recH.  Averaged over xi, the energy
// term c_4 psi_4 of a slope c contributes c_4 (un^2 + ut^2 + s)/2 to the polynomial of G with
// s = <|xi|^2> = x2, and to that of H, whose Maxwellian is x2 times that of G, with
// s = <|xi|^4>/<|xi|^2> = x4/x2: the constant shifts e0, e1 and e2 by c_4 s/2.
// Heat flux q = sum w c |c|^2 f / 2 about (U, V) from raw sums of f: m0 = sum f, mn = sum un f,
// mt = sum ut f, mnn, mnt, mtt = sum un^2 f, un ut f, ut^2 f, Kn = sum un |c|^2 f,
// Kt = sum ut |c|^2 f, K0 = sum |c|^2 f (|c|^2 = un^2 + ut^2).
__device__ __forceinline__ void heat_flux(double m0, double mn, double mt, double mnn,
                                          double mnt, double mtt, double Kn, double Kt,
                                          double K0, double U, double V, double* q) {
  const double UV2 = U * U + V * V;
  const double c2 = K0 - 2.0 * (U * mn + V * mt) + UV2 * m0;  // sum |u - U|^2 f
  q[0] = 0.5 * (Kn - 2.0 * (U * mnn + V * mnt) + UV2 * mn - U * c2);
  q[1] = 0.5 * (Kt - 2.0 * (U * mnt + V * mtt) + UV2 * mt - V * c2);
}

// Shakhov term of an interface: g0 S0 held over the step adds Mt1 g0 S0 to the distribution
// flux, S0 = k (c . q)(2 lambda |c|^2 - 4), k = (1 - Pr) lambda^2/rho, c = (un - U, ut - V);
// expanded in the record's basis {1, un, ut, c2h, un^2, un ut, ut^2, un c2h, ut c2h} it adds
// to every coefficient of both upwind sides.
// Face records are stored field-major: field f of face e of a family of nf faces (the x faces,
// or the y faces) at f nf + e, so that a wavefront's 64 neighbouring faces read or write one
// field as one contiguous access.  RecRef is one face's record in that layout.
struct RecRef {
  UGKS_GLOBAL double* p;  // field 0 of the face
  size_t nf;              // faces of the family: the stride between fields
  __device__ __forceinline__ UGKS_GLOBAL double& operator[](int f) const {
    return p[(size_t)f * nf];
  }
};

__device__ __forceinline__ void fold_shakhov(RecRef rec, const Prim& p0,
                                             const double* q, double km) {
  const double lam = p0.lam, U = p0.U, V = p0.V;
  const double Q0 = q[0] * U + q[1] * V;
  const double C0 = 2.0 * lam * (U * U + V * V) - 4.0;
  const double l4 = 4.0 * lam;
  const double d[9] = {-C0 * Q0,          l4 * U * Q0 + C0 * q[0], l4 * V * Q0 + C0 * q[1],
                       -l4 * Q0,          -l4 * U * q[0],          -l4 * (V * q[0] + U * q[1]),
                       -l4 * V * q[1],    l4 * q[0],               l4 * q[1]};
#pragma unroll
  for (int n = 0; n < 9; ++n) rec[R_E + n] = fma(km, d[n], rec[R_E + n]);
  rec[R_ER + 0] = fma(km, d[1], rec[R_ER + 0]);
  rec[R_ER + 1] = fma(km, d[4], rec[R_ER + 1]);
  rec[R_ER + 2] = fma(km, d[5], rec[R_ER + 2]);
  rec[R_ER + 3] = fma(km, d[7], rec[R_ER + 3]);
}

template <bool kXi>
__device__ void interface_scalars(const KParams& P, double dt, const double* S, const double* WL,
                                  const double* WR, double dn, double len, double* F,
                                  RecRef rec, RecRef recH,
                                  double& U0, double& V0, double T3 = 0.0) {
  const double* W0 = S;
  const double* Wt = S + 4;
  const double* Q1 = S + 8;
  const double* Q2 = S + 12;
  if (P.collisionless) {
    const double Mt4 = dt, Mt5 = 0.5 * dt * dt;
#pragma unroll
    for (int q = 0; q < 4; ++q) F[q] = len * (Mt4 * Q1[q] - Mt5 * Q2[q]);
#pragma unroll
    for (int q = 0; q < 13; ++q) rec[R_E + q] = 0.0;
    rec[R_GC] = 0.0;
    rec[R_LAM] = 0.0;
    rec[R_M4] = len * Mt4;
    rec[R_M5] = len * Mt5;
    rec[R_KIND] = K_FREE;
    if constexpr (kXi) {
#pragma unroll
      for (int q = R_GC; q < kRec; ++q) recH[q] = rec[q];
    }
    U0 = V0 = 0.0;
    return;
  }
  Prim p0;
  if (!prim_of(W0, p0, P.lam_c)) *P.flag = 1;
  Xi xi{0.0, 0.0};
  if constexpr (kXi) {
    xi.x2 = (double)P.dof / (2.0 * p0.lam);
    xi.x4 = (double)(P.dof * (P.dof + 2)) / (4.0 * p0.lam * p0.lam);
  }
  const double tau0 = collision_time(p0, P.mu_ref);
  double Mt[5];
  time_weights(dt, tau0, Mt);
  double swL[4], swR[4], aL[4], aR[4], b[4], A[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    swL[q] = (W0[q] - WL[q]) / (0.5 * dn);
    swR[q] = (WR[q] - W0[q]) / (0.5 * dn);
  }
  micro_slope(p0, swL, aL, P.q_c, P.a4_c);
  micro_slope(p0, swR, aR, P.q_c, P.a4_c);
  micro_slope(p0, Wt, b, P.q_c, P.a4_c);
  double mu[7], mp[7], mn[7], mv[7], tp[7], tn[7];
  axis_moments(p0.U, p0.lam, mu, mp, mn);
  axis_moments(p0.V, p0.lam, mv, tp, tn);
  double m1[4], m2[4], m3[4], sA[4];
  mpsi_c<kXi>(mp, mv, 1, 0, xi, aL, m1);
  mpsi_c<kXi>(mn, mv, 1, 0, xi, aR, m2);
  mpsi_c<kXi>(mu, mv, 0, 1, xi, b, m3);
#pragma unroll
  for (int q = 0; q < 4; ++q) sA[q] = -p0.rho * (m1[q] + m2[q] + m3[q]);
  micro_slope(p0, sA, A, P.q_c, P.a4_c);
  double e0[4], eL[4], eR[4], eb[4], eA[4];
  mpsi<kXi>(mu, mv, 1, 0, xi, e0);
  mpsi_c<kXi>(mp, mv, 2, 0, xi, aL, eL);
  mpsi_c<kXi>(mn, mv, 2, 0, xi, aR, eR);
  mpsi_c<kXi>(mu, mv, 1, 1, xi, b, eb);
  mpsi_c<kXi>(mu, mv, 1, 0, xi, A, eA);
  // Shakhov: heat flux of the reconstruction at the interface (local frame); T3 is the sum of
  // ut c2h f_hat, the other raw sums are W0 and Q1
  double qh[2] = {0.0, 0.0};
  if (P.shak)
    heat_flux(W0[0], W0[1], W0[2], Q1[1], Q1[2], 2.0 * W0[3] - Q1[1], 2.0 * Q1[3], 2.0 * T3,
              2.0 * W0[3], p0.U, p0.V, qh);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double feq = p0.rho * (Mt[0] * e0[q] + Mt[1] * (eL[q] + eR[q] + eb[q]) + Mt[2] * eA[q]);
    if (q == 3 && P.shak) feq = fma(Mt[0] * P.pr_c, qh[0], feq);
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
  if (P.shak) fold_shakhov(rec, p0, qh, Mt[0] * P.pr_c * p0.lam * p0.lam / p0.rho);
  rec[R_GC] = len * p0.rho * p0.lam / kPi;
  rec[R_LAM] = p0.lam;
  rec[R_M4] = len * Mt[3];
  rec[R_M5] = len * Mt[4];
  rec[R_KIND] = K_INTERIOR;
  if constexpr (kXi) {
#pragma unroll
    for (int q = R_GC; q < kRec; ++q) recH[q] = rec[q];
    recH[R_GC] = rec[R_GC] * xi.x2;
    const double sh = 0.5 * xi.x4 / xi.x2, sg = 0.5 * xi.x2;
    const double e3 = rec[R_E + 3], e7 = rec[R_E + 7], e8 = rec[R_E + 8];
    const double e7r = rec[R_ER + 3];
    recH[R_E + 0] = fma(sh, e3, rec[R_E + 0]);
    recH[R_E + 1] = fma(sh, e7, rec[R_E + 1]);
    recH[R_E + 2] = fma(sh, e8, rec[R_E + 2]);
    recH[R_ER + 0] = fma(sh, e7r, rec[R_ER + 0]);
    rec[R_E + 0] = fma(sg, e3, rec[R_E + 0]);
    rec[R_E + 1] = fma(sg, e7, rec[R_E + 1]);
    rec[R_E + 2] = fma(sg, e8, rec[R_E + 2]);
    rec[R_ER + 0] = fma(sg, e7r, rec[R_ER + 0]);
  }
  U0 = p0.U;
  V0 = p0.V;
}

// One thread per interface: x-faces first (ny rows of nx+1), then y-faces (ny+1 rows of nx).
// With internal degrees of freedom each face also gets the record of H, nfx (nfy) records
// after those of G; it repeats the macroscopic flux, so either record serves Eq. (4).
__global__ __launch_bounds__(256) void faces_kernel(PlanView pv) {
  const int b = blockIdx.x;
  const int ii = find_inst(pv.off_face, pv.ninst, b);
  const Inst* __restrict__ I = inst_at(pv, ii);
  const KParams P = I->P;
  const UGKS_GLOBAL double* hs = I->hs;
  const UGKS_GLOBAL double* hsg = I->hsg;
  const UGKS_GLOBAL double* W = I->W[(I->cur + pv.step) & 1];
  const double dt = step_dt(P, (I->cur + pv.step) & 1);
  const UGKS_GLOBAL double* Wg = I->Wg;
  UGKS_GLOBAL double* recx = I->recx;
  UGKS_GLOBAL double* recy = I->recy;
  const long e = (long)(b - first_block(pv.off_face, ii)) * blockDim.x + threadIdx.x;
  // the update kernel of this step takes the max rate of W^{n+1} into the other slot
  if (e == 0) P.rmax[((I->cur + pv.step) & 1) ^ 1] = 0ull;
  const long nfx = (long)P.ny * (P.nx + 1);
  const long nfy = (long)(P.ny + 1) * P.nx;
  const bool chan = P.bc == UGKS_BC_CHANNEL;
  const size_t nc = (size_t)P.nx * P.ny;
  double S[16], F[4];
  double U0, V0, T3 = 0.0;
  if (e < nfx) {
    const int j = (int)(e / (P.nx + 1)), i = (int)(e % (P.nx + 1));
    // a channel's ghost side: the ghost sums the moment kernel left (the chunk-sum kernel has
    // added the parts of the velocity chunks into the first)
    const bool gL = chan && i == 0, gR = chan && i == P.nx;
    const size_t cl = (size_t)j * P.nx + wrap(i - 1, P.nx);
    const size_t cr = (size_t)j * P.nx + wrap(i, P.nx);
    const UGKS_GLOBAL double* sL = gL ? hsg + (size_t)j * kGhostSums : hs + 16 * S_XP * nc + cl;
    const UGKS_GLOBAL double* sR =
        gR ? hsg + ((size_t)P.ny + j) * kGhostSums : hs + 16 * S_XM * nc + cr;
    const size_t stL = gL ? 1 : nc, stR = gR ? 1 : nc;
    const UGKS_GLOBAL double* WL = gL ? Wg + 4 * (size_t)j : W + 4 * cl;
    const UGKS_GLOBAL double* WR = gR ? Wg + 4 * ((size_t)P.ny + j) : W + 4 * cr;
#pragma unroll
    for (int q = 0; q < 16; ++q) S[q] = sL[q * stL] + sR[q * stR];
    if (P.shak)  // the heat sums of the two sides
      T3 = (gL ? sL[16] : hs[(kSlotHeat + S_XP) * nc + cl]) +
           (gR ? sR[16] : hs[(kSlotHeat + S_XM) * nc + cr]);
    double wl[4], wr[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wl[q] = WL[q];
      wr[q] = WR[q];
    }
    const RecRef rec{recx + e, (size_t)nfx};
    const RecRef recH{recx + (size_t)nfx * kRec + e, (size_t)nfx};
    if (P.NC > 1)
      interface_scalars<true>(P, dt, S, wl, wr, P.dx, P.dy, F, rec, recH, U0, V0);
    else
      interface_scalars<false>(P, dt, S, wl, wr, P.dx, P.dy, F, rec, recH, U0, V0, T3);
    for (int c = 0; c < P.NC; ++c) {
      const RecRef r = c ? recH : rec;
#pragma unroll
      for (int q = 0; q < 4; ++q) r[R_FX + q] = F[q];
      r[R_UX] = U0;
      r[R_VY] = V0;
    }
    return;
  }
  if (e >= nfx + nfy) return;
  const long e2 = e - nfx;
  const int j = (int)(e2 / P.nx), i = (int)(e2 % P.nx);
  const RecRef rec{recy + e2, (size_t)nfy};
  const RecRef recH{recy + (size_t)nfy * kRec + e2, (size_t)nfy};
  if (chan && (j == 0 || j == P.ny)) {
    // diffuse wall: sums of the wall-row cell towards the wall; local frame (v, u)
    const bool top = j == P.ny;
    const size_t c = (size_t)(top ? P.ny - 1 : 0) * P.nx + i;
    const UGKS_GLOBAL double* Q1s = hs + (16 * (top ? S_YP : S_YM) + 8) * nc + c;
    const double Q1[4] = {Q1s[0], Q1s[nc], Q1s[2 * nc], Q1s[3 * nc]};
    const double den = top ? P.wall_den_top : P.wall_den_bot;
    const double* Gw = top ? P.wall_G_top : P.wall_G_bot;
    const double rho_w = -Q1[0] / den;
    const double s = P.dx * dt;
    double Fl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) Fl[q] = s * (Q1[q] + rho_w * Gw[q]);
    // H leaves the wall with kap_w times the Maxwellian of G
    for (int c = 0; c < P.NC; ++c) {
      const RecRef r = c ? recH : rec;
      r[R_FX + 0] = Fl[0];
      r[R_FX + 1] = Fl[2];
      r[R_FX + 2] = Fl[1];
      r[R_FX + 3] = Fl[3];
      r[R_GC] = s * rho_w * P.lam_w / kPi * (c ? P.kap_w : 1.0);
      r[R_LAM] = P.lam_w;
      r[R_UX] = 0.0;
      r[R_VY] = 0.0;
      r[R_M4] = s;
      r[R_M5] = 0.0;
      r[R_KIND] = K_WALL;
#pragma unroll
      for (int q = 0; q < 13; ++q) r[R_E + q] = 0.0;  // a wall carries no polynomial
    }
    if (!(rho_w > 0.0) || !isfinite(rho_w)) *P.flag = 1;
    return;
  }
  const size_t cl = (size_t)wrap(j - 1, P.ny) * P.nx + i;
  const size_t cr = (size_t)wrap(j, P.ny) * P.nx + i;
  const UGKS_GLOBAL double* sL = hs + 16 * S_YP * nc + cl;
  const UGKS_GLOBAL double* sR = hs + 16 * S_YM * nc + cr;
#pragma unroll
  for (int q = 0; q < 16; ++q) S[q] = sL[q * nc] + sR[q * nc];
  if (P.shak) T3 = hs[(kSlotHeat + S_YP) * nc + cl] + hs[(kSlotHeat + S_YM) * nc + cr];
  const double wl[4] = {W[4 * cl], W[4 * cl + 2], W[4 * cl + 1], W[4 * cl + 3]};
  const double wr[4] = {W[4 * cr], W[4 * cr + 2], W[4 * cr + 1], W[4 * cr + 3]};
  if (P.NC > 1)
    interface_scalars<true>(P, dt, S, wl, wr, P.dy, P.dx, F, rec, recH, U0, V0);
  else
    interface_scalars<false>(P, dt, S, wl, wr, P.dy, P.dx, F, rec, recH, U0, V0, T3);
  for (int c = 0; c < P.NC; ++c) {
    const RecRef r = c ? recH : rec;
    r[R_FX + 0] = F[0];
    r[R_FX + 1] = F[2];
    r[R_FX + 2] = F[1];
    r[R_FX + 3] = F[3];
    r[R_UX] = V0;  // local (normal, tangential) = global (y, x)
    r[R_VY] = U0;
  }
}

// ------------------------------------------------------------------ update kernel
// A workgroup takes one segment of kTileU cells of two neighbouring rows, jb and jb + 1; its
// lanes hold the segment and two cells on each side.  Wavefront q runs velocity quadrant q
// (signs su, sv) over both rows: u nodes outer, v nodes inner.  The upwind row of the pair
// (jb for sv > 0) comes first: the flux through the face between the two rows is evaluated
// once, as that row's outgoing flux, and taken over in registers as the other row's incoming
// flux.  Per velocity the wavefront loads five row segments of the plane (the pair, the two
// rows upwind of it, the row downwind of it) instead of four per row.
//
// Arithmetic: with f stored in FP64 every step is FP64.  With f stored in FP32 the
// per-velocity work (slopes, reconstruction, face fluxes, Eq. (3)) runs in FP32 on FP32
// copies of the face records and cell constants; Eq. (4), the interface scalars and the
// velocity moments stay FP64.
//
// Rows: the pairs are (0, 1), (2, 3), ...; with ny odd the last pair is (ny - 2, ny - 1), of
// which only row ny - 1 is written (row ny - 2 belongs to the pair before), and with ny = 1
// the only pair is (-1, 0), of which only row 0 is written.  A row outside the mesh reads
// zeros or halo values and writes nothing; the faces it touches are chosen so that no flux
// that a written row takes from it depends on its values (see face_role).
constexpr int kPair = 2;
// Face record fields staged in LDS: R_GC .. R_M5 except R_VY (read once, for the Gauss starts).
constexpr int kSF = R_M5 - R_GC;
__host__ __device__ constexpr int sf(int R) { return R < R_VY ? R - R_GC : R - R_GC - 1; }
// Per-cell state of Eq. (3) (CellField) for the two rows.
enum CellField { C_LAMN, C_UN, C_VN, C_LAM1, C_U1, C_V1, C_AN, C_A1, C_AF, C_ADF, C_COUNT };
template <typename T>
struct PairStage {
  T sx[kPair][kSF][kWave + 1];  // x face i0 - 2 + f of row jb + r (left face of lane f)
  T sy[kPair + 1][kSF][kWave];  // y face row jb + r (bottom face of row jb + r), lane l
  T cell[kPair][C_COUNT][kWave];
  // Gauss starts (value, ratio) at the first node of v half h (0: v > 0, 1: v < 0)
  T xs[2][kPair][2][kWave + 1];   // x faces
  T ys[2][kPair + 1][2][kWave];   // y faces
  T gs[2][kPair][2][2][kWave];    // g^n (0) and g^{n+1} (1) of each cell
};

// A Gaussian factor exp(-lam (x - c)^2) along the uniform nodes x0, x0 + h, x0 + 2h, ...:
// e is its value at the current node and r the ratio to the next one; successive ratios
// differ by the factor exp(-2 lam h^2), applied as r + r (exp(-2 lam h^2) - 1) with the
// second factor from expm1, so that it adds one rounding per node and no drift.
template <typename T>
__device__ __forceinline__ void gauss_next(T& e, T& r, T qm1) {
  e *= r;
  r = fma(r, qm1, r);
}

// Cubic of the folded equilibrium polynomial P(un, ut) of a record (interface scalars) in
// one velocity with the other fixed.  The e1, e4, e5, e7 of the side the particles come from
// are passed in (pos: un > 0).
template <typename T>
struct Cubic {
  T c0, c1, c2, c3;
};
// P as a cubic in the tangential velocity at fixed normal velocity un.
template <typename T>
__device__ __forceinline__ Cubic<T> cubic_in_ut(const T* e, T un) {
  const T h = T(0.5);
  Cubic<T> c;
  c.c0 = fma(un, fma(un, fma(un, h * e[7], e[4] + h * e[3]), e[1]), e[0]);
  c.c1 = fma(un, fma(un, h * e[8], e[5]), e[2]);
  c.c2 = fma(un, h * e[7], e[6] + h * e[3]);
  c.c3 = h * e[8];
  return c;
}
// P as a cubic in the normal velocity at fixed tangential velocity ut.
template <typename T>
__device__ __forceinline__ Cubic<T> cubic_in_un(const T* e, T ut) {
  const T h = T(0.5);
  Cubic<T> c;
  c.c0 = fma(ut, fma(ut, fma(ut, h * e[8], h * e[3] + e[6]), e[2]), e[0]);
  c.c1 = fma(ut, fma(ut, h * e[7], e[5]), e[1]);
  c.c2 = fma(ut, h * e[8], h * e[3] + e[4]);
  c.c3 = h * e[7];
  return c;
}
template <typename T>
__device__ __forceinline__ T horner(const Cubic<T>& c, T x) {
  return fma(x, fma(x, fma(x, c.c3, c.c2), c.c1), c.c0);
}
template <typename T>
__device__ __forceinline__ Cubic<T> scaled(Cubic<T> c, T s) {
  c.c0 *= s;
  c.c1 *= s;
  c.c2 *= s;
  c.c3 *= s;
  return c;
}
// e0..e8 of a staged record for particles with normal velocity of sign s
template <typename T, int N>
__device__ __forceinline__ void load_e(const T (*st)[N], int col, int s, T* e) {
#pragma unroll
  for (int n = 0; n < 9; ++n) e[n] = st[sf(R_E + n)][col];
  if (s < 0) {
    e[1] = st[sf(R_ER + 0)][col];
    e[4] = st[sf(R_ER + 1)][col];
    e[5] = st[sf(R_ER + 2)][col];
    e[7] = st[sf(R_ER + 3)][col];
  }
}

// Shakhov: S of one cell at fixed u as a cubic in v.  kqx, kqy = (1 - Pr)(lambda^2/rho) q;
// S = (A + B v)(a2 v^2 + a1 v + a0) with A + B v = k (c . q), a2 v^2 + a1 v + a0 = 2 lambda |c|^2 - 4.
template <typename T>
__device__ __forceinline__ Cubic<T> shakhov_in_v(T u, T kqx, T kqy, T lam, T U, T V) {
  const T du = u - U;
  const T A = fma(du, kqx, -V * kqy), B = kqy;
  const T a2 = T(2) * lam, a1 = T(-4) * lam * V;
  const T a0 = fma(T(2) * lam, fma(du, du, V * V), T(-4));
  Cubic<T> c;
  c.c0 = A * a0;
  c.c1 = fma(A, a1, B * a0);
  c.c2 = fma(A, a2, B * a1);
  c.c3 = B * a2;
  return c;
}

// Role of y face F (between rows F - 1 and F) for particles moving with the sign sv of v.  A
// channel wall emits its Maxwellian when the particles leave it (F = 0 with sv > 0, F = ny with
// sv < 0): the flux is GC Et(u) E(v) alone, with no polynomial and no free transport, and takes
// nothing from the row beyond the wall.  A wall the particles reach (the other two cases)
// takes the first-order free transport of the wall row (its record has no polynomial and M5 = 0;
// the wall row has no y slope).  Every other face is an interior face.
enum FaceRole { F_INTERIOR = 0, F_EMIT = 1, F_ABSORB = 2 };
__device__ __forceinline__ int face_role(const KParams& P, int F, int sv) {
  if (P.bc != UGKS_BC_CHANNEL) return F_INTERIOR;
  if ((F == 0 && sv > 0) || (F == P.ny && sv < 0)) return F_EMIT;
  if ((F == P.ny && sv > 0) || (F == 0 && sv < 0)) return F_ABSORB;
  return F_INTERIOR;
}

// The equilibrium part of a y face at tangential velocity u as a cubic in v, and its free
// transport weights, for particles of v sign sv, by the face's role.
template <typename T>
__device__ __forceinline__ void y_face(const PairStage<T>& st, int fr, int lane, int sv, int role,
                                       T u, Cubic<T>& c, T& m4, T& m5) {
  const T(*r)[kWave] = st.sy[fr];
  const T d = u - r[sf(R_UX)][lane];
  const T Et = r[sf(R_GC)][lane] * exp_of(-r[sf(R_LAM)][lane] * d * d);
  if (role == F_EMIT) {
    c = Cubic<T>{Et, T(0), T(0), T(0)};
    m4 = m5 = T(0);
    return;
  }
  m4 = r[sf(R_M4)][lane];
  if (role == F_ABSORB) {
    c = Cubic<T>{T(0), T(0), T(0), T(0)};
    m5 = T(0);
    return;
  }
  T e[9];
  load_e(r, lane, sv, e);
  c = scaled(cubic_in_un(e, u), Et);
  m5 = r[sf(R_M5)][lane];
}

// Per velocity quadrant (SU = sign of u, sv = sign of v) of a row pair: Eq. (3) for every
// velocity of the quadrant's chunk of u nodes, in the arithmetic type S of the storage.  Per
// velocity and row a lane (cell i) forms
//   its upwind reconstruction and slope term at its outgoing x and y faces,
//   the flux through its outgoing x face, which the downwind lane takes over as its incoming
//   x flux (x faces of the segment are each evaluated once),
//   the flux through its outgoing y face; the upwind row's is the other row's incoming flux,
//   and the upwind row's incoming flux comes from the reconstruction of the cell below it
//   (i, jb - 1) for sv > 0 (above, (i, jb + 2), for sv < 0).
// The equilibrium part of a face flux is GC En(un) Et(ut) P(un, ut): the Gaussian and cubic
// of the u node are formed once per node, those of the v node follow the node by Gauss
// recurrences.
// kAhead: nodes whose loads are in flight ahead of the node computed.  On the
// 400 x 100 x 40^2 channel 2 measured fastest in both storage types (3 ahead: FP64 1% slower,
// FP32 storage 4% slower, its registers then spill); the Shakhov variant has no registers to
// spare beyond 1.  The ring only works because nothing else in the loop is a vector load: the
// next v node is a scalar load (UGKS_CONST), so waiting for it never waits for f loads.
template <typename S, int SU, bool kShak, int kAhead = kShak ? 1 : 2>
__device__ __forceinline__ void pair_quadrant(const KParams& P, const PairStage<S>& st,
                                              const S (*sk)[4][kWave], int lane, int sv,
                                              int jb, bool store0, int g, int G, int gv, int Gv,
                                              bool writes, bool ghost_lane,
                                              const UGKS_GLOBAL S* fin, UGKS_GLOBAL S* fout,
                                              int i) {
  typedef S T;  // arithmetic type of the per-velocity work
  const bool chan = P.bc == UGKS_BC_CHANNEL;
  const int r0 = sv > 0 ? 0 : 1, r1 = 1 - r0;     // rows of the pair, upwind first
  const int j0 = jb + r0, j1 = jb + r1;           // their mesh rows
  const int jB = j0 - sv;                         // the cell upwind of row j0
  // y face rows of the stage: incoming face of j0, the face between the rows, outgoing of j1
  const int fin_r = sv > 0 ? 0 : 2, fout_r = 2 - fin_r, fmid_r = 1;
  const int role_in = face_role(P, jb + fin_r, sv);
  const int role_mid = face_role(P, jb + fmid_r, sv);
  const int role_out = face_role(P, jb + fout_r, sv);
  auto no_wall = [&](int j) { return !(chan && (j == 0 || j == P.ny - 1)); };
  const bool gm = !ghost_lane;  // ghost columns have zero slopes
  const bool mB = no_wall(jB), m0 = gm && no_wall(j0), m1 = gm && no_wall(j1);
  // cells, and a channel's ghost columns (the ghost Maxwellian of the next step)
  const bool st0 = writes && (r0 == 0 ? store0 : true);
  const bool st1 = writes && (r1 == 0 ? store0 : true);
  // byte offsets of the five rows j0 - 2 sv, j0 - sv, j0, j1 = j0 + sv, j1 + sv
  const unsigned bs = (unsigned)sizeof(S);
  const int ic = i < P.nx + 1 ? i : P.nx + 1;
  const int o0 = pidx(P, ic, j0);
  const int L = sv * P.Lx;
  const unsigned oA = (unsigned)(o0 - 2 * L) * bs, oB = (unsigned)(o0 - L) * bs;
  const unsigned oC = (unsigned)o0 * bs, oD = (unsigned)(o0 + L) * bs;
  const unsigned oE = (unsigned)(o0 + 2 * L) * bs;
  const unsigned w0 = st0 ? oC : kDropOffset, w1 = st1 ? oD : kDropOffset;
  const int xo = lane + (SU > 0 ? 1 : 0);  // staged x face the lane's particles leave by
  const T Af0 = st.cell[r0][C_AF][lane], AdF0 = st.cell[r0][C_ADF][lane];
  const T Af1 = st.cell[r1][C_AF][lane], AdF1 = st.cell[r1][C_ADF][lane];
  const Half hu = axis_half(P.K, SU, false), hv = axis_half(P.M, sv, false);
  const int hf = sv > 0 ? 0 : 1;
  const T hstep = T(sv * P.dv);
  const T h2 = T(-2) * hstep * hstep;
  const T qx0 = expm1_of(h2 * st.sx[r0][sf(R_LAM)][xo]);
  const T qx1 = expm1_of(h2 * st.sx[r1][sf(R_LAM)][xo]);
  const T qyi = expm1_of(h2 * st.sy[fin_r][sf(R_LAM)][lane]);
  const T qym = expm1_of(h2 * st.sy[fmid_r][sf(R_LAM)][lane]);
  const T qyo = expm1_of(h2 * st.sy[fout_r][sf(R_LAM)][lane]);
  const T qn0 = expm1_of(h2 * st.cell[r0][C_LAMN][lane]);
  const T q10 = expm1_of(h2 * st.cell[r0][C_LAM1][lane]);
  const T qn1 = expm1_of(h2 * st.cell[r1][C_LAMN][lane]);
  const T q11 = expm1_of(h2 * st.cell[r1][C_LAM1][lane]);
  const T two_idx = T(2.0 * P.inv_dx), two_idy = T(2.0 * P.inv_dy);
  int a0, a1;
  chunk_range(hu.count, g, G, a0, a1);
  // this workgroup's v nodes of the half: chunk gv of Gv, vn nodes from node vf
  int c0, c1;
  chunk_range(hv.count, gv, Gv, c0, c1);
  const int vn = c1 - c0, vf = hv.first + c0 * hv.step;
  for (int a = a0; a < a1; ++a) {
    const int k = hu.first + a * hu.step;
    const T u = T(((const UGKS_CONST double*)P.uk)[k]);  // a scalar load
    const T au = fabs(u);
    const T ucx = u * two_idx;
    struct Vals {
      S A, B, C, D, E;  // rows j0 - 2 sv, j0 - sv, j0, j1, j1 + sv
    };
    // planes (read and written) and v nodes are walked with running pointers
    const long long pstep = (long long)hv.step * P.PS;
    const UGKS_GLOBAL S* pnext = plane_of(fin, P, k * P.M) + (long long)vf * P.PS;
    UGKS_GLOBAL S* wcur = plane_of(fout, P, k * P.M) + (long long)vf * P.PS;
    const UGKS_CONST double* vp = (const UGKS_CONST double*)(P.vm + vf);
    // loads run kAhead nodes ahead of the node computed; past the last node of the chunk they
    // read its plane again
    int nl = 0;
    auto load_next = [&]() {
      const __amdgpu_buffer_rsrc_t r = plane_rsrc(pnext, P);
      const Vals v{bload_raw(r, oA, S{}), bload_raw(r, oB, S{}), bload_raw(r, oC, S{}),
                   bload_raw(r, oD, S{}), bload_raw(r, oE, S{})};
      if (++nl < vn) pnext += pstep;
      return v;
    };
    // the first nodes' stencil values, requested before the node's tables are formed
    constexpr int NB = kAhead + 1;
    Vals ring[NB];
#pragma unroll
    for (int d = 0; d < kAhead; ++d) ring[d] = load_next();
    // x faces of both rows: cubic in v times GC En(u), with |u| folded in
    Cubic<T> cx0, cx1;
    T m4x0, m5x0, m4x1, m5x1;
    {
      T e[9];
      const T(*x0)[kWave + 1] = st.sx[r0];
      load_e(x0, xo, SU, e);
      const T d = u - x0[sf(R_UX)][xo];
      cx0 = scaled(cubic_in_ut(e, u), x0[sf(R_GC)][xo] * exp_of(-x0[sf(R_LAM)][xo] * d * d) * au);
      m4x0 = x0[sf(R_M4)][xo] * au;
      m5x0 = x0[sf(R_M5)][xo] * au;
    }
    __builtin_amdgcn_sched_barrier(0);
    {
      T e[9];
      const T(*x1)[kWave + 1] = st.sx[r1];
      load_e(x1, xo, SU, e);
      const T d = u - x1[sf(R_UX)][xo];
      cx1 = scaled(cubic_in_ut(e, u), x1[sf(R_GC)][xo] * exp_of(-x1[sf(R_LAM)][xo] * d * d) * au);
      m4x1 = x1[sf(R_M4)][xo] * au;
      m5x1 = x1[sf(R_M5)][xo] * au;
    }
    __builtin_amdgcn_sched_barrier(0);
    // y faces: cubic in v at tangential u, times GC Et(u)
    Cubic<T> ci, cm, co;
    T m4i, m5i, m4m, m5m, m4o, m5o;
    y_face(st, fin_r, lane, sv, role_in, u, ci, m4i, m5i);
    __builtin_amdgcn_sched_barrier(0);
    y_face(st, fmid_r, lane, sv, role_mid, u, cm, m4m, m5m);
    __builtin_amdgcn_sched_barrier(0);
    y_face(st, fout_r, lane, sv, role_out, u, co, m4o, m5o);
    __builtin_amdgcn_sched_barrier(0);
    // g^n and g^{n+1} of both cells: u factors (with the Eq. (3) weights) times the v
    // Gaussians' start values
    T en0, rn0, e10, r10, en1, rn1, e11, r11;
    {
      const T(*c0)[kWave] = st.cell[r0];
      const T dn = u - c0[C_UN][lane], d1 = u - c0[C_U1][lane];
      en0 = c0[C_AN][lane] * exp_of(-c0[C_LAMN][lane] * dn * dn) * st.gs[hf][r0][0][0][lane];
      e10 = c0[C_A1][lane] * exp_of(-c0[C_LAM1][lane] * d1 * d1) * st.gs[hf][r0][1][0][lane];
      rn0 = st.gs[hf][r0][0][1][lane];
      r10 = st.gs[hf][r0][1][1][lane];
    }
    __builtin_amdgcn_sched_barrier(0);
    {
      const T(*c1)[kWave] = st.cell[r1];
      const T dn = u - c1[C_UN][lane], d1 = u - c1[C_U1][lane];
      en1 = c1[C_AN][lane] * exp_of(-c1[C_LAMN][lane] * dn * dn) * st.gs[hf][r1][0][0][lane];
      e11 = c1[C_A1][lane] * exp_of(-c1[C_LAM1][lane] * d1 * d1) * st.gs[hf][r1][1][0][lane];
      rn1 = st.gs[hf][r1][0][1][lane];
      r11 = st.gs[hf][r1][1][1][lane];
    }
    // Shakhov: the factors (1 + S) of g^n and g^{n+1} of both cells as cubics in v
    Cubic<T> sn0{}, s10{}, sn1{}, s11{};
    if constexpr (kShak) {
      const T(*c0)[kWave] = st.cell[r0];
      const T(*c1)[kWave] = st.cell[r1];
      sn0 = shakhov_in_v(u, sk[r0][0][lane], sk[r0][1][lane], c0[C_LAMN][lane], c0[C_UN][lane],
                         c0[C_VN][lane]);
      s10 = shakhov_in_v(u, sk[r0][2][lane], sk[r0][3][lane], c0[C_LAM1][lane], c0[C_U1][lane],
                         c0[C_V1][lane]);
      sn1 = shakhov_in_v(u, sk[r1][0][lane], sk[r1][1][lane], c1[C_LAMN][lane], c1[C_UN][lane],
                         c1[C_VN][lane]);
      s11 = shakhov_in_v(u, sk[r1][2][lane], sk[r1][3][lane], c1[C_LAM1][lane], c1[C_U1][lane],
                         c1[C_V1][lane]);
    }
    __builtin_amdgcn_sched_barrier(0);
    // v-direction Gaussians of the faces at the first node of the chunk, and their ratios
    T ex0 = st.xs[hf][r0][0][xo], rx0 = st.xs[hf][r0][1][xo];
    T ex1 = st.xs[hf][r1][0][xo], rx1 = st.xs[hf][r1][1][xo];
    T ei = st.ys[hf][fin_r][0][lane], ri = st.ys[hf][fin_r][1][lane];
    T em = st.ys[hf][fmid_r][0][lane], rm = st.ys[hf][fmid_r][1][lane];
    T eo = st.ys[hf][fout_r][0][lane], ro = st.ys[hf][fout_r][1][lane];
    T vv = T(*vp);
    auto node = [&](const Vals& x) {
      const T vnext = T(vp[hv.step]);  // the next node (read one ahead; past the end a pad)
      const T av = fabs(vv);
      const T avcy = av * two_idy;
      // upwind neighbour of row j0: half-cell changes towards the pair (y) and in x
      const T fBw = from_lower(x.B), fBe = from_upper(x.B);
      const T HxB = half_limited(fBe - x.B, x.B - fBw);
      const T HyB = half_limited(x.C - x.B, x.B - x.A, mB);
      const T DB = fma(ucx, HxB, avcy * HyB);
      const T fhB = x.B + HyB;
      // row j0
      const T fCw = from_lower(x.C), fCe = from_upper(x.C);
      const T HxC = half_limited(fCe - x.C, x.C - fCw, gm);
      const T HyC = half_limited(x.D - x.C, x.C - x.B, m0);
      const T DC = fma(ucx, HxC, avcy * HyC);
      const T fxC = SU > 0 ? x.C + HxC : x.C - HxC;
      const T fhC = x.C + HyC;
      // row j1
      const T fDw = from_lower(x.D), fDe = from_upper(x.D);
      const T HxD = half_limited(fDe - x.D, x.D - fDw, gm);
      const T HyD = half_limited(x.E - x.D, x.D - x.C, m1);
      const T DD = fma(ucx, HxD, avcy * HyD);
      const T fxD = SU > 0 ? x.D + HxD : x.D - HxD;
      const T fhD = x.D + HyD;
      // x faces: outgoing of this lane, incoming from the upwind lane
      const T Fxo0 = fma(ex0, horner(cx0, vv), fma(m4x0, fxC, -m5x0 * DC));
      const T Fxo1 = fma(ex1, horner(cx1, vv), fma(m4x1, fxD, -m5x1 * DD));
      const T Fxi0 = SU > 0 ? from_lower(Fxo0) : from_upper(Fxo0);
      const T Fxi1 = SU > 0 ? from_lower(Fxo1) : from_upper(Fxo1);
      // y faces: into row j0, between the rows, out of row j1
      const T Fyi = av * fma(ei, horner(ci, vv), fma(m4i, fhB, -m5i * DB));
      const T Fym = av * fma(em, horner(cm, vv), fma(m4m, fhC, -m5m * DC));
      const T Fyo = av * fma(eo, horner(co, vv), fma(m4o, fhD, -m5o * DD));
      T g0, g1;
      if constexpr (kShak) {
        g0 = fma(e10, T(1) + horner(s10, vv), en0 * (T(1) + horner(sn0, vv)));
        g1 = fma(e11, T(1) + horner(s11, vv), en1 * (T(1) + horner(sn1, vv)));
      } else {
        g0 = e10 + en0;
        g1 = e11 + en1;
      }
      const T f0 = fma(Af0, x.C, fma(AdF0, (Fxi0 - Fxo0) + (Fyi - Fym), g0));
      const T f1 = fma(Af1, x.D, fma(AdF1, (Fxi1 - Fxo1) + (Fym - Fyo), g1));
      // lanes and rows without a cell to write store past the plane's range (dropped)
      const __amdgpu_buffer_rsrc_t wr = plane_rsrc(wcur, P);
      bstore(wr, w0, f0, S{});
      bstore(wr, w1, f1, S{});
      wcur += pstep;
      vp += hv.step;
      vv = vnext;
      gauss_next(ex0, rx0, qx0);
      gauss_next(ex1, rx1, qx1);
      gauss_next(ei, ri, qyi);
      gauss_next(em, rm, qym);
      gauss_next(eo, ro, qyo);
      gauss_next(en0, rn0, qn0);
      gauss_next(e10, r10, q10);
      gauss_next(en1, rn1, qn1);
      gauss_next(e11, r11, q11);
    };
    // NB value sets in a ring: slot s holds node c + s, loaded kAhead nodes earlier
    int c = 0;
    for (; c + NB <= vn; c += NB) {
#pragma unroll
      for (int s = 0; s < NB; ++s) {
        ring[(s + kAhead) % NB] = load_next();
        node(ring[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      if (c + s < vn) {
        ring[(s + kAhead) % NB] = load_next();
        node(ring[s]);
      }
    }
  }
}

// Fill mode of the update kernel, quadrant wavefront: the ghost columns of the current f from
// the ghost states of the current W (after the initial state and after a state is set).  It
// forms the ghost lanes' g^{n+1} with the expressions and Gauss recurrences of the update loop,
// where Eq. (3) with every other weight zero leaves f = g^{n+1}, so a state set from a
// checkpoint steps on exactly as a running solver does.
template <typename S, int SU>
__device__ __forceinline__ void ghost_fill_quadrant(const KParams& P, const PairStage<S>& st,
                                                    int lane, int sv, int jb, bool store0,
                                                    int g, int G, int gv, int Gv, bool ghost_w,
                                                    UGKS_GLOBAL S* f, int i) {
  typedef S T;
  const int r0 = sv > 0 ? 0 : 1, r1 = 1 - r0;
  const int j0 = jb + r0;
  const bool st0 = ghost_w && (r0 == 0 ? store0 : true);
  const bool st1 = ghost_w && (r1 == 0 ? store0 : true);
  const unsigned bs = (unsigned)sizeof(S);
  const int ic = i < P.nx + 1 ? i : P.nx + 1;
  const int o0 = pidx(P, ic, j0);
  const unsigned oC = (unsigned)o0 * bs, oD = (unsigned)(o0 + sv * P.Lx) * bs;
  const unsigned w0 = st0 ? oC : kDropOffset, w1 = st1 ? oD : kDropOffset;
  const Half hu = axis_half(P.K, SU, false), hv = axis_half(P.M, sv, false);
  const int hf = sv > 0 ? 0 : 1;
  const T hstep = T(sv * P.dv);
  const T h2 = T(-2) * hstep * hstep;
  const T qn0 = expm1_of(h2 * st.cell[r0][C_LAMN][lane]);
  const T q10 = expm1_of(h2 * st.cell[r0][C_LAM1][lane]);
  const T qn1 = expm1_of(h2 * st.cell[r1][C_LAMN][lane]);
  const T q11 = expm1_of(h2 * st.cell[r1][C_LAM1][lane]);
  const long long pstep = (long long)hv.step * P.PS;
  int a0, a1;
  chunk_range(hu.count, g, G, a0, a1);
  int c0, c1;
  chunk_range(hv.count, gv, Gv, c0, c1);
  const int vn = c1 - c0, vf = hv.first + c0 * hv.step;
  for (int a = a0; a < a1; ++a) {
    const int k = hu.first + a * hu.step;
    const T u = T(((const UGKS_CONST double*)P.uk)[k]);  // a scalar load
    UGKS_GLOBAL S* wcur = plane_of(f, P, k * P.M) + (long long)vf * P.PS;
    T en0, rn0, e10, r10, en1, rn1, e11, r11;
    {
      const T(*c0)[kWave] = st.cell[r0];
      const T dn = u - c0[C_UN][lane], d1 = u - c0[C_U1][lane];
      en0 = c0[C_AN][lane] * exp_of(-c0[C_LAMN][lane] * dn * dn) * st.gs[hf][r0][0][0][lane];
      e10 = c0[C_A1][lane] * exp_of(-c0[C_LAM1][lane] * d1 * d1) * st.gs[hf][r0][1][0][lane];
      rn0 = st.gs[hf][r0][0][1][lane];
      r10 = st.gs[hf][r0][1][1][lane];
    }
    {
      const T(*c1)[kWave] = st.cell[r1];
      const T dn = u - c1[C_UN][lane], d1 = u - c1[C_U1][lane];
      en1 = c1[C_AN][lane] * exp_of(-c1[C_LAMN][lane] * dn * dn) * st.gs[hf][r1][0][0][lane];
      e11 = c1[C_A1][lane] * exp_of(-c1[C_LAM1][lane] * d1 * d1) * st.gs[hf][r1][1][0][lane];
      rn1 = st.gs[hf][r1][0][1][lane];
      r11 = st.gs[hf][r1][1][1][lane];
    }
    for (int c = 0; c < vn; ++c) {
      const T g0 = e10 + en0, g1 = e11 + en1;
      const __amdgpu_buffer_rsrc_t wr = plane_rsrc(wcur, P);
      bstore(wr, w0, g0, S{});
      bstore(wr, w1, g1, S{});
      wcur += pstep;
      gauss_next(en0, rn0, qn0);
      gauss_next(e10, r10, q10);
      gauss_next(en1, rn1, qn1);
      gauss_next(e11, r11, q11);
    }
  }
}

// The body of the update kernel; kShak: the Shakhov collision model.
template <typename S, bool kShak, int kCh, bool kFill = false>
__device__ __forceinline__ void update_body(const PlanView& pv) {
  typedef S T;  // arithmetic type of the per-velocity work (and of the LDS stage)
  __shared__ PairStage<T> st;
  // Shakhov: (1 - Pr)(lambda^2/rho) q of each lane's cell at t^n and t^{n+1}, per row
  __shared__ T sk_raw[kShak ? kPair * 4 * kWave : 1];
  T(*sk)[4][kWave] = reinterpret_cast<T(*)[4][kWave]>(sk_raw);
  const int lane = threadIdx.x & (kWave - 1);
  // wavefront w: quadrant q, and c, which of the workgroup's kCh velocity chunks
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int q = w & 3, c = w >> 2;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int ii = find_inst(pv.off_upd, pv.ninst, b);
  const Inst* __restrict__ I = inst_at(pv, ii);
  const KParams P = I->P;
  const int parity = (I->cur + pv.step) & 1;
  const int G = I->usplit, Gv = P.vsplit;
  int t, gg, pb;
  cell_block(b - first_block(pv.off_upd, ii), (P.ny + 1) / 2, (P.nx + kTileU - 1) / kTileU, t,
             gg, pb);
  const int jb = min(2 * pb, P.ny - 2);       // rows jb, jb + 1
  const bool store0 = jb == 2 * pb && jb >= 0;  // row jb is this pair's to write
  // chunk gg: u chunk g of G fastest, then v chunk gv of Gv; chunks G Gv.. update H: its
  // planes, its face records, its equilibria
  const bool hpart = gg >= G * Gv;
  const int g2 = hpart ? gg - G * Gv : gg;
  const int g = g2 % G, gv = g2 / G;
  const long long hoff = hpart ? (long long)P.NV * P.PS : 0ll;
  const UGKS_GLOBAL S* fin = static_cast<const UGKS_GLOBAL S*>(I->f[parity]) + hoff;
  // fill mode writes the ghost columns of the current f
  UGKS_GLOBAL S* fout = static_cast<UGKS_GLOBAL S*>(I->f[kFill ? parity : parity ^ 1]) + hoff;
  // face records, field-major (RecRef): field f of x face e at f nfx + e, of y face e at
  // f nfy + e; the records of H follow those of G
  const size_t nfx = (size_t)P.ny * (P.nx + 1), nfy = (size_t)(P.ny + 1) * P.nx;
  const UGKS_GLOBAL double* recx = I->recx + (hpart ? nfx * kRec : (size_t)0);
  const UGKS_GLOBAL double* recy = I->recy + (hpart ? nfy * kRec : (size_t)0);
  const UGKS_GLOBAL double* W = I->W[parity];
  UGKS_GLOBAL double* Wout = I->W[parity ^ 1];
  const int i0 = t * kTileU;
  const int i = i0 - kHalo + lane;
  const bool valid = lane >= kHalo && lane < kHalo + kTileU && i < P.nx;
  const bool chan = P.bc == UGKS_BC_CHANNEL;
  const bool ghost_lane = chan && (i == -1 || i == P.nx);
  // the ghost lane whose neighbouring cell is this segment's writes the ghost column (the
  // outlet column can also be the right halo of the segment before the last)
  const bool ghost_w = ghost_lane && (i < 0 || lane <= kHalo + kTileU);
  // the Eq. (4) inputs of wavefronts 0 and 1 (row jb + w), requested before the stage so that
  // their latency overlaps the stage's
  double eWn[4] = {1.0, 0.0, 0.0, 1.0}, eF[4][4] = {};
  if (w < kPair) {
    const int jr = clampi(jb + w, 0, P.ny - 1);
    const int ci = valid ? i : 0;
    const size_t cc = (size_t)jr * P.nx + ci;
    if (valid) {
#pragma unroll
      for (int k = 0; k < 4; ++k) eWn[k] = W[4 * cc + k];
    }
    if constexpr (!kFill) {
      // the fluxes through the cell's left and right x faces and its lower and upper y faces
      const UGKS_GLOBAL double* fl = recx + (size_t)R_FX * nfx + (size_t)jr * (P.nx + 1) + ci;
      const UGKS_GLOBAL double* fb = recy + (size_t)R_FX * nfy + (size_t)jr * P.nx + ci;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        eF[0][k] = fl[k * nfx];
        eF[1][k] = fl[k * nfx + 1];
        eF[2][k] = fb[k * nfy];
        eF[3][k] = fb[k * nfy + P.nx];
      }
    }
  }
  // stage the records of the pair's faces: x faces i0-2 .. i0+62 of both rows, y face rows
  // jb .. jb+2 below / above lanes 0..63; indices clamped into the mesh for lanes and rows
  // outside it.  Every thread issues all its record loads before it writes any to LDS: one
  // trip of a load-then-store loop per value would wait out one memory latency per trip.
  if constexpr (!kFill) {
    constexpr int kThreads = kWave * kQuads * kCh;  // the launch's workgroup size
    constexpr int kNX = kPair * (kWave + 1) * kSF, kNY = (kPair + 1) * kWave * kSF;
    constexpr int kItX = (kNX + kThreads - 1) / kThreads;
    constexpr int kItY = (kNY + kThreads - 1) / kThreads;
    auto fld_of = [](int s) { return s <= sf(R_UX) ? R_GC + s : R_GC + s + 1; };  // skip R_VY
    double vx[kItX], vy[kItY];
#pragma unroll
    for (int it = 0; it < kItX; ++it) {
      const int e = threadIdx.x + it * kThreads;
      if (e < kNX) {
        const int r = e / ((kWave + 1) * kSF), rem = e - r * ((kWave + 1) * kSF);
        const int s = rem / (kWave + 1), fc = rem - s * (kWave + 1);  // faces fastest
        const int fi = clampi(i0 - kHalo + fc, 0, P.nx);
        const int row = clampi(jb + r, 0, P.ny - 1);
        vx[it] = recx[(size_t)fld_of(s) * nfx + (size_t)row * (P.nx + 1) + fi];
      }
    }
#pragma unroll
    for (int it = 0; it < kItY; ++it) {
      const int e = threadIdx.x + it * kThreads;
      if (e < kNY) {
        const int r = e / (kWave * kSF), rem = e - r * (kWave * kSF);
        const int s = rem / kWave, fc = rem - s * kWave;  // faces fastest
        const int fi = clampi(i0 - kHalo + fc, 0, P.nx - 1);
        const int row = clampi(jb + r, 0, P.ny);
        vy[it] = recy[(size_t)fld_of(s) * nfy + (size_t)row * P.nx + fi];
      }
    }
#pragma unroll
    for (int it = 0; it < kItX; ++it) {
      const int e = threadIdx.x + it * kThreads;
      if (e < kNX) {
        const int r = e / ((kWave + 1) * kSF), rem = e - r * ((kWave + 1) * kSF);
        const int s = rem / (kWave + 1), fc = rem - s * (kWave + 1);
        st.sx[r][s][fc] = T(vx[it]);
      }
    }
#pragma unroll
    for (int it = 0; it < kItY; ++it) {
      const int e = threadIdx.x + it * kThreads;
      if (e < kNY) {
        const int r = e / (kWave * kSF), rem = e - r * (kWave * kSF);
        const int s = rem / kWave, fc = rem - s * kWave;
        st.sy[r][s][fc] = T(vy[it]);
      }
    }
  }
  __syncthreads();
  const double hstep = P.dv;
  // A start value below the normal range cannot be carried up to a peak that lies beyond the
  // chunk's first node: such a state (speed ratio |V| lambda^(1/2) above about 26 across v)
  // is flagged.
  bool lost = false;
  // the first v node of this workgroup's chunk in half h (h = 0: v >= 0, walked upwards)
  int vfirst[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const Half hv = axis_half(P.M, h == 0 ? 1 : -1, false);
    int c0, c1;
    chunk_range(hv.count, gv, Gv, c0, c1);
    vfirst[h] = hv.first + c0 * hv.step;
  }
  // Gauss start of exp(-lam (v - c)^2) at that node and its ratio to the next (FP64, stored
  // in the stage's type)
  auto start = [&](double lam, double c, int h, T* e, T* r, int col) {
    const double v0 = ((const UGKS_CONST double*)P.vm)[vfirst[h]];
    const double hs = h == 0 ? hstep : -hstep;
    const double d = v0 - c;
    const double x = lam * d * d;
    e[col] = T(exp(-x));
    r[col] = T(exp(-lam * hs * (2.0 * d + hs)));
    lost = lost || (x > 700.0 && (h == 0 ? c > v0 : c < v0));
  };
  if (w < kPair) {
    // Eq. (4) for row jb + w, and the cell's Maxwellians of W^n and W^{n+1} with the
    // weights of Eq. (3) solved for f^{n+1}: f1 = Af f + AdF dF + (A1 g^{n+1} + An g^n)
    const int r = w;
    const int jr = clampi(jb + r, 0, P.ny - 1);
    const bool mine = valid && (r == 0 ? store0 : true);
    const int ci = valid ? i : 0;
    const size_t cc = (size_t)jr * P.nx + ci;
    double Wn[4], W1[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) Wn[k] = eWn[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if constexpr (kFill) {  // the ghost states of the current W
        W1[k] = Wn[k];
      } else {
        const double dW = (eF[0][k] - eF[1][k] + eF[2][k] - eF[3][k]) / P.area;
        W1[k] = valid ? Wn[k] + dW : Wn[k];
      }
    }
    // every velocity chunk of the segment forms the same W^{n+1}; chunk 0 stores it
    if (!kFill && mine && gg == 0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) Wout[4 * cc + k] = W1[k];
    }
    if (!kFill && P.adaptive && gg == 0) {
      // the adaptive step of the next step: the largest rate over the cells of W^{n+1}
      double rate = 0.0;
      if (mine)
        rate = (P.umax + fabs(W1[1] / W1[0])) / P.dx + (P.vmax + fabs(W1[2] / W1[0])) / P.dy;
      rate = wave_max(rate);
      if (lane == 0)
        atomicMax((unsigned long long*)(P.rmax + (parity ^ 1)),
                  (unsigned long long)__double_as_longlong(rate));
    }
    // the simulated time advances by this step's dt (one thread of the instance)
    if (!kFill && b == first_block(pv.off_upd, ii) && w == 0 && lane == 0)
      *P.tsum += step_dt(P, parity);
    Prim pn{}, p1{};
    double Af = 1.0, AdF = 1.0 / P.area, A1 = 0.0, An = 0.0;
    if (!P.collisionless) {
      const bool ok = prim_of(Wn, pn, P.lam_c) && prim_of(W1, p1, P.lam_c);
      if (!ok && mine) *P.flag = 1;
      const double tn = collision_time(pn, P.mu_ref), t1 = collision_time(p1, P.mu_ref);
      const double hdt = 0.5 * step_dt(P, parity);
      const double den = 1.0 / (1.0 + hdt / t1);
      Af = (1.0 - hdt / tn) * den;
      AdF = den / P.area;
      A1 = (p1.rho * p1.lam / kPi) * (hdt / t1) * den;
      An = (pn.rho * pn.lam / kPi) * (hdt / tn) * den;
      if (hpart) {  // the equilibrium of H: dof/(2 lambda) times that of G
        A1 *= (double)P.dof / (2.0 * p1.lam);
        An *= (double)P.dof / (2.0 * pn.lam);
      }
    }
    // A channel's ghost column (lane of cell -1 or nx) takes the ghost state of step n + 1,
    // formed from W^{n+1} of the cell next to it (Sec. 3.A), as its g^{n+1} with weight one
    // and every other Eq. (3) weight zero: the loop then writes the ghost Maxwellian of the
    // next step into the ghost column of f^{n+1}.  The first velocity chunk stores its W.
    // (both shifts run on every lane: a lane exchange inside a per-lane branch would read
    // the lanes the branch switched off)
    double Wc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double up = from_upper(W1[k]), dn = from_lower(W1[k]);
      Wc[k] = i < 0 ? up : dn;
    }
    if (ghost_w) {
      const int side = i < 0 ? 0 : 1;
      Prim pc;
      (void)prim_of(Wc, pc, P.lam_c);  // an invalid cell state is flagged by its own lane
      p1 = ghost_prim(P, side, jr, pc);
      pn = p1;
      if (gg == 0 && (r == 0 ? store0 : true))
        store_wg(I->Wg + 4 * ((size_t)side * P.ny + jr), p1, P.lam_c);
      Af = 0.0;
      AdF = 0.0;
      An = 0.0;
      A1 = p1.rho * p1.lam / kPi;
      if (hpart) A1 *= (double)P.dof / (2.0 * p1.lam);
    }
    if constexpr (kShak) {
      // heat flux of f^n about U^n from the cell's raw moments (moment kernel, chunk 0)
      const size_t nc = (size_t)P.nx * P.ny;
      const UGKS_GLOBAL double* cm = I->hs + (size_t)kSlotCell * nc + cc;
      double m[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) m[k] = valid ? cm[(size_t)k * nc] : 0.0;
      double qn[2];
      heat_flux(m[0], m[1], m[2], m[3], m[4], m[5], m[6], m[7], m[3] + m[5], pn.U, pn.V, qn);
      // no Shakhov factor on a ghost Maxwellian
      const double kn = P.collisionless || ghost_w ? 0.0 : P.pr_c * pn.lam * pn.lam / pn.rho;
      const double k1 = P.collisionless || ghost_w ? 0.0 : P.pr_c * p1.lam * p1.lam / p1.rho;
      sk[r][0][lane] = T(kn * qn[0]);
      sk[r][1][lane] = T(kn * qn[1]);
      sk[r][2][lane] = T(k1 * qn[0]);
      sk[r][3][lane] = T(k1 * qn[1]);
    }
    const double cell[C_COUNT] = {pn.lam, pn.U, pn.V, p1.lam, p1.U, p1.V, An, A1, Af, AdF};
#pragma unroll
    for (int n = 0; n < C_COUNT; ++n) st.cell[r][n][lane] = T(cell[n]);
    // Gauss starts of g^n and g^{n+1} of this cell in both halves of v
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      start(pn.lam, pn.V, h, st.gs[h][r][0][0], st.gs[h][r][0][1], lane);
      start(p1.lam, p1.V, h, st.gs[h][r][1][0], st.gs[h][r][1][1], lane);
    }
  } else if (!kFill) {
    // Gauss starts of the faces (FP64 records): wavefront 2 + r takes the x faces of row
    // jb + r; the y face rows jb .. jb + 2 go one to a wavefront 4..6 with eight wavefronts,
    // else row jb to wavefront 2 and rows jb + 1, jb + 2 to wavefront 3
    const int r = w - kPair;
    if (r < kPair) {
      const int jr = clampi(jb + r, 0, P.ny - 1);
      for (int fc = lane; fc < kWave + 1; fc += kWave) {
        const int fi = clampi(i0 - kHalo + fc, 0, P.nx);
        const UGKS_GLOBAL double* rec = recx + (size_t)jr * (P.nx + 1) + fi;
        const double lam = rec[(size_t)R_LAM * nfx], vy = rec[(size_t)R_VY * nfx];
#pragma unroll
        for (int h = 0; h < 2; ++h) start(lam, vy, h, st.xs[h][r][0], st.xs[h][r][1], fc);
      }
    }
    const int fr0 = kCh == 2 ? r - kPair : (r == 0 ? 0 : 1);
    const int fr1 = kCh == 2 ? min(r - kPair + 1, kPair + 1) : (r == 0 ? 1 : kPair + 1);
    for (int fr = max(fr0, 0); fr < fr1; ++fr) {
      const int fi = clampi(i0 - kHalo + lane, 0, P.nx - 1);
      const int row = clampi(jb + fr, 0, P.ny);
      const UGKS_GLOBAL double* rec = recy + (size_t)row * P.nx + fi;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        start(rec[(size_t)R_LAM * nfy], rec[(size_t)R_VY * nfy], h, st.ys[h][fr][0],
              st.ys[h][fr][1], lane);
    }
  }
  if (lost && (valid || ghost_w)) *P.flag = 1;
  __syncthreads();
  // the workgroup's chunks kCh g .. kCh g + kCh - 1 of the quadrant's kCh G chunks
  const int sv = quad_sv(q);
  if constexpr (kFill) {
    if (quad_su(q) > 0)
      ghost_fill_quadrant<S, 1>(P, st, lane, sv, jb, store0, kCh * g + c, kCh * G, gv, Gv,
                                ghost_w, fout, i);
    else
      ghost_fill_quadrant<S, -1>(P, st, lane, sv, jb, store0, kCh * g + c, kCh * G, gv, Gv,
                                 ghost_w, fout, i);
    return;
  }
  if (quad_su(q) > 0)
    pair_quadrant<S, 1, kShak>(P, st, sk, lane, sv, jb, store0, kCh * g + c, kCh * G, gv, Gv,
                               valid || ghost_w, ghost_lane, fin, fout, i);
  else
    pair_quadrant<S, -1, kShak>(P, st, sk, lane, sv, jb, store0, kCh * g + c, kCh * G, gv, Gv,
                                valid || ghost_w, ghost_lane, fin, fout, i);
}

// Velocity chunks per update workgroup, kCh (its wavefronts: four quadrants times kCh), which
// share one stage, and the update waves per SIMD.  FP64: the registers of two rows allow two
// waves per SIMD; with two chunks, one workgroup of eight waves per CU (its stage takes 73 KB),
// and sharing the stage halves its cost per velocity node; one chunk serves meshes too small
// to give every CU a workgroup of two.  FP32 storage: four waves per SIMD, four workgroups of
// four waves per CU (37 KB each); the Shakhov form two waves per SIMD.
template <typename S, bool kShak>
constexpr int kUpdateWaves = sizeof(S) == 8 || kShak ? 2 : 4;

template <typename S, int kCh>
__global__ __launch_bounds__(kWave* kQuads* kCh)
__attribute__((amdgpu_waves_per_eu(kUpdateWaves<S, false>)))
void update_kernel(PlanView pv) {
  update_body<S, false, kCh>(pv);
}

template <typename S, int kCh>
__global__ __launch_bounds__(kWave* kQuads* kCh)
__attribute__((amdgpu_waves_per_eu(kUpdateWaves<S, true>)))
void update_kernel_shakhov(PlanView pv) {
  update_body<S, true, kCh>(pv);
}

// The update kernel's fill mode (any collision model: a ghost Maxwellian carries no Shakhov
// factor), launched with the workgroups of the update kernel.
template <typename S, int kCh>
__global__ __launch_bounds__(kWave* kQuads* kCh)
__attribute__((amdgpu_waves_per_eu(kUpdateWaves<S, false>)))
void ghost_fill_kernel(PlanView pv) {
  update_body<S, false, kCh, true>(pv);
}

}  // namespace

// ================================================================== launchers
// Moment-kernel workgroups that a solver's velocity chunks aim for: 3 per CU.
constexpr long long kFillWorkgroups = 256 * 3;

int velocity_chunks(int nx, int ny, int K, int NC) {
  const long long base = (long long)((nx + kTileU - 1) / kTileU) * ny * NC;
  long long G = kFillWorkgroups / base;
  const int half = K / 2;  // nodes of the smaller half of the u axis
  if (G > half) G = half;
  if (G > 16) G = 16;
  return G < 1 ? 1 : (int)G;
}

// Velocity chunks per quadrant of the update kernel, U, for `base` workgroups per chunk and
// `slots` workgroups that run at once.  The update kernel adds nothing across chunks, so its
// chunks do not change any result.
//
// A batch of instances (update_chunks): the fewest chunks whose workgroups fill every round of
// the slots that they start to at least 85%, and at least one full round; at most 16.
int update_chunks(long long base, long long slots) {
  for (int U = 1; U <= 16; ++U) {
    const long long n = base * U;
    const long long rounds = (n + slots - 1) / slots;
    if (n >= slots && n * 100 >= 85 * rounds * slots) return U;
  }
  return 16;
}

// One instance (update_chunks_single): U, at most `cap` and 16, that minimises
// rounds x (2 + u nodes per chunk / vs), with `per_wg` chunks to a workgroup over the `half`
// u nodes of the smaller half and the v range in `vs` chunks: a workgroup's fixed cost (its
// stage and Gauss starts) counts as two u nodes of a whole v half; of equal costs the most
// workgroups.  On the paper's meshes and the 400x100 channel it picks the fastest U of a
// sweep or one within 1% of it.
int update_chunks_single(long long base, long long slots, int cap, int per_wg, int half,
                         int vs) {
  int best = 1;
  long long best_cost = -1;
  for (int U = 1; U <= cap && U <= 16; ++U) {
    const long long rounds = (base * U + slots - 1) / slots;
    const long long chunks = (long long)per_wg * U;
    const long long cost = rounds * (2LL * vs + (half + chunks - 1) / chunks);
    if (best_cost < 0 || cost <= best_cost) {
      best = U;
      best_cost = cost;
    }
  }
  return best;
}

int update_vsplit(int nx, int ny, int K, int M, int NC, int fp32, int shak, int cap) {
  const long long base = (long long)((nx + kTileU - 1) / kTileU) * ((ny + 1) / 2) * NC;
  const int umax = std::max(1, std::min(K / 2, 16));
  // four-wavefront workgroups that run at once: 256 CUs x update waves per SIMD
  const long long slots = 256LL * (fp32 ? (shak ? kUpdateWaves<float, true>
                                                 : kUpdateWaves<float, false>)
                                         : kUpdateWaves<double, false>);
  if (2 * base * umax >= slots) return 1;
  int vs = (int)(slots / (base * umax));
  vs = std::min(vs, (M / 2) / 4);
  if (cap > 0) vs = std::min(vs, cap);
  return std::max(vs, 1);
}

size_t plan_bytes(int n) {
  const size_t inst = ((sizeof(Inst) * (size_t)n + 255) / 256) * 256;
  return inst + 6 * (((size_t)(n + 1) * sizeof(int) + 255) / 256) * 256;
}

PlanTotals build_plan(const Inst* insts, int n, void* buf, const void* dev, PlanView* view) {
  char* h = static_cast<char*>(buf);
  const char* d = static_cast<const char*>(dev);
  const size_t inst_bytes = ((sizeof(Inst) * (size_t)n + 255) / 256) * 256;
  const size_t off_bytes = (((size_t)(n + 1) * sizeof(int) + 255) / 256) * 256;
  std::memcpy(h, insts, sizeof(Inst) * (size_t)n);
  int* off[6];
  for (int a = 0; a < 6; ++a) off[a] = reinterpret_cast<int*>(h + inst_bytes + a * off_bytes);
  PlanTotals t{};
  // each instance keeps the velocity chunks it was created with, in any plan, so that its
  // sums are added in the same order whether it is stepped alone or in a batch
  Inst* img = reinterpret_cast<Inst*>(h);
  long long upd_base = 0;  // update workgroups of all instances with one chunk
  for (int q = 0; q < n; ++q) {
    const KParams& P = insts[q].P;
    upd_base += (long long)((P.nx + kTileU - 1) / kTileU) * ((P.ny + 1) / 2) * P.NC * P.vsplit;
  }
  // velocity chunks per update workgroup (FP64 two, FP32 storage one) and the workgroups
  // that run at once: 256 CUs x waves per CU / waves per workgroup
  const bool shak = n > 0 && insts[0].P.shak;
  const bool f32 = n > 0 && insts[0].fp32;
  const int waves = f32 ? (shak ? kUpdateWaves<float, true> : kUpdateWaves<float, false>)
                        : kUpdateWaves<double, false>;
  int per_wg = f32 ? 1 : 2;
  // each workgroup's chunks take at least one u node each of the smaller half
  auto cap_of = [&](const KParams& P, int ch) {
    const int c = P.K / 2 / ch;
    return c < 1 ? 1 : c;
  };
  auto choose = [&](int ch) {
    const long long slots = 256LL * waves / ch;
    if (n == 1)
      return update_chunks_single(upd_base, slots, cap_of(insts[0].P, ch), ch, insts[0].P.K / 2,
                                  insts[0].P.vsplit);
    return update_chunks(upd_base, slots);
  };
  int U = choose(per_wg);
  // a mesh that leaves more than half the CUs without a workgroup of two chunks takes one
  // chunk per workgroup: twice the workgroups, on twice the CUs
  if (per_wg == 2 && n == 1 && upd_base * U < 128) {
    per_wg = 1;
    U = choose(1);
  }
  t.upd_ch = per_wg;
  for (int q = 0; q < n; ++q) {
    img[q].gsplit = insts[q].P.gmax;
    const int cap = cap_of(insts[q].P, per_wg);
    img[q].usplit = U < cap ? U : cap;
  }
  for (int q = 0; q < n; ++q) {
    const KParams& P = insts[q].P;
    const int G = img[q].gsplit * P.NC;  // chunks of G, then those of H
    const int nf = P.ny * (P.nx + 1) + (P.ny + 1) * P.nx;
    off[0][q] = t.sums;
    off[1][q] = t.upd;
    off[2][q] = t.face;
    off[3][q] = t.ghost;
    off[4][q] = t.red;
    off[5][q] = 0;
    if (G > 1)  // the per-cell sums, and a channel's ghost sums
      t.red += (int)(((long long)P.nslot * P.nx * P.ny +
                      (P.bc == UGKS_BC_CHANNEL ? 2LL * P.ny * kGhostSums : 0) + 255) /
                     256);
    t.shak = t.shak || P.shak;
    t.sums += ((P.nx + kTileS - 1) / kTileS) * P.ny * G;
    t.upd += ((P.nx + kTileU - 1) / kTileU) * ((P.ny + 1) / 2) * img[q].usplit * P.vsplit * P.NC;
    t.face += (nf + 255) / 256;
    if (P.bc == UGKS_BC_CHANNEL) {
      t.channel = 1;
    } else {
      t.periodic = 1;
      const long long frame = (long long)P.Lx * P.Ly - (long long)P.nx * P.ny;
      t.ghost += (int)((frame * P.NV * P.NC + kGhostThreads - 1) / kGhostThreads);
    }
  }
  off[0][n] = t.sums;
  off[1][n] = t.upd;
  off[2][n] = t.face;
  off[3][n] = t.ghost;
  off[4][n] = t.red;
  off[5][n] = 0;
  view->inst = reinterpret_cast<const Inst*>(d);
  view->off_sums = reinterpret_cast<const int*>(d + inst_bytes + 0 * off_bytes);
  view->off_upd = reinterpret_cast<const int*>(d + inst_bytes + 1 * off_bytes);
  view->off_face = reinterpret_cast<const int*>(d + inst_bytes + 2 * off_bytes);
  view->off_ghost = reinterpret_cast<const int*>(d + inst_bytes + 3 * off_bytes);
  view->off_red = reinterpret_cast<const int*>(d + inst_bytes + 4 * off_bytes);
  view->ninst = n;
  view->step = 0;
  return t;
}

hipError_t launch_poison(const PlanView& pv, int fp32, long long nvalues, hipStream_t s) {
  const unsigned blocks = (unsigned)((nvalues + 255) / 256);
  if (fp32)
    poison_kernel<float><<<blocks, 256, 0, s>>>(pv);
  else
    poison_kernel<double><<<blocks, 256, 0, s>>>(pv);
  return hipGetLastError();
}

hipError_t launch_init(const PlanView& pv, int fp32, long long nvalues, hipStream_t s) {
  const unsigned blocks = (unsigned)((nvalues + 255) / 256);
  if (fp32)
    init_kernel<float><<<blocks, 256, 0, s>>>(pv);
  else
    init_kernel<double><<<blocks, 256, 0, s>>>(pv);
  return hipGetLastError();
}

// phase 0 ghosts, 1 moment sums, 2 interface scalars, 3 cell update
hipError_t launch_ghost_fill(const PlanView& pv, const PlanTotals& t, int fp32, hipStream_t s) {
  if (!t.channel) return hipSuccess;
  const unsigned nt = (unsigned)(kWave * kQuads * t.upd_ch);
  if (fp32)
    ghost_fill_kernel<float, 1><<<(unsigned)t.upd, nt, 0, s>>>(pv);
  else if (t.upd_ch == 2)
    ghost_fill_kernel<double, 2><<<(unsigned)t.upd, nt, 0, s>>>(pv);
  else
    ghost_fill_kernel<double, 1><<<(unsigned)t.upd, nt, 0, s>>>(pv);
  return hipGetLastError();
}

hipError_t launch_phase(const PlanView& pv, const PlanTotals& t, int fp32, int phase,
                        hipStream_t s) {
  switch (phase) {
    case 0:
      if (t.ghost == 0) return hipSuccess;  // no periodic instance
      if (fp32)
        ghost_kernel<float><<<(unsigned)t.ghost, kGhostThreads, 0, s>>>(pv);
      else
        ghost_kernel<double><<<(unsigned)t.ghost, kGhostThreads, 0, s>>>(pv);
      break;
    case 1:
      if (t.shak) {
        if (fp32)
          sums_kernel<float, true><<<(unsigned)t.sums, kWave * kQuads, 0, s>>>(pv);
        else
          sums_kernel<double, true><<<(unsigned)t.sums, kWave * kQuads, 0, s>>>(pv);
      } else {
        if (fp32)
          sums_kernel<float, false><<<(unsigned)t.sums, kWave * kQuads, 0, s>>>(pv);
        else
          sums_kernel<double, false><<<(unsigned)t.sums, kWave * kQuads, 0, s>>>(pv);
      }
      if (t.red > 0) {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        chunk_sum_kernel<<<(unsigned)t.red, 256, 0, s>>>(pv);
      }
      break;
    case 2:
      faces_kernel<<<(unsigned)t.face, 256, 0, s>>>(pv);
      break;
    default: {
      // FP32 storage runs one chunk per workgroup (build_plan never asks for two)
      const unsigned nt = (unsigned)(kWave * kQuads * t.upd_ch);
      if (t.shak) {
        if (fp32)
          update_kernel_shakhov<float, 1><<<(unsigned)t.upd, nt, 0, s>>>(pv);
        else if (t.upd_ch == 2)
          update_kernel_shakhov<double, 2><<<(unsigned)t.upd, nt, 0, s>>>(pv);
        else
          update_kernel_shakhov<double, 1><<<(unsigned)t.upd, nt, 0, s>>>(pv);
      } else {
        if (fp32)
          update_kernel<float, 1><<<(unsigned)t.upd, nt, 0, s>>>(pv);
        else if (t.upd_ch == 2)
          update_kernel<double, 2><<<(unsigned)t.upd, nt, 0, s>>>(pv);
        else
          update_kernel<double, 1><<<(unsigned)t.upd, nt, 0, s>>>(pv);
      }
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
