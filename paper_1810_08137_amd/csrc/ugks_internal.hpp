// Internal declarations shared by the host library and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "ugks.h"

namespace ugks {

// Device buffers are declared in the global address space, so that pointers the kernels read
// from a launch plan still compile to global (scalar-base) loads rather than flat ones.
#define UGKS_GLOBAL __attribute__((address_space(1)))
// Tables that no kernel writes while another reads them (velocity nodes, weights), read at a
// wavefront-uniform address through the constant address space: scalar loads, counted apart
// from the vector loads of f, so waiting for a table value never waits for f loads in flight.
#define UGKS_CONST __attribute__((address_space(4)))
template <typename T>
inline UGKS_GLOBAL T* gp(T* p) {
  return (UGKS_GLOBAL T*)p;
}

constexpr int kWave = 64;      // CDNA wavefront
constexpr int kSlots = 64;     // per-cell outgoing moment sums: 4 faces x 16
// Shakhov model: after the 64 sums, one more per face side (sum of ut (un^2 + ut^2)/2 f_hat, for
// the interface heat flux) and eight raw moments of the cell's f (sum of f, u f, v f, u^2 f,
// u v f, v^2 f, u |c|^2 f, v |c|^2 f with |c|^2 = u^2 + v^2) for its heat flux
constexpr int kSlotHeat = 64;
constexpr int kSlotCell = 68;
constexpr int kSlotsShakhov = 76;
constexpr int kGhostSums = 17;  // sums of a channel ghost cell towards the domain: 16 + the heat sum
constexpr int kRec = 32;       // doubles per interface record
constexpr int kHalo = 2;       // halo columns / rows on each side of a velocity plane
constexpr int kMaxNodes = 1024;  // nodes per velocity axis

// Interface record (doubles), written by the interface kernel, read by the cell update.
// Frame: "normal"/"tangential" velocity of the face; for x-faces (u, v), for y-faces (v, u).
// The time-integrated distribution flux of one velocity is
//   un * ( GC Ek[k] Em[m] P(un, ut) + M4 fhat - M5 (un sn + ut st) )
// with P(un, ut) = e0 + e3 c2h + un (e1 + e4 un + e5 ut + e7 c2h) + ut (e2 + e6 ut + e8 c2h),
// c2h = (un^2 + ut^2)/2: the time weights Mt1..Mt3 and the slopes a, b, A of S4 folded into
// nine coefficients (e1, e4, e5, e7 depend on the side the particle comes from).
enum RecField {
  R_FX = 0,     // [0..3] macroscopic flux, global frame (rho, rho U, rho V, rho E)
  R_GC = 4,     // len * rho0 lambda0 / pi (interior); len * dt * rho_w lambda_w / pi (wall)
  R_LAM = 5,    // lambda of the interface (or wall) Maxwellian
  R_UX = 6,     // its velocity, global x component
  R_VY = 7,     // its velocity, global y component
  R_E = 8,      // [8..16] e0..e8 for un > 0 (normal slope aL)
  R_ER = 17,    // [17..20] e1, e4, e5, e7 for un < 0 (normal slope aR)
  R_M4 = 21,    // len * Mt4 (wall: len * dt)
  R_M5 = 22,    // len * Mt5 (wall: 0)
  R_KIND = 23,  // 0 interior, 1 wall, 2 collisionless interior
};
enum FaceKind { K_INTERIOR = 0, K_WALL = 1, K_FREE = 2 };

// Slot layout of the outgoing sums of one cell: face f in {+x, -x, +y, -y} at 16*f, each
// [W0(4), Wt(4), Q1(4), Q2(4)] in the local frame of that face.
enum FaceSide { S_XP = 0, S_XM = 1, S_YP = 2, S_YM = 3 };

// f is stored velocity-major: plane p = k M + m holds f(u_k, v_m) of every cell, laid out as
// (ny + 4) rows of Lx = nx + 4 values (cell (i, j) at (j + 2) Lx + i + 2), with two halo
// columns and rows on each side; planes are PS values apart.  With internal degrees of
// freedom the NV planes of H (the distribution's internal energy) follow those of G.
struct KParams {
  int nx, ny, K, M, NV;
  int NC;           // reduced distributions: 1 (G), or 2 (G, H) with internal degrees of freedom
  int dof;          // internal degrees of freedom
  double lam_c;     // (2 + dof)/4: lambda = lam_c rho / (rho E - rho |U|^2/2)
  double q_c;       // (2 + dof)/2: the energy row of the micro-slope solve, q2 = |U|^2 + q_c/lambda
  double a4_c;      // 4/(2 + dof): its energy coefficient, a4 = a4_c lambda^2/rho (...)
  int shak;         // Shakhov collision model (else BGK)
  int nslot;        // per-cell sums per velocity chunk: kSlots, or kSlotsShakhov
  double pr_c;      // 1 - Prandtl number (Shakhov)
  int Lx, Ly;       // padded row length and row count of a plane
  int bc, collisionless, inlet_fixed_u;
  int gmax;         // velocity chunks per quadrant the moment-sum buffer has room for
  int vsplit;       // v-range chunks per half of the update kernel, fixed at create: each
                    // chunk starts its Gauss recurrences at its own first node, so the count
                    // decides the rounding and is kept in every launch plan
  long long PS;     // values per plane
  double dx, dy, dt, inv_dx, inv_dy, area, mu_ref;
  double du, dv;    // node spacing of the uniform u and v grids
  double p_in, p_out, T_in, lam_w;
  double kap_w;     // H / G of the wall Maxwellian: dof/(2 lambda_w)
  double U_in, U_noise;
  double wall_den_bot, wall_den_top;  // sum over wall-leaving velocities of w v g_w
  double wall_G_bot[4], wall_G_top[4];  // sum of w v psi_local g_w over the same velocities
                                        // (energy: with the wall's H)
  const UGKS_GLOBAL double* uk;    // [K]
  const UGKS_GLOBAL double* vm;    // [M], with one zero before and after (vm[-1], vm[M])
  const UGKS_GLOBAL double* wk;    // [K] weights of the u nodes
  const UGKS_GLOBAL double* wm;    // [M] weights of the v nodes
  const UGKS_GLOBAL double* vmom;  // [M][5] w_m v_m^n (n = 0..4), halved at v_m = 0
  const UGKS_GLOBAL double* xi_in;  // [ny] inlet noise
  UGKS_GLOBAL int* flag;           // device flag: set to 1 on an invalid state
  // adaptive step: dt^n = cfl / rmax[n & 1], rmax the largest (umax + |U|)/dx + (vmax + |V|)/dy
  // over the cells of W^n, kept as the bits of a non-negative double (ordered like the
  // integers, so an integer atomic max is the max of the doubles)
  int adaptive;
  double cfl, umax, vmax;
  UGKS_GLOBAL unsigned long long* rmax;  // [2]
  UGKS_GLOBAL double* tsum;              // simulated time: the sum of the steps taken
};

// Device buffers carved out of one workspace.
struct Buffers {
  void* f[2];       // [NC NV][PS] storage type
  double* W[2];     // [nx*ny][4], ping-pong with f
  double* Wg;       // [2][ny][4]
  double* hs;       // [NC gmax][nslot][nx*ny]: partial g of sum q of face side s of cell c at
                    // ((g nslot) + 16 s + q) nx ny + c; chunks of H after those of G
  double* hsg;      // [NC G][2][ny][kGhostSums]: the chunks' parts, added into the first
  double* recx;     // [NC][32][ny (nx+1)]: records of G, then of H, field-major
  double* recy;     // [NC][32][(ny+1) nx]
  double* wk;       // [K], followed by wm [M], then vmom [M][5]
  double* uk;       // [K]
  double* vm;       // [M + 2]: zero, the M nodes, zero
  double* xi_in;    // [ny]
  int* flag;
  unsigned long long* rmax;  // [2] (adaptive step)
  double* tsum;              // simulated time
};

struct Layout {
  size_t off[15];
  size_t total;
};

// One solver instance as the kernels see it: constants, buffers, and which f buffer holds the
// state when the launch sequence's step counter is 0.
struct Inst {
  KParams P;
  UGKS_GLOBAL void* f[2];
  UGKS_GLOBAL double* W[2];
  UGKS_GLOBAL double* Wg;
  UGKS_GLOBAL double* hs;
  UGKS_GLOBAL double* hsg;
  UGKS_GLOBAL double* recx;
  UGKS_GLOBAL double* recy;
  int cur;   // f[(cur + step) & 1] and W[(cur + step) & 1] are read, the others written
  int fp32;  // storage type of f
  int gsplit;  // velocity chunks per quadrant and reduced distribution of the moment kernel
               // (P.gmax; set by build_plan); a segment has NC gsplit workgroups, those of H
               // after those of G
  int usplit;  // the same for the update kernel (set by build_plan for the whole launch)
};

// A launch plan: instances plus, per kernel, the prefix sum of the workgroups each instance
// takes, so that one launch per phase covers every instance (instance search is uniform per
// workgroup).  Device-resident; the kernels read it through PlanView.
struct PlanView {
  const Inst* inst;
  const int* off_sums;   // one workgroup per (row segment, velocity chunk) of the moment kernel
  const int* off_upd;    // one workgroup per (row segment, velocity chunk) of the update kernel
  const int* off_face;   // 256 faces per workgroup
  const int* off_ghost;  // periodic: the halo frame of every plane (a channel has none)
  const int* off_red;    // chunk-sum workgroups (instances with more than one chunk)
  int ninst;
  int step;              // steps enqueued since the plan's `cur` values were taken
};

struct PlanTotals {
  int sums, upd, face, ghost;  // workgroups of each launch
  int red;                     // workgroups of the chunk-sum launch (0: not launched)
  int shak;                    // the instances use the Shakhov model (all or none)
  int upd_ch;                  // velocity chunks per update workgroup (1 or 2)
  int periodic;                // some instance has a periodic halo (the ghost kernel runs)
  int channel;                 // some instance is a channel (ghost columns from the update)
};

// Bytes of a device plan with n instances, and its host image (offsets into one buffer).
size_t plan_bytes(int n);
// Velocity chunks per quadrant of an instance: enough update workgroups to fill the GPU
// when the instance runs alone (NC reduced distributions each take their own chunks), at
// least one u node per chunk and at most 16 chunks.
int velocity_chunks(int nx, int ny, int K, int NC);
// v-range chunks per half of the update kernel for a solver: 1 unless its update workgroups,
// with the u ranges split as far as they go, would leave more than half the GPU idle; then as
// many as fill it, each chunk at least four v nodes of the smaller half, at most `cap` (> 0).
int update_vsplit(int nx, int ny, int K, int M, int NC, int fp32, int shak, int cap);
// Build the host image of a plan for `n` instances into `buf` (plan_bytes(n) bytes) and return
// the totals; `dev` is the device address the image will be copied to.
PlanTotals build_plan(const Inst* insts, int n, void* buf, const void* dev, PlanView* view);

// Launchers (ugks_kernels.hip).  All enqueue on `s` and return the launch error.
hipError_t launch_init(const PlanView& pv, int fp32, long long nvalues, hipStream_t s);
// Debug: NaN into every cell value of the f and W buffers the next step writes.
hipError_t launch_poison(const PlanView& pv, int fp32, long long nvalues, hipStream_t s);
// Fill the channel ghost columns of the current f and the ghost states Wg from the current W
// (after the initial state and after ugks_set_state; the update kernel writes those of the
// next step in every step), with the update kernel's own arithmetic.
hipError_t launch_ghost_fill(const PlanView& pv, const PlanTotals& t, int fp32, hipStream_t s);
hipError_t launch_step(const PlanView& pv, const PlanTotals& t, int fp32, hipStream_t s,
                       hipEvent_t* ev /* 8 events or NULL */);
hipError_t launch_phase(const PlanView& pv, const PlanTotals& t, int fp32, int phase,
                        hipStream_t s);

}  // namespace ugks
