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
template <typename T>
inline UGKS_GLOBAL T* gp(T* p) {
  return (UGKS_GLOBAL T*)p;
}

constexpr int kWave = 64;      // CDNA wavefront
constexpr int kSlots = 64;     // per-cell outgoing moment sums: 4 faces x 16
constexpr int kRec = 32;       // doubles per interface record
// nu + nv limit: the update kernel keeps 13 (nu + 1) + 13 (nv + 1) doubles of tables per cell
// and nu + nv + 2 node values in LDS, which must fit one 64 KB workgroup
constexpr int kMaxTable = 582;

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

struct KParams {
  int nx, ny, K, M, NV, NVP;
  int bc, collisionless, inlet_fixed_u, pad0;
  double dx, dy, dt, inv_dx, inv_dy, area, mu_ref;
  double p_in, p_out, T_in, lam_w;
  double U_in, U_noise;
  double wall_den_bot, wall_den_top;  // sum over wall-leaving velocities of w v g_w
  double wall_G_bot[4], wall_G_top[4];  // sum of w v psi_local g_w over the same velocities
  const UGKS_GLOBAL double* U;     // [NVP] u of each velocity slot (0 in pads)
  const UGKS_GLOBAL double* V;     // [NVP]
  const UGKS_GLOBAL double* Wq;    // [NVP] quadrature weight (0 in pads)
  const UGKS_GLOBAL int* km;       // [NVP] k | m << 16 of each velocity slot (K | M << 16 in pads)
  const UGKS_GLOBAL int* chunk_sign;  // [NVP/64] per 64-slot chunk: bit0/1 all u > 0 / < 0,
                                      // bit2/3 the same for v
  const UGKS_GLOBAL double* uk;    // [K]
  const UGKS_GLOBAL double* vm;    // [M]
  const UGKS_GLOBAL double* wk;    // [K] weights of the u nodes
  const UGKS_GLOBAL double* wm;    // [M] weights of the v nodes
  const UGKS_GLOBAL double* xi_in;  // [ny] inlet noise
  UGKS_GLOBAL int* flag;           // device flag: set to 1 on an invalid state
};

// Device buffers carved out of one workspace.
struct Buffers {
  void* f[2];       // [nx*ny][NVP] storage type
  double* W;        // [nx*ny][4]
  double* Wg;       // [2][ny][4]
  void* fg;         // [2][ny][NVP] storage type
  double* hs;       // [nx*ny][64]
  double* hsg;      // [2][ny][16]
  double* recx;     // [ny][nx+1][32]
  double* recy;     // [ny+1][nx][32]
  double* U;        // [NVP]
  double* V;
  double* Wq;
  int* km;          // [NVP]
  double* wk;       // [K], followed by wm [M]
  int* chunk_sign;  // [NVP/64]
  double* uk;       // [K]
  double* vm;       // [M]
  double* xi_in;    // [ny]
  int* flag;
};

struct Layout {
  size_t off[19];
  size_t total;
};

// One solver instance as the kernels see it: constants, buffers, and which f buffer holds the
// state when the launch sequence's step counter is 0.
struct Inst {
  KParams P;
  UGKS_GLOBAL void* f[2];
  UGKS_GLOBAL double* W;
  UGKS_GLOBAL double* Wg;
  UGKS_GLOBAL void* fg;
  UGKS_GLOBAL double* hs;
  UGKS_GLOBAL double* hsg;
  UGKS_GLOBAL double* recx;
  UGKS_GLOBAL double* recy;
  int cur;   // f[(cur + step) & 1] is read, the other buffer written
  int fp32;  // storage type of f
};

// A launch plan: instances plus, per kernel, the prefix sum of the workgroups each instance
// takes, so that one launch per phase covers every instance (instance search is uniform per
// workgroup).  Device-resident; the kernels read it through PlanView.
struct PlanView {
  const Inst* inst;
  const int* off_sums;   // kCellsPerBlock cells per workgroup
  const int* off_upd;    // cpb_upd cells per workgroup
  const int* off_face;   // 256 faces per workgroup
  const int* off_ghost;  // 2 ny workgroups for a channel, 0 for a periodic box
  int ninst;
  int step;              // steps enqueued since the plan's `cur` values were taken
  int cpb_upd;
  int lds_per_cell;      // bytes of update-kernel LDS per cell
};

struct PlanTotals {
  int sums, upd, face, ghost;  // workgroups of each launch
  int cpb_upd;
  int lds_per_cell;
  int lds_upd, lds_sums;       // bytes of dynamic LDS per workgroup
};

// Bytes of a device plan with n instances, and its host image (offsets into one buffer).
size_t plan_bytes(int n);
// Build the host image of a plan for `n` instances into `buf` (plan_bytes(n) bytes) and return
// the totals; `dev` is the device address the image will be copied to.
PlanTotals build_plan(const Inst* insts, int n, void* buf, const void* dev, PlanView* view);

// Launchers (ugks_kernels.hip).  All enqueue on `s` and return the launch error.
hipError_t launch_init(const PlanView& pv, int fp32, int ncells, hipStream_t s);
hipError_t launch_step(const PlanView& pv, const PlanTotals& t, int fp32, hipStream_t s,
                       hipEvent_t* ev /* 8 events or NULL */);
hipError_t launch_phase(const PlanView& pv, const PlanTotals& t, int fp32, int phase,
                        hipStream_t s);

}  // namespace ugks
