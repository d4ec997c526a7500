// Host side of the C ABI declared in include/ugks.h: argument checks, the velocity grid and
// boundary constants, one device workspace carved into all buffers, and the per-step launch
// sequence on the caller's stream.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ugks_internal.hpp"

using namespace ugks;

struct ugks_batch {
  hipStream_t stream = nullptr;
  int cap = 0;
  int fp32 = 0;
  void* plan_dev = nullptr;   // device plan of up to cap instances
  void* plan_host = nullptr;  // pinned staging of the same size
  hipEvent_t uploaded = nullptr;
  bool upload_pending = false;
  std::vector<uint64_t> members;      // ids of the handles of the current plan, in order
  std::vector<int64_t> base_steps;     // their step counts when the plan was built
  int64_t counter = 0;                 // steps enqueued with the current plan
  PlanView pv{};
  PlanTotals pt{};
  std::string err;
};

static std::atomic<uint64_t> g_next_handle_id{1};

struct ugks_handle {
  uint64_t uid = g_next_handle_id.fetch_add(1);  // never reused, unlike the address
  KParams P{};
  int prec = 0;
  size_t ssize = 8;
  hipStream_t stream = nullptr;
  int device = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool owns_ws = false;
  Buffers B{};
  Inst inst{};       // this solver as the kernels see it (cur = 0: f[steps & 1] is current)
  void* plan_dev = nullptr;  // its one-instance launch plan, inside the workspace
  PlanView pv{};
  PlanTotals pt{};
  // ugks_step_static: a second one-instance plan (also inside the workspace) whose transient
  // buffers are the device's static scratch array; built at create when they fit
  void* plan_static = nullptr;
  PlanView pv_static{};
  bool static_ok = false;
  std::string static_why;    // why not, when static_ok is false
  bool last_static = false;  // the last step ran on the static scratch
  int moment_chunks = 1, update_chunks = 1, update_ch = 1;  // the plan's choices (ugks_info)
  int64_t steps = 0;
  double tau_ref = 0.0;
  std::string err;
  std::atomic<int> busy{0};
  // a launch failed part-way through a step: the device state is unknown (which f/W buffer
  // is current cannot be trusted), so every later call except destroy returns UGKS_E_DEVICE
  bool poisoned = false;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> pool;
  struct Pending {
    int kernel;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  double total_ms[4] = {0, 0, 0, 0};
  int64_t launches[4] = {0, 0, 0, 0};
};

namespace {

thread_local char g_create_error[512] = "";

constexpr size_t kAlign = 256;
constexpr double kPiHost = 3.14159265358979323846;

// Static scratch of ugks_step_static: the transient buffers of one step (ghost states,
// per-cell moment sums, face records) of whichever handle that call steps.  One copy per GPU,
// held from the library's first use on that GPU until the process ends.  Host code never
// passes this name to a kernel or a copy: it is a host-side stand-in for the device array,
// whose address on each device comes from hipGetSymbolAddress (scratch_address).
constexpr size_t kStaticScratchBytes = (size_t)48 << 20;
static_assert(kStaticScratchBytes == UGKS_STATIC_SCRATCH_BYTES, "header and library disagree");
__device__ __align__(256) static unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the static scratch on `device`, which must be the current device; looked
// up once per device.  nullptr (and a message) if the lookup fails.
void* scratch_address(int device, std::string& why) {
  if (device < 0 || device >= kMaxDevices) {
    why = "device index beyond the static scratch table";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      why = std::string("hipGetSymbolAddress of the static scratch: ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int fail(ugks_handle* h, int code, const char* fmt, const char* detail = "") {
  char buf[512];
  std::snprintf(buf, sizeof buf, fmt, detail);
  if (h)
    h->err = buf;
  else
    std::memcpy(g_create_error, buf, sizeof buf);
  return code;
}

// Position of cell c = j nx + i inside a velocity plane.
size_t plane_index(const KParams& P, size_t c) {
  const size_t j = c / (size_t)P.nx, i = c - j * (size_t)P.nx;
  return (j + kHalo) * (size_t)P.Lx + i + kHalo;
}

int hip_fail(ugks_handle* h, hipError_t e, const char* what) {
  char buf[512];
  std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
  if (h)
    h->err = buf;
  else
    std::memcpy(g_create_error, buf, sizeof buf);
  return UGKS_E_DEVICE;
}

int poisoned_fail(ugks_handle* h) {
  return fail(h, UGKS_E_DEVICE,
              "a kernel launch failed part-way through a step; the state is unknown%s");
}

struct Busy {
  ugks_handle* h;
  bool ok;
  explicit Busy(ugks_handle* hh) : h(hh) {
    int z = 0;
    ok = h->busy.compare_exchange_strong(z, 1);
  }
  ~Busy() {
    if (ok) h->busy.store(0);
  }
};

// Uniform nodes on [-a, a] with both ends, made exactly mirror-symmetric; trapezoid weights.
void velocity_nodes(int n, double a, double* x, double* w) {
  const double h = 2.0 * a / (double)(n - 1);
  for (int k = 0; k < n; ++k) x[k] = -a + (double)k * h;
  for (int k = 0; k < n / 2; ++k) x[n - 1 - k] = -x[k];
  if (n & 1) x[n / 2] = 0.0;
  for (int k = 0; k < n; ++k) w[k] = (k == 0 || k == n - 1) ? 0.5 * h : h;
}

// SplitMix64, counter form: output k of the generator seeded with s.
uint64_t splitmix(uint64_t s, uint64_t k) {
  uint64_t z = s + (k + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double noise_unit(uint64_t s, uint64_t k) {
  return 2.0 * ((double)(splitmix(s, k) >> 11) * 0x1.0p-53) - 1.0;
}

struct Shape {
  int nx, ny, K, M, NV;
  int dof, NC;  // internal degrees of freedom; reduced distributions per velocity
  int Lx, Ly;
  size_t PS;  // values per velocity plane
  size_t nc;
};

bool shape_ok(const ugks_mesh* mesh, const ugks_vgrid* vg, Shape& s, std::string& why) {
  if (!mesh || !vg) {
    why = "mesh and vgrid are required";
    return false;
  }
  if (mesh->nx < 1 || mesh->ny < 1) {
    why = "nx and ny must be >= 1";
    return false;
  }
  if (!(mesh->lx > 0) || !(mesh->ly > 0) || !std::isfinite(mesh->lx) || !std::isfinite(mesh->ly)) {
    why = "lx and ly must be positive and finite";
    return false;
  }
  if (vg->nu < 2 || vg->nv < 2) {
    why = "nu and nv must be >= 2";
    return false;
  }
  if (vg->nu > kMaxNodes || vg->nv > kMaxNodes) {
    why = "nu and nv must be <= 1024";
    return false;
  }
  if (!(vg->umax > 0) || !(vg->vmax > 0) || !std::isfinite(vg->umax) || !std::isfinite(vg->vmax)) {
    why = "umax and vmax must be positive and finite";
    return false;
  }
  if (vg->internal_dof < 0 || vg->internal_dof > 16) {
    why = "internal_dof must be in 0..16";
    return false;
  }
  // the kernels address a plane (cells and halo) with 32-bit byte offsets
  if (((double)mesh->nx + 2 * kHalo) * ((double)mesh->ny + 2 * kHalo) > (double)(1 << 28)) {
    why = "too many cells: (nx + 4)(ny + 4) must not exceed 2^28";
    return false;
  }
  s.nx = mesh->nx;
  s.ny = mesh->ny;
  s.K = vg->nu;
  s.M = vg->nv;
  s.NV = vg->nu * vg->nv;
  s.dof = vg->internal_dof;
  s.NC = s.dof > 0 ? 2 : 1;
  s.Lx = s.nx + 2 * kHalo;
  s.Ly = s.ny + 2 * kHalo;
  s.PS = round_up((size_t)s.Lx * (size_t)s.Ly, (size_t)kWave);
  s.nc = (size_t)s.nx * s.ny;
  return true;
}

// Offsets of every buffer inside the workspace.
// Velocity chunks of a solver: the automatic choice, capped at the requested number.
int chunks_of(const Shape& s, int cap) {
  const int a = velocity_chunks(s.nx, s.ny, s.K, s.NC);
  return cap > 0 && cap < a ? cap : a;
}

// Collision model of the options: BGK for prandtl 0 or 1, Shakhov for 0 < prandtl < 1 (gas
// without internal degrees of freedom only).  false with a message otherwise.
bool collision_of(const ugks_opts* o, const Shape& s, bool& shak, std::string& why) {
  const double pr = o ? o->prandtl : 0.0;
  shak = false;
  if (pr == 0.0 || pr == 1.0) return true;
  if (!(pr > 0.0 && pr < 1.0)) {
    why = "prandtl must be 0, 1 (BGK) or in (0, 1) (Shakhov)";
    return false;
  }
  if (s.dof != 0) {
    why = "the Shakhov model needs internal_dof = 0";
    return false;
  }
  shak = true;
  return true;
}

Layout layout_of(const Shape& s, int prec, int chunks, bool shak) {
  const size_t ss = prec == UGKS_FP32_STORE ? 4 : 8;
  const size_t sizes[15] = {
      (size_t)s.NC * s.NV * s.PS * ss,          // f0: NC NV planes
      (size_t)s.NC * s.NV * s.PS * ss,          // f1
      s.nc * 4 * 8,                             // W0
      s.nc * 4 * 8,                             // W1
      2 * (size_t)s.ny * 4 * 8,                 // Wg
      (size_t)s.NC * chunks * s.nc * (shak ? kSlotsShakhov : kSlots) * 8,  // hs: partial sums
      (size_t)s.NC * chunks * 2 * s.ny * kGhostSums * 8,  // hsg: parts of the ghost sums
      (size_t)s.NC * s.ny * (s.nx + 1) * kRec * 8,  // recx
      (size_t)s.NC * (s.ny + 1) * s.nx * kRec * 8,  // recy
      (size_t)(s.K + 6 * s.M) * 8,              // wk, wm, vmom
      (size_t)s.K * 8,                          // uk
      (size_t)(s.M + 2) * 8,                    // vm, padded with a zero on each side
      (size_t)s.ny * 8 + 128,                   // xi_in, flag, rmax[2], tsum
      plan_bytes(1),                            // one-instance launch plan
      plan_bytes(1),                            // the same on the static scratch
  };
  Layout L{};
  size_t off = 0;
  for (int b = 0; b < 15; ++b) {
    L.off[b] = off;
    off += round_up(sizes[b], kAlign);
  }
  L.total = off;
  return L;
}

void carve(ugks_handle* h, const Layout& L, const Shape& s) {
  char* base = static_cast<char*>(h->ws);
  Buffers& B = h->B;
  B.f[0] = base + L.off[0];
  B.f[1] = base + L.off[1];
  B.W[0] = reinterpret_cast<double*>(base + L.off[2]);
  B.W[1] = reinterpret_cast<double*>(base + L.off[3]);
  B.Wg = reinterpret_cast<double*>(base + L.off[4]);
  B.hs = reinterpret_cast<double*>(base + L.off[5]);
  B.hsg = reinterpret_cast<double*>(base + L.off[6]);
  B.recx = reinterpret_cast<double*>(base + L.off[7]);
  B.recy = reinterpret_cast<double*>(base + L.off[8]);
  B.wk = reinterpret_cast<double*>(base + L.off[9]);
  B.uk = reinterpret_cast<double*>(base + L.off[10]);
  B.vm = reinterpret_cast<double*>(base + L.off[11]);
  B.xi_in = reinterpret_cast<double*>(base + L.off[12]);
  B.flag = reinterpret_cast<int*>(base + L.off[12] + round_up((size_t)s.ny * 8, 64));
  B.rmax = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(B.flag) + 64);
  B.tsum = reinterpret_cast<double*>(reinterpret_cast<char*>(B.flag) + 80);
  h->plan_dev = base + L.off[13];
  h->plan_static = base + L.off[14];
}

// The transient buffers of one step (hs, hsg, recx, recy: layout entries 5..8) are
// contiguous in the workspace; their size, and the same buffers carved out of `base`.  The
// ghost states Wg (entry 4) are not transient: the update kernel of a step writes those of
// the next.
size_t transient_bytes(const Layout& L) { return L.off[9] - L.off[5]; }
void carve_transient(const Layout& L, char* base, Inst& I) {
  I.hs = gp(reinterpret_cast<double*>(base + (L.off[5] - L.off[5])));
  I.hsg = gp(reinterpret_cast<double*>(base + (L.off[6] - L.off[5])));
  I.recx = gp(reinterpret_cast<double*>(base + (L.off[7] - L.off[5])));
  I.recy = gp(reinterpret_cast<double*>(base + (L.off[8] - L.off[5])));
}

hipEvent_t pool_get(ugks_handle* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Enqueue one step of a plan: four launches, each bracketed by timing events when enabled.
int enqueue_plan_step(ugks_handle* h, const PlanView& pv, const PlanTotals& pt, int fp32,
                      hipStream_t stream) {
  static const char* names[4] = {"ghost kernel launch", "moment kernel launch",
                                 "interface kernel launch", "update kernel launch"};
  for (int phase = 0; phase < 4; ++phase) {
    hipEvent_t a = nullptr, b = nullptr;
    const bool timed = h && h->timing && (phase != 0 || pt.ghost > 0);
    if (timed) {
      a = pool_get(h);
      b = pool_get(h);
      if (a) (void)hipEventRecord(a, stream);
    }
    const hipError_t e = launch_phase(pv, pt, fp32, phase, stream);
    if (timed) {
      if (b) (void)hipEventRecord(b, stream);
      if (a && b) h->pending.push_back({phase, a, b});
    }
    if (e != hipSuccess) return hip_fail(h, e, names[phase]);
  }
  return UGKS_OK;
}

int collect_timing(ugks_handle* h) {
  for (auto& p : h->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      h->total_ms[p.kernel] += ms;
      h->launches[p.kernel] += 1;
    }
    h->pool.push_back(p.a);
    h->pool.push_back(p.b);
  }
  h->pending.clear();
  return UGKS_OK;
}


// Every check of ugks_create's arguments; false with a message.
bool problem_ok(const ugks_mesh* mesh, const ugks_vgrid* vgrid, double kn, const ugks_bc* bc,
                const ugks_opts* opts, Shape& s, bool& shak, std::string& why) {
  if (!shape_ok(mesh, vgrid, s, why)) return false;
  why.clear();
  if (!bc || !opts)
    why = "bc and opts are required";
  else if (!(kn > 0))
    why = "kn must be > 0 (or +inf)";
  else if (bc->kind != UGKS_BC_PERIODIC && bc->kind != UGKS_BC_CHANNEL)
    why = "unknown boundary kind";
  else if (bc->kind == UGKS_BC_CHANNEL &&
           (!(bc->p_ratio > 0) || !(bc->T_in > 0) || !(bc->T_wall > 0) ||
            !std::isfinite(bc->p_ratio) || !std::isfinite(bc->T_in) || !std::isfinite(bc->T_wall)))
    why = "channel needs p_ratio, T_in, T_wall > 0";
  else if (opts->precision != UGKS_FP64 && opts->precision != UGKS_FP32_STORE)
    why = "unknown precision";
  else if (opts->velocity_chunks < 0 || opts->velocity_chunks > 16)
    why = "velocity_chunks must be in 0..16";
  else if (!(opts->rho0 > 0) || !(opts->T0 > 0) || !(std::fabs(opts->noise) < 1.0))
    why = "need rho0 > 0, T0 > 0, |noise| < 1";
  else if (!(opts->dt_override > 0) && !(opts->cfl > 0 && std::isfinite(opts->cfl)))
    why = "need cfl > 0 or dt_override > 0";
  else if (opts->adaptive_dt != 0 && (opts->adaptive_dt != 1 || opts->dt_override > 0))
    why = "adaptive_dt must be 0 or 1, and 1 needs dt_override = 0";
  if (!why.empty()) return false;
  return collision_of(opts, s, shak, why);
}

// Host copies of the velocity tables and the inlet noise.
struct HostTables {
  double uk[kMaxNodes], wk[kMaxNodes], vm[kMaxNodes], wm[kMaxNodes], vmom[5 * kMaxNodes];
  double vm_padded[kMaxNodes + 2];  // zero, vm[0..M), zero: the device copy of the v nodes
};

// Seeded inlet noise of row j (output nx*ny + j of the generator).
double inlet_noise(const ugks_opts* opts, const Shape& s, int j) {
  return noise_unit(opts->seed, s.nc + (uint64_t)j);
}

// The kernels' constants for a problem (everything of KParams but the device pointers), and
// the tables the device copies of which the pointers will address.
void fill_constants(const ugks_mesh* mesh, const ugks_vgrid* vgrid, double kn, const ugks_bc* bc,
                    const ugks_opts* opts, const Shape& s, bool shak, int chunks, KParams& P,
                    HostTables& T) {
  P.nx = s.nx;
  P.ny = s.ny;
  P.K = s.K;
  P.M = s.M;
  P.NV = s.NV;
  P.NC = s.NC;
  P.dof = s.dof;
  P.lam_c = 0.25 * (double)(2 + s.dof);
  P.q_c = 0.5 * (double)(2 + s.dof);
  P.a4_c = 4.0 / (double)(2 + s.dof);
  P.shak = shak ? 1 : 0;
  P.nslot = shak ? kSlotsShakhov : kSlots;
  P.pr_c = shak ? 1.0 - opts->prandtl : 0.0;
  P.Lx = s.Lx;
  P.Ly = s.Ly;
  P.gmax = chunks;
  P.vsplit = update_vsplit(s.nx, s.ny, s.K, s.M, s.NC, opts->precision == UGKS_FP32_STORE ? 1 : 0,
                           shak ? 1 : 0, opts->velocity_chunks);
  P.PS = (long long)s.PS;
  P.bc = bc->kind;
  P.collisionless = std::isinf(kn) ? 1 : 0;
  P.inlet_fixed_u = bc->inlet_fixed_u ? 1 : 0;
  P.dx = mesh->lx / s.nx;
  P.dy = mesh->ly / s.ny;
  P.dt = opts->dt_override > 0 ? opts->dt_override
                               : opts->cfl / (vgrid->umax / P.dx + vgrid->vmax / P.dy);
  P.inv_dx = 1.0 / P.dx;
  P.inv_dy = 1.0 / P.dy;
  P.area = P.dx * P.dy;
  P.mu_ref = P.collisionless ? 0.0 : 5.0 * std::sqrt(kPiHost) * kn / 16.0;
  const double p0 = 0.5 * opts->rho0 * opts->T0;
  const double r = bc->kind == UGKS_BC_CHANNEL ? bc->p_ratio : 1.0;
  P.p_in = 2.0 * r * p0 / (r + 1.0);
  P.p_out = 2.0 * p0 / (r + 1.0);
  P.T_in = bc->kind == UGKS_BC_CHANNEL ? bc->T_in : 1.0;
  const double Tw = bc->kind == UGKS_BC_CHANNEL ? bc->T_wall : 1.0;
  P.lam_w = 1.0 / Tw;
  P.kap_w = (double)s.dof / (2.0 * P.lam_w);
  P.U_in = bc->U_in;
  P.U_noise = bc->U_noise;
  P.adaptive = opts->adaptive_dt ? 1 : 0;
  P.cfl = opts->cfl;
  P.umax = vgrid->umax;
  P.vmax = vgrid->vmax;

  const double* uk = T.uk;
  const double* wk = T.wk;
  const double* vm = T.vm;
  const double* wm = T.wm;
  velocity_nodes(s.K, vgrid->umax, T.uk, T.wk);
  velocity_nodes(s.M, vgrid->vmax, T.vm, T.wm);
  T.vm_padded[0] = 0.0;
  for (int m = 0; m < s.M; ++m) T.vm_padded[m + 1] = T.vm[m];
  T.vm_padded[s.M + 1] = 0.0;
  P.du = 2.0 * vgrid->umax / (double)(s.K - 1);
  P.dv = 2.0 * vgrid->vmax / (double)(s.M - 1);
  // diffuse-wall constants: moments of the unit-density wall Maxwellian over the velocities
  // that leave each wall, in the wall's local frame (v, u)
  P.wall_den_bot = P.wall_den_top = 0.0;
  for (int q = 0; q < 4; ++q) P.wall_G_bot[q] = P.wall_G_top[q] = 0.0;
  for (int k = 0; k < s.K; ++k)
    for (int m = 0; m < s.M; ++m) {
      const double u = uk[k], v = vm[m], w = wk[k] * wm[m];
      const double gw = P.lam_w / kPiHost * std::exp(-P.lam_w * (u * u + v * v));
      const double psi[4] = {1.0, v, u, 0.5 * (u * u + v * v)};
      if (v > 0) {
        P.wall_den_bot += w * v * gw;
        for (int q = 0; q < 4; ++q) P.wall_G_bot[q] += w * v * psi[q] * gw;
      } else if (v < 0) {
        P.wall_den_top += w * v * gw;
        for (int q = 0; q < 4; ++q) P.wall_G_top[q] += w * v * psi[q] * gw;
      }
    }
  // the wall's H (kap_w times its G) carries energy: psi = (0, 0, 0, 1/2)
  P.wall_G_bot[3] += 0.5 * P.kap_w * P.wall_den_bot;
  P.wall_G_top[3] += 0.5 * P.kap_w * P.wall_den_top;
  // moment-kernel weights w_m v_m^n; a node at v = 0 is visited by both halves of v
  for (int m = 0; m < s.M; ++m) {
    double w = wm[m] * (vm[m] == 0.0 ? 0.5 : 1.0);
    for (int n = 0; n < 5; ++n) {
      T.vmom[5 * (size_t)m + n] = w;
      w *= vm[m];
    }
  }
}

// The adaptive step's rate of a host state W (nx*ny cells): the largest
// (umax + |U|)/dx + (vmax + |V|)/dy over the cells, as the bits the kernels keep.
unsigned long long rate_bits(const KParams& P, const double* W, size_t nc) {
  double r = 0.0;
  for (size_t c = 0; c < nc; ++c) {
    const double rho = W[4 * c], U = W[4 * c + 1] / rho, V = W[4 * c + 2] / rho;
    const double x = (P.umax + std::fabs(U)) / P.dx + (P.vmax + std::fabs(V)) / P.dy;
    if (x > r) r = x;
  }
  unsigned long long b;
  std::memcpy(&b, &r, sizeof b);
  return b;
}

// Point the constants at the device tables of a set of buffers.
void bind_tables(KParams& P, const Buffers& B, const Shape& s) {
  P.wk = gp(B.wk);
  P.wm = gp(B.wk + s.K);
  P.vmom = gp(B.wk + s.K + s.M);
  P.uk = gp(B.uk);
  P.vm = gp(B.vm + 1);
  P.xi_in = gp(B.xi_in);
  P.flag = gp(B.flag);
  P.rmax = gp(B.rmax);
  P.tsum = gp(B.tsum);
}

// One solver as the kernels see it; f[0] and W[0] hold the state when its step counter is 0.
void make_inst(const KParams& P, const Buffers& B, int prec, Inst& I) {
  I = Inst{};
  I.P = P;
  I.f[0] = gp(B.f[0]);
  I.f[1] = gp(B.f[1]);
  I.W[0] = gp(B.W[0]);
  I.W[1] = gp(B.W[1]);
  I.gsplit = 1;
  I.Wg = gp(B.Wg);
  I.hs = gp(B.hs);
  I.hsg = gp(B.hsg);
  I.recx = gp(B.recx);
  I.recy = gp(B.recy);
  I.cur = 0;
  I.fp32 = prec == UGKS_FP32_STORE ? 1 : 0;
}

struct Copy {
  void* dst;
  const void* src;
  size_t n;
};

// Host-to-device copies of the velocity tables into a set of buffers; returns their number (5).
int table_copies(const Buffers& B, const HostTables& T, const Shape& s, Copy* out) {
  out[0] = {B.wk, T.wk, (size_t)s.K * 8};
  out[1] = {B.wk + s.K, T.wm, (size_t)s.M * 8};
  out[2] = {B.wk + s.K + s.M, T.vmom, (size_t)s.M * 5 * 8};
  out[3] = {B.uk, T.uk, (size_t)s.K * 8};
  out[4] = {B.vm, T.vm_padded, (size_t)(s.M + 2) * 8};
  return 5;
}

}  // namespace

extern "C" {

int ugks_required_bytes(const ugks_mesh* mesh, const ugks_vgrid* vgrid, const ugks_opts* opts,
                        size_t* out_bytes) {
  if (!out_bytes) return fail(nullptr, UGKS_E_INVAL, "out_bytes is NULL%s");
  Shape s;
  std::string why;
  if (!shape_ok(mesh, vgrid, s, why)) return fail(nullptr, UGKS_E_INVAL, "%s", why.c_str());
  const int prec = opts ? opts->precision : UGKS_FP64;
  if (prec != UGKS_FP64 && prec != UGKS_FP32_STORE)
    return fail(nullptr, UGKS_E_INVAL, "unknown precision%s");
  if (opts && (opts->velocity_chunks < 0 || opts->velocity_chunks > 16))
    return fail(nullptr, UGKS_E_INVAL, "velocity_chunks must be in 0..16%s");
  bool shak = false;
  if (!collision_of(opts, s, shak, why)) return fail(nullptr, UGKS_E_INVAL, "%s", why.c_str());
  *out_bytes = layout_of(s, prec, chunks_of(s, opts ? opts->velocity_chunks : 0), shak).total;
  return UGKS_OK;
}

int ugks_create(const ugks_mesh* mesh, const ugks_vgrid* vgrid, double kn, const ugks_bc* bc,
                const ugks_opts* opts, ugks_handle** out) {
  if (!out) return fail(nullptr, UGKS_E_INVAL, "out is NULL%s");
  *out = nullptr;
  Shape s;
  std::string why;
  bool shak = false;
  if (!problem_ok(mesh, vgrid, kn, bc, opts, s, shak, why))
    return fail(nullptr, UGKS_E_INVAL, "%s", why.c_str());
  const int chunks = chunks_of(s, opts->velocity_chunks);
  const Layout L = layout_of(s, opts->precision, chunks, shak);
  if (opts->workspace && opts->workspace_bytes < L.total)
    return fail(nullptr, UGKS_E_NOMEM, "workspace smaller than ugks_required_bytes()%s");
  if (opts->workspace && (reinterpret_cast<uintptr_t>(opts->workspace) % kAlign) != 0)
    return fail(nullptr, UGKS_E_INVAL, "workspace must be 256-byte aligned%s");

  ugks_handle* h = new (std::nothrow) ugks_handle();
  if (!h) return fail(nullptr, UGKS_E_NOMEM, "host allocation failed%s");
  h->prec = opts->precision;
  h->ssize = h->prec == UGKS_FP32_STORE ? 4 : 8;
  h->stream = static_cast<hipStream_t>(opts->stream);
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(nullptr, e, "hipGetDevice");
  }
  if (opts->workspace) {
    h->ws = opts->workspace;
    h->ws_bytes = opts->workspace_bytes;
  } else {
    e = hipMalloc(&h->ws, L.total);
    if (e != hipSuccess) {
      delete h;
      (void)hipGetLastError();
      return fail(nullptr, UGKS_E_NOMEM, "hipMalloc of the workspace failed%s");
    }
    h->ws_bytes = L.total;
    h->owns_ws = true;
  }
  carve(h, L, s);

  // ---- constants
  KParams& P = h->P;
  std::unique_ptr<HostTables> tables(new (std::nothrow) HostTables);
  if (!tables) {
    if (h->owns_ws) (void)hipFree(h->ws);
    delete h;
    return fail(nullptr, UGKS_E_NOMEM, "host allocation failed%s");
  }
  HostTables& T = *tables;
  fill_constants(mesh, vgrid, kn, bc, opts, s, shak, chunks, P, T);
  std::vector<double> xi(s.ny);
  for (int j = 0; j < s.ny; ++j) xi[j] = inlet_noise(opts, s, j);
  h->tau_ref = P.collisionless ? std::numeric_limits<double>::infinity() : 2.0 * P.mu_ref;
  std::vector<double> W0(4 * s.nc);
  for (int j = 0; j < s.ny; ++j) {
    for (int i = 0; i < s.nx; ++i) {
      const size_t c = (size_t)j * s.nx + i;
      const double rho = opts->rho0 * (1.0 + opts->noise * noise_unit(opts->seed, c));
      W0[4 * c + 0] = rho;
      W0[4 * c + 1] = 0.0;
      W0[4 * c + 2] = 0.0;
      W0[4 * c + 3] = P.lam_c * rho * opts->T0;  // (2 + dof) rho/(4 lambda)
    }
  }
  Buffers& B = h->B;
  bind_tables(P, B, s);
  Inst& I = h->inst;
  make_inst(P, B, h->prec, I);
  std::vector<char> plan_host(plan_bytes(1));
  h->pt = build_plan(&I, 1, plan_host.data(), h->plan_dev, &h->pv);
  {
    const Inst* img = reinterpret_cast<const Inst*>(plan_host.data());
    h->moment_chunks = img->gsplit;
    h->update_chunks = img->usplit;
    h->update_ch = h->pt.upd_ch;
  }
  // the plan of ugks_step_static: the same instance with its transient buffers on this
  // device's static scratch (looked up here, once per device)
  std::vector<char> plan_static_host(plan_bytes(1));
  {
    std::string why;
    void* sp = scratch_address(h->device, why);
    if (!sp) {
      h->static_why = why;
    } else if (transient_bytes(L) > kStaticScratchBytes) {
      char msg[256];
      std::snprintf(msg, sizeof msg,
                    "the transient buffers of this shape need %zu bytes, more than the "
                    "static scratch's %zu",
                    transient_bytes(L), kStaticScratchBytes);
      h->static_why = msg;
    } else {
      Inst Is = I;
      carve_transient(L, static_cast<char*>(sp), Is);
      (void)build_plan(&Is, 1, plan_static_host.data(), h->plan_static, &h->pv_static);
      h->static_ok = true;
    }
  }

  Copy copies[10];
  int nt = table_copies(B, T, s, copies);
  copies[nt++] = {B.xi_in, xi.data(), xi.size() * 8};
  copies[nt++] = {B.W[0], W0.data(), W0.size() * 8};
  // rmax[0] of the initial state (adaptive step), rmax[1] and the simulated time zero
  const unsigned long long rmax_tsum[3] = {rate_bits(P, W0.data(), s.nc), 0ull, 0ull};
  copies[nt++] = {B.rmax, rmax_tsum, sizeof rmax_tsum};
  copies[nt++] = {h->plan_dev, plan_host.data(), plan_host.size()};
  if (h->static_ok) copies[nt++] = {h->plan_static, plan_static_host.data(), plan_static_host.size()};
  int rc = UGKS_OK;
  for (int c = 0; c < nt; ++c) {
    const Copy& cp = copies[c];
    e = hipMemcpyAsync(cp.dst, cp.src, cp.n, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) {
      rc = hip_fail(nullptr, e, "hipMemcpyAsync of the tables");
      break;
    }
  }
  if (rc == UGKS_OK) {
    e = hipMemsetAsync(B.flag, 0, sizeof(int), h->stream);

    if (e != hipSuccess) rc = hip_fail(nullptr, e, "hipMemsetAsync of the state flag");
  }
  if (rc == UGKS_OK) {
    // the halo rows and columns start at zero; in a channel only the ghost columns are
    // written (by the fill below, then by every step's update kernel), the rest is read as
    // zero
    const size_t fbytes = (size_t)s.NC * s.NV * s.PS * h->ssize;
    e = hipMemsetAsync(B.f[0], 0, fbytes, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(B.f[1], 0, fbytes, h->stream);
    if (e == hipSuccess)
      e = launch_init(h->pv, I.fp32, (long long)s.nc * (long long)s.NV * s.NC, h->stream);
    if (e == hipSuccess) e = launch_ghost_fill(h->pv, h->pt, I.fp32, h->stream);
    // debug option: every cell value of the buffers the first step writes starts as NaN
    const char* poison = std::getenv("UGKS_DEBUG_POISON");
    if (e == hipSuccess && poison && poison[0] == '1')
      e = launch_poison(h->pv, I.fp32, (long long)s.nc * (long long)s.NV * s.NC, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) rc = hip_fail(nullptr, e, "initial state");
  }
  if (rc != UGKS_OK) {
    if (h->owns_ws) (void)hipFree(h->ws);
    delete h;
    return rc;
  }
  *out = h;
  return UGKS_OK;
}

int ugks_step(ugks_handle* h, int n) {
  if (!h) return UGKS_E_INVAL;
  if (n < 0) return fail(h, UGKS_E_INVAL, "n must be >= 0%s");
  Busy b(h);
  if (!b.ok) return fail(h, UGKS_E_BUSY, "handle in use%s");
  if (h->poisoned) return poisoned_fail(h);
  for (int s = 0; s < n; ++s) {
    h->pv.step = (int)(h->steps & 1);
    const int rc = enqueue_plan_step(h, h->pv, h->pt, h->inst.fp32, h->stream);
    if (rc != UGKS_OK) {
      h->poisoned = true;
      return rc;
    }
    h->steps += 1;
    h->last_static = false;
  }
  return UGKS_OK;
}

int ugks_step_static(ugks_handle* h, int n) {
  if (!h) return UGKS_E_INVAL;
  if (n < 0) return fail(h, UGKS_E_INVAL, "n must be >= 0%s");
  Busy b(h);
  if (!b.ok) return fail(h, UGKS_E_BUSY, "handle in use%s");
  if (h->poisoned) return poisoned_fail(h);
  if (!h->static_ok)
    return fail(h, UGKS_E_INVAL, "ugks_step_static: %s", h->static_why.c_str());
  static const char* names[4] = {"ghost kernel launch", "moment kernel launch",
                                 "interface kernel launch", "update kernel launch"};
  for (int s = 0; s < n; ++s) {
    h->pv_static.step = (int)(h->steps & 1);
    // no timing events here: creating them would allocate
    for (int phase = 0; phase < 4; ++phase) {
      const hipError_t e = launch_phase(h->pv_static, h->pt, h->inst.fp32, phase, h->stream);
      if (e != hipSuccess) {
        h->poisoned = true;
        return hip_fail(h, e, names[phase]);
      }
    }
    h->steps += 1;
    h->last_static = true;
  }
  return UGKS_OK;
}

int ugks_moments(ugks_handle* h, double* host_out) {
  if (!h) return UGKS_E_INVAL;
  if (!host_out) return fail(h, UGKS_E_INVAL, "host_out is NULL%s");
  Busy b(h);
  if (!b.ok) return fail(h, UGKS_E_BUSY, "handle in use%s");
  if (h->poisoned) return poisoned_fail(h);
  const size_t nc = (size_t)h->P.nx * h->P.ny;
  std::vector<double> W(4 * nc);
  int flag = 0;
  hipError_t e = hipMemcpyAsync(W.data(), h->B.W[h->steps & 1], W.size() * 8,
                                hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&flag, h->B.flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reading W");
  bool bad = flag != 0;
  for (size_t c = 0; c < nc; ++c) {
    const double* w = &W[4 * c];
    const double rho = w[0], U = w[1] / rho, V = w[2] / rho;
    const double T = (w[3] - 0.5 * rho * (U * U + V * V)) / (h->P.lam_c * rho);
    host_out[4 * c + 0] = rho;
    host_out[4 * c + 1] = U;
    host_out[4 * c + 2] = V;
    host_out[4 * c + 3] = T;
    if (!(rho > 0) || !(T > 0) || !std::isfinite(U) || !std::isfinite(V) || !std::isfinite(T))
      bad = true;
  }
  if (bad) return fail(h, UGKS_E_STATE, "invalid state (NaN, rho <= 0 or T <= 0)%s");
  return UGKS_OK;
}

int ugks_destroy(ugks_handle* h) {
  if (!h) return UGKS_OK;
  (void)hipStreamSynchronize(h->stream);
  for (auto& p : h->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : h->pool) (void)hipEventDestroy(e);
  if (h->owns_ws) (void)hipFree(h->ws);
  delete h;
  return UGKS_OK;
}

const char* ugks_last_error(const ugks_handle* h) {
  return h ? h->err.c_str() : g_create_error;
}

int ugks_get_info(const ugks_handle* h, ugks_info* out) {
  if (!h || !out) return UGKS_E_INVAL;
  out->nx = h->P.nx;
  out->ny = h->P.ny;
  out->nu = h->P.K;
  out->nv = h->P.M;
  out->plane_stride = h->P.PS;
  out->precision = h->prec;
  out->internal_dof = h->P.dof;
  out->prandtl = h->P.shak ? 1.0 - h->P.pr_c : 1.0;
  out->dx = h->P.dx;
  out->dy = h->P.dy;
  out->dt = h->P.dt;
  out->tau_ref = h->tau_ref;
  out->steps = h->steps;
  out->device_bytes = h->ws_bytes;
  out->moment_chunks = h->moment_chunks;
  out->update_chunks = h->update_chunks;
  out->update_chunks_per_workgroup = h->update_ch;
  out->update_v_chunks = h->P.vsplit;
  return UGKS_OK;
}

int ugks_get_time(ugks_handle* h, double* time, double* dt_next) {
  if (!h || !time || !dt_next) return UGKS_E_INVAL;
  Busy b(h);
  if (!b.ok) return fail(h, UGKS_E_BUSY, "handle in use%s");
  if (h->poisoned) return poisoned_fail(h);
  unsigned long long rt[3];
  hipError_t e = hipMemcpyAsync(rt, h->B.rmax, sizeof rt, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reading the time");
  std::memcpy(time, &rt[2], sizeof(double));
  double r;
  std::memcpy(&r, &rt[h->steps & 1], sizeof r);
  *dt_next = h->P.adaptive ? h->P.cfl / r : h->P.dt;
  return UGKS_OK;
}

int ugks_get_state(ugks_handle* h, double* f, double* W) {
  if (!h) return UGKS_E_INVAL;
  Busy b(h);
  if (!b.ok) return fail(h, UGKS_E_BUSY, "handle in use%s");
  if (h->poisoned) return poisoned_fail(h);
  const size_t nc = (size_t)h->P.nx * h->P.ny, NV = (size_t)h->P.NV * h->P.NC;
  const size_t PS = (size_t)h->P.PS;
  hipError_t e = hipSuccess;
  std::vector<char> raw;
  if (f) {
    raw.resize(NV * PS * h->ssize);
    e = hipMemcpyAsync(raw.data(), h->B.f[h->steps & 1], raw.size(), hipMemcpyDeviceToHost,
                       h->stream);
  }
  if (e == hipSuccess && W)
    e = hipMemcpyAsync(W, h->B.W[h->steps & 1], nc * 4 * 8, hipMemcpyDeviceToHost, h->stream);
  int flag = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&flag, h->B.flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reading the state");
  if (f) {
    for (size_t c = 0; c < nc; ++c) {
      const size_t at = plane_index(h->P, c);
      for (size_t v = 0; v < NV; ++v) {
        const size_t sl = v * PS + at;
        f[c * NV + v] = h->prec == UGKS_FP32_STORE
                            ? (double)reinterpret_cast<const float*>(raw.data())[sl]
                            : reinterpret_cast<const double*>(raw.data())[sl];
      }
    }
  }
  if (flag) return fail(h, UGKS_E_STATE, "invalid state flagged on the device%s");
  return UGKS_OK;
}

int ugks_set_state(ugks_handle* h, const double* f, const double* W) {
  if (!h) return UGKS_E_INVAL;
  Busy b(h);
  if (!b.ok) return fail(h, UGKS_E_BUSY, "handle in use%s");
  if (h->poisoned) return poisoned_fail(h);
  const size_t nc = (size_t)h->P.nx * h->P.ny, NV = (size_t)h->P.NV * h->P.NC;
  const size_t PS = (size_t)h->P.PS;
  std::vector<char> raw;
  hipError_t e = hipSuccess;
  if (f) {
    raw.assign(NV * PS * h->ssize, 0);
    for (size_t c = 0; c < nc; ++c) {
      const size_t at = plane_index(h->P, c);
      for (size_t v = 0; v < NV; ++v) {
        const size_t sl = v * PS + at;
        if (h->prec == UGKS_FP32_STORE)
          reinterpret_cast<float*>(raw.data())[sl] = (float)f[c * NV + v];
        else
          reinterpret_cast<double*>(raw.data())[sl] = f[c * NV + v];
      }
    }
    e = hipMemcpyAsync(h->B.f[h->steps & 1], raw.data(), raw.size(), hipMemcpyHostToDevice,
                       h->stream);
  }
  if (e == hipSuccess && W)
    e = hipMemcpyAsync(h->B.W[h->steps & 1], W, nc * 4 * 8, hipMemcpyHostToDevice, h->stream);
  // the adaptive step of the next step follows the new W
  const unsigned long long rb = W ? rate_bits(h->P, W, nc) : 0ull;
  if (e == hipSuccess && W)
    e = hipMemcpyAsync(h->B.rmax + (h->steps & 1), &rb, sizeof rb, hipMemcpyHostToDevice,
                       h->stream);
  // the ghost columns and ghost states of the new state (the host image's halo is zero)
  if (e == hipSuccess) {
    PlanView pv = h->pv;
    pv.step = (int)(h->steps & 1);
    e = launch_ghost_fill(pv, h->pt, h->inst.fp32, h->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "writing the state");
  return UGKS_OK;
}

int ugks_get_face_flux(ugks_handle* h, double* Fx, double* Fy) {
  if (!h) return UGKS_E_INVAL;
  Busy b(h);
  if (!b.ok) return fail(h, UGKS_E_BUSY, "handle in use%s");
  if (h->poisoned) return poisoned_fail(h);
  if (h->last_static)
    return fail(h, UGKS_E_INVAL,
                "the last step ran with ugks_step_static, whose face records are not kept%s");
  const size_t nfx = (size_t)h->P.ny * (h->P.nx + 1), nfy = (size_t)(h->P.ny + 1) * h->P.nx;
  std::vector<double> rx(Fx ? nfx * kRec : 0), ry(Fy ? nfy * kRec : 0);
  hipError_t e = hipSuccess;
  if (Fx) e = hipMemcpyAsync(rx.data(), h->B.recx, rx.size() * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess && Fy)
    e = hipMemcpyAsync(ry.data(), h->B.recy, ry.size() * 8, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "reading the face records");
  // the records are field-major: field f of face k at f nf + k
  for (size_t k = 0; Fx && k < nfx; ++k)
    for (int q = 0; q < 4; ++q) Fx[4 * k + q] = rx[(R_FX + q) * nfx + k];
  for (size_t k = 0; Fy && k < nfy; ++k)
    for (int q = 0; q < 4; ++q) Fy[4 * k + q] = ry[(R_FX + q) * nfy + k];
  return UGKS_OK;
}

int ugks_set_kernel_timing(ugks_handle* h, int on) {
  if (!h) return UGKS_E_INVAL;
  Busy b(h);
  if (!b.ok) return fail(h, UGKS_E_BUSY, "handle in use%s");
  (void)hipStreamSynchronize(h->stream);
  collect_timing(h);
  for (int k = 0; k < 4; ++k) {
    h->total_ms[k] = 0.0;
    h->launches[k] = 0;
  }
  h->timing = on != 0;
  return UGKS_OK;
}

int ugks_get_kernel_timing(ugks_handle* h, int kernel, double* total_ms, int64_t* launches) {
  if (!h || kernel < 0 || kernel > 3 || !total_ms || !launches) return UGKS_E_INVAL;
  Busy b(h);
  if (!b.ok) return fail(h, UGKS_E_BUSY, "handle in use%s");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(h, e, "synchronising for timing");
  collect_timing(h);
  *total_ms = h->total_ms[kernel];
  *launches = h->launches[kernel];
  return UGKS_OK;
}


int ugks_batch_create(void* stream, int max_instances, ugks_batch** out) {
  if (!out) return fail(nullptr, UGKS_E_INVAL, "out is NULL%s");
  *out = nullptr;
  if (max_instances < 1 || max_instances > (1 << 20))
    return fail(nullptr, UGKS_E_INVAL, "max_instances out of range%s");
  ugks_batch* b = new (std::nothrow) ugks_batch();
  if (!b) return fail(nullptr, UGKS_E_NOMEM, "host allocation failed%s");
  b->stream = static_cast<hipStream_t>(stream);
  b->cap = max_instances;
  const size_t bytes = plan_bytes(max_instances);
  hipError_t e = hipMalloc(&b->plan_dev, bytes);
  if (e == hipSuccess) e = hipHostMalloc(&b->plan_host, bytes, hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (b->plan_dev) (void)hipFree(b->plan_dev);
    if (b->plan_host) (void)hipHostFree(b->plan_host);
    delete b;
    (void)hipGetLastError();
    return fail(nullptr, UGKS_E_NOMEM, "batch plan allocation failed%s");
  }
  *out = b;
  return UGKS_OK;
}

int ugks_step_batch(ugks_batch* b, ugks_handle* const* hs, int count, int n) {
  if (!b) return UGKS_E_INVAL;
  if (!hs || count < 1 || count > b->cap || n < 0) {
    b->err = "need 1 <= count <= max_instances, n >= 0 and a handle array";
    return UGKS_E_INVAL;
  }
  for (int q = 0; q < count; ++q) {
    if (!hs[q]) {
      b->err = "NULL handle in the batch";
      return UGKS_E_INVAL;
    }
    if (hs[q]->inst.P.shak != hs[0]->inst.P.shak) {
      b->err = "a batch holds handles of one collision model";
      return UGKS_E_INVAL;
    }
    if (hs[q]->inst.fp32 != hs[0]->inst.fp32) {
      b->err = "a batch holds handles of one precision";
      return UGKS_E_INVAL;
    }
    for (int r = 0; r < q; ++r)
      if (hs[r] == hs[q]) {
        b->err = "a handle appears twice in the batch";
        return UGKS_E_INVAL;
      }
    if (hs[q]->poisoned) {
      b->err = "a handle of the batch had a failed launch; its state is unknown";
      return UGKS_E_DEVICE;
    }
  }
  // claim every handle for the duration of the call
  int claimed = 0;
  for (; claimed < count; ++claimed) {
    int z = 0;
    if (!hs[claimed]->busy.compare_exchange_strong(z, 1)) break;
  }
  auto release = [&] {
    for (int q = 0; q < claimed; ++q) hs[q]->busy.store(0);
  };
  if (claimed < count) {
    release();
    b->err = "a handle of the batch is in use";
    return UGKS_E_BUSY;
  }
  // adopt members created on another stream: the batch stream first waits for their work,
  // then they live on the batch stream
  for (int q = 0; q < count; ++q) {
    ugks_handle* h = hs[q];
    if (h->stream == b->stream) continue;
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, h->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, ev, 0);
    if (ev) (void)hipEventDestroy(ev);
    if (e != hipSuccess) {
      release();
      b->err = hipGetErrorString(e);
      return UGKS_E_DEVICE;
    }
    h->stream = b->stream;
  }
  // rebuild the plan when the members changed or were stepped outside this batch
  bool same = (int)b->members.size() == count;
  for (int q = 0; same && q < count; ++q)
    same = b->members[q] == hs[q]->uid && hs[q]->steps == b->base_steps[q] + b->counter;
  if (!same) {
    if (b->upload_pending) {
      const hipError_t e = hipEventSynchronize(b->uploaded);
      if (e != hipSuccess) {
        release();
        b->err = hipGetErrorString(e);
        return UGKS_E_DEVICE;
      }
    }
    std::vector<Inst> insts(count);
    b->members.resize(count);
    b->base_steps.resize(count);
    for (int q = 0; q < count; ++q) {
      insts[q] = hs[q]->inst;
      insts[q].cur = (int)(hs[q]->steps & 1);
      b->members[q] = hs[q]->uid;
      b->base_steps[q] = hs[q]->steps;
    }
    b->counter = 0;
    b->fp32 = hs[0]->inst.fp32;
    b->pt = build_plan(insts.data(), count, b->plan_host, b->plan_dev, &b->pv);
    hipError_t e = hipMemcpyAsync(b->plan_dev, b->plan_host, plan_bytes(count),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->uploaded, b->stream);
    if (e != hipSuccess) {
      release();
      b->members.clear();
      b->err = hipGetErrorString(e);
      return UGKS_E_DEVICE;
    }
    b->upload_pending = true;
  }
  int rc = UGKS_OK;
  int done = 0;  // steps whose launches were all enqueued
  for (; done < n; ++done) {
    b->pv.step = (int)((b->counter + done) & 1);
    rc = enqueue_plan_step(nullptr, b->pv, b->pt, b->fp32, b->stream);
    if (rc != UGKS_OK) break;
  }
  // the steps enqueued in full advance every member; a step that failed part-way leaves each
  // member's state unknown, so the members are poisoned
  b->counter += done;
  for (int q = 0; q < count; ++q) {
    hs[q]->steps += done;
    if (done > 0) hs[q]->last_static = false;
  }
  if (rc != UGKS_OK) {
    for (int q = 0; q < count; ++q) hs[q]->poisoned = true;
    b->err = g_create_error;
    b->members.clear();
    rc = UGKS_E_DEVICE;
  }
  release();
  return rc;
}

int ugks_batch_destroy(ugks_batch* b) {
  if (!b) return UGKS_OK;
  (void)hipStreamSynchronize(b->stream);
  if (b->uploaded) (void)hipEventDestroy(b->uploaded);
  if (b->plan_dev) (void)hipFree(b->plan_dev);
  if (b->plan_host) (void)hipHostFree(b->plan_host);
  delete b;
  return UGKS_OK;
}

const char* ugks_batch_last_error(const ugks_batch* b) { return b ? b->err.c_str() : ""; }

}  // extern "C"
