// Host runtime of libhd.so: contexts, batch layout in device memory, the
// schedulers (persistent launches of the LDS-resident or one-workgroup
// kernels replayed as graphs of 2000-step chunks; grid kernels captured in
// graphs of 50 steps), the autotuner, checkpoints and read-outs.  Every function exported here is declared in
// include/hd.h.  Host arithmetic is limited to laying out inputs (cell grids,
// rigid-body offsets); every step of the method runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/hd.h"
#include "hd_device.h"
#include "hd_launch.h"

using hdk::SysDesc;
using hdk::SysState;

// Static device scratch of hd_quench_noalloc (FIRE state, system list and
// reduction partials), for callers that cannot allocate device memory.  Each
// device holds its own copy for the life of the process; in host code the
// array's name is not a device address, so its per-device address is taken
// once (hd_create) and only that address is used.  Calls that overlap on one
// device share it and race.
constexpr size_t kScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void *g_scratch[kMaxDevices] = {};
static std::mutex g_scratch_mutex;

namespace {

constexpr int64_t kChunkSteps = 2000;   // steps per batched launch
constexpr int kGraphSteps = 50;         // steps per captured grid graph

struct SysHost {
  int dim = 0, n = 0;
  double box[3] = {0, 0, 0};
  int periodic[3] = {0, 0, 0};
  double mass = 1.0;
  std::vector<double> pos, rO, cofs;
  std::vector<uint8_t> type, role;
  hd_lj_params lj{};
  hd_thermo_params th{};
  hd_drive_params dr{};
  hd_bias_params bias{};
  int tip_bonds = 0;
  double k_bond = 0.0, r_bond = 0.0, r_bond_cut = 0.0;
  // bias variables (hd_set_bias_variables): var1 drives the switch of
  // hd_bias_params, var2 (-1: none) a second one, combined by eq. 13
  int bias_var1 = HD_BIAS_SLOPE, bias_var2 = -1;
  double b2_lo = 0.0, b2_hi = 1.0;
  // thermostat (hd_set_nose_hoover): 0 Langevin, else a Nose-Hoover chain
  // of nhc_len thermostats with relaxation time nhc_tau
  int nhc_len = 0;
  double nhc_tau = 0.5;
  // eigenvalue variable (hd_set_min_mode): the mode estimate, [dim][n]
  // (mobile atoms and the rigid body's component on its atoms), and the step
  // of its rotation
  std::vector<double> mode;
  double mode_alpha = 0.0;
  // schedule: the system is in a grid plan that keeps 16-bit list entries;
  // lists_wide: its list still holds the 32-bit entries of a curvature
  // evaluation (hd_min_mode_gradient) until the next step or evaluation
  int list16 = 0, lists_wide = 0;
  int n_rigid = 0, first_rigid = -1;
  double XR[3] = {0, 0, 0}, XR0[3] = {0, 0, 0};
  bool init_vel = false;
  std::vector<double> vel;  // explicit velocities set before finalize
};

// Systems the LDS-resident kernel does not cover: models with tip bonds and
// biases beyond the slope alone.  The one-workgroup kernel does not cover
// those nor the Nose-Hoover chain: they take the grid kernels.
static bool lds_excluded(const SysHost &h) {
  return h.tip_bonds || h.bias_var1 != HD_BIAS_SLOPE || h.bias_var2 >= 0;
}
static bool grid_only(const SysHost &h) { return lds_excluded(h) || h.nhc_len > 0; }

struct Plan {
  std::vector<int> ids;  // systems of the plan
  hdk::Tile *d_tiles = nullptr;
  int32_t *d_sys = nullptr;
  int32_t *d_tile0 = nullptr;
  hdk::GridPlan gp{};
  hipGraphExec_t exec = nullptr;   // kGraphSteps steps
  int graph_steps = 0;
  int launches_per_graph = 0;
  // the remainder of a call shorter than kGraphSteps, captured at the length
  // last asked for (re-captured when a call needs another length)
  hipGraphExec_t tail_exec = nullptr;
  int tail_steps = 0;
  int tail_launches = 0;
};

double minimg_h(double dx, double L, int periodic) {
  if (!periodic) return dx;
  if (dx > 0.5 * L) dx -= L;
  else if (dx < -0.5 * L) dx += L;
  return dx;
}

double wrap_h(double x, double L, int periodic) {
  if (!periodic) return x;
  if (x >= L) x -= L;
  else if (x < 0.0) x += L;
  return x;
}

}  // namespace

struct hd_ctx {
  hd_precision prec = HD_FP64;
  int device = 0;
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;
  hd_exec exec = HD_EXEC_BATCHED;
  int block_threads = 0, max_nb = 0;
  int small_block = 0;           // LDS-resident workgroup size floor (0: smallest that fits)
  bool small_half = true;        // float32 LDS-resident pair pass on half lists
  bool small_disabled = false;
  bool persistent_big = false;  // large systems on the one-workgroup global kernel
  std::vector<SysHost> sys;
  bool finalized = false, poisoned = false, need_eval = false;
  std::string err;
  // device memory
  std::vector<void *> allocs;
  std::vector<void *> sched_allocs;  // schedule-owned (groups, plans, partials)
  hdk::Arrays A{};
  SysDesc *d_desc = nullptr;
  SysState *d_state = nullptr;
  int32_t *d_all = nullptr;
  // batched scheduler: groups of systems of one dimension, resident in LDS
  // (small) or in global memory
  struct Group {
    int dim = 2;
    bool small = false;
    std::vector<int32_t> ids;
    int32_t *d_ids = nullptr;
    int nmax = 0, cellmax = 1, maxnb = 32;
    int block = 0;   // threads per workgroup
    bool nhc = false;   // some system runs the Nose-Hoover chain
  };
  std::vector<Group> groups;
  std::vector<int32_t> small_ids, big_ids;
  int maxnb2 = 32, maxnb3 = 128;
  size_t lds_limit = 0;
  hipStream_t stream2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::vector<SysDesc> h_desc;
  int block = 256;
  int64_t ntot = 0;
  // grid plans: [0] all systems (GRID), or one per system (SEQUENTIAL)
  std::vector<Plan> plans;
  void *d_gscal = nullptr;
  hipGraphExec_t batched_graph = nullptr;  // one chunk of the batched scheduler
  int64_t batched_graph_launches = 0;
  bool all_frozen = false;
  // per system: its neighbour list was last written by the grid kernels
  // (rows and entries are cell-sorted positions) rather than by a
  // one-workgroup kernel (atom indices)
  std::vector<uint8_t> sorted_lists;
  bool any_eig = false;   // some system is biased on the eigenvalue variable
  // hd_bind_device: the context's own storage of each bindable batch field
  // (x, v, ftot, flj, fb, hu), kept while the field lives in caller memory
  double *own_field[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  int64_t last_launches = 0;
  double tuned_ms = 0.0;
};

namespace {

hd_status fail(hd_ctx *c, hd_status st, const std::string &msg) {
  if (c) {
    c->err = msg;
    if (st == HD_E_HIP) c->poisoned = true;
  }
  return st;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, HD_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define CHECK_CTX()                                                                      \
  do {                                                                                   \
    if (!ctx) return HD_E_ARG;                                                           \
    if (ctx->poisoned) return fail(ctx, HD_E_HIP, "context poisoned by an earlier HIP error"); \
  } while (0)

template <typename T>
hd_status dalloc(hd_ctx *ctx, T **p, size_t count, bool sched = false) {
  void *q = nullptr;
  size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return fail(ctx, HD_E_OOM, "hipMalloc failed: " + std::string(hipGetErrorString(e)));
  e = hipMemsetAsync(q, 0, bytes, ctx->stream);
  if (e != hipSuccess) return fail(ctx, HD_E_HIP, "hipMemsetAsync failed");
  (sched ? ctx->sched_allocs : ctx->allocs).push_back(q);
  *p = (T *)q;
  return HD_OK;
}

// Rigid body from the current rigid atoms: COM unwrapped about the first rigid
// atom, offsets c_i = x_i - X_R, atoms re-placed at X_R + c_i.
void init_rigid(SysHost &s) {
  const int n = s.n;
  s.n_rigid = 0;
  s.first_rigid = -1;
  for (int i = 0; i < n; ++i)
    if (s.role[i] == HD_ROLE_RIGID) { if (s.first_rigid < 0) s.first_rigid = i; s.n_rigid++; }
  s.cofs.assign((size_t)s.dim * n, 0.0);
  for (int k = 0; k < 3; ++k) { s.XR[k] = 0; s.XR0[k] = 0; }
  if (s.n_rigid == 0) return;
  const int f = s.first_rigid;
  for (int k = 0; k < s.dim; ++k) {
    const double xf = s.pos[(size_t)k * n + f];
    double sum = 0.0;
    for (int i = 0; i < n; ++i)
      if (s.role[i] == HD_ROLE_RIGID) sum += xf + minimg_h(s.pos[(size_t)k * n + i] - xf, s.box[k], s.periodic[k]);
    s.XR[k] = sum / s.n_rigid;
    for (int i = 0; i < n; ++i)
      if (s.role[i] == HD_ROLE_RIGID)
        s.cofs[(size_t)k * n + i] = (xf + minimg_h(s.pos[(size_t)k * n + i] - xf, s.box[k], s.periodic[k])) - s.XR[k];
    s.XR0[k] = s.XR[k];
  }
  for (int i = 0; i < n; ++i)
    if (s.role[i] == HD_ROLE_RIGID)
      for (int k = 0; k < s.dim; ++k)
        s.pos[(size_t)k * n + i] = wrap_h(s.XR[k] + s.cofs[(size_t)k * n + i], s.box[k], s.periodic[k]);
}

void fill_desc(const hd_ctx *ctx, const SysHost &s, SysDesc &D) {
  D.dim = s.dim;
  D.n = s.n;
  D.n_rigid = s.n_rigid;
  D.first_rigid = s.first_rigid;
  for (int k = 0; k < 3; ++k) {
    D.periodic[k] = (k < s.dim) ? s.periodic[k] : 0;
    D.box[k] = s.box[k];
    D.hbox[k] = 0.5 * s.box[k];
    D.inv_box[k] = (k < s.dim && s.periodic[k]) ? 1.0 / s.box[k] : 0.0;
    D.XR0[k] = s.XR0[k];
  }
  D.mass = s.mass;
  D.inv_mass = 1.0 / s.mass;
  D.massR = s.mass * (s.n_rigid > 0 ? s.n_rigid : 1);
  D.inv_massR = 1.0 / D.massR;
  const double rc = s.lj.rc;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int t = a * 2 + b;
      const double eps = s.lj.eps[a][b], s2 = s.lj.sig[a][b] * s.lj.sig[a][b];
      const double sr2 = s2 / (rc * rc), sr6 = sr2 * sr2 * sr2;
      D.eps[t] = eps;
      D.sig2[t] = s2;
      D.shift[t] = 4.0 * eps * (sr6 * sr6 - sr6);
      D.eps_f[t] = (float)eps;
      D.sig2_f[t] = (float)s2;
      D.shift_f[t] = (float)D.shift[t];
    }
  D.rc2 = rc * rc;
  const double rl = rc + s.lj.skin;
  D.rl2 = rl * rl;
  D.skin_half2 = 0.25 * s.lj.skin * s.lj.skin;
  D.dt = s.th.dt;
  D.hdt = 0.5 * s.th.dt;
  D.c1 = std::exp(-s.th.gamma * s.th.dt);
  D.c2 = std::sqrt((1.0 - D.c1 * D.c1) * s.th.kT / s.mass);
  D.c2R = std::sqrt((1.0 - D.c1 * D.c1) * s.th.kT / D.massR);
  D.kT = s.th.kT;
  D.seed = s.th.seed;
  D.k_spring = s.dr.k_spring;
  D.f_normal = s.dr.f_normal;
  D.x_slider = s.dr.x_slider;
  D.v_slider = s.dr.v_slider;
  D.tip_bonds = s.tip_bonds;
  D.k_bond = s.k_bond;
  D.r_bond = s.r_bond;
  D.rbc2 = s.r_bond_cut * s.r_bond_cut;
  D.k_bond_f = (float)s.k_bond;
  D.r_bond_f = (float)s.r_bond;
  D.rbc2_f = (float)D.rbc2;
  D.bias_on = s.bias.enabled;
  D.m_b = s.bias.m_b;
  D.dv_max = s.bias.dv_max;
  D.g_lo = s.bias.g_lo;
  D.g_hi = s.bias.g_hi;
  D.inv_kT = 1.0 / s.th.kT;
  D.inv_glh = (s.bias.g_lo != s.bias.g_hi) ? 1.0 / (s.bias.g_lo - s.bias.g_hi) : 0.0;
  D.bias_var1 = s.bias_var1;
  D.bias_var2 = s.bias_var2;
  D.gen_bias = (s.bias_var1 != HD_BIAS_SLOPE || s.bias_var2 >= 0) ? 1 : 0;
  D.curv = (s.bias_var1 == HD_BIAS_CURVATURE || s.bias_var2 == HD_BIAS_CURVATURE) ? 1 : 0;
  D.b2_lo = s.b2_lo;
  D.b2_hi = s.b2_hi;
  D.inv_glh2 = (s.b2_lo != s.b2_hi) ? 1.0 / (s.b2_lo - s.b2_hi) : 0.0;
  D.thermostat = s.nhc_len > 0 ? 1 : 0;
  D.nhc_len = s.nhc_len;
  {
    // N_f: the mobile atoms' coordinates and the rigid body's
    int nm = 0;
    for (int i = 0; i < s.n; ++i) nm += s.role[i] == hdk::ROLE_MOBILE;
    const int nf = s.dim * (nm + (s.n_rigid > 0 ? 1 : 0));
    const double t2 = s.nhc_tau * s.nhc_tau;
    D.nhc_NfkT = nf * s.th.kT;
    D.nhc_Q1 = D.nhc_NfkT * t2;
    D.nhc_Q = s.th.kT * t2;
  }
  D.eig = (s.bias_var1 == HD_BIAS_EIGENVALUE || s.bias_var2 == HD_BIAS_EIGENVALUE) ? 1 : 0;
  D.mode_alpha = s.mode_alpha;
  D.list16 = s.list16;
  D.inv_nR = s.n_rigid > 0 ? 1.0 / s.n_rigid : 0.0;
  D.k_nR2 = s.n_rigid > 0 ? s.dr.k_spring / ((double)s.n_rigid * s.n_rigid) : 0.0;
  (void)ctx;
}

// Cell grid: cells of edge strictly above rc + skin (so atoms closer than the
// list radius always land in the same or adjacent cells); a periodic axis with
// room for fewer than three cells uses one; open axes span the initial extent
// plus a margin, atoms beyond it are clamped into the edge cells.
void fill_cells(const SysHost &s, SysDesc &D) {
  const double rl = (s.lj.rc + s.lj.skin) * (1.0 + 1e-9);
  for (int k = 0; k < 3; ++k) { D.nc[k] = 1; D.lo[k] = 0.0; D.inv_h[k] = 0.0; }
  for (int k = 0; k < s.dim; ++k) {
    if (s.periodic[k]) {
      int m = (int)std::floor(s.box[k] / rl);
      if (m < 3) m = 1;
      D.nc[k] = m;
      D.lo[k] = 0.0;
      D.inv_h[k] = m / s.box[k];
    } else {
      double mn = s.pos[(size_t)k * s.n], mx = mn;
      for (int i = 1; i < s.n; ++i) {
        mn = std::min(mn, s.pos[(size_t)k * s.n + i]);
        mx = std::max(mx, s.pos[(size_t)k * s.n + i]);
      }
      const double margin = 2.0 * rl + 5.0;
      const double span = (mx - mn) + 2.0 * margin;
      int m = (int)std::floor(span / rl);
      if (m < 1) m = 1;
      D.nc[k] = m;
      D.lo[k] = mn - margin;
      D.inv_h[k] = m / span;
    }
  }
  D.ncell = D.nc[0] * D.nc[1] * D.nc[2];
}

hd_status upload_desc(hd_ctx *ctx, int s) {
  SysDesc &D = ctx->h_desc[s];
  fill_desc(ctx, ctx->sys[s], D);
  HIPCHK(hipMemcpyAsync(ctx->d_desc + s, &D, sizeof(SysDesc), hipMemcpyHostToDevice, ctx->stream));
  return HD_OK;
}

hd_status sync_in(hd_ctx *ctx) {
  // order our stream after the caller's stream
  if (ctx->user_stream && ctx->user_stream != ctx->stream) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipEventRecord(e, ctx->user_stream));
    HIPCHK(hipStreamWaitEvent(ctx->stream, e, 0));
    HIPCHK(hipEventDestroy(e));
  }
  return HD_OK;
}

hd_status sync_out(hd_ctx *ctx) {
  if (ctx->user_stream && ctx->user_stream != ctx->stream) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    HIPCHK(hipEventRecord(e, ctx->stream));
    HIPCHK(hipStreamWaitEvent(ctx->user_stream, e, 0));
    HIPCHK(hipEventDestroy(e));
  }
  return HD_OK;
}

hd_status check_sys(hd_ctx *ctx, int32_t s) {
  if (s < 0 || s >= (int32_t)ctx->sys.size()) return fail(ctx, HD_E_ARG, "system index out of range");
  return HD_OK;
}

hd_status build_plan(hd_ctx *ctx, const std::vector<int> &systems, Plan &P) {
  const int B = ctx->block;
  std::vector<hdk::Tile> tiles;
  std::vector<int32_t> tile0;
  int max_ncell = 1;
  for (int s : systems) {
    const int n = ctx->sys[s].n;
    const int nt = (n + B - 1) / B;
    tile0.push_back((int32_t)tiles.size());
    for (int t = 0; t < nt; ++t) {
      hdk::Tile T{};
      T.sys = s;
      T.first = t * B;
      T.count = std::min(B, n - t * B);
      T.tile_in_sys = t;
      T.tiles_in_sys = nt;
      tiles.push_back(T);
    }
    max_ncell = std::max(max_ncell, ctx->h_desc[s].ncell);
    P.gp.max_n = std::max(P.gp.max_n, n);
    if (ctx->sys[s].tip_bonds) P.gp.any_bonds = 1;
    if (ctx->h_desc[s].curv) P.gp.any_curv = 1;
    if (ctx->h_desc[s].thermostat == 1) P.gp.any_nhc = 1;
    if (ctx->h_desc[s].eig) P.gp.any_eig = 1;
  }
  // LJ-only plans whose systems' sorted positions fit 15 bits keep 16-bit
  // list entries (half the list traffic of the pair pass)
  P.gp.list16 = (!P.gp.any_bonds && !P.gp.any_curv && !P.gp.any_eig) ? 1 : 0;
  for (int s : systems)
    if (ctx->sys[s].n > 32767) P.gp.list16 = 0;
  hd_status st = dalloc(ctx, &P.d_tiles, tiles.size(), true);
  if (st != HD_OK) return st;
  st = dalloc(ctx, &P.d_sys, systems.size(), true);
  if (st != HD_OK) return st;
  st = dalloc(ctx, &P.d_tile0, systems.size(), true);
  if (st != HD_OK) return st;
  HIPCHK(hipMemcpyAsync(P.d_tiles, tiles.data(), tiles.size() * sizeof(hdk::Tile), hipMemcpyHostToDevice, ctx->stream));
  std::vector<int32_t> ids(systems.begin(), systems.end());
  HIPCHK(hipMemcpyAsync(P.d_sys, ids.data(), ids.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(P.d_tile0, tile0.data(), tile0.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  P.ids = systems;
  P.gp.tiles = P.d_tiles;
  P.gp.ntiles = (int)tiles.size();
  P.gp.block = B;
  P.gp.sys_ids = P.d_sys;
  P.gp.sys_tile0 = P.d_tile0;
  P.gp.nsys = (int)systems.size();
  P.gp.max_ncell = max_ncell;
  P.gp.gscal = ctx->d_gscal;
  return HD_OK;
}

hd_status capture_plan(hd_ctx *ctx, Plan &P, int steps, hipGraphExec_t *exec, int *n_launches) {
  hipStream_t cs;
  HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  int launches = 0;
  hipError_t e = hipSuccess;
  e = hdk::grid_steps(ctx->prec == HD_FP64 ? 0 : 1, ctx->d_desc, ctx->d_state, ctx->A, P.gp, steps, cs, &launches);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(cs, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    hipStreamDestroy(cs);
    return fail(ctx, HD_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  }
  HIPCHK(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
  HIPCHK(hipGraphDestroy(g));
  HIPCHK(hipStreamDestroy(cs));
  *n_launches = launches;
  return HD_OK;
}

// Pair-pass variant of the LDS-resident kernel: float64 (full lists), float32
// with half lists and float64 LDS accumulation of the partner's share, or
// float32 with full lists.
int small_kind(const hd_ctx *ctx) { return ctx->prec == HD_FP64 ? 0 : (ctx->small_half ? 1 : 2); }

// One persistent launch per group (LDS-resident groups, and large systems
// when they run on the one-workgroup global kernel), on `stream`.
hd_status launch_groups(hd_ctx *ctx, int64_t nsteps, int mode, hipStream_t stream, int64_t *launches) {
  const int prec = ctx->prec == HD_FP64 ? 0 : 1;
  for (auto &G : ctx->groups) {
    if (G.ids.empty()) continue;
    for (int s : G.ids) ctx->sorted_lists[s] = 0;
    if (G.small)
      HIPCHK(hdk::launch_small(small_kind(ctx), G.dim, ctx->d_desc, ctx->d_state, ctx->A, G.d_ids, (int)G.ids.size(),
                               G.nmax, G.maxnb, G.cellmax, G.block, nsteps, (mode == 0 && G.nhc) ? 2 : mode,
                               stream));
    else
      HIPCHK(hdk::launch_batched(prec, G.dim, ctx->d_desc, ctx->d_state, ctx->A, G.d_ids, (int)G.ids.size(),
                                 ctx->block, nsteps, mode, stream));
    if (launches) ++*launches;
  }
  return HD_OK;
}

// Evaluate at the current positions for every system.  Lists are rebuilt
// from the current positions, or (force_rebuild false, grid systems) only
// where an atom left half the skin: the LDS-resident kernel builds its lists
// at every launch either way.
hd_status evaluate_all(hd_ctx *ctx, bool force_rebuild = true) {
  const int prec = ctx->prec == HD_FP64 ? 0 : 1;
  hd_status st = launch_groups(ctx, 0, 1, ctx->stream, nullptr);
  if (st != HD_OK) return st;
  for (auto &P : ctx->plans) {
    int l = 0;
    for (int s : P.ids) { ctx->sorted_lists[s] = 1; ctx->sys[s].lists_wide = 0; }
    HIPCHK(hdk::grid_step(prec, ctx->d_desc, ctx->d_state, ctx->A, P.gp, true, ctx->stream, &l, force_rebuild));
    HIPCHK(hdk::grid_ekin(ctx->d_desc, ctx->d_state, ctx->A, P.gp, ctx->stream));
  }
  ctx->need_eval = false;
  return HD_OK;
}

// Graphs a call of n_steps replays on the grid plans: kGraphSteps steps, and
// the remainder at its own length (re-captured when a call needs another
// length).  Captured before the call's work is enqueued, so that the capture
// stays outside the call's timed region.
hd_status prepare_plans(hd_ctx *ctx, int64_t n_steps) {
  hd_status st;
  for (auto &P : ctx->plans) {
    if (n_steps >= kGraphSteps && !P.exec) {
      if ((st = capture_plan(ctx, P, kGraphSteps, &P.exec, &P.launches_per_graph)) != HD_OK) return st;
      P.graph_steps = kGraphSteps;
    }
    const int left = (int)(n_steps % kGraphSteps);
    if (left > 0 && (!P.tail_exec || P.tail_steps != left)) {
      if (P.tail_exec) {
        HIPCHK(hipStreamSynchronize(ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream2));
        HIPCHK(hipGraphExecDestroy(P.tail_exec));
        P.tail_exec = nullptr;
      }
      if ((st = capture_plan(ctx, P, left, &P.tail_exec, &P.tail_launches)) != HD_OK) return st;
      P.tail_steps = left;
    }
  }
  return HD_OK;
}

// Grid plans: replays of the graphs prepare_plans captured, then the kinetic
// energy.
hd_status run_plans(hd_ctx *ctx, int64_t n_steps, hipStream_t stream, int64_t *launches) {
  for (auto &P : ctx->plans) {
    for (int s : P.ids) {
      ctx->sorted_lists[s] = 1;
      if (n_steps > 0) ctx->sys[s].lists_wide = 0;   // the first step rebuilds a restored list
    }
    for (int64_t g = 0; g < n_steps / kGraphSteps; ++g) {
      HIPCHK(hipGraphLaunch(P.exec, stream));
      *launches += P.launches_per_graph;
    }
    if (n_steps % kGraphSteps) {
      HIPCHK(hipGraphLaunch(P.tail_exec, stream));
      *launches += P.tail_launches;
    }
    HIPCHK(hdk::grid_ekin(ctx->d_desc, ctx->d_state, ctx->A, P.gp, stream));
    ++*launches;
  }
  return HD_OK;
}

// Persistent groups: full chunks replay a captured graph of one chunk, the
// rest is launched directly.
hd_status run_groups(hd_ctx *ctx, int64_t n_steps, hipStream_t stream, int64_t *launches) {
  if (ctx->groups.empty()) return HD_OK;
  hd_status st;
  int64_t left = n_steps;
  if (left >= kChunkSteps && !ctx->batched_graph) {
    HIPCHK(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    int64_t nl = 0;
    const hd_status cst = launch_groups(ctx, kChunkSteps, 0, stream, &nl);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(stream, &g);
    if (cst != HD_OK) return cst;
    if (e2 != hipSuccess) return fail(ctx, HD_E_HIP, std::string("batched graph capture: ") + hipGetErrorString(e2));
    HIPCHK(hipGraphInstantiate(&ctx->batched_graph, g, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(g));
    ctx->batched_graph_launches = nl;
  }
  while (left >= kChunkSteps) {
    HIPCHK(hipGraphLaunch(ctx->batched_graph, stream));
    *launches += ctx->batched_graph_launches;
    left -= kChunkSteps;
  }
  if (left > 0 && (st = launch_groups(ctx, left, 0, stream, launches)) != HD_OK) return st;
  return HD_OK;
}


// Workgroup size of the LDS-resident kernel for a group whose largest system
// has nmax atoms: one thread per atom, at least the tuned floor.
int small_block_for(const hd_ctx *ctx, int nmax) {
  int b = nmax <= 256 ? 256 : (nmax <= 512 ? 512 : 1024);
  while (b < ctx->small_block && b < 1024) b *= 2;
  return b;
}

// Drop the schedule (graphs, groups, plans and their device buffers).
void clear_schedule(hd_ctx *ctx) {
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipStreamSynchronize(ctx->stream2);
  for (auto &P : ctx->plans) {
    if (P.exec) (void)hipGraphExecDestroy(P.exec);
    if (P.tail_exec) (void)hipGraphExecDestroy(P.tail_exec);
  }
  ctx->plans.clear();
  if (ctx->batched_graph) (void)hipGraphExecDestroy(ctx->batched_graph);
  ctx->batched_graph = nullptr;
  for (void *q : ctx->sched_allocs) (void)hipFree(q);
  ctx->sched_allocs.clear();
  ctx->groups.clear();
  ctx->small_ids.clear();
  ctx->big_ids.clear();
  ctx->A.partials = nullptr;
  ctx->A.rb_tiles = nullptr;
}

// Assign systems to the LDS-resident groups, the one-workgroup kernel or the
// grid plans, following the scheduler and launch knobs of the context.
hd_status build_schedule(hd_ctx *ctx) {
  const int S = (int)ctx->sys.size();
  hdk::Arrays &A = ctx->A;
  hd_status st;
#define ALLOC(p, cnt) do { st = dalloc(ctx, &(p), (cnt), true); if (st != HD_OK) return st; } while (0)
  // batched scheduler: systems of <= 1024 atoms whose state fits in LDS run
  // LDS-resident (one thread per atom), the rest from global memory
  ctx->small_ids.clear();
  ctx->big_ids.clear();
  ctx->groups.clear();
  if (ctx->exec == HD_EXEC_BATCHED) {
    const int prec = small_kind(ctx);
    const size_t budget = ctx->lds_limit > 8192 ? ctx->lds_limit - 8192 : 0;  // static LDS of the kernel
    std::vector<int> cand;
    for (int s = 0; s < S; ++s) {
      const SysHost &h = ctx->sys[s];
      const int maxnb = h.dim == 2 ? ctx->maxnb2 : ctx->maxnb3;
      // models with tip bonds or a bias beyond the slope alone run on the
      // grid kernels only (the Nose-Hoover chain may stay LDS-resident)
      const bool ok = h.n <= 1024 && maxnb <= 32767 && !lds_excluded(h) &&
                      hdk::small_lds_bytes(h.dim, prec, h.n, maxnb, ctx->h_desc[s].ncell) <= budget &&
                      !ctx->small_disabled;
      if (ok) cand.push_back(s);
      else ctx->big_ids.push_back(s);
    }
    // admit candidates (by size) while the group's common layout fits
    std::sort(cand.begin(), cand.end(), [&](int a, int b) { return ctx->sys[a].n < ctx->sys[b].n; });
    int gn[2] = {0, 0}, gc[2] = {1, 1};
    std::vector<int32_t> sm[2];
    for (int s : cand) {
      const int d = ctx->sys[s].dim - 2;
      const int maxnb = d == 0 ? ctx->maxnb2 : ctx->maxnb3;
      const int n2 = std::max(gn[d], ctx->sys[s].n), c2 = std::max(gc[d], ctx->h_desc[s].ncell);
      if (hdk::small_lds_bytes(d + 2, prec, n2, maxnb, c2) <= budget) {
        sm[d].push_back(s); gn[d] = n2; gc[d] = c2;
      } else {
        ctx->big_ids.push_back(s);
      }
    }
    for (int d = 0; d < 2; ++d) {
      std::sort(sm[d].begin(), sm[d].end());
      for (int s : sm[d]) ctx->small_ids.push_back(s);
      if (sm[d].empty()) continue;
      hd_ctx::Group G;
      G.dim = d + 2; G.small = true; G.ids = sm[d]; G.nmax = gn[d]; G.cellmax = gc[d];
      G.maxnb = d == 0 ? ctx->maxnb2 : ctx->maxnb3;
      for (int s : sm[d]) G.nhc = G.nhc || ctx->sys[s].nhc_len > 0;
      ctx->groups.push_back(G);
    }
    std::sort(ctx->big_ids.begin(), ctx->big_ids.end());
    if (ctx->persistent_big) {
      for (int d = 0; d < 2; ++d) {
        hd_ctx::Group G;
        G.dim = d + 2;
        for (int s : ctx->big_ids)
          if (ctx->sys[s].dim == d + 2 && !grid_only(ctx->sys[s])) G.ids.push_back(s);
        if (!G.ids.empty()) ctx->groups.push_back(G);
      }
    }
  }
  // block size of the global-memory batched kernel / grid tiles
  int maxn = 0;
  for (int s : ctx->big_ids) maxn = std::max(maxn, ctx->sys[s].n);
  if (ctx->block_threads > 0) ctx->block = ctx->block_threads;
  else if (ctx->exec == HD_EXEC_BATCHED && ctx->persistent_big) ctx->block = maxn <= 256 ? 256 : 512;
  else ctx->block = 256;
  for (auto &G : ctx->groups) {
    ALLOC(G.d_ids, G.ids.size());
    G.block = G.small ? small_block_for(ctx, G.nmax) : ctx->block;
    HIPCHK(hipMemcpyAsync(G.d_ids, G.ids.data(), G.ids.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                          ctx->stream));
    if (G.small) {
      const int prec = small_kind(ctx);
      HIPCHK(hdk::small_allow_lds(prec, G.dim,
                                  hdk::small_group_bytes(prec, G.dim, G.nmax, G.maxnb, G.cellmax)));
    }
  }
  HIPCHK(hdk::grid_allow_lds());
  // grid plans (with the one-workgroup kernel for the large systems, the
  // models with tip bonds or a general bias still take the grid)
  std::vector<int> grid_big;
  for (int s : ctx->big_ids)
    if (!ctx->persistent_big || grid_only(ctx->sys[s])) grid_big.push_back(s);
  if (ctx->exec == HD_EXEC_BATCHED && !grid_big.empty()) {
    ctx->plans.resize(1);
    if ((st = build_plan(ctx, grid_big, ctx->plans[0])) != HD_OK) return st;
  } else if (ctx->exec == HD_EXEC_GRID) {
    std::vector<int> sys_all(S);
    for (int s = 0; s < S; ++s) sys_all[s] = s;
    ctx->plans.resize(1);
    if ((st = build_plan(ctx, sys_all, ctx->plans[0])) != HD_OK) return st;
  } else if (ctx->exec == HD_EXEC_SEQUENTIAL) {
    ctx->plans.resize(S);
    for (int s = 0; s < S; ++s)
      if ((st = build_plan(ctx, std::vector<int>{s}, ctx->plans[s])) != HD_OK) return st;
  }
  // list format of each system: 16-bit entries in list16 plans
  for (int s = 0; s < S; ++s) ctx->sys[s].list16 = 0;
  for (auto &P : ctx->plans)
    if (P.gp.list16)
      for (int s : P.ids) ctx->sys[s].list16 = 1;
  for (int s = 0; s < S; ++s)
    if ((st = upload_desc(ctx, s)) != HD_OK) return st;
  {
    int max_tiles = 1;
    for (auto &P : ctx->plans) max_tiles = std::max(max_tiles, P.gp.ntiles);
    ALLOC(A.partials, (size_t)max_tiles * hdk::NPART);
    ALLOC(A.rb_tiles, (size_t)max_tiles);
  }
  if (!ctx->plans.empty()) {
    // grid path: the first step rebuilds every list from the recorded build
    // positions (equal to the positions at hd_finalize), so that a schedule
    // change in the middle of a run keeps the list an uninterrupted run has
    std::vector<int32_t> twos(S, 2);
    HIPCHK(hipMemcpyAsync(A.rebuild_flag, twos.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HD_OK;
#undef ALLOC
}
}  // namespace

// ===========================================================================
extern "C" {

hd_status hd_create(hd_precision prec, int device, void *hip_stream, hd_ctx **out) {
  if (!out || (prec != HD_FP64 && prec != HD_FP32C)) return HD_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return HD_E_NOGPU;
  if (device < 0 || device >= ndev) return HD_E_ARG;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HD_E_NOGPU;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return HD_E_NOGPU;
  hd_ctx *ctx = new (std::nothrow) hd_ctx();
  if (!ctx) return HD_E_OOM;
  ctx->prec = prec;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) { delete ctx; return HD_E_HIP; }
  if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) { delete ctx; return HD_E_HIP; }
  ctx->user_stream = (hipStream_t)hip_stream;
  if (hipStreamCreateWithFlags(&ctx->stream2, hipStreamNonBlocking) != hipSuccess) { delete ctx; return HD_E_HIP; }
  std::unique_lock<std::mutex> scratch_lock(g_scratch_mutex);
  if (device < kMaxDevices && !g_scratch[device]) {
    // the static scratch array's address on this device (current above)
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      hipStreamDestroy(ctx->stream);
      hipStreamDestroy(ctx->stream2);
      delete ctx;
      return HD_E_HIP;
    }
    g_scratch[device] = ptr;
  }
  scratch_lock.unlock();
  hipEventCreate(&ctx->ev0);
  hipEventCreate(&ctx->ev1);
  hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming);
  hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming);
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) lds = 65536;
  ctx->lds_limit = (size_t)lds;
  *out = ctx;
  return HD_OK;
}

hd_status hd_set_exec(hd_ctx *ctx, hd_exec exec) {
  CHECK_CTX();
  if (ctx->finalized) return fail(ctx, HD_E_STATE, "hd_set_exec after hd_finalize");
  if (exec != HD_EXEC_BATCHED && exec != HD_EXEC_GRID && exec != HD_EXEC_SEQUENTIAL)
    return fail(ctx, HD_E_ARG, "unknown scheduler");
  ctx->exec = exec;
  return HD_OK;
}

hd_status hd_set_launch(hd_ctx *ctx, int32_t block_threads, int32_t max_neighbors, int32_t flags) {
  CHECK_CTX();
  if (ctx->finalized) return fail(ctx, HD_E_STATE, "hd_set_launch after hd_finalize");
  if (block_threads != 0 && (block_threads < 64 || block_threads > 1024 || block_threads % 64 != 0))
    return fail(ctx, HD_E_ARG, "block_threads must be a multiple of 64 in [64, 1024]");
  if (max_neighbors < 0 || max_neighbors > 4096) return fail(ctx, HD_E_ARG, "max_neighbors out of range");
  if (flags & ~(HD_LAUNCH_LDS | HD_LAUNCH_PERSISTENT_LARGE)) return fail(ctx, HD_E_ARG, "unknown launch flag");
  ctx->block_threads = block_threads;
  ctx->max_nb = max_neighbors;
  ctx->small_disabled = (flags & HD_LAUNCH_LDS) == 0;
  ctx->persistent_big = (flags & HD_LAUNCH_PERSISTENT_LARGE) != 0;
  return HD_OK;
}

hd_status hd_add_system(hd_ctx *ctx, const hd_system_desc *desc, const hd_lj_params *lj,
                        const hd_thermo_params *thermo, const hd_drive_params *drive, int32_t *sys_id) {
  CHECK_CTX();
  if (ctx->finalized) return fail(ctx, HD_E_STATE, "systems must be added before hd_finalize");
  if (!desc || !lj || !thermo || !drive) return fail(ctx, HD_E_ARG, "null parameter block");
  if (desc->dim != 2 && desc->dim != 3) return fail(ctx, HD_E_ARG, "dim must be 2 or 3");
  if (desc->n_atoms <= 0 || desc->n_atoms > (1 << 28)) return fail(ctx, HD_E_ARG, "n_atoms out of range");
  if (!desc->pos || !desc->type || !desc->role) return fail(ctx, HD_E_ARG, "null per-atom array");
  if (!(desc->mass > 0)) return fail(ctx, HD_E_ARG, "mass must be positive");
  if (!(lj->rc > 0) || !(lj->skin >= 0)) return fail(ctx, HD_E_ARG, "bad cutoff or skin");
  const double rl = lj->rc + lj->skin;
  for (int k = 0; k < desc->dim; ++k)
    if (desc->periodic[k] && !(desc->box[k] >= 2.0 * rl))
      return fail(ctx, HD_E_ARG, "periodic box shorter than twice the list radius");
  if (!(thermo->dt > 0) || thermo->gamma < 0 || thermo->kT < 0) return fail(ctx, HD_E_ARG, "bad thermostat");
  SysHost s;
  s.dim = desc->dim;
  s.n = desc->n_atoms;
  for (int k = 0; k < 3; ++k) { s.box[k] = desc->box[k]; s.periodic[k] = (k < s.dim) ? desc->periodic[k] : 0; }
  s.mass = desc->mass;
  const size_t nd = (size_t)s.dim * s.n;
  s.pos.assign(desc->pos, desc->pos + nd);
  s.type.assign(desc->type, desc->type + s.n);
  s.role.assign(desc->role, desc->role + s.n);
  for (int i = 0; i < s.n; ++i) {
    if (s.type[i] > 1) return fail(ctx, HD_E_ARG, "type must be 0 or 1");
    if (s.role[i] > 2) return fail(ctx, HD_E_ARG, "role must be 0, 1 or 2");
  }
  for (int k = 0; k < s.dim; ++k)
    if (s.periodic[k])
      for (int i = 0; i < s.n; ++i) {
        double &x = s.pos[(size_t)k * s.n + i];
        if (!(x >= 0.0 && x < s.box[k])) x = x - s.box[k] * std::floor(x / s.box[k]);
        if (x >= s.box[k]) x = 0.0;
      }
  s.lj = *lj;
  s.th = *thermo;
  s.dr = *drive;
  s.bias = hd_bias_params{0, 2, 0.0, 0.0, 1.0};
  init_rigid(s);
  s.rO = s.pos;
  ctx->sys.push_back(std::move(s));
  if (sys_id) *sys_id = (int32_t)ctx->sys.size() - 1;
  return HD_OK;
}

// Critical values of a switch: "lower" below "upper" for the slope and the
// curvature, above it for the distance (which grows towards the dividing
// surface).
static bool thresholds_ok(int var, double lo, double hi) {
  return var == HD_BIAS_DISTANCE ? lo > hi : lo < hi;
}

// An enabled bias with variables var1 (and var2): m_b >= 1, dv_max >= 0
// (> 0 with two variables: eq. 13 divides by it), both switches' critical
// values in their variable's order.  A disabled bias is not checked.
static const char *bias_problem(const hd_bias_params &b, int var1, int var2, double lo2, double hi2) {
  if (!b.enabled) return nullptr;
  if (b.m_b < 1 || b.dv_max < 0) return "bias needs m_b >= 1 and dv_max >= 0";
  if (!thresholds_ok(var1, b.g_lo, b.g_hi))
    return "bias needs g_lo < g_hi (g_lo > g_hi when the first variable is the distance)";
  if (var2 >= 0 && !thresholds_ok(var2, lo2, hi2))
    return "second switch needs lo2 < hi2 (lo2 > hi2 for the distance)";
  if (var2 >= 0 && !(b.dv_max > 0)) return "two bias variables need dv_max > 0 (eq. 13 divides by it)";
  return nullptr;
}

hd_status hd_set_bias(hd_ctx *ctx, int32_t sys, const hd_bias_params *bias) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK || !bias) return fail(ctx, HD_E_ARG, "bad system or null bias");
  const SysHost &h = ctx->sys[sys];
  if (const char *why = bias_problem(*bias, h.bias_var1, h.bias_var2, h.b2_lo, h.b2_hi))
    return fail(ctx, HD_E_ARG, why);
  if (bias->enabled && ctx->sys[sys].th.kT > 0 && bias->dv_max / ctx->sys[sys].th.kT > 700.0)
    return fail(ctx, HD_E_ARG, "dv_max/kT above 700 overflows the boosted clock");
  ctx->sys[sys].bias = *bias;
  if (ctx->finalized) { ctx->need_eval = true; return upload_desc(ctx, sys); }
  return HD_OK;
}

hd_status hd_set_slider(hd_ctx *ctx, int32_t sys, double x_slider) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK) return HD_E_ARG;
  ctx->sys[sys].dr.x_slider = x_slider;
  if (ctx->finalized) { ctx->need_eval = true; return upload_desc(ctx, sys); }
  return HD_OK;
}

hd_status hd_set_thermo(hd_ctx *ctx, int32_t sys, const hd_thermo_params *thermo) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK || !thermo) return fail(ctx, HD_E_ARG, "bad system or null thermo");
  if (!(thermo->dt > 0) || thermo->gamma < 0 || thermo->kT < 0) return fail(ctx, HD_E_ARG, "bad thermostat");
  if (ctx->sys[sys].nhc_len > 0 && !(thermo->kT > 0))
    return fail(ctx, HD_E_ARG, "the Nose-Hoover chain needs kT > 0");
  ctx->sys[sys].th = *thermo;
  if (ctx->finalized) { ctx->need_eval = true; return upload_desc(ctx, sys); }
  return HD_OK;
}

hd_status hd_set_tip_bonds(hd_ctx *ctx, int32_t sys, int32_t enabled, double k_bond, double r_bond,
                           double r_cut) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK) return fail(ctx, HD_E_ARG, "bad system");
  SysHost &s = ctx->sys[sys];
  if (enabled && !(k_bond >= 0.0 && r_bond > 0.0 && r_cut > 0.0 && r_cut <= s.lj.rc))
    return fail(ctx, HD_E_ARG, "tip bonds need k >= 0, r0 > 0 and 0 < cut <= rc");
  if (ctx->finalized) return fail(ctx, HD_E_STATE, "hd_set_tip_bonds after hd_finalize");
  s.tip_bonds = enabled ? 1 : 0;
  s.k_bond = k_bond;
  s.r_bond = r_bond;
  s.r_bond_cut = r_cut;
  return HD_OK;
}

hd_status hd_set_bias_variables(hd_ctx *ctx, int32_t sys, int32_t var1, int32_t var2, double lo2, double hi2) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK) return fail(ctx, HD_E_ARG, "bad system");
  SysHost &s = ctx->sys[sys];
  if (var1 < HD_BIAS_SLOPE || var1 > HD_BIAS_EIGENVALUE || var2 < -1 || var2 > HD_BIAS_EIGENVALUE || var2 == var1)
    return fail(ctx, HD_E_ARG,
                "bias variables: var1 in {slope, curvature, distance, eigenvalue}, var2 another one or -1");
  if ((var1 == HD_BIAS_CURVATURE && var2 == HD_BIAS_EIGENVALUE) ||
      (var1 == HD_BIAS_EIGENVALUE && var2 == HD_BIAS_CURVATURE))
    return fail(ctx, HD_E_ARG, "the curvature and the eigenvalue cannot be combined");
  if (const char *why = bias_problem(s.bias, var1, var2, lo2, hi2)) return fail(ctx, HD_E_ARG, why);
  if (ctx->finalized) return fail(ctx, HD_E_STATE, "hd_set_bias_variables after hd_finalize");
  s.bias_var1 = var1;
  s.bias_var2 = var2;
  s.b2_lo = var2 >= 0 ? lo2 : 0.0;
  s.b2_hi = var2 >= 0 ? hi2 : 1.0;
  return HD_OK;
}

hd_status hd_set_min_mode(hd_ctx *ctx, int32_t sys, const double *mode, double alpha) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK || !mode) return fail(ctx, HD_E_ARG, "bad system or null mode");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(ctx, HD_E_ARG, "mode step alpha must be >= 0");
  SysHost &h = ctx->sys[sys];
  if (h.bias_var1 != HD_BIAS_EIGENVALUE && h.bias_var2 != HD_BIAS_EIGENVALUE)
    return fail(ctx, HD_E_STATE, "hd_set_min_mode: the system is not biased on the eigenvalue");
  const size_t nd = (size_t)h.dim * h.n;
  h.mode.assign(nd, 0.0);
  double q2 = 0.0;
  for (int i = 0; i < h.n; ++i) {
    const int src = h.role[i] == HD_ROLE_RIGID ? h.first_rigid : i;
    if (h.role[i] == HD_ROLE_FIXED) continue;
    for (int k = 0; k < h.dim; ++k) {
      const double q = mode[(size_t)k * h.n + src];
      if (!std::isfinite(q)) return fail(ctx, HD_E_ARG, "mode must be finite");
      h.mode[(size_t)k * h.n + i] = q;
      if (h.role[i] == HD_ROLE_MOBILE || i == h.first_rigid) q2 += q * q;
    }
  }
  // stored unit over the degrees of freedom
  if (q2 > 0.0)
    for (double &q : h.mode) q /= std::sqrt(q2);
  h.mode_alpha = alpha;
  if (!ctx->finalized) return HD_OK;
  // into the running batch: the mobile atoms' components and the rigid body's
  hd_status st = sync_in(ctx);
  if (st != HD_OK) return st;
  const SysDesc &D = ctx->h_desc[sys];
  std::vector<double> q(h.mode);
  for (int i = 0; i < h.n; ++i)
    if (h.role[i] != HD_ROLE_MOBILE)
      for (int k = 0; k < h.dim; ++k) q[(size_t)k * h.n + i] = 0.0;
  for (int k = 0; k < h.dim; ++k)
    HIPCHK(hipMemcpyAsync(ctx->A.qm + k * ctx->ntot + D.off, q.data() + (size_t)k * h.n, sizeof(double) * h.n,
                          hipMemcpyHostToDevice, ctx->stream));
  SysState T;
  HIPCHK(hipMemcpyAsync(&T, ctx->d_state + sys, sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < 3; ++k) T.qR[k] = (h.n_rigid > 0 && k < h.dim) ? h.mode[(size_t)k * h.n + h.first_rigid] : 0.0;
  HIPCHK(hipMemcpyAsync(ctx->d_state + sys, &T, sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->need_eval = true;
  return upload_desc(ctx, sys);
}

hd_status hd_set_nose_hoover(hd_ctx *ctx, int32_t sys, int32_t chain_len, double tau) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK) return fail(ctx, HD_E_ARG, "bad system");
  SysHost &s = ctx->sys[sys];
  if (chain_len < 0 || chain_len > 4) return fail(ctx, HD_E_ARG, "chain length 0 (Langevin) to 4");
  if (chain_len > 0 && !(tau > 0 && s.th.kT > 0))
    return fail(ctx, HD_E_ARG, "the Nose-Hoover chain needs tau > 0 and kT > 0");
  if (ctx->finalized) return fail(ctx, HD_E_STATE, "hd_set_nose_hoover after hd_finalize");
  s.nhc_len = chain_len;
  s.nhc_tau = chain_len > 0 ? tau : 0.5;
  return HD_OK;
}

hd_status hd_set_reference(hd_ctx *ctx, int32_t sys, const double *rO) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK || !rO) return fail(ctx, HD_E_ARG, "bad system or null r_O");
  SysHost &s = ctx->sys[sys];
  s.rO.assign(rO, rO + (size_t)s.dim * s.n);
  if (ctx->finalized) {
    for (int k = 0; k < s.dim; ++k)
      HIPCHK(hipMemcpyAsync(ctx->A.rO + k * ctx->ntot + ctx->h_desc[sys].off, s.rO.data() + (size_t)k * s.n,
                            sizeof(double) * s.n, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->need_eval = true;
  }
  return HD_OK;
}

hd_status hd_finalize(hd_ctx *ctx);

static hd_status run_init_velocities(hd_ctx *ctx, int32_t sys);

hd_status hd_init_velocities(hd_ctx *ctx, int32_t sys) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK) return HD_E_ARG;
  if (!ctx->finalized) {
    ctx->sys[sys].init_vel = true;
    ctx->sys[sys].vel.clear();
    return HD_OK;
  }
  return run_init_velocities(ctx, sys);
}

hd_status hd_sync(hd_ctx *ctx) {
  CHECK_CTX();
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ctx->finalized) {
    std::vector<SysState> st(ctx->sys.size());
    HIPCHK(hipMemcpy(st.data(), ctx->d_state, st.size() * sizeof(SysState), hipMemcpyDeviceToHost));
    bool all = !st.empty();
    for (auto &t : st) all = all && (t.flags & HD_FLAG_UNSTABLE);
    ctx->all_frozen = all;
    if (all) return fail(ctx, HD_E_UNSTABLE, "every system is frozen as unstable");
  }
  return HD_OK;
}

}  // extern "C"

namespace hdk {
hipError_t launch_init_velocities(const SysDesc *descs, SysState *states, const Arrays &A, int sys,
                                  int n, int block, hipStream_t stream);
}

static hd_status run_init_velocities(hd_ctx *ctx, int32_t sys) {
  HIPCHK(hdk::launch_init_velocities(ctx->d_desc, ctx->d_state, ctx->A, sys, ctx->sys[sys].n, 256, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HD_OK;
}

extern "C" {

hd_status hd_finalize(hd_ctx *ctx) {
  CHECK_CTX();
  if (ctx->finalized) return fail(ctx, HD_E_STATE, "already finalized");
  const int S = (int)ctx->sys.size();
  if (S == 0) return fail(ctx, HD_E_STATE, "no systems");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, HD_E_HIP, "hipSetDevice");
  // layout
  ctx->h_desc.assign(S, SysDesc{});
  int64_t off = 0, cell_off = 0, cstart_off = 0, nbr_off = 0;
  int max_dim = 2;
  for (int s = 0; s < S; ++s) {
    SysHost &h = ctx->sys[s];
    SysDesc &D = ctx->h_desc[s];
    fill_desc(ctx, h, D);
    fill_cells(h, D);
    D.off = off;
    D.cell_off = cell_off;
    D.cstart_off = cstart_off;
    D.maxnb = ctx->max_nb > 0 ? ctx->max_nb : (h.dim == 2 ? 32 : 128);
    D.nbr_off = nbr_off;
    off += h.n;
    cell_off += D.ncell;
    cstart_off += D.ncell + 1;
    nbr_off += (int64_t)((D.maxnb + 3) / 4 * 4) * h.n;   // grid lists come in blocks of four slots
    max_dim = std::max(max_dim, h.dim);
  }
  const int64_t N = off;
  ctx->ntot = N;
  hdk::Arrays &A = ctx->A;
  A.ntot = N;
  A.rec_f32 = ctx->prec == HD_FP64 ? 0 : 1;
  hd_status st;
#define ALLOC(p, cnt) do { st = dalloc(ctx, &(p), (cnt)); if (st != HD_OK) return st; } while (0)
  ALLOC(A.x, 3 * N); ALLOC(A.v, 3 * N); ALLOC(A.rO, 3 * N); ALLOC(A.xb, 3 * N); ALLOC(A.cofs, 3 * N);
  ALLOC(A.ftot, 3 * N); ALLOC(A.flj, 3 * N); ALLOC(A.hu, 3 * N); ALLOC(A.fb, 3 * N);
  if (ctx->prec != HD_FP64) { ALLOC(A.flj_f, 3 * N); ALLOC(A.hu_f, 3 * N); }
  ALLOC(A.rec, (size_t)N * hdk::kRecDoubles);
  ALLOC(A.brec, (size_t)N * 4);
  ALLOC(A.tuu, 3 * N);
  {
    // eigenvalue bias arrays, only when some system uses it
    bool any_eig = false;
    for (const auto &h : ctx->sys)
      any_eig = any_eig || h.bias_var1 == HD_BIAS_EIGENVALUE || h.bias_var2 == HD_BIAS_EIGENVALUE;
    const size_t ne = any_eig ? (size_t)N : 1;
    ALLOC(A.qm, 3 * ne); ALLOC(A.hw, 3 * ne); ALLOC(A.recw, 4 * ne);
    ctx->any_eig = any_eig;
  }
  ALLOC(A.pos, N);
  if (ctx->prec == HD_FP64) { double *u; ALLOC(u, 3 * N); A.u = u; }
  else { float *u; ALLOC(u, 3 * N); A.u = u; }
  ALLOC(A.tr, N); ALLOC(A.nbr, nbr_off); ALLOC(A.nnb, N);
  ALLOC(A.cell_count, cell_off); ALLOC(A.cell_start, cstart_off); ALLOC(A.cell_atoms, N); ALLOC(A.cidx, N);
  ALLOC(A.sys_of, N);
  ALLOC(A.XR_next, 6 * S); ALLOC(A.rebuild_flag, S);
  ALLOC(A.rb_sys, S); ALLOC(A.rb_count, 2);
  ALLOC(ctx->d_desc, S); ALLOC(ctx->d_state, S); ALLOC(ctx->d_all, S);
  {
    char *g;
    ALLOC(g, hdk::grid_scal_bytes() * S);
    ctx->d_gscal = g;
  }
  ctx->maxnb2 = ctx->max_nb > 0 ? ctx->max_nb : 32;
  ctx->maxnb3 = ctx->max_nb > 0 ? ctx->max_nb : 128;
  // host staging
  std::vector<double> x(3 * N, 0.0), rO(3 * N, 0.0), cofs(3 * N, 0.0), v(3 * N, 0.0);
  std::vector<uint8_t> tr(N);
  std::vector<int32_t> sys_of(N), all(S), pos0(N);
  std::vector<SysState> states(S);
  for (int s = 0; s < S; ++s) {
    SysHost &h = ctx->sys[s];
    const SysDesc &D = ctx->h_desc[s];
    for (int k = 0; k < h.dim; ++k)
      for (int i = 0; i < h.n; ++i) {
        x[k * N + D.off + i] = h.pos[(size_t)k * h.n + i];
        rO[k * N + D.off + i] = h.rO[(size_t)k * h.n + i];
        cofs[k * N + D.off + i] = h.cofs[(size_t)k * h.n + i];
        if (!h.vel.empty()) v[k * N + D.off + i] = h.vel[(size_t)k * h.n + i];
      }
    for (int i = 0; i < h.n; ++i) {
      tr[D.off + i] = (uint8_t)(h.type[i] | (h.role[i] << 1));
      sys_of[D.off + i] = s;
      pos0[D.off + i] = i;
    }
    all[s] = s;
    SysState &T = states[s];
    std::memset(&T, 0, sizeof(T));
    for (int k = 0; k < 3; ++k) T.XR[k] = h.XR[k];
    if (!h.vel.empty() && h.n_rigid > 0) {
      for (int k = 0; k < h.dim; ++k) {
        double sum = 0.0;
        for (int i = 0; i < h.n; ++i)
          if (h.role[i] == HD_ROLE_RIGID) sum += h.vel[(size_t)k * h.n + i];
        T.VR[k] = sum / h.n_rigid;
      }
    }
    T.rebuild = 1;
    if (!h.mode.empty() && h.n_rigid > 0)
      for (int k = 0; k < h.dim; ++k) T.qR[k] = h.mode[(size_t)k * h.n + h.first_rigid];
  }
  if (ctx->any_eig) {
    std::vector<double> qm(3 * N, 0.0);
    for (int s = 0; s < S; ++s) {
      const SysHost &h = ctx->sys[s];
      if (h.mode.empty()) continue;
      for (int k = 0; k < h.dim; ++k)
        for (int i = 0; i < h.n; ++i)
          if (h.role[i] == HD_ROLE_MOBILE) qm[k * N + ctx->h_desc[s].off + i] = h.mode[(size_t)k * h.n + i];
    }
    HIPCHK(hipMemcpyAsync(A.qm, qm.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  HIPCHK(hipMemcpyAsync(A.x, x.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(A.xb, x.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(A.rO, rO.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(A.cofs, cofs.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(A.v, v.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(A.tr, tr.data(), N, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(A.sys_of, sys_of.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(A.pos, pos0.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  ctx->sorted_lists.assign(S, 0);
  HIPCHK(hipMemcpyAsync(ctx->d_all, all.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->d_desc, ctx->h_desc.data(), S * sizeof(SysDesc), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->d_state, states.data(), S * sizeof(SysState), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->finalized = true;
  if ((st = build_schedule(ctx)) != HD_OK) return st;
  for (int s = 0; s < S; ++s)
    if (ctx->sys[s].init_vel) {
      if ((st = run_init_velocities(ctx, s)) != HD_OK) return st;
    }
  if ((st = evaluate_all(ctx)) != HD_OK) return st;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HD_OK;
#undef ALLOC
}

hd_status hd_compute(hd_ctx *ctx) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "hd_compute before hd_finalize");
  hd_status st = sync_in(ctx);
  if (st != HD_OK) return st;
  if ((st = evaluate_all(ctx)) != HD_OK) return st;
  return sync_out(ctx);
}

hd_status hd_step(hd_ctx *ctx, int64_t n_steps) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "hd_step before hd_finalize");
  if (n_steps < 0) return fail(ctx, HD_E_ARG, "negative step count");
  if (n_steps == 0) return HD_OK;
  if (ctx->all_frozen) return fail(ctx, HD_E_UNSTABLE, "every system is frozen as unstable");
  hd_status st = sync_in(ctx);
  if (st != HD_OK) return st;
  if (ctx->need_eval && (st = evaluate_all(ctx)) != HD_OK) return st;
  if ((st = prepare_plans(ctx, n_steps)) != HD_OK) return st;
  int64_t launches = 0;
  HIPCHK(hipEventRecord(ctx->ev0, ctx->stream));
  // persistent groups on the context stream, grid plans concurrently on the
  // second stream, joined before the closing event
  const bool both = !ctx->groups.empty() && !ctx->plans.empty();
  if (both) {
    HIPCHK(hipEventRecord(ctx->fork, ctx->stream));
    HIPCHK(hipStreamWaitEvent(ctx->stream2, ctx->fork, 0));
  }
  if ((st = run_groups(ctx, n_steps, ctx->stream, &launches)) != HD_OK) return st;
  if ((st = run_plans(ctx, n_steps, both ? ctx->stream2 : ctx->stream, &launches)) != HD_OK) return st;
  if (both) {
    HIPCHK(hipEventRecord(ctx->join, ctx->stream2));
    HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->join, 0));
  }
  HIPCHK(hipEventRecord(ctx->ev1, ctx->stream));
  ctx->last_launches = launches;
  ctx->last_ms = -1.0;
  return sync_out(ctx);
}

hd_status hd_get_schedule(hd_ctx *ctx, hd_schedule *out) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (!out) return fail(ctx, HD_E_ARG, "null output");
  out->lds_resident = ctx->small_disabled ? 0 : 1;
  out->small_block = 0;
  for (const auto &G : ctx->groups)
    if (G.small) out->small_block = std::max(out->small_block, G.block);
  out->persistent_large = ctx->persistent_big ? 1 : 0;
  out->large_block = ctx->block;
  out->small_half_lists = (ctx->prec != HD_FP64 && ctx->small_half) ? 1 : 0;
  out->ms_per_step = ctx->tuned_ms;
  return HD_OK;
}

namespace {

hd_status apply_schedule(hd_ctx *ctx, const hd_schedule &c) {
  clear_schedule(ctx);
  ctx->small_disabled = c.lds_resident == 0;
  ctx->small_block = c.small_block;
  ctx->persistent_big = c.persistent_large != 0;
  ctx->block_threads = c.large_block;
  ctx->small_half = c.small_half_lists != 0;
  hd_status st = build_schedule(ctx);
  if (st != HD_OK) return st;
  // a system may now run on another kernel, whose list format differs (half
  // or full lists): every kernel rebuilds from the recorded build positions
  std::vector<SysState> T(ctx->sys.size());
  HIPCHK(hipMemcpyAsync(T.data(), ctx->d_state, T.size() * sizeof(SysState), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (auto &t : T) t.rebuild = 2;
  HIPCHK(hipMemcpyAsync(ctx->d_state, T.data(), T.size() * sizeof(SysState), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HD_OK;
}

hd_status restore_all(hd_ctx *ctx, const std::vector<std::vector<char>> &ck) {
  for (size_t s = 0; s < ck.size(); ++s) {
    const hd_status st = hd_set_state(ctx, (int32_t)s, ck[s].data(), ck[s].size());
    if (st != HD_OK) return st;
  }
  return HD_OK;
}

}  // namespace

hd_status hd_set_schedule(hd_ctx *ctx, const hd_schedule *shape) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "hd_set_schedule before hd_finalize");
  if (!shape) return fail(ctx, HD_E_ARG, "null schedule");
  if (ctx->exec == HD_EXEC_SEQUENTIAL) return fail(ctx, HD_E_STATE, "the sequential scheduler has no launch shapes");
  const int sb = shape->small_block, lb = shape->large_block;
  if ((sb != 0 && sb != 256 && sb != 512 && sb != 1024) || lb < 64 || lb > 1024 || lb % 64 != 0)
    return fail(ctx, HD_E_ARG, "small_block must be 0, 256, 512 or 1024; large_block a multiple of 64 in [64, 1024]");
  hd_status st;
  if (ctx->need_eval && (st = evaluate_all(ctx)) != HD_OK) return st;
  if ((st = apply_schedule(ctx, *shape)) != HD_OK) return st;
  ctx->tuned_ms = shape->ms_per_step;
  return HD_OK;
}

hd_status hd_autotune(hd_ctx *ctx, double min_ms, int64_t max_steps, hd_schedule *trials, int32_t cap,
                      int32_t *n_trials) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "hd_autotune before hd_finalize");
  if (ctx->exec == HD_EXEC_SEQUENTIAL) return fail(ctx, HD_E_STATE, "the sequential scheduler has no launch shapes to tune");
  if (!(min_ms > 0) || max_steps < 8 || cap < 0 || (cap > 0 && !trials))
    return fail(ctx, HD_E_ARG, "hd_autotune needs min_ms > 0, max_steps >= 8, a trial buffer when cap > 0");
  const int S = (int)ctx->sys.size();
  hd_status st;
  if (ctx->need_eval && (st = evaluate_all(ctx)) != HD_OK) return st;
  // checkpoint every system
  std::vector<std::vector<char>> ck(S);
  for (int s = 0; s < S; ++s) {
    size_t b = 0;
    if ((st = hd_get_state(ctx, s, nullptr, &b)) != HD_OK) return st;
    ck[s].resize(b);
    if ((st = hd_get_state(ctx, s, ck[s].data(), &b)) != HD_OK) return st;
  }
  hd_schedule prev{};
  if ((st = hd_get_schedule(ctx, &prev)) != HD_OK) return st;
  // candidates: LDS-resident or not for the systems that fit, its workgroup
  // size, and the shape of the rest (grid tile size, or one workgroup per
  // system on the global kernel)
  bool any_fit = false, any_large = false;
  int nmax_fit = 0;
  for (int s = 0; s < S; ++s) {
    if (ctx->sys[s].n <= 1024) { any_fit = true; nmax_fit = std::max(nmax_fit, ctx->sys[s].n); }
    else any_large = true;
  }
  std::vector<hd_schedule> cand;
  const int large_grid[4] = {64, 128, 256, 512}, large_pers[3] = {256, 512, 1024};
  auto add_large = [&](hd_schedule c, bool need) {
    if (!need) { c.persistent_large = 0; c.large_block = 256; cand.push_back(c); return; }
    for (int b : large_grid) { c.persistent_large = 0; c.large_block = b; cand.push_back(c); }
    if (ctx->exec == HD_EXEC_BATCHED)
      for (int b : large_pers) { c.persistent_large = 1; c.large_block = b; cand.push_back(c); }
  };
  if (ctx->exec == HD_EXEC_BATCHED && any_fit) {
    for (int half = (ctx->prec == HD_FP64 ? 0 : 1); half >= 0; --half)
      for (int b : {256, 512, 1024}) {
        if (b < nmax_fit && b != 1024) continue;
        add_large(hd_schedule{1, b, 0, 256, half, 0.0}, any_large);
      }
  }
  add_large(hd_schedule{0, 0, 0, 256, 0, 0.0}, true);
  // measure
  std::vector<hd_schedule> done;
  double best_ms = 0.0;
  int best = -1;
  for (const hd_schedule &c0 : cand) {
    hd_schedule c = c0;
    if ((st = apply_schedule(ctx, c)) != HD_OK) return st;
    if ((st = restore_all(ctx, ck)) != HD_OK) return st;
    if ((st = hd_step(ctx, 4)) != HD_OK) break;         // warm-up: code objects, first rebuild
    double ms_step = 0.0;
    for (int64_t k = 8;; k *= 4) {
      if ((st = hd_step(ctx, std::min(k, max_steps))) != HD_OK) break;
      double ms = 0.0;
      if ((st = hd_last_step_timing(ctx, &ms, nullptr)) != HD_OK) return st;
      ms_step = ms / (double)std::min(k, max_steps);
      if (ms >= min_ms || k >= max_steps) break;
      if (best >= 0 && ms_step > 3.0 * best_ms) break;
    }
    if (st != HD_OK) break;
    c.ms_per_step = ms_step;
    if (best < 0 || ms_step < best_ms) { best = (int)done.size(); best_ms = ms_step; }
    done.push_back(c);
  }
  // keep the fastest shape (or the previous one after a failure) and put
  // every system back where it was
  const hd_status trial_st = st;
  if (trial_st != HD_OK && trial_st != HD_E_UNSTABLE) return trial_st;
  const hd_schedule keep = (trial_st == HD_OK && best >= 0) ? done[best] : prev;
  if ((st = apply_schedule(ctx, keep)) != HD_OK) return st;
  if ((st = restore_all(ctx, ck)) != HD_OK) return st;
  ctx->tuned_ms = trial_st == HD_OK ? keep.ms_per_step : 0.0;
  if (n_trials) *n_trials = (int32_t)done.size();
  for (int32_t q = 0; q < cap && q < (int32_t)done.size(); ++q) trials[q] = done[q];
  if (trial_st != HD_OK) return fail(ctx, trial_st, "a trial froze every system; previous launch shape kept");
  return HD_OK;
}

hd_status hd_last_step_timing(hd_ctx *ctx, double *ms, int64_t *launches) {
  CHECK_CTX();
  HIPCHK(hipEventSynchronize(ctx->ev1));
  float t = 0.f;
  HIPCHK(hipEventElapsedTime(&t, ctx->ev0, ctx->ev1));
  if (ms) *ms = t;
  if (launches) *launches = ctx->last_launches;
  return HD_OK;
}

static hd_status copy_field(hd_ctx *ctx, int32_t sys, const double *base, double *out, hipMemcpyKind kind) {
  const SysHost &s = ctx->sys[sys];
  const SysDesc &D = ctx->h_desc[sys];
  for (int k = 0; k < s.dim; ++k)
    HIPCHK(hipMemcpyAsync(out + (size_t)k * s.n, base + k * ctx->ntot + D.off, sizeof(double) * s.n, kind, ctx->stream));
  return HD_OK;
}

hd_status hd_read_forces(hd_ctx *ctx, int32_t sys, int32_t which, double *out) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !out) return fail(ctx, HD_E_ARG, "bad system or null output");
  const double *src = which == HD_FORCE_TOTAL ? ctx->A.ftot : which == HD_FORCE_LJ ? ctx->A.flj
                    : which == HD_FORCE_BIAS ? ctx->A.fb : which == HD_HU ? ctx->A.hu
                    : which == HD_TUU ? ctx->A.tuu : nullptr;
  if (!src) return fail(ctx, HD_E_ARG, "unknown force selector");
  hd_status st = copy_field(ctx, sys, src, out, hipMemcpyDeviceToHost);
  if (st != HD_OK) return st;
  SysState T;
  HIPCHK(hipMemcpyAsync(&T, ctx->d_state + sys, sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (which == HD_TUU && ctx->h_desc[sys].eig) {
    // the kernels keep T[q,q] of the mode as stored; along the unit mode:
    const size_t nd = (size_t)ctx->sys[sys].dim * ctx->sys[sys].n;
    for (size_t q = 0; q < nd; ++q) out[q] *= T.eig_inv_q2;
  }
  return HD_OK;
}

hd_status hd_read_positions(hd_ctx *ctx, int32_t sys, double *out) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !out) return fail(ctx, HD_E_ARG, "bad system or null output");
  hd_status st = copy_field(ctx, sys, ctx->A.x, out, hipMemcpyDeviceToHost);
  if (st != HD_OK) return st;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HD_OK;
}

hd_status hd_read_min_mode(hd_ctx *ctx, int32_t sys, double *out) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !out) return fail(ctx, HD_E_ARG, "bad system or null output");
  const SysHost &h = ctx->sys[sys];
  if (!ctx->h_desc[sys].eig) return fail(ctx, HD_E_STATE, "the system is not biased on the eigenvalue");
  hd_status st = copy_field(ctx, sys, ctx->A.qm, out, hipMemcpyDeviceToHost);
  if (st != HD_OK) return st;
  SysState T;
  HIPCHK(hipMemcpyAsync(&T, ctx->d_state + sys, sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  // normalised over the degrees of freedom: mobile atoms and the rigid body
  double q2 = 0.0;
  for (int i = 0; i < h.n; ++i)
    for (int k = 0; k < h.dim; ++k) {
      double &q = out[(size_t)k * h.n + i];
      if (h.role[i] == HD_ROLE_RIGID) q = T.qR[k];
      else if (h.role[i] == HD_ROLE_FIXED) q = 0.0;
      else q2 += q * q;
    }
  if (h.n_rigid > 0)
    for (int k = 0; k < h.dim; ++k) q2 += T.qR[k] * T.qR[k];
  const double inv = q2 > 0.0 ? 1.0 / std::sqrt(q2) : 0.0;
  for (size_t q = 0; q < (size_t)h.dim * h.n; ++q) out[q] *= inv;
  return HD_OK;
}

hd_status hd_read_velocities(hd_ctx *ctx, int32_t sys, double *out) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !out) return fail(ctx, HD_E_ARG, "bad system or null output");
  hd_status st = copy_field(ctx, sys, ctx->A.v, out, hipMemcpyDeviceToHost);
  if (st != HD_OK) return st;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HD_OK;
}

hd_status hd_copy_positions_device(hd_ctx *ctx, int32_t sys, double *dev_out) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !dev_out) return fail(ctx, HD_E_ARG, "bad system or null output");
  return copy_field(ctx, sys, ctx->A.x, dev_out, hipMemcpyDeviceToDevice);
}

hd_status hd_copy_forces_device(hd_ctx *ctx, int32_t sys, int32_t which, double *dev_out) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !dev_out) return fail(ctx, HD_E_ARG, "bad system or null output");
  const double *src = which == HD_FORCE_TOTAL ? ctx->A.ftot : which == HD_FORCE_LJ ? ctx->A.flj
                    : which == HD_FORCE_BIAS ? ctx->A.fb : which == HD_HU ? ctx->A.hu
                    : which == HD_TUU ? ctx->A.tuu : nullptr;
  if (!src) return fail(ctx, HD_E_ARG, "unknown force selector");
  return copy_field(ctx, sys, src, dev_out, hipMemcpyDeviceToDevice);
}

// The Arrays member of each bindable field, in HD_FIELD_* order.
static double *&bound_field(hd_ctx *ctx, int field) {
  hdk::Arrays &A = ctx->A;
  switch (field) {
    case HD_FIELD_POSITIONS: return A.x;
    case HD_FIELD_VELOCITIES: return A.v;
    case HD_FIELD_FORCES: return A.ftot;
    case HD_FIELD_FORCES_LJ: return A.flj;
    case HD_FIELD_FORCES_BIAS: return A.fb;
    default: return A.hu;
  }
}

// Captured graphs hold the batch arrays' addresses as kernel arguments: drop
// them so that the next call captures the current ones.
static hd_status drop_graphs(hd_ctx *ctx) {
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream2));
  for (auto &P : ctx->plans) {
    if (P.exec) HIPCHK(hipGraphExecDestroy(P.exec));
    if (P.tail_exec) HIPCHK(hipGraphExecDestroy(P.tail_exec));
    P.exec = nullptr;
    P.tail_exec = nullptr;
    P.tail_steps = 0;
  }
  if (ctx->batched_graph) HIPCHK(hipGraphExecDestroy(ctx->batched_graph));
  ctx->batched_graph = nullptr;
  return HD_OK;
}

hd_status hd_batch_layout(hd_ctx *ctx, int32_t sys, int64_t *offset, int64_t *ntot) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !offset || !ntot) return fail(ctx, HD_E_ARG, "bad system or null output");
  *offset = ctx->h_desc[sys].off;
  *ntot = ctx->ntot;
  return HD_OK;
}

hd_status hd_bind_device(hd_ctx *ctx, int32_t sys, int32_t field, void *dev_ptr) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "hd_bind_device before hd_finalize");
  if (sys != HD_ALL_SYSTEMS)
    return fail(ctx, HD_E_ARG, "fields are bound for the whole batch (sys = HD_ALL_SYSTEMS)");
  if (field < HD_FIELD_POSITIONS || field > HD_FIELD_HU) return fail(ctx, HD_E_ARG, "unknown field");
  if (dev_ptr) {
    if (((uintptr_t)dev_ptr & 7u) != 0) return fail(ctx, HD_E_ARG, "device pointer not 8-byte aligned");
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, dev_ptr) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, HD_E_ARG, "not a HIP device allocation");
    }
    if (at.type != hipMemoryTypeDevice || at.device != ctx->device)
      return fail(ctx, HD_E_ARG, "not device memory of the context's device");
  }
  hd_status st = sync_in(ctx);
  if (st != HD_OK) return st;
  double *&cur = bound_field(ctx, field);
  double *&own = ctx->own_field[field];
  double *target = dev_ptr ? (double *)dev_ptr : (own ? own : cur);
  if (target == cur) return HD_OK;
  if ((st = drop_graphs(ctx)) != HD_OK) return st;
  // the field's current contents move to its new storage
  HIPCHK(hipMemcpyAsync(target, cur, sizeof(double) * 3 * ctx->ntot, hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (!own) own = cur;
  cur = target;
  if (cur == own) own = nullptr;
  return HD_OK;
}

static void scalars_of(const SysState &T, hd_scalars *out) {
  out->e_pot = T.e_pot;
  out->e_kin = T.e_kin;
  out->dv = T.dv;
  out->dvp = T.dvp;
  out->g = T.g;
  out->d = T.d;
  out->t_md = T.t_md;
  out->t_hyper = T.t_hyper;
  out->x_slider = T.x_slider;
  out->x_tip = T.x_tip;
  out->f_lat = T.f_lat;
  out->step = T.step;
  out->flags = T.flags;
  out->n_rebuilds = T.n_rebuilds;
  out->kappa = T.kappa;
  out->dv1 = T.dv1;
  out->dv2 = T.dv2;
  out->e_nhc = T.e_nhc;
  out->lambda = T.lambda;
}

hd_status hd_read_scalars(hd_ctx *ctx, int32_t sys, hd_scalars *out) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !out) return fail(ctx, HD_E_ARG, "bad system or null output");
  SysState T;
  HIPCHK(hipMemcpyAsync(&T, ctx->d_state + sys, sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  scalars_of(T, out);
  return HD_OK;
}

// The states of consecutive systems lie side by side: one copy for all.
hd_status hd_read_scalars_batch(hd_ctx *ctx, int32_t first, int32_t count, hd_scalars *out) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  const int32_t S = (int32_t)ctx->sys.size();
  if (first < 0 || count < 0 || first > S - count || (count > 0 && !out))
    return fail(ctx, HD_E_ARG, "hd_read_scalars_batch needs 0 <= first, first + count <= systems and an output");
  if (count == 0) return HD_OK;
  std::vector<SysState> T(count);
  HIPCHK(hipMemcpyAsync(T.data(), ctx->d_state + first, sizeof(SysState) * count, hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int32_t k = 0; k < count; ++k) scalars_of(T[k], out + k);
  return HD_OK;
}

// Replace positions of one system: the rigid body follows its first atom.
hd_status hd_set_positions(hd_ctx *ctx, int32_t sys, const double *pos) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK || !pos) return fail(ctx, HD_E_ARG, "bad system or null positions");
  SysHost &s = ctx->sys[sys];
  const int n = s.n;
  std::vector<double> cur((size_t)s.dim * n);
  double XR[3] = {s.XR[0], s.XR[1], s.XR[2]};
  SysState T{};
  if (ctx->finalized) {
    hd_status st = copy_field(ctx, sys, ctx->A.x, cur.data(), hipMemcpyDeviceToHost);
    if (st != HD_OK) return st;
    HIPCHK(hipMemcpyAsync(&T, ctx->d_state + sys, sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 3; ++k) XR[k] = T.XR[k];
  } else {
    cur = s.pos;
  }
  if (s.n_rigid > 0) {
    const int f = s.first_rigid;
    for (int k = 0; k < s.dim; ++k)
      XR[k] = XR[k] + minimg_h(pos[(size_t)k * n + f] - cur[(size_t)k * n + f], s.box[k], s.periodic[k]);
  }
  std::vector<double> nx((size_t)s.dim * n);
  for (int k = 0; k < s.dim; ++k)
    for (int i = 0; i < n; ++i) {
      const size_t q = (size_t)k * n + i;
      nx[q] = (s.role[i] == HD_ROLE_RIGID) ? wrap_h(XR[k] + s.cofs[q], s.box[k], s.periodic[k]) : pos[q];
    }
  if (!ctx->finalized) {
    s.pos = nx;
    for (int k = 0; k < 3; ++k) s.XR[k] = XR[k];
    return HD_OK;
  }
  const SysDesc &D = ctx->h_desc[sys];
  for (int k = 0; k < s.dim; ++k)
    HIPCHK(hipMemcpyAsync(ctx->A.x + k * ctx->ntot + D.off, nx.data() + (size_t)k * n, sizeof(double) * n,
                          hipMemcpyHostToDevice, ctx->stream));
  for (int k = 0; k < 3; ++k) T.XR[k] = XR[k];
  T.rebuild = 1;
  T.flags &= ~HD_FLAG_UNSTABLE;  // new positions: the system runs again
  ctx->all_frozen = false;
  HIPCHK(hipMemcpyAsync(ctx->d_state + sys, &T, sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  if (!ctx->plans.empty()) {
    int32_t one = 1;
    HIPCHK(hipMemcpyAsync(ctx->A.rebuild_flag + sys, &one, sizeof(one), hipMemcpyHostToDevice, ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->need_eval = true;
  return HD_OK;
}

hd_status hd_set_velocities(hd_ctx *ctx, int32_t sys, const double *vel) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK || !vel) return fail(ctx, HD_E_ARG, "bad system or null velocities");
  SysHost &s = ctx->sys[sys];
  const int n = s.n;
  std::vector<double> nv((size_t)s.dim * n, 0.0);
  double VR[3] = {0, 0, 0};
  for (int k = 0; k < s.dim; ++k) {
    double sum = 0.0;
    for (int i = 0; i < n; ++i) {
      const size_t q = (size_t)k * n + i;
      if (s.role[i] == HD_ROLE_MOBILE) nv[q] = vel[q];
      else if (s.role[i] == HD_ROLE_RIGID) sum += vel[q];
    }
    if (s.n_rigid > 0) VR[k] = sum / s.n_rigid;
    for (int i = 0; i < n; ++i)
      if (s.role[i] == HD_ROLE_RIGID) nv[(size_t)k * n + i] = VR[k];
  }
  if (!ctx->finalized) {
    s.vel = nv;
    s.init_vel = false;
    return HD_OK;
  }
  const SysDesc &D = ctx->h_desc[sys];
  for (int k = 0; k < s.dim; ++k)
    HIPCHK(hipMemcpyAsync(ctx->A.v + k * ctx->ntot + D.off, nv.data() + (size_t)k * n, sizeof(double) * n,
                          hipMemcpyHostToDevice, ctx->stream));
  SysState T;
  HIPCHK(hipMemcpyAsync(&T, ctx->d_state + sys, sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < 3; ++k) T.VR[k] = VR[k];
  HIPCHK(hipMemcpyAsync(ctx->d_state + sys, &T, sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HD_OK;
}

// Checkpoint layout: header, then x, v, rO, xb, ftot and the mode estimate
// as [dim][n] doubles.
// params_fp fingerprints the parameters the stored forces were evaluated
// with (the potential, the drive and the bias), so that a state restored into
// a system with other parameters gets its forces re-evaluated.
struct CkptHeader {
  uint32_t magic, version;
  int32_t dim, n;
  uint64_t params_fp;
  SysState state;
};
static const uint32_t kMagic = 0x68644350u;  // "hdCP"
static const uint32_t kCkptVersion = 3;

// FNV-1a over the parameters that shape a system's forces (not the seed,
// the time step or the thermostat, which only shape the dynamics).
static uint64_t params_fingerprint(const SysHost &h) {
  uint64_t f = 1469598103934665603ull;
  auto mix = [&f](const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) { f ^= b[i]; f *= 1099511628211ull; }
  };
  mix(&h.dim, sizeof h.dim); mix(&h.n, sizeof h.n);
  mix(h.box, sizeof h.box); mix(h.periodic, sizeof h.periodic); mix(&h.mass, sizeof h.mass);
  mix(&h.lj, sizeof h.lj); mix(&h.dr, sizeof h.dr); mix(&h.bias, sizeof h.bias);
  mix(&h.tip_bonds, sizeof h.tip_bonds); mix(&h.k_bond, sizeof h.k_bond); mix(&h.r_bond, sizeof h.r_bond);
  mix(&h.r_bond_cut, sizeof h.r_bond_cut); mix(&h.bias_var1, sizeof h.bias_var1);
  mix(&h.bias_var2, sizeof h.bias_var2); mix(&h.b2_lo, sizeof h.b2_lo); mix(&h.b2_hi, sizeof h.b2_hi);
  mix(h.XR0, sizeof h.XR0);
  return f;
}

hd_status hd_get_state(hd_ctx *ctx, int32_t sys, void *buf, size_t *bytes) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !bytes) return fail(ctx, HD_E_ARG, "bad system or null size");
  const SysHost &s = ctx->sys[sys];
  const size_t nd = (size_t)s.dim * s.n;
  const size_t need = sizeof(CkptHeader) + 6 * nd * sizeof(double);
  if (!buf) { *bytes = need; return HD_OK; }
  if (*bytes < need) return fail(ctx, HD_E_ARG, "checkpoint buffer too small");
  CkptHeader h{};
  h.magic = kMagic;
  h.version = kCkptVersion;
  h.dim = s.dim;
  h.n = s.n;
  h.params_fp = params_fingerprint(s);
  HIPCHK(hipMemcpyAsync(&h.state, ctx->d_state + sys, sizeof(SysState), hipMemcpyDeviceToHost, ctx->stream));
  double *p = (double *)((char *)buf + sizeof(CkptHeader));
  // the eigenvalue variable's mode estimate (mobile atoms) rides along as a
  // sixth field, zero for systems without it
  const double *fields[6] = {ctx->A.x, ctx->A.v, ctx->A.rO, ctx->A.xb, ctx->A.ftot, ctx->A.qm};
  const int nf = ctx->any_eig ? 6 : 5;
  for (int f = 0; f < nf; ++f) {
    hd_status st = copy_field(ctx, sys, fields[f], p + f * nd, hipMemcpyDeviceToHost);
    if (st != HD_OK) return st;
  }
  if (nf == 5) std::memset(p + 5 * nd, 0, nd * sizeof(double));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::memcpy(buf, &h, sizeof(h));
  *bytes = need;
  return HD_OK;
}

hd_status hd_set_state(hd_ctx *ctx, int32_t sys, const void *buf, size_t bytes) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !buf) return fail(ctx, HD_E_ARG, "bad system or null buffer");
  const SysHost &s = ctx->sys[sys];
  const size_t nd = (size_t)s.dim * s.n;
  if (bytes < sizeof(CkptHeader) + 6 * nd * sizeof(double)) return fail(ctx, HD_E_ARG, "checkpoint too short");
  CkptHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kMagic || h.version != kCkptVersion || h.dim != s.dim || h.n != s.n)
    return fail(ctx, HD_E_ARG, "checkpoint does not match this system");
  const double *p = (const double *)((const char *)buf + sizeof(CkptHeader));
  double *fields[6] = {ctx->A.x, ctx->A.v, ctx->A.rO, ctx->A.xb, ctx->A.ftot, ctx->A.qm};
  const SysDesc &D = ctx->h_desc[sys];
  for (int f = 0; f < (ctx->any_eig ? 6 : 5); ++f)
    for (int k = 0; k < s.dim; ++k)
      HIPCHK(hipMemcpyAsync(fields[f] + k * ctx->ntot + D.off, p + f * nd + (size_t)k * s.n, sizeof(double) * s.n,
                            hipMemcpyHostToDevice, ctx->stream));
  SysState T = h.state;
  T.rebuild = 2;  // rebuild the list from the recorded build positions
  HIPCHK(hipMemcpyAsync(ctx->d_state + sys, &T, sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  if (!ctx->plans.empty()) {
    // the grid scheduler rebuilds its list from the restored build positions
    int32_t two = 2;
    HIPCHK(hipMemcpyAsync(ctx->A.rebuild_flag + sys, &two, sizeof(two), hipMemcpyHostToDevice, ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->all_frozen = false;
  // forces evaluated under other parameters (another slider position, bias,
  // ...) are re-evaluated before the next step, as after a parameter change
  if (h.params_fp != params_fingerprint(s)) ctx->need_eval = true;
  return HD_OK;
}

// FIRE quench of the listed systems (hd_quench).  With no_alloc, the FIRE
// state, the system list and the reduction partials are carved out of the
// device's static scratch array and nothing is allocated on the device; the
// read-out arrays (LJ and bias forces, H u, u) are then
// re-evaluated at the restored positions instead of being saved and copied
// back.
static hd_status quench_run(hd_ctx *ctx, const int32_t *systems, int32_t count, double ftol, int64_t max_iters,
                            int32_t mode, int64_t *iters, double *max_disp, double *x_min, bool no_alloc) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "hd_quench before hd_finalize");
  if (!systems || count <= 0 || !iters || !max_disp || !(ftol > 0) || max_iters < 1 ||
      (mode != HD_QUENCH_CHECK && mode != HD_QUENCH_SET_REFERENCE))
    return fail(ctx, HD_E_ARG, "hd_quench needs systems, count > 0, ftol > 0, max_iters >= 1, a known mode");
  const int S = (int)ctx->sys.size();
  std::vector<char> seen(S, 0);
  int nmax = 0;
  for (int k = 0; k < count; ++k) {
    const int s = systems[k];
    if (s < 0 || s >= S || seen[s]) return fail(ctx, HD_E_ARG, "quench systems must be distinct valid indices");
    seen[s] = 1;
    nmax = std::max(nmax, ctx->sys[s].n);
  }
  const size_t list_bytes = (sizeof(int32_t) * count + 255) & ~(size_t)255;
  const size_t fire_bytes = (sizeof(hdk::FireSys) * count + 255) & ~(size_t)255;
  const size_t part_bytes = sizeof(double) * hdk::fire_partials_doubles(count, nmax);
  char *scratch = nullptr;
  if (no_alloc) {
    if (list_bytes + fire_bytes + part_bytes > kScratchBytes)
      return fail(ctx, HD_E_ARG, "hd_quench_noalloc: " + std::to_string(count) + " systems of up to " +
                                     std::to_string(nmax) + " atoms need " +
                                     std::to_string(list_bytes + fire_bytes + part_bytes) +
                                     " bytes of scratch, above the " + std::to_string(kScratchBytes) +
                                     "-byte limit");
    scratch = (char *)g_scratch[ctx->device];
    if (!scratch) return fail(ctx, HD_E_STATE, "hd_quench_noalloc: the device's scratch address is not known");
  }
  hd_status st = sync_in(ctx);
  if (st != HD_OK) return st;
  if (ctx->need_eval && (st = evaluate_all(ctx)) != HD_OK) return st;
  // every system's state is checkpointed (the quench moves the listed ones
  // and re-evaluates all), and the read-out arrays saved, so the run
  // continues afterwards exactly as it would have
  std::vector<std::vector<char>> ck(S);
  for (int s = 0; s < S; ++s) {
    size_t b = 0;
    if ((st = hd_get_state(ctx, s, nullptr, &b)) != HD_OK) return st;
    ck[s].resize(b);
    if ((st = hd_get_state(ctx, s, ck[s].data(), &b)) != HD_OK) return st;
  }
  for (int k = 0; k < count; ++k) {
    SysState T;
    std::memcpy(&T, ck[systems[k]].data() + offsetof(CkptHeader, state), sizeof(T));
    if (T.flags & hdk::FLAG_UNSTABLE) return fail(ctx, HD_E_STATE, "cannot quench a system frozen as unstable");
  }
  const size_t N = (size_t)ctx->ntot;
  const size_t ubytes = 3 * N * (ctx->prec == HD_FP64 ? sizeof(double) : sizeof(float));
  struct Saved { void *dev; void *copy; size_t bytes; };
  std::vector<Saved> saved;
  if (!no_alloc)
    saved = {{ctx->A.flj, nullptr, 3 * N * sizeof(double)},
             {ctx->A.hu, nullptr, 3 * N * sizeof(double)},
             {ctx->A.fb, nullptr, 3 * N * sizeof(double)},
             {ctx->A.u, nullptr, ubytes}};
  int32_t *d_list = nullptr;
  hdk::FireSys *d_fire = nullptr;
  double *d_fpart = nullptr;
  auto release = [&]() {
    for (auto &v : saved)
      if (v.copy) (void)hipFree(v.copy);
    if (no_alloc) return;
    if (d_list) (void)hipFree(d_list);
    if (d_fire) (void)hipFree(d_fire);
    if (d_fpart) (void)hipFree(d_fpart);
  };
  auto hip_fail = [&](hipError_t e) {
    release();
    return fail(ctx, HD_E_HIP, std::string("hd_quench: ") + hipGetErrorString(e));
  };
  hipError_t e = hipSuccess;
  for (auto &v : saved) {
    if ((e = hipMalloc(&v.copy, v.bytes)) != hipSuccess) return hip_fail(e);
    if ((e = hipMemcpyAsync(v.copy, v.dev, v.bytes, hipMemcpyDeviceToDevice, ctx->stream)) != hipSuccess)
      return hip_fail(e);
  }
  if (no_alloc) {
    d_list = (int32_t *)scratch;
    d_fire = (hdk::FireSys *)(scratch + list_bytes);
    d_fpart = (double *)(scratch + list_bytes + fire_bytes);
  } else {
    if ((e = hipMalloc(&d_list, list_bytes)) != hipSuccess) return hip_fail(e);
    if ((e = hipMalloc(&d_fire, fire_bytes)) != hipSuccess) return hip_fail(e);
    if ((e = hipMalloc(&d_fpart, part_bytes)) != hipSuccess) return hip_fail(e);
  }
  // LDS-resident systems first, group by group: each group's listed systems
  // take the whole quench in one launch of the LDS kernel's FIRE mode; the
  // others (grid plans, the one-workgroup global kernel) follow, iterated
  // from here.  ord is the order of d_list and of the FIRE states.
  using Group = std::remove_reference<decltype(ctx->groups[0])>::type;
  struct LdsRun { const Group *G; int first, n; };
  std::vector<int> at(S, -1);
  for (int k = 0; k < count; ++k) at[systems[k]] = k;
  std::vector<char> in_lds(S, 0);
  std::vector<int32_t> ord;
  std::vector<LdsRun> lds_runs;
  for (const auto &G : ctx->groups) {
    if (!G.small) continue;
    const int f = (int)ord.size();
    for (int s : G.ids)
      if (at[s] >= 0) { ord.push_back(s); in_lds[s] = 1; }
    if ((int)ord.size() > f) lds_runs.push_back({&G, f, (int)ord.size() - f});
  }
  const int n_lds = (int)ord.size();
  int nmax_rest = 0;
  for (int k = 0; k < count; ++k)
    if (!in_lds[systems[k]]) {
      ord.push_back(systems[k]);
      nmax_rest = std::max(nmax_rest, ctx->sys[systems[k]].n);
    }
  const int n_rest = count - n_lds;
  std::vector<hdk::FireSys> fs(count);
  for (int k = 0; k < count; ++k) {
    fs[k] = hdk::FireSys{};
    fs[k].dt = ctx->sys[ord[k]].th.dt;
    fs[k].alpha = hdk::kFireAlpha0;
  }
  if ((e = hipMemcpyAsync(d_list, ord.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice, ctx->stream)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(d_fire, fs.data(), sizeof(hdk::FireSys) * count, hipMemcpyHostToDevice, ctx->stream)) !=
          hipSuccess)
    return hip_fail(e);
  // FIRE starts at rest: the listed systems' velocities and rigid-body
  // velocity are zeroed (the checkpoint restores them)
  for (int k = 0; k < count; ++k) {
    const int s = systems[k];
    for (int d = 0; d < ctx->sys[s].dim; ++d)
      if ((e = hipMemsetAsync(ctx->A.v + d * ctx->ntot + ctx->h_desc[s].off, 0, sizeof(double) * ctx->sys[s].n,
                              ctx->stream)) != hipSuccess)
        return hip_fail(e);
    SysState T;
    std::memcpy(&T, ck[s].data() + offsetof(CkptHeader, state), sizeof(T));
    for (int d = 0; d < 3; ++d) T.VR[d] = 0.0;
    if ((e = hipMemcpyAsync(ctx->d_state + s, &T, sizeof(T), hipMemcpyHostToDevice, ctx->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(ctx->stream)) != hipSuccess)
      return hip_fail(e);
  }
  // the unbiased potential: the bias is off for the quench
  std::vector<int32_t> bias_was(S);
  for (int s = 0; s < S; ++s) {
    bias_was[s] = ctx->sys[s].bias.enabled;
    ctx->sys[s].bias.enabled = 0;
    if ((st = upload_desc(ctx, s)) != HD_OK) { release(); return st; }
  }
  // iterations: forces, then the FIRE step; convergence read back every 32.
  // Grid lists are rebuilt only when atoms leave half the skin.
  st = evaluate_all(ctx, false);
  for (const auto &R : lds_runs) {
    if (st != HD_OK || e != hipSuccess) break;
    for (int q = 0; q < R.n; ++q) ctx->sorted_lists[ord[R.first + q]] = 0;
    e = hdk::launch_small_fire(small_kind(ctx), R.G->dim, ctx->d_desc, ctx->d_state, ctx->A, d_list + R.first, R.n,
                               R.G->nmax, R.G->maxnb, R.G->cellmax, max_iters, d_fire + R.first, ftol, ctx->stream);
  }
  int64_t it = 0;
  for (; n_rest > 0 && st == HD_OK && e == hipSuccess && it < max_iters; ++it) {
    if ((e = hdk::fire_iteration(ctx->d_desc, ctx->d_state, ctx->A, d_list + n_lds, n_rest, nmax_rest,
                                 d_fire + n_lds, ftol, it, d_fpart, ctx->stream)) != hipSuccess)
      break;
    if ((st = evaluate_all(ctx, false)) != HD_OK) break;
    if ((it & 31) == 31) {
      if ((e = hipMemcpyAsync(fs.data() + n_lds, d_fire + n_lds, sizeof(hdk::FireSys) * n_rest,
                              hipMemcpyDeviceToHost, ctx->stream)) != hipSuccess ||
          (e = hipStreamSynchronize(ctx->stream)) != hipSuccess)
        break;
      bool all = true;
      for (int k = n_lds; k < count; ++k) all = all && fs[k].done;
      if (all) break;
    }
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(fs.data(), d_fire, sizeof(hdk::FireSys) * count, hipMemcpyDeviceToHost, ctx->stream);
  // the minima (rigid atoms sit at the rigid body's final position)
  size_t tot = 0;
  for (int k = 0; k < count; ++k) tot += (size_t)ctx->sys[systems[k]].dim * ctx->sys[systems[k]].n;
  std::vector<double> xm(tot);
  if (e == hipSuccess && st == HD_OK) {
    size_t o = 0;
    for (int k = 0; k < count && st == HD_OK; ++k) {
      st = copy_field(ctx, systems[k], ctx->A.x, xm.data() + o, hipMemcpyDeviceToHost);
      o += (size_t)ctx->sys[systems[k]].dim * ctx->sys[systems[k]].n;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  // restore the bias, the saved arrays and every system's state
  for (int s = 0; s < S; ++s) {
    ctx->sys[s].bias.enabled = bias_was[s];
    const hd_status su = upload_desc(ctx, s);
    if (st == HD_OK) st = su;
  }
  for (auto &v : saved)
    if (e == hipSuccess) e = hipMemcpyAsync(v.dev, v.copy, v.bytes, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  release();
  if (e != hipSuccess) return fail(ctx, HD_E_HIP, std::string("hd_quench: ") + hipGetErrorString(e));
  if (st != HD_OK) return st;
  if ((st = restore_all(ctx, ck)) != HD_OK) return st;
  // without saved copies the read-out arrays are evaluated again at the
  // restored positions (lists rebuilt from the restored build positions,
  // which reproduces them bit for bit), and the states restored once more so
  // that the pending rebuild from the build positions is as hd_quench leaves it
  if (no_alloc) {
    if ((st = evaluate_all(ctx, false)) != HD_OK) return st;
    if ((st = restore_all(ctx, ck)) != HD_OK) return st;
  }
  // results: iterations, the largest displacement from r_O (check) or from
  // the starting positions (set reference), the minima
  std::vector<int> pos(count);   // listed system k's FIRE state is fs[pos[k]]
  for (int q = 0; q < count; ++q) pos[at[ord[q]]] = q;
  size_t o = 0;
  for (int k = 0; k < count; ++k) {
    const int s = systems[k];
    const SysHost &h = ctx->sys[s];
    const size_t nd = (size_t)h.dim * h.n;
    const double *ref = (const double *)(ck[s].data() + sizeof(CkptHeader)) + (mode == HD_QUENCH_CHECK ? 2 : 0) * nd;
    double worst = 0.0;
    for (int i = 0; i < h.n; ++i) {
      double d2 = 0.0;
      for (int d = 0; d < h.dim; ++d) {
        double dx = xm[o + (size_t)d * h.n + i] - ref[(size_t)d * h.n + i];
        if (h.periodic[d]) dx = minimg_h(dx, h.box[d], 1);
        d2 += dx * dx;
      }
      worst = std::max(worst, std::sqrt(d2));
    }
    const hdk::FireSys &f = fs[pos[k]];
    iters[k] = f.done ? f.iters : -max_iters;
    max_disp[k] = worst;
    if (x_min) std::memcpy(x_min + o, xm.data() + o, sizeof(double) * nd);
    if (mode == HD_QUENCH_SET_REFERENCE && (st = hd_set_reference(ctx, s, xm.data() + o)) != HD_OK) return st;
    o += nd;
  }
  return sync_out(ctx);
}

hd_status hd_quench(hd_ctx *ctx, const int32_t *systems, int32_t count, double ftol, int64_t max_iters,
                    int32_t mode, int64_t *iters, double *max_disp, double *x_min) {
  return quench_run(ctx, systems, count, ftol, max_iters, mode, iters, max_disp, x_min, false);
}

hd_status hd_quench_noalloc(hd_ctx *ctx, const int32_t *systems, int32_t count, double ftol, int64_t max_iters,
                            int32_t mode, int64_t *iters, double *max_disp, double *x_min) {
  return quench_run(ctx, systems, count, ftol, max_iters, mode, iters, max_disp, x_min, true);
}

namespace {

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal a[0..k) and off-diagonal b[0..k-1) (Sturm sequence of its LDL^T
// factors).
int sturm_below(const std::vector<double> &a, const std::vector<double> &b, int k, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    d = a[i] - x - (i > 0 ? off / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// Smallest eigenvalue of that matrix, by bisection between Gershgorin bounds.
double tridiag_min_eig(const std::vector<double> &a, const std::vector<double> &b, int k) {
  double lo = a[0], hi = a[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(lo) + std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(a, b, k, mid) >= 1) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Eigenvector of that matrix for the eigenvalue theta: inverse iteration
// with a slightly shifted tridiagonal solve.
std::vector<double> tridiag_vec(const std::vector<double> &a, const std::vector<double> &b, int k, double theta) {
  std::vector<double> y(k, 1.0), c(k), d(k), z(k);
  const double shift = theta - 1e-10 * std::max(1.0, std::fabs(theta));
  for (int rep = 0; rep < 3; ++rep) {
    // Thomas algorithm on (T - shift I) z = y
    for (int i = 0; i < k; ++i) d[i] = a[i] - shift;
    c = y;
    for (int i = 1; i < k; ++i) {
      const double m = b[i - 1] / d[i - 1];
      d[i] -= m * b[i - 1];
      c[i] -= m * c[i - 1];
    }
    z[k - 1] = c[k - 1] / d[k - 1];
    for (int i = k - 2; i >= 0; --i) z[i] = (c[i] - b[i] * z[i + 1]) / d[i];
    double nz = 0.0;
    for (double v : z) nz += v * v;
    nz = std::sqrt(nz);
    for (int i = 0; i < k; ++i) y[i] = z[i] / nz;
  }
  return y;
}

}  // namespace

hd_status hd_min_mode(hd_ctx *ctx, int32_t sys, int32_t max_iter, double tol, uint64_t seed, double *eps,
                      int32_t *iters, double *mode) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "hd_min_mode before hd_finalize");
  if (check_sys(ctx, sys) != HD_OK || !eps || !iters || max_iter < 1 || !(tol > 0))
    return fail(ctx, HD_E_ARG, "hd_min_mode needs a valid system, eps and iters outputs, max_iter >= 1, tol > 0");
  const SysHost &h = ctx->sys[sys];
  const int dim = h.dim, n = h.n;
  std::vector<int> mob;
  for (int i = 0; i < n; ++i)
    if (h.role[i] == HD_ROLE_MOBILE) mob.push_back(i);
  const bool rigid = h.n_rigid > 0;
  const int m = dim * (int)mob.size() + (rigid ? dim : 0);   // degrees of freedom
  if (m == 0) return fail(ctx, HD_E_ARG, "the system has no degrees of freedom");
  hd_status st = sync_in(ctx);
  if (st != HD_OK) return st;
  if (ctx->need_eval && (st = evaluate_all(ctx)) != HD_OK) return st;
  const int S = (int)ctx->sys.size();
  std::vector<std::vector<char>> ck(S);
  for (int s = 0; s < S; ++s) {
    size_t b = 0;
    if ((st = hd_get_state(ctx, s, nullptr, &b)) != HD_OK) return st;
    ck[s].resize(b);
    if ((st = hd_get_state(ctx, s, ck[s].data(), &b)) != HD_OK) return st;
  }
  const size_t N = (size_t)ctx->ntot;
  const size_t ubytes = 3 * N * (ctx->prec == HD_FP64 ? sizeof(double) : sizeof(float));
  struct Saved { void *dev; void *copy; size_t bytes; };
  std::vector<Saved> saved = {{ctx->A.flj, nullptr, 3 * N * sizeof(double)},
                              {ctx->A.hu, nullptr, 3 * N * sizeof(double)},
                              {ctx->A.fb, nullptr, 3 * N * sizeof(double)},
                              {ctx->A.u, nullptr, ubytes}};
  auto release = [&]() {
    for (auto &v : saved)
      if (v.copy) (void)hipFree(v.copy);
  };
  hipError_t e = hipSuccess;
  for (auto &v : saved) {
    if ((e = hipMalloc(&v.copy, v.bytes)) != hipSuccess ||
        (e = hipMemcpyAsync(v.copy, v.dev, v.bytes, hipMemcpyDeviceToDevice, ctx->stream)) != hipSuccess) {
      release();
      return fail(ctx, HD_E_HIP, std::string("hd_min_mode: ") + hipGetErrorString(e));
    }
  }
  const size_t nd = (size_t)dim * n;
  const double *x = (const double *)(ck[sys].data() + sizeof(CkptHeader));   // positions
  std::vector<double> rO_tmp(nd), hu(nd), w_atoms(nd);
  // reduced Hessian times q: the displacement q of the degrees of freedom
  // (each rigid atom takes the rigid body's) becomes u = x - r_O by moving
  // r_O, one evaluation gives H u per atom, projected back (the rigid body
  // collects its atoms' rows, which include the drive's Hessian)
  auto matvec = [&](const std::vector<double> &q, std::vector<double> &out) -> hd_status {
    std::fill(w_atoms.begin(), w_atoms.end(), 0.0);
    for (size_t t = 0; t < mob.size(); ++t)
      for (int d = 0; d < dim; ++d) w_atoms[(size_t)d * n + mob[t]] = q[t * dim + d];
    if (rigid)
      for (int i = 0; i < n; ++i)
        if (h.role[i] == HD_ROLE_RIGID)
          for (int d = 0; d < dim; ++d) w_atoms[(size_t)d * n + i] = q[mob.size() * dim + d];
    for (size_t k = 0; k < nd; ++k) rO_tmp[k] = x[k] - w_atoms[k];
    for (int d = 0; d < dim; ++d)
      HIPCHK(hipMemcpyAsync(ctx->A.rO + d * ctx->ntot + ctx->h_desc[sys].off, rO_tmp.data() + (size_t)d * n,
                            sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
    hd_status r = evaluate_all(ctx);
    if (r != HD_OK) return r;
    if ((r = copy_field(ctx, sys, ctx->A.hu, hu.data(), hipMemcpyDeviceToHost)) != HD_OK) return r;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    out.assign(m, 0.0);
    for (size_t t = 0; t < mob.size(); ++t)
      for (int d = 0; d < dim; ++d) out[t * dim + d] = hu[(size_t)d * n + mob[t]];
    if (rigid)
      for (int i = 0; i < n; ++i)
        if (h.role[i] == HD_ROLE_RIGID)
          for (int d = 0; d < dim; ++d) out[mob.size() * dim + d] += hu[(size_t)d * n + i];
    return HD_OK;
  };
  // Lanczos with full reorthogonalisation from a seeded random start
  const int kmax = std::min(max_iter, m);
  std::vector<std::vector<double>> Q;
  std::vector<double> alpha, beta, q(m), wv;
  uint64_t rs = seed * 0x9E3779B97F4A7C15ull + 1;
  double nq = 0.0;
  for (int i = 0; i < m; ++i) {
    rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;   // xorshift64
    q[i] = (double)(rs >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    nq += q[i] * q[i];
  }
  for (double &v : q) v /= std::sqrt(nq);
  double theta = 0.0, prev = 0.0;
  int used = 0;
  bool converged = false;
  for (int j = 0; j < kmax && st == HD_OK; ++j) {
    Q.push_back(q);
    if ((st = matvec(q, wv)) != HD_OK) break;
    double a = 0.0;
    for (int i = 0; i < m; ++i) a += q[i] * wv[i];
    alpha.push_back(a);
    for (int rep = 0; rep < 2; ++rep)
      for (const auto &v : Q) {
        double c = 0.0;
        for (int i = 0; i < m; ++i) c += v[i] * wv[i];
        for (int i = 0; i < m; ++i) wv[i] -= c * v[i];
      }
    double bnorm = 0.0;
    for (double v : wv) bnorm += v * v;
    bnorm = std::sqrt(bnorm);
    used = j + 1;
    theta = tridiag_min_eig(alpha, beta, used);
    // converged, or the Krylov space is invariant (H q within the span)
    if ((j > 0 && std::fabs(theta - prev) <= tol * std::max(1.0, std::fabs(theta))) ||
        bnorm <= 1e-12 * std::max(std::fabs(a), std::fabs(theta))) {
      converged = true;
      break;
    }
    prev = theta;
    beta.push_back(bnorm);
    for (int i = 0; i < m; ++i) q[i] = wv[i] / bnorm;
  }
  // restore the run state
  for (auto &v : saved)
    if (e == hipSuccess) e = hipMemcpyAsync(v.dev, v.copy, v.bytes, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  release();
  if (e != hipSuccess) return fail(ctx, HD_E_HIP, std::string("hd_min_mode: ") + hipGetErrorString(e));
  if (st != HD_OK) return st;
  if ((st = restore_all(ctx, ck)) != HD_OK) return st;
  *eps = theta;
  *iters = converged ? used : -used;
  if (mode) {
    // the Ritz vector, unit norm over the degrees of freedom, as atom
    // displacements [dim][n] (fixed atoms 0, rigid atoms the body's)
    const std::vector<double> y = tridiag_vec(alpha, beta, used, theta);
    std::vector<double> v(m, 0.0);
    for (int j = 0; j < used; ++j)
      for (int i = 0; i < m; ++i) v[i] += y[j] * Q[j][i];
    double nv = 0.0;
    for (double c : v) nv += c * c;
    nv = std::sqrt(nv);
    std::fill(mode, mode + nd, 0.0);
    for (size_t t = 0; t < mob.size(); ++t)
      for (int d = 0; d < dim; ++d) mode[(size_t)d * n + mob[t]] = v[t * dim + d] / nv;
    if (rigid)
      for (int i = 0; i < n; ++i)
        if (h.role[i] == HD_ROLE_RIGID)
          for (int d = 0; d < dim; ++d) mode[(size_t)d * n + i] = v[mob.size() * dim + d] / nv;
  }
  return sync_out(ctx);
}

hd_status hd_min_mode_gradient(hd_ctx *ctx, int32_t sys, const double *mode, double *grad) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "hd_min_mode_gradient before hd_finalize");
  if (check_sys(ctx, sys) != HD_OK || !mode || !grad)
    return fail(ctx, HD_E_ARG, "hd_min_mode_gradient needs a valid system, a mode and an output");
  Plan *plan = nullptr;
  for (auto &P : ctx->plans)
    if (std::find(P.ids.begin(), P.ids.end(), sys) != P.ids.end()) plan = &P;
  if (!plan)
    return fail(ctx, HD_E_STATE, "hd_min_mode_gradient needs the system on the grid kernels (HD_EXEC_GRID, "
                                 "or a system with tip bonds, a general bias or the Nose-Hoover chain)");
  const SysHost &h = ctx->sys[sys];
  const int dim = h.dim, n = h.n;
  const size_t nd = (size_t)dim * n;
  // w = P q from the mode (mobile atoms' entries, the rigid body's taken from
  // its first atom), normalised over the degrees of freedom
  std::vector<double> w(nd, 0.0);
  double nq = 0.0;
  for (int i = 0; i < n; ++i)
    if (h.role[i] == HD_ROLE_MOBILE)
      for (int d = 0; d < dim; ++d) nq += mode[(size_t)d * n + i] * mode[(size_t)d * n + i];
  if (h.n_rigid > 0)
    for (int d = 0; d < dim; ++d) nq += mode[(size_t)d * n + h.first_rigid] * mode[(size_t)d * n + h.first_rigid];
  if (!(nq > 0.0) || !std::isfinite(nq)) return fail(ctx, HD_E_ARG, "the mode is zero or not finite");
  const double inv = 1.0 / std::sqrt(nq);
  for (int i = 0; i < n; ++i) {
    const int src = h.role[i] == HD_ROLE_RIGID ? h.first_rigid : i;
    if (h.role[i] != HD_ROLE_FIXED)
      for (int d = 0; d < dim; ++d) w[(size_t)d * n + i] = mode[(size_t)d * n + src] * inv;
  }
  hd_status st = sync_in(ctx);
  if (st != HD_OK) return st;
  if (ctx->need_eval && (st = evaluate_all(ctx)) != HD_OK) return st;
  const int S = (int)ctx->sys.size();
  std::vector<std::vector<char>> ck(S);
  for (int s = 0; s < S; ++s) {
    size_t b = 0;
    if ((st = hd_get_state(ctx, s, nullptr, &b)) != HD_OK) return st;
    ck[s].resize(b);
    if ((st = hd_get_state(ctx, s, ck[s].data(), &b)) != HD_OK) return st;
  }
  const size_t N = (size_t)ctx->ntot;
  const size_t ubytes = 3 * N * (ctx->prec == HD_FP64 ? sizeof(double) : sizeof(float));
  struct Saved { void *dev; void *copy; size_t bytes; };
  std::vector<Saved> saved = {{ctx->A.flj, nullptr, 3 * N * sizeof(double)},
                              {ctx->A.hu, nullptr, 3 * N * sizeof(double)},
                              {ctx->A.fb, nullptr, 3 * N * sizeof(double)},
                              {ctx->A.tuu, nullptr, 3 * N * sizeof(double)},
                              {ctx->A.u, nullptr, ubytes}};
  auto release = [&]() {
    for (auto &v : saved)
      if (v.copy) (void)hipFree(v.copy);
  };
  hipError_t e = hipSuccess;
  for (auto &v : saved) {
    if ((e = hipMalloc(&v.copy, v.bytes)) != hipSuccess ||
        (e = hipMemcpyAsync(v.copy, v.dev, v.bytes, hipMemcpyDeviceToDevice, ctx->stream)) != hipSuccess) {
      release();
      return fail(ctx, HD_E_HIP, std::string("hd_min_mode_gradient: ") + hipGetErrorString(e));
    }
  }
  // one evaluation with u = w (r_O moved) in the pair kernels that also
  // accumulate T[u,u]
  const double *x = (const double *)(ck[sys].data() + sizeof(CkptHeader));
  std::vector<double> rO_tmp(nd), t(nd);
  for (size_t k = 0; k < nd; ++k) rO_tmp[k] = x[k] - w[k];
  for (int d = 0; d < dim && e == hipSuccess; ++d)
    e = hipMemcpyAsync(ctx->A.rO + d * ctx->ntot + ctx->h_desc[sys].off, rO_tmp.data() + (size_t)d * n,
                       sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream);
  // the curvature kernels read 32-bit lists: the plan's systems build those
  // for this evaluation (every list is rebuilt by it), and 16-bit ones again
  // from the restored build positions at the next step
  const int curv_was = plan->gp.any_curv, eig_was = plan->gp.any_eig, l16_was = plan->gp.list16;
  plan->gp.any_curv = 1;
  plan->gp.any_eig = 0;
  plan->gp.list16 = 0;
  for (int q : plan->ids)
    if (l16_was && st == HD_OK) { ctx->sys[q].list16 = 0; st = upload_desc(ctx, q); }
  if (e == hipSuccess && st == HD_OK) st = evaluate_all(ctx);
  plan->gp.any_curv = curv_was;
  plan->gp.any_eig = eig_was;
  plan->gp.list16 = l16_was;
  for (int q : plan->ids)
    if (l16_was) {
      ctx->sys[q].list16 = 1;
      ctx->sys[q].lists_wide = 1;
      const hd_status su = upload_desc(ctx, q);
      if (st == HD_OK) st = su;
    }
  if (e == hipSuccess && st == HD_OK) st = copy_field(ctx, sys, ctx->A.tuu, t.data(), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  // restore the run state
  for (auto &v : saved)
    if (e == hipSuccess) e = hipMemcpyAsync(v.dev, v.copy, v.bytes, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  release();
  if (e != hipSuccess) return fail(ctx, HD_E_HIP, std::string("hd_min_mode_gradient: ") + hipGetErrorString(e));
  if (st != HD_OK) return st;
  if ((st = restore_all(ctx, ck)) != HD_OK) return st;
  // d eps / d y = P^T T[w, w]: mobile atoms' rows, the rigid body's the sum
  // over its atoms (written on each rigid atom)
  double tR[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < n; ++i)
    if (h.role[i] == HD_ROLE_RIGID)
      for (int d = 0; d < dim; ++d) tR[d] += t[(size_t)d * n + i];
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < dim; ++d)
      grad[(size_t)d * n + i] = h.role[i] == HD_ROLE_MOBILE ? t[(size_t)d * n + i]
                                : h.role[i] == HD_ROLE_RIGID ? tR[d] : 0.0;
  return sync_out(ctx);
}

hd_status hd_debug_pairs(hd_ctx *ctx, int32_t sys, int32_t *ij, int64_t cap, int64_t *n_pairs) {
  CHECK_CTX();
  if (!ctx->finalized) return fail(ctx, HD_E_STATE, "not finalized");
  if (check_sys(ctx, sys) != HD_OK || !n_pairs || (cap > 0 && !ij)) return fail(ctx, HD_E_ARG, "bad arguments");
  const SysHost &s = ctx->sys[sys];
  const SysDesc &D = ctx->h_desc[sys];
  std::vector<int32_t> nnb(s.n), list((size_t)(D.maxnb + 3) / 4 * 4 * s.n), cat(s.n);
  HIPCHK(hipMemcpyAsync(nnb.data(), ctx->A.nnb + D.off, sizeof(int32_t) * s.n, hipMemcpyDeviceToHost, ctx->stream));
  if (D.list16 && ctx->sorted_lists[sys] && !s.lists_wide) {
    // 16-bit entries (grid plans of small LJ-only systems)
    std::vector<uint16_t> l16(list.size());
    HIPCHK(hipMemcpyAsync(l16.data(), ctx->A.nbr + D.nbr_off, sizeof(uint16_t) * l16.size(), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (size_t q = 0; q < list.size(); ++q) list[q] = l16[q];
  } else {
    HIPCHK(hipMemcpyAsync(list.data(), ctx->A.nbr + D.nbr_off, sizeof(int32_t) * list.size(), hipMemcpyDeviceToHost,
                          ctx->stream));
  }
  HIPCHK(hipMemcpyAsync(cat.data(), ctx->A.cell_atoms + D.off, sizeof(int32_t) * s.n, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  // grid lists are indexed by cell-sorted position (cat maps it to the atom)
  const bool sorted = ctx->sorted_lists[sys] != 0;
  // full lists hold each pair under both atoms, half lists under one of them
  // (either one): collect (min, max) and drop duplicates
  std::vector<std::pair<int32_t, int32_t>> pr;
  for (int r = 0; r < s.n; ++r)
    for (int q = 0; q < nnb[r]; ++q) {
      const int e = list[sorted ? (size_t)hdk::grid_list_index(q, s.n, r) : (size_t)q * s.n + r] >> 1;
      const int i = sorted ? cat[r] : r, j = sorted ? cat[e] : e;
      if (j == i) continue;
      pr.emplace_back(std::min(i, j), std::max(i, j));
    }
  std::sort(pr.begin(), pr.end());
  pr.erase(std::unique(pr.begin(), pr.end()), pr.end());
  const int64_t cnt = (int64_t)pr.size();
  for (int64_t k = 0; k < cnt && k < cap; ++k) { ij[2 * k] = pr[k].first; ij[2 * k + 1] = pr[k].second; }
  *n_pairs = cnt;
  return HD_OK;
}

hd_status hd_system_info(hd_ctx *ctx, int32_t sys, int32_t *dim, int32_t *n_atoms) {
  CHECK_CTX();
  if (check_sys(ctx, sys) != HD_OK) return HD_E_ARG;
  if (dim) *dim = ctx->sys[sys].dim;
  if (n_atoms) *n_atoms = ctx->sys[sys].n;
  return HD_OK;
}

int32_t hd_num_systems(const hd_ctx *ctx) { return ctx ? (int32_t)ctx->sys.size() : 0; }

const char *hd_last_error(const hd_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void hd_destroy(hd_ctx *ctx) {
  if (!ctx) return;
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  for (auto &P : ctx->plans)
    if (P.exec) hipGraphExecDestroy(P.exec);
  for (auto &P : ctx->plans)
    if (P.tail_exec) hipGraphExecDestroy(P.tail_exec);
  if (ctx->batched_graph) hipGraphExecDestroy(ctx->batched_graph);
  for (void *p : ctx->sched_allocs) hipFree(p);
  for (void *p : ctx->allocs) hipFree(p);
  if (ctx->ev0) hipEventDestroy(ctx->ev0);
  if (ctx->ev1) hipEventDestroy(ctx->ev1);
  if (ctx->stream2) { hipStreamSynchronize(ctx->stream2); hipStreamDestroy(ctx->stream2); }
  if (ctx->fork) hipEventDestroy(ctx->fork);
  if (ctx->join) hipEventDestroy(ctx->join);
  if (ctx->stream) hipStreamDestroy(ctx->stream);
  delete ctx;
}

}  // extern "C"
