// C ABI of the COLA library: plan construction (host, FP64) and the enqueue-only
// entry points that drive the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/cola.h"
#include "cosmology.hpp"
#include "internal.hpp"

using namespace cola;

struct cola_plan_s {
  cola_config cfg;
  Cosmo cosmo;
  std::vector<StepRow> table;
  Growth g_init;                  // growth at a_init (true values, any variant)
  std::vector<float> tw_nm, tw_np;
  std::vector<float> lpt_tab;     // sqrt(P/dp^3) / (kf n^2 np^3) indexed by n^2
  Bins bins;                      // Eulerian tiles of the force mesh
  int fft_width[2] = {0, 0};      // columns per tile of the mesh-size y passes and x pass (0: default)
  int fft_rot = -1;               // rotate the mesh-size half spectrum between y and x: 1 / 0 (-1: default)
  // resident steps (cola_plan_set_resident_steps): what the last resident step left in
  // its workspace, and the workspace generation of the current call
  int resident = 0;
  uint64_t ws_gen = 0;
  struct Resident {
    bool valid = false;
    const void* ws = nullptr;
    const float *s = nullptr, *v = nullptr, *s1 = nullptr, *s2 = nullptr;
    int next = 0;       // the step index the state is ready for
    int which = 0;      // sorted workspace copy holding it
    int parity = 0;     // bin buffers holding its tile counts
    uint64_t gen = 0;   // workspace generation of the call that left it
  } res;
  // stage tracing (hipEvent pairs around each launch, on the launch stream)
  int trace = 0;   // trace level: 0 off, 1 every kernel, 2 each cola_run step
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_stage;       // stage id of event pair k (events 2k, 2k+1)
  size_t ev_used = 0;              // pairs recorded since the last read
  // device copies
  int device = -1;
  float2* d_tw_nm = nullptr;
  float2* d_tw_np = nullptr;
  float* d_lpt_tab = nullptr;
};

namespace {

thread_local int g_last_hip = 0;

int hip_status(hipError_t e) {
  if (e == hipSuccess) return COLA_OK;
  g_last_hip = (int)e;
  return COLA_ERR_HIP;
}

// Stage ids reported by cola_trace_read.
enum Stage : int {
  kStBinCount = 0, kStBinScan, kStBinScatter, kStDeposit, kStZFwd, kStYFwd, kStXPoisson,
  kStYInv, kStZInv, kStGatherKickDrift, kStGatherForce, kStFinish, kStLptZFwd, kStLptYFwd, kStLptX,
  kStLptYInv, kStLptZInv, kStLptHessian, kStNoise, kStFft, kStAdjKick, kStAdjDeposit, kStAdjFft, kStAdjGather,
  kStAdjLpt, kStCheckpoint, kStRunStep, kStUnsort, kStYInvPair, kStAnalysis, kStWriteback, kNumStages
};
const char* const kStageNames[kNumStages] = {
  "bin_count", "bin_scan", "bin_scatter", "deposit", "fft_z_fwd", "fft_y_fwd",
  "fft_x_poisson", "fft_y_inv", "fft_z_inv", "gather_kick_drift", "gather_force", "gather_finish",
  "lpt_fft_z_fwd", "lpt_fft_y_fwd", "lpt_fft_x_mul", "lpt_fft_y_inv", "lpt_fft_z_inv", "lpt_hessian", "noise",
  "fft_test", "adj_kick_drift", "adj_deposit", "adj_fft", "adj_gather", "adj_lpt", "checkpoint", "run_step", "unsort",
  "fft_y_inv_pair", "analysis", "writeback"};

// Trace levels: 1 records an event pair around every kernel launch, 2 only around
// each whole COLA step of cola_run (stage run_step), so step times carry no
// per-kernel event overhead.
// trace_open returns the event slot of a span at `level`, or -1 when that level is
// not being traced; trace_close records its end.
long trace_open(cola_plan p, int level, int stage, hipStream_t st, hipError_t& rc) {
  rc = hipSuccess;
  if (p->trace != level) return -1;
  const size_t need = 2 * (p->ev_used + 1);
  while (p->ev_pool.size() < need) {
    hipEvent_t e;
    rc = hipEventCreate(&e);
    if (rc != hipSuccess) return -1;
    p->ev_pool.push_back(e);
  }
  const size_t slot = p->ev_used++;
  if (p->ev_stage.size() <= slot) p->ev_stage.resize(slot + 1);
  p->ev_stage[slot] = stage;
  rc = hipEventRecord(p->ev_pool[2 * slot], st);
  return (long)slot;
}
hipError_t trace_close(cola_plan p, long slot, hipStream_t st) {
  return slot < 0 ? hipSuccess : hipEventRecord(p->ev_pool[2 * slot + 1], st);
}

// Runs launch `fn` inside a level-1 span.
template <class F>
hipError_t traced(cola_plan p, int stage, hipStream_t st, F&& fn) {
  hipError_t rc;
  const long slot = trace_open(p, 1, stage, st, rc);
  if (rc != hipSuccess) return rc;
  rc = fn();
  if (rc != hipSuccess) return rc;
  return trace_close(p, slot, st);
}

#define COLA_TRY(expr)                      \
  do {                                      \
    const int rc_ = (expr);                 \
    if (rc_ != COLA_OK) return rc_;         \
  } while (0)
#define COLA_HIP(expr) COLA_TRY(hip_status(expr))

std::vector<float> twiddles(int n) {
  std::vector<float> t(2 * n);
  for (int m = 0; m < n; ++m) {
    const double ang = -2.0 * M_PI * (double)m / (double)n;
    t[2 * m] = (float)std::cos(ang);
    t[2 * m + 1] = (float)std::sin(ang);
  }
  return t;
}

int validate(const cola_config* c) {
  if (!c) return COLA_ERR_INVALID;
  if (!fft_size_supported(c->np) || !fft_size_supported(c->nm)) return COLA_ERR_UNSUPPORTED_SIZE;
  if (c->nm % c->np) return COLA_ERR_INVALID;
  if (!(c->box > 0) || !(c->omega_m > 0) || !(c->sigma8 > 0) || !(c->h > 0)) return COLA_ERR_INVALID;
  if (!(c->a_init > 0) || !(c->a_final > c->a_init)) return COLA_ERR_INVALID;
  if (c->n_steps < 1 || c->n_steps > 100000) return COLA_ERR_INVALID;
  if (c->n_lpt == 0.0 || !std::isfinite(c->n_lpt)) return COLA_ERR_INVALID;
  if (c->flags & ~(uint32_t)(COLA_FLAG_KDK_STD | COLA_FLAG_NO_LPT_FRAME | COLA_FLAG_LOG_A_STEPS | COLA_FLAG_U1_DRIFT))
    return COLA_ERR_INVALID;
  // E(a)^2 must stay positive on [a_init, a_final]
  const double ok = 1.0 - c->omega_m - c->omega_l;
  for (int i = 0; i <= 64; ++i) {
    const double a = c->a_init + (c->a_final - c->a_init) * i / 64.0;
    if (!(c->omega_m / (a * a * a) + ok / (a * a) + c->omega_l > 0)) return COLA_ERR_INVALID;
  }
  return COLA_OK;
}

template <class T>
int upload(T** dst, const std::vector<float>& src) {
  COLA_HIP(hipMalloc((void**)dst, src.size() * sizeof(float)));
  COLA_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(float), hipMemcpyHostToDevice));
  return COLA_OK;
}

// Uploads the plan's tables on first use; later calls must come from the same device.
int ensure_device(cola_plan p) {
  int dev = 0;
  COLA_HIP(hipGetDevice(&dev));
  if (p->device >= 0) return dev == p->device ? COLA_OK : COLA_ERR_DEVICE;
  COLA_TRY(upload(&p->d_tw_nm, p->tw_nm));
  COLA_TRY(upload(&p->d_tw_np, p->tw_np));
  COLA_TRY(upload(&p->d_lpt_tab, p->lpt_tab));
  p->device = dev;
  return COLA_OK;
}

const float2* twiddle_for(cola_plan p, int n) { return n == p->cfg.nm ? p->d_tw_nm : p->d_tw_np; }

inline long cube(long n) { return n * n * n; }

FieldPtrs fields(std::initializer_list<float*> l) {
  FieldPtrs f{};
  int i = 0;
  for (float* x : l) f.p[i++] = reinterpret_cast<float2*>(x);
  return f;
}

Lattice lattice(cola_plan p) {
  Lattice l;
  l.np = p->cfg.np;
  l.nm = p->cfg.nm;
  l.ratio = p->cfg.nm / p->cfg.np;
  const double inv_dx = p->cfg.nm / p->cfg.box;
  l.inv_dx = (float)inv_dx;
  l.inv_dx_lo = (float)(inv_dx - (double)l.inv_dx);
  l.npart = cube(p->cfg.np);
  set_lattice_divisor(l);
  return l;
}

int width_for(cola_plan p, int n, int pass) { return n == p->cfg.nm ? p->fft_width[pass] : 0; }
// Row rotation of the half spectrum that the method's y -> x -> y chains hold between
// their y and x passes (the public FFT and the spectrum analysis use plain planes).
int rot_for(cola_plan p, int n) {
  const bool on = (n == p->cfg.nm && p->fft_rot >= 0) ? p->fft_rot == 1 : fft_rot_default_on(n);
  return on ? fft_rot_rows(n) : 0;
}

// y pass (in place) over nf fields of an n^3 half-spectrum layout; the k-space side
// (output of dir < 0, input of dir > 0) has its planes rotated by rot.
int ypass(cola_plan p, int stage, int n, int dir, FieldPtrs f, int nf, const float2* tw, hipStream_t st, int rot,
          int reverse = 0) {
  const long h = n / 2;
  const int w = width_for(p, n, 0);
  return hip_status(traced(p, stage, st, [&] {
    return launch_col(n, dir, f, f, nf, n, (long)n * h, h, (int)h, tw, w, rot, st, reverse);
  }));
}

// Workspace: four real nm^3 meshes (the three force components and the scalar field
// of the force passes), then the binning buffers.
size_t mesh_floats(cola_plan p) { return 4 * (size_t)cube(p->cfg.nm); }

// parity selects which of the two tile-count arrays holds the current counts
// (cola_run alternates them: a step's gather counts into the other one).
BinBuffers bin_buffers(cola_plan p, float* ws, int parity = 0) {
  BinBuffers bb = carve_bins(ws + mesh_floats(p), cube(p->cfg.np), p->bins);
  if (parity) std::swap(bb.count, bb.count_next);
  return bb;
}

// Two tile-sorted copies of the particle state (13 words per particle each) after
// the binning buffers; used by cola_run.
SortedState sorted_state(cola_plan p, float* ws, int which) {
  const long n = cube(p->cfg.np);
  char* c = reinterpret_cast<char*>(ws + mesh_floats(p)) + bin_workspace_bytes(n, p->bins);
  float* f = reinterpret_cast<float*>(c) + (long)which * 13 * n;
  SortedState ss;
  ss.s = f;
  ss.v = f + 3 * n;
  ss.s1 = f + 6 * n;
  ss.s2 = f + 9 * n;
  ss.lag = reinterpret_cast<int*>(f + 12 * n);
  return ss;
}

// Bins the particles at q + s (caller's Lagrangian-order arrays) by Eulerian tile and
// deposits their CIC density (mean 1) into rho; the bins stay valid for a gather from
// the same s.
int deposit_with(cola_plan p, const float* s, float* rho, const BinBuffers& bb, hipStream_t st) {
  const Lattice lat = lattice(p);
  const Bins& b = p->bins;
  const double ratio = (double)lat.ratio;
  COLA_HIP(traced(p, kStBinCount, st, [&] { return launch_bin_count(lat, b, s, bb, st); }));
  COLA_HIP(traced(p, kStBinScan, st, [&] { return launch_bin_scan(b, bb, false, st); }));
  COLA_HIP(traced(p, kStBinScatter, st, [&] { return launch_bin_scatter(lat, bb, st); }));
  COLA_HIP(traced(p, kStDeposit, st,
                  [&] { return launch_deposit(lat, b, s, bb, rho, (float)(ratio * ratio * ratio), st); }));
  return COLA_OK;
}

int deposit_into(cola_plan p, const float* s, float* rho, float* ws, hipStream_t st) {
  return deposit_with(p, s, rho, bin_buffers(p, ws), st);
}

// Poisson solve on the density in ws mesh 0: g_d = (3/2) Om a irfft(i k_d delta_k / k^2),
// d = 0..2, left in ws meshes 0, 1, 2 as real nm^3 fields (mesh 3 is scratch).
int fft_force(cola_plan p, double a, float* ws, hipStream_t st) {
  const int n = p->cfg.nm;
  const long r = cube(n);
  float* g0 = ws;
  float* g1 = ws + r;
  float* g2 = ws + 2 * r;
  const float2* tw = p->d_tw_nm;
  COLA_HIP(traced(p, kStZFwd, st,
                  [&] { return launch_zfwd(n, g0, reinterpret_cast<float2*>(g0), (long)n * n, tw, st); }));
  // The y pass walks the rows the z pass wrote last first, and each force field goes
  // through its y and z inverse passes back to back (the z pass again walking
  // backwards), so those passes start on data still held by the memory-side cache.
  const int rot = rot_for(p, n);
  COLA_TRY(ypass(p, kStYFwd, n, -1, fields({g0}), 1, tw, st, rot, 1));
  const double kf = 2.0 * M_PI / p->cfg.box;
  MulArgs m{};
  m.c = (float)(1.5 * p->cfg.omega_m * a / (kf * (double)r));
  // The gradient i k_j phi_k needs its factor k_j while axis j is still in k-space:
  // the x pass writes i n_x Phi (into g0) and Phi (into g3), Phi = c X / n^2 after the
  // inverse x transform; the y pass of Phi writes i n_y Phi (g1) and Phi (g2); the z
  // pass applies i n_z to g2.  Two x outputs and one y input fewer than three separate
  // gradient chains, the same operators.
  float* g3 = ws + 3 * r;
  COLA_HIP(traced(p, kStXPoisson, st, [&] {
    return launch_xmul(n, kMulGradPair, reinterpret_cast<float2*>(g0), fields({g0, g3}), 2, m, tw,
                       p->fft_width[1], rot, st);
  }));
  EpiArgs e{};
  e.scale = 1.0f;
  e.reverse = 1;
  const int h = n / 2;
  // the y pass reads the tail the x pass wrote last first; the z pass then takes
  // both of its outputs together from their heads
  COLA_HIP(traced(p, kStYInvPair, st, [&] {
    return launch_col_pair(n, reinterpret_cast<const float2*>(g3), reinterpret_cast<float2*>(g2),
                           reinterpret_cast<float2*>(g1), n, (long)n * h, h, h, tw, width_for(p, n, 0), rot, st,
                           1);
  }));
  e.reverse = 0;
  e.deriv = 2;   // field 1 (g2): the z component
  COLA_HIP(traced(p, kStZInv, st, [&] {
    return launch_zinv(n, fields({g1, g2}), fields({g1, g2}), 2, (long)n * n, tw, kEpiStore, e, st);
  }));
  e.deriv = 0;
  e.reverse = 1;
  COLA_TRY(ypass(p, kStYInv, n, 1, fields({g0}), 1, tw, st, rot));
  COLA_HIP(traced(p, kStZInv, st, [&] {
    return launch_zinv(n, fields({g0}), fields({g0}), 1, (long)n * n, tw, kEpiStore, e, st);
  }));
  return COLA_OK;
}

// The force mesh of particles at q + s (binned first).
int pm_mesh(cola_plan p, const float* s, double a, float* ws, hipStream_t st) {
  COLA_TRY(deposit_into(p, s, ws, ws, st));
  return fft_force(p, a, ws, st);
}

GatherArgs gather_args(cola_plan p, float* ws) {
  const long r = cube(p->cfg.nm);
  GatherArgs g{};
  g.g0 = ws;
  g.g1 = ws + r;
  g.g2 = ws + 2 * r;
  return g;
}

// Workspace generations: every call that takes a workspace moves that workspace's
// generation on by one, so a plan can tell whether a workspace still holds what the
// plan's previous call left there (its generation then moved by exactly this call).
std::mutex g_ws_mu;
std::unordered_map<const void*, uint64_t> g_ws_gen;

uint64_t ws_bump(const void* ws) {
  std::lock_guard<std::mutex> lock(g_ws_mu);
  return ++g_ws_gen[ws];
}

int check_common(cola_plan p, const void* ws) {
  if (!p || !ws) return COLA_ERR_INVALID;
  p->ws_gen = ws_bump(ws);
  return ensure_device(p);
}

int check_particles(const cola_particles* q) {
  if (!q || !q->s || !q->v || !q->s1 || !q->s2) return COLA_ERR_INVALID;
  return COLA_OK;
}

// The caller's Lagrangian-order particles binned by tile and packed into the tile-sorted
// workspace copy pk (slot = list position; the caller's arrays are read in order), the
// CIC density deposited from pk and the force meshes solved: the state a cola_run step
// starts from, so the public calls run the same deposit and gather kernels.
int packed_mesh(cola_plan p, const cola_particles* q, double a, float* ws, hipStream_t st, SortedState& pk) {
  const Lattice lat = lattice(p);
  const Bins& b = p->bins;
  const BinBuffers bb = bin_buffers(p, ws);
  const SortedState lagr{q->s, q->v, q->s1, q->s2, nullptr};
  pk = sorted_state(p, ws, 0);
  const double ratio = (double)lat.ratio;
  COLA_HIP(traced(p, kStBinCount, st, [&] { return launch_bin_count(lat, b, q->s, bb, st); }));
  COLA_HIP(traced(p, kStBinScan, st, [&] { return launch_bin_scan(b, bb, false, st); }));
  COLA_HIP(traced(p, kStBinScatter, st, [&] { return launch_bin_scatter_pack(lat, bb, lagr, pk, st); }));
  COLA_HIP(traced(p, kStDeposit, st, [&] {
    return launch_deposit(lat, b, pk.s, bb, ws, (float)(ratio * ratio * ratio), st, pk.lag);
  }));
  return fft_force(p, a, ws, st);
}

// Kick and drift factors of step i (eq. KDKALC) and of the closing half-kick with
// L+(a_n) (eq. ALCtimestep, Lops).
KickArgs step_kick(cola_plan p, const StepRow& row) {
  const bool plain = p->cfg.flags & COLA_FLAG_NO_LPT_FRAME;
  KickArgs k{};
  k.alpha = (float)row.alpha;
  k.t2d1 = plain ? 0.0f : (float)row.g.t2d1;
  k.t2d2 = plain ? 0.0f : (float)row.g.t2d2;
  k.beta = (float)row.beta;
  k.dd1 = plain ? 0.0f : (float)row.dd1;
  k.dd2 = plain ? 0.0f : (float)row.dd2;
  return k;
}

KickArgs finish_kick(cola_plan p, const StepRow& row) {
  const bool plain = p->cfg.flags & COLA_FLAG_NO_LPT_FRAME;
  KickArgs k{};
  k.alpha = (float)row.alpha;
  k.t2d1 = plain ? 0.0f : (float)row.g.t2d1;
  k.t2d2 = plain ? 0.0f : (float)row.g.t2d2;
  k.td1 = plain ? 0.0f : (float)row.g.td1;
  k.td2 = plain ? 0.0f : (float)row.g.td2;
  k.box = (float)p->cfg.box;
  return k;
}

// One COLA step: PM force at a_i, merged kick, drift (eq. KDKALC).  The kick and drift
// read the packed copy in tile order and write s, v back to the caller's arrays by
// Lagrangian index; the arithmetic is the cola_run gather's, so both paths agree bit
// for bit.
int step_impl(cola_plan p, int i, const cola_particles* q, float* ws, hipStream_t st) {
  p->res.valid = false;
  const StepRow& row = p->table[i];
  SortedState pk;
  COLA_TRY(packed_mesh(p, q, row.a, ws, st, pk));
  const KickArgs k = step_kick(p, row);
  const GatherArgs g = gather_args(p, ws);
  const SortedState lagr{q->s, q->v, q->s1, q->s2, nullptr};
  return hip_status(traced(p, kStGatherKickDrift, st, [&] {
    return launch_gather_sorted(lattice(p), p->bins, pk, lagr, bin_buffers(p, ws), kGatherKickDriftLag, g, k, st);
  }));
}

// Resident steps.  A step that finds in the workspace the tile-sorted state and bins
// that the previous resident step left there (same particle arrays and workspace, the
// next step index, and no other call on that workspace since) starts from them as a
// cola_run step does: scan and scatter of the bins, no re-binning and no packing.
// Otherwise it bins and packs the caller's arrays.  Its gather writes the next state in
// this step's tile order, bins it for the next step and writes s and v to the caller's
// arrays, which are therefore current after every step.
bool resident_ready(cola_plan p, int i, const cola_particles* q, const float* ws) {
  const auto& r = p->res;
  return r.valid && r.ws == ws && r.s == q->s && r.v == q->v && r.s1 == q->s1 && r.s2 == q->s2 && r.next == i &&
         (r.gen == p->ws_gen || r.gen + 1 == p->ws_gen);
}

// Deposit from the sorted state src through the bins bb, then the force meshes.
int sorted_mesh(cola_plan p, const SortedState& src, const BinBuffers& bb, double a, float* ws, hipStream_t st) {
  const double ratio = (double)lattice(p).ratio;
  COLA_HIP(traced(p, kStDeposit, st, [&] {
    return launch_deposit(lattice(p), p->bins, src.s, bb, ws, (float)(ratio * ratio * ratio), st, src.lag);
  }));
  return fft_force(p, a, ws, st);
}

// The sorted source of step i and its bins (clear_next: the step's gather bins for the
// next step); which_dst and parity name the copy and bins the gather writes into.
int resident_source(cola_plan p, int i, const cola_particles* q, float* ws, hipStream_t st, bool clear_next,
                    BinBuffers& bb, SortedState& src, int& which_dst, int& parity) {
  const Lattice lat = lattice(p);
  const Bins& b = p->bins;
  const bool ready = resident_ready(p, i, q, ws);
  p->res.valid = false;
  if (ready) {
    parity = p->res.parity;
    bb = bin_buffers(p, ws, parity);
    src = sorted_state(p, ws, p->res.which);
    which_dst = p->res.which ^ 1;
    COLA_HIP(traced(p, kStBinScan, st, [&] { return launch_bin_scan(b, bb, clear_next, st); }));
    return hip_status(traced(p, kStBinScatter, st, [&] { return launch_bin_scatter(lat, bb, st); }));
  }
  parity = 0;
  bb = bin_buffers(p, ws, 0);
  src = sorted_state(p, ws, 0);
  which_dst = 1;
  const SortedState lagr{q->s, q->v, q->s1, q->s2, nullptr};
  COLA_HIP(traced(p, kStBinCount, st, [&] { return launch_bin_count(lat, b, q->s, bb, st); }));
  COLA_HIP(traced(p, kStBinScan, st, [&] { return launch_bin_scan(b, bb, clear_next, st); }));
  return hip_status(traced(p, kStBinScatter, st, [&] { return launch_bin_scatter_pack(lat, bb, lagr, src, st); }));
}

int resident_step(cola_plan p, int i, const cola_particles* q, float* ws, hipStream_t st) {
  const StepRow& row = p->table[i];
  BinBuffers bb;
  SortedState src;
  int which_dst, parity;
  COLA_TRY(resident_source(p, i, q, ws, st, true, bb, src, which_dst, parity));
  COLA_TRY(sorted_mesh(p, src, bb, row.a, ws, st));
  const KickArgs k = step_kick(p, row);
  GatherArgs g = gather_args(p, ws);
  // the slot of every Lagrangian index goes to force mesh 3, free once the forces are
  // solved, for the write-back of s and v to the caller's arrays in their order
  g.inv = reinterpret_cast<int*>(ws + 3 * cube(p->cfg.nm));
  const SortedState dst = sorted_state(p, ws, which_dst);
  const Lattice lat = lattice(p);
  COLA_HIP(traced(p, kStGatherKickDrift, st, [&] {
    return launch_gather_sorted(lat, p->bins, src, dst, bb, kGatherKickDriftInv, g, k, st);
  }));
  COLA_HIP(traced(p, kStWriteback, st, [&] { return launch_writeback(lat, dst, g.inv, q->s, q->v, st); }));
  auto& r = p->res;
  r.valid = true;
  r.ws = ws;
  r.s = q->s;
  r.v = q->v;
  r.s1 = q->s1;
  r.s2 = q->s2;
  r.next = i + 1;
  r.which = which_dst;
  r.parity = parity ^ 1;
  r.gen = p->ws_gen;
  return COLA_OK;
}

// Closing half-kick at a_n and L+(a_n) (eq. ALCtimestep, Lops), as the closing step of
// cola_run: the kick in tile order into the other workspace copy, then back to
// Lagrangian order with L+ and the positions.  Starts from the resident state when the
// last step left one.
int finish_impl(cola_plan p, const cola_particles* q, float* x_out, float* v_out, float* ws, hipStream_t st) {
  const StepRow& row = p->table[p->cfg.n_steps];
  BinBuffers bb;
  SortedState src, out;
  if (resident_ready(p, p->cfg.n_steps, q, ws)) {
    int which_dst, parity;
    COLA_TRY(resident_source(p, p->cfg.n_steps, q, ws, st, false, bb, src, which_dst, parity));
    COLA_TRY(sorted_mesh(p, src, bb, row.a, ws, st));
    out = sorted_state(p, ws, which_dst);
  } else {
    p->res.valid = false;
    COLA_TRY(packed_mesh(p, q, row.a, ws, st, src));
    bb = bin_buffers(p, ws);
    out = sorted_state(p, ws, 1);
  }
  const KickArgs k = finish_kick(p, row);
  GatherArgs g = gather_args(p, ws);
  g.s = q->s;
  g.v = q->v;
  g.s1 = q->s1;
  g.s2 = q->s2;
  g.out_a = x_out;
  g.out_b = v_out;
  const Lattice lat = lattice(p);
  COLA_HIP(traced(p, kStFinish, st, [&] {
    return launch_gather_sorted(lat, p->bins, src, out, bb, kGatherFinish, g, k, st);
  }));
  return hip_status(traced(p, kStUnsort, st, [&] { return launch_unsort(lat, out, g, k, st); }));
}

// ---------------------------------------------------------------------------------
// Adjoint of the whole run with respect to the white noise.
//
// Workspace layout: [3 nm^3 force meshes | bins | 3 nm^3 adjoint meshes |
// lam_s, lam_v, lam_s1, lam_s2 (4 x 3 np^3) | 10 np^3 of 2LPT scratch].
// ---------------------------------------------------------------------------------
struct AdjLayout {
  float* amesh[3];
  float* lam_s;
  float* lam_v;
  float* lam_s1;
  float* lam_s2;
  float* lpt;       // 10 np^3
  unsigned* wmax;   // four words: max |weight| of the weighted deposit
  size_t bytes;
};

AdjLayout adj_layout(cola_plan p, float* ws) {
  const long r = cube(p->cfg.nm), n = cube(p->cfg.np);
  const size_t head = mesh_floats(p) * sizeof(float) + bin_workspace_bytes(n, p->bins);
  AdjLayout L;
  float* f = ws ? reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + head) : nullptr;
  for (int d = 0; d < 3; ++d) L.amesh[d] = f ? f + d * r : nullptr;
  float* q = f ? f + 3 * r : nullptr;
  L.lam_s = q;
  L.lam_v = q ? q + 3 * n : nullptr;
  L.lam_s1 = q ? q + 6 * n : nullptr;
  L.lam_s2 = q ? q + 9 * n : nullptr;
  L.lpt = q ? q + 12 * n : nullptr;
  L.wmax = q ? reinterpret_cast<unsigned*>(q + 22 * n) : nullptr;
  L.bytes = head + (3 * (size_t)r + 22 * (size_t)n + 4) * sizeof(float);
  return L;
}

// Bins the particles at q + s (no deposit).
int bin_only(cola_plan p, const float* s, float* ws, hipStream_t st) {
  const Lattice lat = lattice(p);
  const BinBuffers bb = bin_buffers(p, ws);
  COLA_HIP(traced(p, kStBinCount, st, [&] { return launch_bin_count(lat, p->bins, s, bb, st); }));
  COLA_HIP(traced(p, kStBinScan, st, [&] { return launch_bin_scan(p->bins, bb, false, st); }));
  COLA_HIP(traced(p, kStBinScatter, st, [&] { return launch_bin_scatter(lat, bb, st); }));
  return COLA_OK;
}

// z and y forward passes over nf real fields of an n^3 grid, in place.
int fwd_zy(cola_plan p, int stage, int n, std::initializer_list<float*> f, const float2* tw, hipStream_t st) {
  for (float* x : f)
    COLA_HIP(traced(p, stage, st,
                    [&] { return launch_zfwd(n, x, reinterpret_cast<float2*>(x), (long)n * n, tw, st); }));
  return ypass(p, stage, n, -1, fields(f), (int)f.size(), tw, st, rot_for(p, n));
}

// y and z inverse passes of one field, in place (scale 1).
int inv_yz(cola_plan p, int stage, int n, float* x, const float2* tw, hipStream_t st) {
  COLA_TRY(ypass(p, stage, n, 1, fields({x}), 1, tw, st, rot_for(p, n)));
  EpiArgs e{};
  e.scale = 1.0f;
  return hip_status(traced(p, stage, st, [&] {
    return launch_zinv(n, fields({x}), fields({x}), 1, (long)n * n, tw, kEpiStore, e, st);
  }));
}

int run_adjoint(cola_plan p, const float* w, const float* ckpt, const float* dL_drho, float* dL_dw, float* ws,
                hipStream_t st) {
  const int ns = p->cfg.n_steps;
  const long n = cube(p->cfg.np), n3 = 3 * n;
  const Lattice lat = lattice(p);
  const Bins& b = p->bins;
  const AdjLayout L = adj_layout(p, ws);
  const float inv_dx = lat.inv_dx;
  const float mass = (float)std::pow((double)lat.ratio, 3);
  const bool plain = p->cfg.flags & COLA_FLAG_NO_LPT_FRAME;
  const int nm = p->cfg.nm;
  for (float* x : {L.lam_s, L.lam_v, L.lam_s1, L.lam_s2})
    COLA_HIP(traced(p, kStAdjKick, st, [&] { return launch_fill(x, n3, 0.0f, st); }));
  // dL/ds at the end: derivative of the CIC density of s_n against dL/drho.
  const float* s_end = ckpt + (long)ns * n3;
  COLA_TRY(bin_only(p, s_end, ws, st));
  {
    AdjGatherArgs ga{};
    ga.rbar = dL_drho;
    ga.lam_s = L.lam_s;
    ga.f1 = 0.0f;
    ga.f2 = mass * inv_dx;
    COLA_HIP(traced(p, kStAdjGather, st, [&] { return launch_grad_gather(lat, b, bin_buffers(p, ws), s_end, ga, st); }));
  }
  const double kf = 2.0 * M_PI / p->cfg.box;
  for (int i = ns - 1; i >= 0; --i) {
    const StepRow& row = p->table[i];
    const float* s_i = ckpt + (long)i * n3;
    AdjStepArgs a{};
    a.alpha = (float)row.alpha;
    a.beta = (float)row.beta;
    a.t2d1 = plain ? 0.0f : (float)row.g.t2d1;
    a.t2d2 = plain ? 0.0f : (float)row.g.t2d2;
    a.dd1 = plain ? 0.0f : (float)row.dd1;
    a.dd2 = plain ? 0.0f : (float)row.dd2;
    COLA_HIP(traced(p, kStAdjKick, st,
                    [&] { return launch_adj_kick_drift(n3, a, L.lam_s, L.lam_v, L.lam_s1, L.lam_s2, st); }));
    // recompute the force mesh at s_i (bins for s_i stay valid)
    COLA_TRY(pm_mesh(p, s_i, row.a, ws, st));
    // nu_d = mass-weighted CIC deposit of mu_d = lam_v_d
    const BinBuffers bb = bin_buffers(p, ws);
    // the three components in one particle walk (amesh[d] = amesh[0] + d nm^3)
    COLA_HIP(traced(p, kStAdjDeposit, st, [&] {
      return launch_deposit3(lat, b, s_i, bb, L.amesh[0], mass, L.lam_v, L.wmax, st);
    }));
    // rbar = sum_d K_d^T nu_d (conjugate multiplier), into amesh[0]
    const float2* tw = p->d_tw_nm;
    COLA_TRY(fwd_zy(p, kStAdjFft, nm, {L.amesh[0], L.amesh[1], L.amesh[2]}, tw, st));
    MulArgs m{};
    m.c = (float)(1.5 * p->cfg.omega_m * row.a / (kf * (double)cube(nm)));
    COLA_HIP(traced(p, kStAdjFft, st, [&] {
      return launch_xmul_adj(nm, kMulGrad, fields({L.amesh[0], L.amesh[1], L.amesh[2]}), 3,
                             reinterpret_cast<float2*>(L.amesh[0]), m, tw, rot_for(p, nm), st);
    }));
    COLA_TRY(inv_yz(p, kStAdjFft, nm, L.amesh[0], tw, st));
    // lam_s += alpha [ (1/dx) grad(mu . g) + (1/dx) grad(rbar) ]
    AdjGatherArgs ga{};
    ga.g0 = ws;
    ga.g1 = ws + cube(nm);
    ga.g2 = ws + 2 * cube(nm);
    ga.mu = L.lam_v;
    ga.rbar = L.amesh[0];
    ga.lam_s = L.lam_s;
    ga.f1 = (float)row.alpha * inv_dx;
    ga.f2 = (float)row.alpha * inv_dx;
    COLA_HIP(traced(p, kStAdjGather, st, [&] { return launch_grad_gather(lat, b, bb, s_i, ga, st); }));
  }
  // initial state s_0 = D1 s1 + D2 s2 (and, without the LPT frame, v_0 = T[D1] s1 + T[D2] s2)
  const Growth& g0 = p->g_init;
  COLA_HIP(traced(p, kStAdjLpt, st, [&] { return launch_axpy(n3, (float)g0.d1, L.lam_s, L.lam_s1, st); }));
  COLA_HIP(traced(p, kStAdjLpt, st, [&] { return launch_axpy(n3, (float)g0.d2, L.lam_s, L.lam_s2, st); }));
  if (plain) {
    COLA_HIP(traced(p, kStAdjLpt, st, [&] { return launch_axpy(n3, (float)g0.td1, L.lam_v, L.lam_s1, st); }));
    COLA_HIP(traced(p, kStAdjLpt, st, [&] { return launch_axpy(n3, (float)g0.td2, L.lam_v, L.lam_s2, st); }));
  }
  // 2LPT VJP.  Recompute the Hessian phi_ab of the linear potential into lpt[3..8].
  const int np_ = p->cfg.np;
  const float2* twp = p->d_tw_np;
  float* sc[10];
  for (int k = 0; k < 10; ++k) sc[k] = L.lpt + k * n;
  COLA_HIP(traced(p, kStAdjLpt, st,
                  [&] { return launch_zfwd(np_, w, reinterpret_cast<float2*>(sc[9]), (long)np_ * np_, twp, st); }));
  const int rot_p = rot_for(p, np_);
  COLA_TRY(ypass(p, kStAdjLpt, np_, -1, fields({sc[9]}), 1, twp, st, rot_p));
  MulArgs ml{};
  ml.kf = (float)kf;
  ml.tab = p->d_lpt_tab;
  const FieldPtrs all9 = fields({sc[0], sc[1], sc[2], sc[3], sc[4], sc[5], sc[6], sc[7], sc[8]});
  COLA_HIP(traced(p, kStAdjLpt, st, [&] {
    return launch_xmul(np_, kMulLpt1, reinterpret_cast<float2*>(sc[9]), all9, 9, ml, twp, 0, rot_p, st);
  }));
  const FieldPtrs phi = fields({sc[3], sc[4], sc[5], sc[6], sc[7], sc[8]});
  COLA_TRY(ypass(p, kStAdjLpt, np_, 1, phi, 6, twp, st, rot_p));
  EpiArgs e1{};
  e1.scale = 1.0f;
  COLA_HIP(traced(p, kStAdjLpt, st,
                  [&] { return launch_zinv(np_, phi, phi, 6, (long)np_ * np_, twp, kEpiStore, e1, st); }));
  // sigma = sum_j G_j^T lam_s2_j, G_j the s2 operator (multiplier -i k_j / k^2)
  float* l2[3] = {L.lam_s2, L.lam_s2 + n, L.lam_s2 + 2 * n};
  COLA_TRY(fwd_zy(p, kStAdjLpt, np_, {l2[0], l2[1], l2[2]}, twp, st));
  MulArgs m2{};
  m2.c = (float)(-1.0 / (kf * (double)n));
  COLA_HIP(traced(p, kStAdjLpt, st, [&] {
    return launch_xmul_adj(np_, kMulGrad, fields({l2[0], l2[1], l2[2]}), 3, reinterpret_cast<float2*>(sc[9]), m2,
                           twp, rot_p, st);
  }));
  COLA_TRY(inv_yz(p, kStAdjLpt, np_, sc[9], twp, st));
  // tau_ab = dS/dphi_ab^T sigma, in place over phi
  HessPtrs hp{};
  for (int k = 0; k < 6; ++k) hp.p[k] = sc[3 + k];
  COLA_HIP(traced(p, kStAdjLpt, st, [&] { return launch_hessian_adjoint(n, sc[9], hp, st); }));
  // dL/dw = A^T lam_s1 + H^T tau: transposed LPT multipliers summed in k space
  float* l1[3] = {L.lam_s1, L.lam_s1 + n, L.lam_s1 + 2 * n};
  COLA_TRY(fwd_zy(p, kStAdjLpt, np_, {l1[0], l1[1], l1[2]}, twp, st));
  COLA_TRY(fwd_zy(p, kStAdjLpt, np_, {sc[3], sc[4], sc[5], sc[6], sc[7], sc[8]}, twp, st));
  const FieldPtrs in9 = fields({l1[0], l1[1], l1[2], sc[3], sc[4], sc[5], sc[6], sc[7], sc[8]});
  COLA_HIP(traced(p, kStAdjLpt, st, [&] {
    return launch_xmul_adj(np_, kMulLpt1, in9, 9, reinterpret_cast<float2*>(sc[9]), ml, twp, rot_p, st);
  }));
  COLA_TRY(ypass(p, kStAdjLpt, np_, 1, fields({sc[9]}), 1, twp, st, rot_p));
  EpiArgs e2{};
  e2.scale = 1.0f;
  return hip_status(traced(p, kStAdjLpt, st, [&] {
    return launch_zinv(np_, fields({sc[9]}), fields({dL_dw}), 1, (long)np_ * np_, twp, kEpiStore, e2, st);
  }));
}

}  // namespace

namespace cola {

int record_hip(hipError_t e) { return hip_status(e); }

size_t plan_bin_bytes(cola_plan_s* p) { return bin_workspace_bytes(cube(p->cfg.np), p->bins); }

int density_with_bins(cola_plan_s* p, const float* s, float* rho, void* bin_base, hipStream_t st) {
  if (p->trace) return COLA_ERR_INVALID;   // trace events are created on demand
  const BinBuffers bb = carve_bins(bin_base, cube(p->cfg.np), p->bins);
  return deposit_with(p, s, rho, bb, st);
}

}  // namespace cola

extern "C" {

int cola_plan_create(const cola_config* cfg, cola_plan* out) {
  if (!out) return COLA_ERR_INVALID;
  *out = nullptr;
  COLA_TRY(validate(cfg));
  cola_plan p = new (std::nothrow) cola_plan_s();
  if (!p) return COLA_ERR_INVALID;
  p->cfg = *cfg;
  Cosmo& c = p->cosmo;
  c.omega_m = cfg->omega_m;
  c.omega_l = cfg->omega_l;
  c.h = cfg->h;
  c.n_s = cfg->n_s;
  c.sigma8 = cfg->sigma8;
  c.n_lpt = cfg->n_lpt;
  c.normalise_sigma8();
  p->table = build_step_table(c, cfg->a_init, cfg->a_final, cfg->n_steps, cfg->flags);
  p->g_init = p->table[0].g;
  p->bins = make_bins(cfg->nm);
  p->tw_nm = twiddles(cfg->nm);
  p->tw_np = twiddles(cfg->np);
  // 2LPT multiplier: sqrt(P(k) / dp^3) / (kf n^2 np^3) at k = kf |n|, per integer n^2.
  const long h = cfg->np / 2;
  const long nmax = 3 * h * h;
  p->lpt_tab.assign(nmax + 1, 0.0f);
  const double kf = 2.0 * M_PI / cfg->box;
  const double dp3 = std::pow(cfg->box / cfg->np, 3);
  const double np3 = (double)cube(cfg->np);
  for (long q = 1; q <= nmax; ++q) {
    const double k = kf * std::sqrt((double)q);
    p->lpt_tab[q] = (float)(std::sqrt(c.power(k) / dp3) / (kf * (double)q * np3));
  }
  *out = p;
  return COLA_OK;
}

int cola_plan_destroy(cola_plan p) {
  if (!p) return COLA_OK;
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->device >= 0) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    (void)hipFree(p->d_tw_nm);
    (void)hipFree(p->d_tw_np);
    (void)hipFree(p->d_lpt_tab);
    (void)hipSetDevice(cur);
  }
  delete p;
  return COLA_OK;
}

int cola_workspace_bytes(cola_plan p, size_t* bytes) {
  if (!p || !bytes) return COLA_ERR_INVALID;
  // 3 nm^3 floats of meshes (np^3 <= nm^3 covers the 2LPT scratch), then the bins
  const size_t mesh = mesh_floats(p) * sizeof(float);
  const size_t sorted = 2 * 13 * (size_t)cube(p->cfg.np) * sizeof(float);
  *bytes = mesh + bin_workspace_bytes(cube(p->cfg.np), p->bins) + sorted;
  return COLA_OK;
}

int cola_step_table(cola_plan p, double* out, size_t len) {
  if (!p || !out) return COLA_ERR_INVALID;
  const int n = p->cfg.n_steps;
  if (len < (size_t)13 * (n + 1)) return COLA_ERR_INVALID;
  for (int i = 0; i <= n; ++i) {
    const StepRow& r = p->table[i];
    double* o = out + 13 * i;
    o[0] = r.a;
    o[1] = r.g.d1;
    o[2] = r.g.d2;
    o[3] = r.g.td1;
    o[4] = r.g.td2;
    o[5] = r.g.t2d1;
    o[6] = r.g.t2d2;
    o[7] = r.alpha;
    o[8] = r.beta;
    o[9] = r.dd1;
    o[10] = r.dd2;
    o[11] = r.a_mid;
    o[12] = r.force;
  }
  return COLA_OK;
}

int cola_noise(cola_plan p, uint64_t seed, float* w, void* stream) {
  if (!p || !w) return COLA_ERR_INVALID;
  COLA_TRY(ensure_device(p));
  hipStream_t st = (hipStream_t)stream;
  return hip_status(traced(p, kStNoise, st, [&] { return launch_noise(seed, w, cube(p->cfg.np), st); }));
}

int cola_init_2lpt(cola_plan p, const float* w, const cola_particles* q, void* ws_, void* stream) {
  COLA_TRY(check_common(p, ws_));
  COLA_TRY(check_particles(q));
  if (!w) return COLA_ERR_INVALID;
  p->res.valid = false;
  hipStream_t st = (hipStream_t)stream;
  const int n = p->cfg.np;
  const long r = cube(n);
  float* w0 = static_cast<float*>(ws_);
  const float2* tw = p->d_tw_np;
  // delta_k and its derivatives: s1 into q->s1, Hessian into q->s and q->v.
  COLA_HIP(traced(p, kStLptZFwd, st,
                  [&] { return launch_zfwd(n, w, reinterpret_cast<float2*>(w0), (long)n * n, tw, st); }));
  const int rot = rot_for(p, n);
  COLA_TRY(ypass(p, kStLptYFwd, n, -1, fields({w0}), 1, tw, st, rot));
  MulArgs m{};
  const double kf = 2.0 * M_PI / p->cfg.box;
  m.kf = (float)kf;
  m.tab = p->d_lpt_tab;
  float* s1[3] = {q->s1, q->s1 + r, q->s1 + 2 * r};
  float* hs[6] = {q->s, q->s + r, q->s + 2 * r, q->v, q->v + r, q->v + 2 * r};
  FieldPtrs outs = fields({s1[0], s1[1], s1[2], hs[0], hs[1], hs[2], hs[3], hs[4], hs[5]});
  COLA_HIP(traced(p, kStLptX, st,
                  [&] { return launch_xmul(n, kMulLpt1, reinterpret_cast<float2*>(w0), outs, 9, m, tw, 0, rot, st); }));
  COLA_TRY(ypass(p, kStLptYInv, n, 1, outs, 9, tw, st, rot));
  EpiArgs e{};
  e.scale = 1.0f;
  FieldPtrs f_s1 = fields({s1[0], s1[1], s1[2]});
  COLA_HIP(traced(p, kStLptZInv, st,
                  [&] { return launch_zinv(n, f_s1, f_s1, 3, (long)n * n, tw, kEpiStore, e, st); }));
  COLA_HIP(traced(p, kStLptHessian, st, [&] {
    return launch_zinv_hessian(n, fields({hs[0], hs[1], hs[2], hs[3], hs[4], hs[5]}), w0, (long)n * n, tw, 1.0f,
                               st);
  }));
  // second order: s2_k = -i k S_k / k^2
  COLA_HIP(traced(p, kStLptZFwd, st,
                  [&] { return launch_zfwd(n, w0, reinterpret_cast<float2*>(w0), (long)n * n, tw, st); }));
  COLA_TRY(ypass(p, kStLptYFwd, n, -1, fields({w0}), 1, tw, st, rot));
  float* s2[3] = {q->s2, q->s2 + r, q->s2 + 2 * r};
  FieldPtrs f_s2 = fields({s2[0], s2[1], s2[2]});
  MulArgs m2{};
  m2.c = (float)(-1.0 / (kf * (double)r));
  COLA_HIP(traced(p, kStLptX, st,
                  [&] { return launch_xmul(n, kMulGrad, reinterpret_cast<float2*>(w0), f_s2, 3, m2, tw, 0, rot, st); }));
  COLA_TRY(ypass(p, kStLptYInv, n, 1, f_s2, 3, tw, st, rot));
  // s2, then s = D1 s1 + D2 s2 and the initial velocity.
  EpiArgs ef{};
  ef.scale = 1.0f;
  ef.d1 = (float)p->g_init.d1;
  ef.d2 = (float)p->g_init.d2;
  ef.s1 = q->s1;
  ef.s = q->s;
  ef.v = q->v;
  ef.comp_stride = r;
  const bool plain = p->cfg.flags & COLA_FLAG_NO_LPT_FRAME;
  ef.v1 = plain ? (float)p->g_init.td1 : 0.0f;   // L-(a_init) cancels the 2LPT velocity
  ef.v2 = plain ? (float)p->g_init.td2 : 0.0f;
  COLA_HIP(traced(p, kStLptZInv, st,
                  [&] { return launch_zinv(n, f_s2, f_s2, 3, (long)n * n, tw, kEpiLptFinal, ef, st); }));
  return COLA_OK;
}

int cola_density(cola_plan p, const float* s, float* rho, void* ws, void* stream) {
  COLA_TRY(check_common(p, ws));
  if (!s || !rho) return COLA_ERR_INVALID;
  return deposit_into(p, s, rho, static_cast<float*>(ws), (hipStream_t)stream);
}

// Forward 3D transform of the real field in ws mesh m (in place, half spectrum).
int fft_forward(cola_plan p, float* g, hipStream_t st) {
  const int n = p->cfg.nm;
  const long h = n / 2;
  const float2* tw = p->d_tw_nm;
  COLA_HIP(traced(p, kStZFwd, st,
                  [&] { return launch_zfwd(n, g, reinterpret_cast<float2*>(g), (long)n * n, tw, st); }));
  COLA_TRY(ypass(p, kStYFwd, n, -1, fields({g}), 1, tw, st, 0));
  // x: columns along x (stride n h) in tiles of kz at fixed y
  return hip_status(traced(p, kStAnalysis, st, [&] {
    return launch_col(n, -1, fields({g}), fields({g}), 1, n, h, (long)n * h, (int)h, tw, p->fft_width[1], 0, st);
  }));
}

int cola_cross_power(cola_plan p, const float* s_a, const float* s_b, double* out, void* ws_, void* stream) {
  COLA_TRY(check_common(p, ws_));
  if (!s_a || !out) return COLA_ERR_INVALID;
  float* ws = static_cast<float*>(ws_);
  hipStream_t st = (hipStream_t)stream;
  const int n = p->cfg.nm;
  const long r = cube(n);
  float* ga = ws;
  float* gb = ws + r;
  COLA_TRY(deposit_into(p, s_a, ga, ws, st));
  COLA_TRY(fft_forward(p, ga, st));
  if (s_b) {
    COLA_TRY(deposit_into(p, s_b, gb, ws, st));
    COLA_TRY(fft_forward(p, gb, st));
  }
  // delta_k = rho_k / mean(rho) with mean 1 (particle mass (nm/np)^3); the k = 0 mode
  // is not reported.  P = <|delta_k|^2> L^3 / nm^6.
  const double norm = std::pow(p->cfg.box, 3) / std::pow((double)n, 6);
  double* part = reinterpret_cast<double*>(ws + 2 * r);   // meshes 2 and 3
  return hip_status(traced(p, kStAnalysis, st, [&] {
    return launch_shell_stats(n, reinterpret_cast<const float2*>(ga), s_b ? reinterpret_cast<const float2*>(gb) : nullptr,
                              part, r, norm, out, st);
  }));
}

int cola_pm_force(cola_plan p, const float* s, double a, float* acc, void* ws_, void* stream) {
  COLA_TRY(check_common(p, ws_));
  if (!s || !acc || !(a > 0)) return COLA_ERR_INVALID;
  hipStream_t st = (hipStream_t)stream;
  float* ws = static_cast<float*>(ws_);
  COLA_TRY(pm_mesh(p, s, a, ws, st));
  GatherArgs g = gather_args(p, ws);
  g.s = const_cast<float*>(s);
  g.out_a = acc;
  return hip_status(
      traced(p, kStGatherForce, st, [&] {
        return launch_gather_force(lattice(p), p->bins, bin_buffers(p, ws), g, st);
      }));
}

int cola_step(cola_plan p, int32_t i, const cola_particles* q, void* ws_, void* stream) {
  COLA_TRY(check_common(p, ws_));
  COLA_TRY(check_particles(q));
  if (i < 0 || i >= p->cfg.n_steps) return COLA_ERR_RANGE;
  float* ws = static_cast<float*>(ws_);
  return p->resident ? resident_step(p, i, q, ws, (hipStream_t)stream) : step_impl(p, i, q, ws, (hipStream_t)stream);
}

int cola_finish(cola_plan p, const cola_particles* q, float* x_out, float* v_out, void* ws_, void* stream) {
  COLA_TRY(check_common(p, ws_));
  COLA_TRY(check_particles(q));
  if (!x_out || !v_out) return COLA_ERR_INVALID;
  return finish_impl(p, q, x_out, v_out, static_cast<float*>(ws_), (hipStream_t)stream);
}

int cola_run(cola_plan p, const float* w, const cola_particles* q, float* x_out, float* v_out, void* ws_,
             void* stream) {
  COLA_TRY(cola_init_2lpt(p, w, q, ws_, stream));
  if (!x_out || !v_out) return COLA_ERR_INVALID;
  float* ws = static_cast<float*>(ws_);
  hipStream_t st = (hipStream_t)stream;
  const Lattice lat = lattice(p);
  const Bins& b = p->bins;
  const float mass = (float)std::pow((double)lat.ratio, 3);
  const bool plain = p->cfg.flags & COLA_FLAG_NO_LPT_FRAME;
  // The state is kept sorted by tile in two workspace copies: every step reads the
  // copy ordered by the previous step's tiles through this step's tile lists, and its
  // gather writes the updated state, ordered by this step's tiles, to the other copy
  // while binning the drifted particles for the next step.
  int parity = 0;
  BinBuffers bb = bin_buffers(p, ws, parity);
  COLA_HIP(traced(p, kStBinCount, st, [&] { return launch_bin_count(lat, b, q->s, bb, st); }));
  SortedState src{q->s, q->v, q->s1, q->s2, nullptr};
  int which = 0;
  GatherArgs g = gather_args(p, ws);
  for (int i = 0; i <= p->cfg.n_steps; ++i) {
    const bool last = i == p->cfg.n_steps;
    const StepRow& row = p->table[i];
    hipError_t trc;
    const long span = last ? -1 : trace_open(p, 2, kStRunStep, st, trc);
    if (!last) COLA_HIP(trc);
    bb = bin_buffers(p, ws, parity);
    COLA_HIP(traced(p, kStBinScan, st, [&] { return launch_bin_scan(b, bb, !last, st); }));
    COLA_HIP(traced(p, kStBinScatter, st, [&] { return launch_bin_scatter(lat, bb, st); }));
    COLA_HIP(traced(p, kStDeposit, st,
                    [&] { return launch_deposit(lat, b, src.s, bb, ws, mass, st, src.lag); }));
    COLA_TRY(fft_force(p, row.a, ws, st));
    KickArgs k{};
    k.alpha = (float)row.alpha;
    k.t2d1 = plain ? 0.0f : (float)row.g.t2d1;
    k.t2d2 = plain ? 0.0f : (float)row.g.t2d2;
    if (!last) {
      k.beta = (float)row.beta;
      k.dd1 = plain ? 0.0f : (float)row.dd1;
      k.dd2 = plain ? 0.0f : (float)row.dd2;
      const SortedState dst = sorted_state(p, ws, which);
      COLA_HIP(traced(p, kStGatherKickDrift, st,
                      [&] { return launch_gather_sorted(lat, b, src, dst, bb, kGatherKickDrift, g, k, st); }));
      COLA_HIP(trace_close(p, span, st));
      parity ^= 1;
      src = dst;
      which ^= 1;
    } else {
      k.td1 = plain ? 0.0f : (float)row.g.td1;
      k.td2 = plain ? 0.0f : (float)row.g.td2;
      k.box = (float)p->cfg.box;
      g.s = q->s;
      g.v = q->v;
      g.s1 = q->s1;
      g.s2 = q->s2;
      g.out_a = x_out;
      g.out_b = v_out;
      const SortedState out = sorted_state(p, ws, which);
      COLA_HIP(traced(p, kStFinish, st,
                      [&] { return launch_gather_sorted(lat, b, src, out, bb, kGatherFinish, g, k, st); }));
      COLA_HIP(traced(p, kStUnsort, st, [&] { return launch_unsort(lat, out, g, k, st); }));
    }
  }
  return COLA_OK;
}

int cola_run_checkpointed(cola_plan p, const float* w, const cola_particles* q, float* x_out, float* v_out,
                          float* ckpt, void* ws_, void* stream) {
  COLA_TRY(cola_init_2lpt(p, w, q, ws_, stream));
  if (!x_out || !v_out || !ckpt) return COLA_ERR_INVALID;
  float* ws = static_cast<float*>(ws_);
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = 3 * (size_t)cube(p->cfg.np) * sizeof(float);
  for (int i = 0; i < p->cfg.n_steps; ++i) {
    float* dst = ckpt + (size_t)i * 3 * cube(p->cfg.np);
    COLA_HIP(traced(p, kStCheckpoint, st,
                    [&] { return hipMemcpyAsync(dst, q->s, bytes, hipMemcpyDeviceToDevice, st); }));
    COLA_TRY(resident_step(p, i, q, ws, st));
  }
  float* last = ckpt + (size_t)p->cfg.n_steps * 3 * cube(p->cfg.np);
  COLA_HIP(traced(p, kStCheckpoint, st, [&] { return hipMemcpyAsync(last, q->s, bytes, hipMemcpyDeviceToDevice, st); }));
  return finish_impl(p, q, x_out, v_out, ws, st);
}

int cola_adjoint_workspace_bytes(cola_plan p, size_t* bytes) {
  if (!p || !bytes) return COLA_ERR_INVALID;
  *bytes = adj_layout(p, nullptr).bytes;
  return COLA_OK;
}

int cola_run_adjoint(cola_plan p, const float* w, const float* ckpt, const float* dL_drho, float* dL_dw, void* ws,
                     void* stream) {
  COLA_TRY(check_common(p, ws));
  if (!w || !ckpt || !dL_drho || !dL_dw) return COLA_ERR_INVALID;
  return run_adjoint(p, w, ckpt, dL_drho, dL_dw, static_cast<float*>(ws), (hipStream_t)stream);
}

int cola_fft_r2c(cola_plan p, int32_t n, const float* in, float* out, void* stream) {
  if (!p || !in || !out) return COLA_ERR_INVALID;
  if (n != p->cfg.nm && n != p->cfg.np) return COLA_ERR_INVALID;
  COLA_TRY(ensure_device(p));
  hipStream_t st = (hipStream_t)stream;
  const float2* tw = twiddle_for(p, n);
  COLA_HIP(traced(p, kStFft, st,
                  [&] { return launch_zfwd(n, in, reinterpret_cast<float2*>(out), (long)n * n, tw, st); }));
  COLA_TRY(ypass(p, kStFft, n, -1, fields({out}), 1, tw, st, 0));
  const long h = n / 2;
  FieldPtrs f = fields({out});
  return hip_status(
      traced(p, kStFft, st, [&] { return launch_col(n, -1, f, f, 1, n, h, (long)n * h, (int)h, tw, 0, 0, st); }));
}

int cola_fft_c2r(cola_plan p, int32_t n, const float* in, float* out, void* stream) {
  if (!p || !in || !out) return COLA_ERR_INVALID;
  if (n != p->cfg.nm && n != p->cfg.np) return COLA_ERR_INVALID;
  COLA_TRY(ensure_device(p));
  hipStream_t st = (hipStream_t)stream;
  const float2* tw = twiddle_for(p, n);
  const long h = n / 2;
  FieldPtrs fi = fields({const_cast<float*>(in)});
  FieldPtrs fo = fields({out});
  COLA_HIP(
      traced(p, kStFft, st, [&] { return launch_col(n, 1, fi, fo, 1, n, h, (long)n * h, (int)h, tw, 0, 0, st); }));
  COLA_TRY(ypass(p, kStFft, n, 1, fo, 1, tw, st, 0));
  EpiArgs e{};
  e.scale = (float)(1.0 / (double)cube(n));
  return hip_status(
      traced(p, kStFft, st, [&] { return launch_zinv(n, fo, fo, 1, (long)n * n, tw, kEpiStore, e, st); }));
}

int cola_plan_set_fft_tile(cola_plan p, int32_t pass, int32_t width) {
  if (!p || pass < 0 || pass > 1) return COLA_ERR_INVALID;
  if (!fft_width_supported(p->cfg.nm, width)) return COLA_ERR_UNSUPPORTED_SIZE;
  p->fft_width[pass] = width;
  return COLA_OK;
}

int cola_plan_set_bin_depth(cola_plan p, int32_t tz) {
  if (!p || (tz != 8 && tz != 16 && tz != 32 && tz != 64)) return COLA_ERR_INVALID;
  if (p->cfg.nm % tz) return COLA_ERR_UNSUPPORTED_SIZE;
  p->bins = make_bins(p->cfg.nm, tz);
  p->res.valid = false;
  return COLA_OK;
}

int cola_plan_set_resident_steps(cola_plan p, int32_t on) {
  if (!p || (on != 0 && on != 1)) return COLA_ERR_INVALID;
  p->resident = on;
  p->res.valid = false;
  return COLA_OK;
}

int cola_plan_set_fft_rotation(cola_plan p, int32_t on) {
  if (!p || on < -1 || on > 1) return COLA_ERR_INVALID;
  p->fft_rot = on;
  return COLA_OK;
}

int cola_plan_get_fft_rotation(cola_plan p, int32_t* rot) {
  if (!p || !rot) return COLA_ERR_INVALID;
  *rot = rot_for(p, p->cfg.nm);
  return COLA_OK;
}

int cola_plan_get_tuning(cola_plan p, int32_t* y_width, int32_t* x_width, int32_t* bin_depth) {
  if (!p || !y_width || !x_width || !bin_depth) return COLA_ERR_INVALID;
  *y_width = p->fft_width[0];
  *x_width = p->fft_width[1];
  *bin_depth = p->bins.tz;
  return COLA_OK;
}

int cola_tuning_workspace_bytes(cola_plan p, size_t* bytes) {
  if (!p || !bytes) return COLA_ERR_INVALID;
  size_t worst = 0;
  for (int tz : {8, 16, 32, 64})
    if (p->cfg.nm % tz == 0) worst = std::max(worst, bin_workspace_bytes(cube(p->cfg.np), make_bins(p->cfg.nm, tz)));
  *bytes = mesh_floats(p) * sizeof(float) + worst;
  return COLA_OK;
}

int cola_autotune(cola_plan p, const cola_particles* q, void* ws_, size_t ws_bytes, void* stream,
                  const char* cache_path, int32_t* used_cache) {
  COLA_TRY(check_common(p, ws_));
  COLA_TRY(check_particles(q));
  p->res.valid = false;
  if (used_cache) *used_cache = 0;
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  COLA_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  COLA_HIP(hipGetDeviceProperties(&prop, dev));
  char key[256];
  std::snprintf(key, sizeof(key), "np=%d nm=%d arch=%s", p->cfg.np, p->cfg.nm, prop.gcnArchName);
  // cached choice?
  if (cache_path) {
    if (FILE* fh = std::fopen(cache_path, "r")) {
      char line[512];
      while (std::fgets(line, sizeof(line), fh)) {
        int y = 0, x = 0, tz = 0;
        char k[256] = {0};
        if (std::sscanf(line, "%255[^|]| y=%d x=%d tz=%d", k, &y, &x, &tz) == 4) {
          std::string ks(k);
          while (!ks.empty() && ks.back() == ' ') ks.pop_back();
          if (ks == key && fft_width_supported(p->cfg.nm, y) && fft_width_supported(p->cfg.nm, x) &&
              p->cfg.nm % tz == 0 && (tz == 8 || tz == 16 || tz == 32 || tz == 64)) {
            std::fclose(fh);
            p->fft_width[0] = y;
            p->fft_width[1] = x;
            p->bins = make_bins(p->cfg.nm, tz);
            if (used_cache) *used_cache = 1;
            return COLA_OK;
          }
        }
      }
      std::fclose(fh);
    }
  }
  // Measure every valid combination on the PM force of the given particles; tile
  // depths whose binning buffers would not fit the given workspace are skipped.
  const bool was_tracing = p->trace;
  if (ws_bytes < mesh_floats(p) * sizeof(float)) return COLA_ERR_INVALID;
  const size_t bin_cap = ws_bytes - mesh_floats(p) * sizeof(float);
  p->trace = false;
  hipEvent_t e0, e1;
  COLA_HIP(hipEventCreate(&e0));
  COLA_HIP(hipEventCreate(&e1));
  float* ws = static_cast<float*>(ws_);
  float best = 1e30f;
  int by = 0, bx = 0, btz = p->bins.tz;
  const int default_tz = p->bins.tz;
  int rc = COLA_OK;
  const int widths[] = {4, 8, 16};
  (void)default_tz;
  for (int tz : {8, 16, 32, 64}) {
    if (p->cfg.nm % tz) continue;
    if (bin_workspace_bytes(cube(p->cfg.np), make_bins(p->cfg.nm, tz)) > bin_cap) continue;
    p->bins = make_bins(p->cfg.nm, tz);
    for (int y : widths) {
      if (!fft_width_supported(p->cfg.nm, y)) continue;
      for (int x : widths) {
        if (!fft_width_supported(p->cfg.nm, x)) continue;
        p->fft_width[0] = y;
        p->fft_width[1] = x;
        float t_min = 1e30f;
        for (int rep = 0; rep < 3 && rc == COLA_OK; ++rep) {
          rc = hip_status(hipEventRecord(e0, st));
          if (rc == COLA_OK) rc = pm_mesh(p, q->s, p->table[0].a, ws, st);
          if (rc == COLA_OK) rc = hip_status(hipEventRecord(e1, st));
          if (rc == COLA_OK) rc = hip_status(hipEventSynchronize(e1));
          float ms = 0.f;
          if (rc == COLA_OK) rc = hip_status(hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) t_min = std::min(t_min, ms);
        }
        if (rc != COLA_OK) break;
        if (t_min < best) {
          best = t_min;
          by = y;
          bx = x;
          btz = tz;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->trace = was_tracing;
  p->fft_width[0] = by;
  p->fft_width[1] = bx;
  p->bins = make_bins(p->cfg.nm, btz);
  if (rc != COLA_OK) return rc;
  if (cache_path) {
    if (FILE* fh = std::fopen(cache_path, "a")) {
      std::fprintf(fh, "%s | y=%d x=%d tz=%d ms=%.4f\n", key, by, bx, btz, best);
      std::fclose(fh);
    }
  }
  return COLA_OK;
}

// ---------------------------------------------------------------------------------
// Ensembles: whole runs of many plans captured once into one hipGraph, one parallel
// branch per member, and replayed with a single graph launch.
// ---------------------------------------------------------------------------------
struct cola_ensemble_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = -1;
  int members = 0;
  std::vector<const void*> ws;   // member workspaces (each replay writes them)
};

int cola_ensemble_create(int32_t n, const cola_plan* plans, const float* const* w, const cola_particles* parts,
                         float* const* x_out, float* const* v_out, void* const* ws, cola_ensemble* out) {
  if (!out || n <= 0 || !plans || !w || !parts || !x_out || !v_out || !ws) return COLA_ERR_INVALID;
  *out = nullptr;
  for (int k = 0; k < n; ++k) {
    COLA_TRY(check_common(plans[k], ws[k]));
    COLA_TRY(check_particles(&parts[k]));
    if (!w[k] || !x_out[k] || !v_out[k]) return COLA_ERR_INVALID;
    if (plans[k]->trace) return COLA_ERR_INVALID;   // no event records inside a graph
  }
  hipStream_t s0 = nullptr;
  std::vector<hipStream_t> side(n, nullptr);
  std::vector<hipEvent_t> done(n, nullptr);
  hipEvent_t fork = nullptr;
  int rc = hip_status(hipStreamCreate(&s0));
  for (int k = 0; k < n && rc == COLA_OK; ++k) {
    rc = hip_status(hipStreamCreate(&side[k]));
    if (rc == COLA_OK) rc = hip_status(hipEventCreateWithFlags(&done[k], hipEventDisableTiming));
  }
  if (rc == COLA_OK) rc = hip_status(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  hipGraph_t graph = nullptr;
  bool capturing = false;
  if (rc == COLA_OK) {
    rc = hip_status(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
    capturing = rc == COLA_OK;
  }
  if (rc == COLA_OK) rc = hip_status(hipEventRecord(fork, s0));
  for (int k = 0; k < n && rc == COLA_OK; ++k) {
    rc = hip_status(hipStreamWaitEvent(side[k], fork, 0));
    if (rc == COLA_OK) rc = cola_run(plans[k], w[k], &parts[k], x_out[k], v_out[k], ws[k], side[k]);
    if (rc == COLA_OK) rc = hip_status(hipEventRecord(done[k], side[k]));
    if (rc == COLA_OK) rc = hip_status(hipStreamWaitEvent(s0, done[k], 0));
  }
  if (capturing) {
    const int rc_end = hip_status(hipStreamEndCapture(s0, &graph));
    if (rc == COLA_OK) rc = rc_end;
  }
  cola_ensemble e = nullptr;
  if (rc == COLA_OK) {
    e = new (std::nothrow) cola_ensemble_s();
    if (!e) rc = COLA_ERR_INVALID;
  }
  if (rc == COLA_OK) {
    e->graph = graph;
    e->members = n;
    e->ws.assign(ws, ws + n);
    (void)hipGetDevice(&e->device);
    rc = hip_status(hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0));
  }
  for (int k = 0; k < n; ++k) {
    if (done[k]) (void)hipEventDestroy(done[k]);
    if (side[k]) (void)hipStreamDestroy(side[k]);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (s0) (void)hipStreamDestroy(s0);
  if (rc != COLA_OK) {
    if (e) {
      if (e->exec) (void)hipGraphExecDestroy(e->exec);
      delete e;
    }
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  *out = e;
  return COLA_OK;
}

int cola_run_batched(int32_t n, const cola_plan* plans, const float* const* w, const cola_particles* parts,
                     float* const* x_out, float* const* v_out, void* const* ws, void* stream) {
  cola_ensemble e = nullptr;
  COLA_TRY(cola_ensemble_create(n, plans, w, parts, x_out, v_out, ws, &e));
  int rc = cola_ensemble_launch(e, stream);
  // the graph is freed only after its launch has finished
  if (rc == COLA_OK) rc = hip_status(hipStreamSynchronize((hipStream_t)stream));
  const int rc_destroy = cola_ensemble_destroy(e);
  return rc != COLA_OK ? rc : rc_destroy;
}

int cola_ensemble_launch(cola_ensemble e, void* stream) {
  if (!e || !e->exec) return COLA_ERR_INVALID;
  for (const void* w : e->ws) ws_bump(w);
  return hip_status(hipGraphLaunch(e->exec, (hipStream_t)stream));
}

int cola_ensemble_destroy(cola_ensemble e) {
  if (!e) return COLA_OK;
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  delete e;
  return COLA_OK;
}

int cola_trace_enable(cola_plan p, int enable) {
  if (!p || enable < 0 || enable > 2) return COLA_ERR_INVALID;
  p->trace = enable;
  p->ev_used = 0;
  return COLA_OK;
}

int cola_trace_read(cola_plan p, double* ms, int32_t* launches, int32_t n) {
  if (!p || !ms || !launches || n < kNumStages) return COLA_ERR_INVALID;
  for (int k = 0; k < kNumStages; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  for (size_t j = 0; j < p->ev_used; ++j) {
    COLA_HIP(hipEventSynchronize(p->ev_pool[2 * j + 1]));
    float t = 0.f;
    COLA_HIP(hipEventElapsedTime(&t, p->ev_pool[2 * j], p->ev_pool[2 * j + 1]));
    ms[p->ev_stage[j]] += t;
    launches[p->ev_stage[j]] += 1;
  }
  p->ev_used = 0;
  return COLA_OK;
}

const char* cola_trace_stage_name(int32_t stage) {
  return (stage >= 0 && stage < kNumStages) ? kStageNames[stage] : nullptr;
}

int32_t cola_trace_stage_count(void) { return kNumStages; }

const char* cola_strerror(int status) {
  switch (status) {
    case COLA_OK:
      return "success";
    case COLA_ERR_INVALID:
      return "invalid argument (null pointer or inconsistent parameter)";
    case COLA_ERR_UNSUPPORTED_SIZE:
      return "unsupported size: np and nm must be one of 16 24 32 48 64 96 128 192 256 384 512 768 1024";
    case COLA_ERR_RANGE:
      return "step index out of range";
    case COLA_ERR_HIP:
      return "HIP runtime error (see cola_last_hip_error)";
    case COLA_ERR_DEVICE:
      return "plan tables live on another device";
    case COLA_ERR_WORKSPACE:
      return "the configuration needs more than the library's static scratch (256 MiB of binning buffers)";
    default:
      return "unknown status";
  }
}

int cola_last_hip_error(void) { return g_last_hip; }

}  // extern "C"
