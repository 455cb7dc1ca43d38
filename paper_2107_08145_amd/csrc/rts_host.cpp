// Host side of librts: the C ABI declared in include/rts.h.
//
// Validates the problem statement, turns every box's rays into sweep tasks
// (rays grouped by dominant axis and direction, at most four per task, as the
// paper's ray groups of "a similar dependency pattern"), lays out the caller's
// workspace, and enqueues prep -> sweep -> reduce on the caller's stream
// (optionally as one replayed hipGraph).  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rts.h"
#include "rts_internal.h"

namespace rts {
// kernels (rts_sweep.hpp, rts_reverse.hpp, rts_misc.hip)
template <class Real>
hipError_t launch_prep(const void*, const void*, const void*, void*, int64_t, int64_t, int64_t,
                       int, int, int, int, hipStream_t);
hipError_t launch_zero(int*, int64_t, hipStream_t);
template <class Real, int H>
size_t sweep_lds_bytes(int threads);
template <class Real, int H, bool UNI>
const void* sweep_fn();
template <class Real, int H, bool UNI>
const void* sweep_fn_ext(int ext);
template <class Real, int H, bool UNI>
hipError_t launch_sweep_h(const SweepArgs&, int, int, hipStream_t);
template <class Real>
hipError_t launch_reduce(const char*, const Task*, const BoxGeo&, const BoxPtrs&, hipStream_t);
template <class Real>
hipError_t launch_scan_nonfinite(const void*, int64_t, int*, int, hipStream_t);

hipError_t launch_gs_init(const GsArgs&, hipStream_t);
hipError_t launch_gs_ghost(const GsArgs&, int, int, hipStream_t);
hipError_t launch_gs_plane(const GsArgs&, int, int, int, int, int, int, hipStream_t);
hipError_t launch_gs_step(const GsArgs&, int, int, int, hipStream_t);
hipError_t launch_gs_finish(const GsArgs&, hipStream_t);

template <class Real>
hipError_t launch_block_init(const BlockArgs&, int64_t, hipStream_t);
template <class Real>
hipError_t launch_block_sweep(const BlockArgs&, int, int, hipStream_t);

template <class Real>
size_t reverse_lds_bytes(int, bool);
template <class Real>
const void* reverse_fn(int cols, bool small);
template <class Real>
int reverse_rows(int cols, bool small);
template <class Real>
hipError_t launch_reverse(const RevArgs&, int, int, bool, hipStream_t);
template <class Real>
hipError_t launch_adj_seed(const void*, const void*, const double*, const void*, void*, void*,
                           double, int, int, int, hipStream_t);
template <class Real>
hipError_t launch_adj_reduce(const char*, const Task*, const AdjTask*, const BoxGeo&,
                             const double*, const void*, const void*, const void*, void*, void*,
                             hipStream_t);
}  // namespace rts

using namespace rts;

namespace {

thread_local std::string g_last_hip;

int hip_fail(hipError_t e, const char* where) {
  g_last_hip = std::string(where) + ": " + hipGetErrorString(e);
  return RTS_E_HIP;
}

#define RTS_HIP(call)                              \
  do {                                             \
    hipError_t _e = (call);                        \
    if (_e != hipSuccess) return hip_fail(_e, #call); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxTimed = 512;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct RayGeo {
  int axis, sa;
  double ds;
  double mu[3];
};

// Dominant axis: the one reached first along the ray (smallest delta/|mu|);
// ties prefer z, then y, then x.
RayGeo ray_geo(const rts_grid& g, const double* m) {
  const double d[3] = {g.dx, g.dy, g.dz};
  RayGeo r;
  r.axis = -1;
  r.ds = INFINITY;
  for (int a = 0; a < 3; ++a) {
    r.mu[a] = m[a];
    if (m[a] == 0.0) continue;
    const double s = d[a] / std::fabs(m[a]);
    if (s <= r.ds) { r.ds = s; r.axis = a; }
  }
  r.sa = m[r.axis] > 0 ? 1 : -1;
  return r;
}

struct Box {
  rts_desc d;
  std::vector<double> mu, w, qw;
  int64_t N = 0;
  int n_up = 0;
  int tasks_per_band = 0;
  std::vector<std::array<int, 4>> groups;  // ray index per slot (-1 unused), same for every band
  int64_t chi_off = 0, chiT_off = 0, sT_off = 0;  // Real-element offsets
  int64_t seed_off = 0, seedT_off = 0;            // adjoint seeds [nbands][N], both layouts
  int64_t btol_off = -1;  // decomposed with tol: 64-bit word offset of [n_iter][2] maxima
};

struct Plan {
  std::vector<Box> boxes;
  int prec = RTS_FP64;
  size_t esz = 8;
  rts_schedule sched{4, 0, 0, 0, 0, 0};
  // layout (bytes)
  size_t off_flags = 0, off_tasks = 0, off_queue = 0, off_atasks = 0, off_rqueue = 0,
         off_data = 0, total = 0;
  // adjoint: the solve layout, then stored D planes, the reverse sweep's
  // reverse exchange rings [off_grads, off_xrev_end) (cleared per call), gradient
  // partials [off_xrev_end, off_grads_end), seeds
  size_t off_grads = 0, off_xrev_end = 0, off_grads_end = 0, total_adj = 0;
  std::vector<AdjTask> atasks;
  std::vector<int32_t> rqueue;
  int rev_blocks = 0;
  std::vector<Task> tasks;
  std::vector<int32_t> queue;
  int total_strips = 0;
  int max_strips = 1;  // strips of the largest task
  // forward sweep launches: one per workgroup width (unless sched.single_launch),
  // widest first; each owns a contiguous segment of the queue with its own tickets
  struct WidthClass {
    int width;       // padded columns that select the class (0: every task)
    int threads;     // workgroup size: the padded columns of its widest task
    int q0, nq;      // queue entries [q0, q0 + nq)
    int strips;      // tickets of the launch
    int max_strips;  // strips of its largest task
    int blocks;      // resident workgroups per CU
    bool uni;        // every task of the launch has four uniform slots
  };
  std::vector<WidthClass> wclasses;
  std::vector<WidthClass> rclasses;  // the same for the reverse sweep (threads: padded columns)
  std::map<int, bool> rev_small;     // reverse launch width -> short strips (small problems)
  int threads = 64;
  bool uni = true;  // every task's four slots share f1, f2, ds and w
  // subdomain decomposition: every box of the plan is divided (rts_desc.sub)
  bool decomposed = false;
  // scattering with Gauss-Seidel source updates (rts_desc.gs_iter > 0)
  int gs_iter = 0;
  std::vector<GsGroup> gsg;
  size_t off_gsg = 0;             // the group table (with the task tables)
  int64_t gs_s = 0, gs_j = 0, gs_p = 0, gs_l = 0, gs_i = 0;  // double offsets of the state
  int max_blocks = 1;      // blocks of the most divided box
  int64_t max_cells = 0;   // cells of the largest box
  int max_iter = 1;        // the largest n_iter
  // device-dependent state, filled on first use
  bool dev_ready = false;
  int device = -1, cus = 0, occupancy_blocks = 0;
  std::string arch;  // the device's architecture name, e.g. gfx950:sramecc+:xnack-
  int64_t timeout_ticks = 0;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  std::vector<void*> old_pinned;
  // graph cache
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;           // the captured graph of gexec
  hipEvent_t cap_ev[4] = {};            // events recorded at capture (timed graphs)
  hipGraphNode_t ev_nodes[4] = {};      // their event-record nodes
  std::vector<const void*> gkey;
  // timing: events of up to kMaxTimed calls (call start, sweep start, sweep end, call end)
  bool timing = false;
  std::vector<std::array<hipEvent_t, 4>> ev;
  int ev_used = 0;
};

bool finite(double v) { return std::isfinite(v); }

// A box cut into subdomains with lagged exchange (rts_desc.sub).
bool decomposed(const rts_desc& d) { return d.sub[0] > 0 || d.sub[1] > 0 || d.sub[2] > 0; }

int validate_desc(const rts_desc& d) {
  const rts_grid& g = d.g;
  if (g.nx < 2 || g.ny < 2 || g.nz < 2) return RTS_E_ARG;
  if (!(g.dx > 0) || !(g.dy > 0) || !(g.dz > 0) || !finite(g.dx) || !finite(g.dy) ||
      !finite(g.dz))
    return RTS_E_ARG;
  if (d.nbands < 1 || d.nrays < 1 || !d.mu || !d.w) return RTS_E_ARG;
  if (d.n_iter < 1) return RTS_E_ARG;
  if (d.bot != RTS_BOT_THERMAL && d.bot != RTS_BOT_FIXED) return RTS_E_ARG;
  if (d.top != RTS_TOP_ZERO && d.top != RTS_TOP_THERMAL) return RTS_E_ARG;
  if (d.prec != RTS_FP64 && d.prec != RTS_FP32) return RTS_E_ARG;
  if (d.flux != 0 && d.flux != 1) return RTS_E_ARG;
  if (!finite(d.tol) || d.tol < 0) return RTS_E_ARG;
  if (!finite(d.i_bot)) return RTS_E_ARG;
  for (int r = 0; r < d.nrays; ++r) {
    const double* m = d.mu + 3 * r;
    if (!finite(m[0]) || !finite(m[1]) || !finite(m[2]) || !finite(d.w[r])) return RTS_E_ARG;
    const double n2 = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    if (std::fabs(n2 - 1.0) > 1e-6) return RTS_E_ARG;
    if (m[2] == 0.0) return RTS_E_ARG;
  }
  if (d.qweight)
    for (int b = 0; b < d.nbands; ++b)
      if (!finite(d.qweight[b])) return RTS_E_ARG;
  const int n3[3] = {g.nx, g.ny, g.nz};
  for (int a = 0; a < 3; ++a)
    if (d.sub[a] < 0 || d.sub[a] > n3[a]) return RTS_E_ARG;
  if (decomposed(d) && d.flux) return RTS_E_UNSUPPORTED;
  if (d.gs_iter < 0) return RTS_E_ARG;
  if (d.gs_iter > 0 && (d.prec != RTS_FP64 || decomposed(d) || d.flux || d.tol > 0)) {
    g_last_hip = "scattering (gs_iter > 0) needs FP64, no flux, no tolerance and no subdomains";
    return RTS_E_UNSUPPORTED;
  }
  if (d.nbands > 16 || d.nrays > 64) return RTS_E_UNSUPPORTED;
  if (g.nx > kMaxCols || g.ny > kMaxCols) return RTS_E_UNSUPPORTED;
  if ((int64_t)g.nx * g.ny * g.nz > ((int64_t)1 << 31)) return RTS_E_UNSUPPORTED;
  if ((int64_t)g.nz * d.nbands > 65535) return RTS_E_UNSUPPORTED;  // grid z of prep and reduce
  return RTS_OK;
}

// Build every task of every box and the workspace layout for the current schedule.
void build_layout(Plan& P) {
  P.tasks.clear();
  P.queue.clear();
  const int H = P.sched.rows_per_strip;
  const size_t esz = P.esz;
  size_t off = align_up(sizeof(WsHeader));
  // first pass: count tasks and strips
  struct Pending { int box, band, g; };
  std::vector<Pending> order;
  for (size_t b = 0; b < P.boxes.size(); ++b)
    for (int band = 0; band < P.boxes[b].d.nbands; ++band)
      for (int g = 0; g < P.boxes[b].tasks_per_band; ++g) order.push_back({(int)b, band, g});
  P.tasks.resize(order.size());
  int max_cols = 1;
  // data region offsets computed after headers
  for (size_t t = 0; t < order.size(); ++t) {
    const Box& B = P.boxes[order[t].box];
    const rts_desc& d = B.d;
    const int nx = d.g.nx, ny = d.g.ny, nz = d.g.nz;
    const std::array<int, 4>& slots = B.groups[order[t].g];
    int first_ray = -1;
    for (int k = 0; k < 4; ++k)
      if (slots[k] >= 0) { first_ray = slots[k]; break; }
    RayGeo g0 = ray_geo(d.g, &B.mu[3 * first_ray]);
    Task T;
    std::memset(&T, 0, sizeof(T));
    T.box = order[t].box;
    T.band = order[t].band;
    T.sa = g0.sa;
    T.nrays = 0;
    if (g0.axis == 2) {
      T.n_planes = nz; T.n_rows = ny; T.n_cols = nx;
      T.plane_stride = (int64_t)nx * ny; T.row_stride = nx;
      T.z_planes = 1; T.row_periodic = 1; T.laps = 1; T.transposed = 0;
      T.it_top = nz - 1; T.itp = 0; T.itr = nx; T.itc = 1;
    } else if (g0.axis == 1) {
      T.n_planes = ny; T.n_rows = nz; T.n_cols = nx;
      T.plane_stride = nx; T.row_stride = (int64_t)nx * ny;
      T.z_planes = 0; T.row_periodic = 0; T.laps = d.n_iter; T.transposed = 0;
      T.it_top = nz - 1; T.itp = nx; T.itr = 0; T.itc = 1;
    } else {
      T.n_planes = nx; T.n_rows = nz; T.n_cols = ny;
      T.plane_stride = (int64_t)nz * ny; T.row_stride = ny;
      T.z_planes = 0; T.row_periodic = 0; T.laps = d.n_iter; T.transposed = 1;
      T.it_top = nz - 1; T.itp = 1; T.itr = 0; T.itc = nx;
    }
    // boundary values D = I - S = a S + b of the bottom (thermal: 0; fixed:
    // i_bot - S) and top (zero: -S; thermal: 0) layers
    const double bot_a = d.bot == RTS_BOT_THERMAL ? 0.0 : -1.0;
    const double bot_b = d.bot == RTS_BOT_THERMAL ? 0.0 : d.i_bot;
    const double top_a = d.top == RTS_TOP_ZERO ? -1.0 : 0.0, top_b = 0.0;
    if (T.z_planes) {
      T.pl_a = T.sa > 0 ? bot_a : top_a;
      T.pl_b = T.sa > 0 ? bot_b : top_b;
    }
    T.bu_a = bot_a; T.bu_b = bot_b; T.bd_a = top_a; T.bd_b = top_b;
    const int col_axis = g0.axis == 0 ? 1 : 0;
    const int row_axis = g0.axis == 2 ? 1 : 2;
    const double dd[3] = {d.g.dx, d.g.dy, d.g.dz};
    std::vector<int> up_index(d.nrays, -1);
    for (int r = 0, u = 0; r < d.nrays; ++r)
      if (B.mu[3 * r + 2] > 0) up_index[r] = u++;
    bool uni = true;
    for (int k = 0; k < 4; ++k) {
      TaskRay& y = T.ray[k];
      const int r = slots[k];
      y.ray = r;
      if (r < 0) {  // unused slot: contributes nothing
        y.f1 = y.f2 = y.hds = y.w = 0.0;
        y.itop = -1;
        uni = false;
        continue;
      }
      ++T.nrays;
      RayGeo g = ray_geo(d.g, &B.mu[3 * r]);
      y.wm[0] = B.w[r] * B.mu[3 * r + col_axis];
      y.wm[1] = B.w[r] * B.mu[3 * r + row_axis];
      y.wm[2] = B.w[r] * B.mu[3 * r + g0.axis];
      y.f1 = g.ds * std::fabs(g.mu[col_axis]) / dd[col_axis];
      y.f2 = g.ds * std::fabs(g.mu[row_axis]) / dd[row_axis];
      y.hds = 0.5 * g.ds;
      y.w = B.w[r];
      y.itop = up_index[r];
    }
    for (int k = 1; k < 4 && uni; ++k)
      uni = T.ray[k].f1 == T.ray[0].f1 && T.ray[k].f2 == T.ray[0].f2 &&
            T.ray[k].hds == T.ray[0].hds && T.ray[k].w == T.ray[0].w;
    T.uni = uni ? 1 : 0;
    T.frame[0] = col_axis;
    T.frame[1] = row_axis;
    T.frame[2] = g0.axis;
    T.it_ray = (int64_t)nx * ny;
    T.it_off = (int64_t)T.band * B.n_up * nx * ny;
    T.rows_per_strip = std::min(H, T.n_rows);
    T.strips = (T.n_rows + T.rows_per_strip - 1) / T.rows_per_strip;
    T.n_unrolled = T.z_planes ? T.n_planes : T.laps * T.n_planes;
    T.gh_M = std::max(nx, ny);
    T.gh_off = (int64_t)T.band * d.nrays * nz * T.gh_M;
    max_cols = std::max(max_cols, T.n_cols);
    P.tasks[t] = T;
  }
  // scattering: the ray groups of the (single) box, from its band-0 tasks
  P.gsg.clear();
  if (P.gs_iter > 0)
    for (int g = 0; g < P.boxes[0].tasks_per_band; ++g) {
      const Task& T = P.tasks[g];
      GsGroup G;
      std::memset(&G, 0, sizeof(G));
      G.axis = T.frame[2];
      G.sa = T.sa;
      G.ea = T.frame[0];  // (the column axis is the lower one)
      G.eb = T.frame[1];
      G.laps = T.laps;
      for (int k = 0; k < kMaxRaysPerTask; ++k) {
        const TaskRay& y = T.ray[k];
        GsRay& z = G.ray[k];
        z.used = y.ray >= 0 ? 1 : 0;
        z.fa = y.f1;
        z.fb = y.f2;
        z.hds = y.hds;
        z.w = y.w;
        z.sea = k < 2 ? 1 : -1;  // (slot k: upwind column c - 1 for k < 2, row i - 1 for even k)
        z.seb = (k & 1) == 0 ? 1 : -1;
        z.up = y.itop >= 0 ? 1 : 0;
        z.itop = y.itop;
        G.wsum += y.w;
      }
      P.gsg.push_back(G);
    }
  // Queue: tasks grouped by workgroup width (a workgroup has one thread per
  // padded column of the widest task it may claim, so narrow tasks in a wide
  // launch leave waves idle), widest first; inside a group the longest sweeps
  // (most plane steps x cells) first, or input order; stable.
  auto width_of = [&](const Task& T) {
    return P.sched.single_launch ? 0 : (T.n_cols + 63) / 64 * 64;
  };
  std::vector<int> q(P.tasks.size());
  for (size_t i = 0; i < q.size(); ++i) q[i] = (int)i;
  std::stable_sort(q.begin(), q.end(), [&](int a, int b) {
    const Task& A = P.tasks[a];
    const Task& Bt = P.tasks[b];
    if (width_of(A) != width_of(Bt)) return width_of(A) > width_of(Bt);
    if (P.sched.order != 0) return false;
    const int64_t sa = (int64_t)A.laps * A.n_planes, sb = (int64_t)Bt.laps * Bt.n_planes;
    if (sa != sb) return sa > sb;
    return (int64_t)A.n_rows * A.n_cols > (int64_t)Bt.n_rows * Bt.n_cols;
  });
  P.wclasses.clear();
  int ticket = 0;
  P.total_strips = 0;
  for (size_t k = 0; k < q.size(); ++k) {
    Task& T = P.tasks[q[k]];
    if (P.wclasses.empty() || P.wclasses.back().width != width_of(T)) {
      P.wclasses.push_back(Plan::WidthClass{width_of(T), 64, (int)k, 0, 0, 1, 0, true});
      ticket = 0;  // every launch counts its own tickets from 0
    }
    Plan::WidthClass& c = P.wclasses.back();
    T.ticket0 = ticket;
    P.queue.push_back(ticket);
    P.queue.push_back(q[k]);
    ticket += T.strips;
    P.total_strips += T.strips;
    c.nq += 1;
    c.strips = ticket;
    c.max_strips = std::max(c.max_strips, (int)T.strips);
    c.threads = std::max(c.threads, (T.n_cols + 63) / 64 * 64);
    c.uni = c.uni && T.uni != 0;
  }
  P.max_strips = 1;
  for (const Task& T : P.tasks) P.max_strips = std::max(P.max_strips, (int)T.strips);
  P.threads = ((max_cols + 63) / 64) * 64;
  P.uni = true;
  for (const Task& T : P.tasks) P.uni = P.uni && T.uni;

  // layout: header, then the neighbour exchange buffers (both zeroed by every
  // call: exchanged words carry step tags that must not survive a call), the
  // task table and queue, the per-box arrays and the per-task partial sums
  const size_t words = P.prec == RTS_FP32 ? 1 : 2;  // 64-bit words per exchanged value
  P.off_flags = off;
  for (Task& T : P.tasks) {
    T.xbuf_off = (int64_t)(off / sizeof(uint64_t));
    off = align_up(off + (size_t)T.strips * 2 * 2 * kMaxRaysPerTask * T.n_cols * words * sizeof(uint64_t));
  }
  for (Task& T : P.tasks) {  // tolerance-driven laps: per-lap maxima and arrival counts
    T.tol = T.z_planes || P.decomposed ? 0.0 : P.boxes[T.box].d.tol;
    T.tolw_off = -1;
    if (T.tol > 0) {
      T.tolw_off = (int64_t)(off / sizeof(uint64_t));
      off = align_up(off + (size_t)T.laps * 3 * sizeof(uint64_t));
    }
  }
  // decomposed boxes with a tolerance: the box's per-iteration maxima (zeroed by every call)
  for (Box& B : P.boxes) {
    B.btol_off = -1;
    if (P.decomposed && B.d.tol > 0) {
      B.btol_off = (int64_t)(off / sizeof(uint64_t));
      off = align_up(off + (size_t)B.d.n_iter * 2 * sizeof(uint64_t));
    }
  }
  P.max_blocks = 1;
  P.max_cells = 0;
  P.max_iter = 1;
  for (Task& T : P.tasks) {  // blocks along the task's cols, rows and planes
    const rts_desc& d = P.boxes[T.box].d;
    for (int m = 0; m < 3; ++m) T.nblk[m] = P.decomposed ? std::max(1, d.sub[T.frame[m]]) : 1;
    T.btol_off = P.boxes[T.box].btol_off;
    T.iters = d.n_iter;
    if (P.decomposed) T.tol = d.tol;
    P.max_blocks = std::max(P.max_blocks, T.nblk[0] * T.nblk[1] * T.nblk[2]);
    P.max_cells = std::max(P.max_cells, P.boxes[T.box].N);
    P.max_iter = std::max(P.max_iter, (int)d.n_iter);
  }
  P.off_tasks = off;
  off = align_up(off + sizeof(Task) * P.tasks.size());
  P.off_queue = off;
  off = align_up(off + sizeof(int32_t) * P.queue.size());
  P.off_atasks = off;  // (room for two slot-pair passes per task)
  off = align_up(off + 2 * sizeof(AdjTask) * P.tasks.size());
  P.off_rqueue = off;
  off = align_up(off + 2 * 2 * sizeof(int32_t) * P.tasks.size());
  P.off_gsg = off;
  off = align_up(off + sizeof(GsGroup) * P.gsg.size());
  P.off_data = off;
  for (Box& B : P.boxes) {
    const size_t arr = (size_t)B.d.nbands * B.N * esz;
    B.chi_off = (int64_t)(off / esz); off = align_up(off + arr);
    B.chiT_off = (int64_t)(off / esz); off = align_up(off + arr);
    B.sT_off = (int64_t)(off / esz); off = align_up(off + arr);
  }
  for (Task& T : P.tasks) {
    const Box& B = P.boxes[T.box];
    const int64_t bandN = (int64_t)T.band * B.N;
    if (T.transposed) {
      T.chi_off = B.chiT_off + bandN;
      T.s_off = B.sT_off + bandN;
    } else {
      T.chi_off = B.chi_off + bandN;
      T.s_off = bandN;  // into the caller's S
    }
    T.part_off = (int64_t)(off / esz);
    off = align_up(off + (size_t)B.N * esz);
    T.n_cells = B.N;
    T.gbuf_off = -1;
    T.dfield_off = -1;
    if (P.decomposed) {  // D of every slot and cell, two iteration parities
      T.dfield_off = (int64_t)(off / esz);
      off = align_up(off + 2 * (size_t)kMaxRaysPerTask * B.N * esz);
    } else if (T.tol > 0) {  // the previous last plane of the strips' rows, every slot
      T.gbuf_off = (int64_t)(off / esz);
      off = align_up(off + (size_t)T.n_rows * T.n_cols * kMaxRaysPerTask * esz);
    }
    T.flux_off = -1;
    if (B.d.flux) {  // flux partials along cols, rows and, unless uni, the plane axis
      T.flux_off = (int64_t)(off / esz);
      off = align_up(off + (T.uni ? 2 : 3) * (size_t)B.N * esz);
    }
  }
  if (P.gs_iter > 0) {  // scattering state (double): S, J, the group contributions, L, I
    const Box& B = P.boxes[0];
    const size_t arr = (size_t)B.d.nbands * B.N * sizeof(double);
    P.gs_s = (int64_t)(off / 8); off = align_up(off + arr);
    P.gs_j = (int64_t)(off / 8); off = align_up(off + arr);
    P.gs_p = (int64_t)(off / 8); off = align_up(off + P.gsg.size() * arr);
    P.gs_l = (int64_t)(off / 8); off = align_up(off + arr);
    P.gs_i = (int64_t)(off / 8); off = align_up(off + P.gsg.size() * kMaxRaysPerTask * arr);
  }
  P.total = off;

  // adjoint region
  P.atasks.assign(P.tasks.size(), AdjTask{});
  for (size_t t = 0; t < P.tasks.size(); ++t) {
    Task& T = P.tasks[t];
    const size_t pc = (size_t)T.n_rows * T.n_cols;
    T.dstore_off = (int64_t)(off / esz);
    off = align_up(off + (size_t)T.n_unrolled * kMaxRaysPerTask * pc * esz);
  }
  P.off_grads = off;
  // Every task is reversed as two slot-pair passes (slots 0, 2 and 1, 3: the
  // rays of a task are independent in reverse and their gradients only add),
  // each with strips of the reverse launch's rows for its width class.
  const int ntask = (int)P.tasks.size();
  auto rev_cols = [&](const Task& T) {
    return P.sched.single_launch ? P.threads : (T.n_cols + 63) / 64 * 64;
  };
  auto rev_rows = [&](int cols, bool small) {
    // (0 for a width the reverse sweep does not support: refused at the call)
    return std::max(1, P.prec == RTS_FP32 ? reverse_rows<float>(cols, small)
                                          : reverse_rows<double>(cols, small));
  };
  // Per launch width, the tall strips, or the short ones where the tall
  // strips' workgroups would give the 256 CUs fewer than two waves per SIMD
  // (a small grid: its passes' strip chains are the only parallelism).
  constexpr int64_t kRevMinWaves = 2 * 4 * 256;
  std::map<int, int64_t> tall_waves;
  for (const Task& T : P.tasks) {
    const int cols = rev_cols(T), h = rev_rows(cols, false);
    tall_waves[cols] += 2 * (int64_t)((T.n_rows + h - 1) / h) * ((cols + 63) / 64);
  }
  P.rev_small.clear();
  for (const auto& kv : tall_waves) P.rev_small[kv.first] = kv.second < kRevMinWaves;
  for (int t = 0; t < ntask; ++t) {
    const Task& T = P.tasks[t];
    AdjTask& AT = P.atasks[t];
    const int cols = rev_cols(T);
    const int hr = rev_rows(cols, P.rev_small[cols]);
    AT.task = t;
    AT.u_init = T.z_planes ? 0 : -1;
    AT.part = 0;
    AT.strips = (T.n_rows + hr - 1) / hr;
    AT.nparts = 2;
    AdjTask second = AT;
    second.part = 1;
    P.atasks.push_back(second);
  }
  // exchange rings and progress words of every pass (cleared by every call)
  for (AdjTask& AT : P.atasks) {
    const Task& T = P.tasks[AT.task];
    AT.xbuf_off = (int64_t)(off / sizeof(uint64_t));
    off = align_up(off + (size_t)rev_ring_words(AT.strips, T.n_cols, (int)words) * sizeof(uint64_t) +
                   (size_t)AT.strips * sizeof(int32_t));
  }
  P.off_xrev_end = off;
  // gradient partials, one per pass (each pass writes every cell at its first
  // visit, so they are not cleared)
  for (int t = 0; t < ntask; ++t) {
    const Box& B = P.boxes[P.tasks[t].box];
    P.atasks[t].gs_off = (int64_t)(off / esz);
    off = align_up(off + 2 * (size_t)B.N * esz);
    P.atasks[t].gc_off = (int64_t)(off / esz);
    off = align_up(off + 2 * (size_t)B.N * esz);
  }
  for (size_t a = ntask; a < P.atasks.size(); ++a) {  // second passes share the partials
    const AdjTask& first = P.atasks[P.atasks[a].task];
    P.atasks[a].gs_off = first.gs_off;
    P.atasks[a].gc_off = first.gc_off;
  }
  P.off_grads_end = off;
  for (Box& B : P.boxes) {
    const size_t arr = (size_t)B.d.nbands * B.N * esz;
    B.seed_off = (int64_t)(off / esz); off = align_up(off + arr);
    B.seedT_off = (int64_t)(off / esz); off = align_up(off + arr);
  }
  P.total_adj = off;
  for (AdjTask& AT : P.atasks) {
    const Task& T = P.tasks[AT.task];
    const Box& B = P.boxes[T.box];
    AT.seed_off = (T.transposed ? B.seedT_off : B.seed_off) + (int64_t)T.band * B.N;
  }
  // reverse queue: grouped by width (and pass form) as the forward one,
  // longest sweeps first
  auto rwidth = [&](int a) {
    return P.sched.single_launch ? 0 : (P.tasks[P.atasks[a].task].n_cols + 63) / 64 * 64;
  };
  auto rlen = [&](int a) { return P.tasks[P.atasks[a].task].n_unrolled - P.atasks[a].u_init; };
  std::vector<int> rq(P.atasks.size());
  for (size_t i = 0; i < rq.size(); ++i) rq[i] = (int)i;
  std::stable_sort(rq.begin(), rq.end(), [&](int a, int b) {
    if (rwidth(a) != rwidth(b)) return rwidth(a) > rwidth(b);
    return rlen(a) > rlen(b);
  });
  P.rqueue.clear();
  P.rclasses.clear();
  int rticket = 0;
  for (size_t k = 0; k < rq.size(); ++k) {
    const int i = rq[k];
    if (P.rclasses.empty() || P.rclasses.back().width != rwidth(i)) {
      P.rclasses.push_back(Plan::WidthClass{rwidth(i), 64, (int)k, 0, 0, 1, 0, true});
      rticket = 0;
    }
    Plan::WidthClass& c = P.rclasses.back();
    P.rqueue.push_back(rticket);
    P.rqueue.push_back(i);
    rticket += P.atasks[i].strips;
    c.nq += 1;
    c.strips = rticket;
    c.max_strips = std::max(c.max_strips, (int)P.atasks[i].strips);
    c.threads = P.sched.single_launch
                    ? P.threads
                    : std::max(c.threads, (P.tasks[P.atasks[i].task].n_cols + 63) / 64 * 64);
  }
  P.rev_blocks = 0;
  if (P.gexec) (void)hipGraphExecDestroy(P.gexec);
  if (P.graph) (void)hipGraphDestroy(P.graph);
  P.gexec = nullptr;
  P.graph = nullptr;
  for (auto& n : P.ev_nodes) n = nullptr;
}

int dev_init(Plan& P) {
  int dev = 0;
  RTS_HIP(hipGetDevice(&dev));
  if (P.dev_ready && dev == P.device) return RTS_OK;
  hipDeviceProp_t prop;
  RTS_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_last_hip = std::string("device is ") + prop.gcnArchName + ", library built for gfx950";
    return RTS_E_NOT_BUILT;
  }
  P.device = dev;
  P.cus = prop.multiProcessorCount;
  P.arch = prop.gcnArchName;
  int clk_khz = 0;
  if (hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      clk_khz <= 0)
    clk_khz = 100000;
  P.timeout_ticks = (int64_t)clk_khz * 1000 * 5;  // 5 s
  P.dev_ready = true;
  return RTS_OK;
}

// Workgroups of `fn` that can be resident on one CU: the runtime's estimate,
// capped by how a workgroup's waves are placed: each of the CU's four SIMDs
// must take ceil(waves / 4) of them, and a SIMD holds 512 / VGPRs waves (a
// five-wave workgroup with 128 VGPRs therefore fits twice, not three times).
int resident_blocks(const void* fn, int threads, size_t lds, int* out) {
  int nb = 0;
  RTS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, lds));
  hipFuncAttributes fa;
  RTS_HIP(hipFuncGetAttributes(&fa, fn));
  const int vgpr = std::max(8, (fa.numRegs + 7) / 8 * 8);
  const int per_simd = std::min(8, 512 / vgpr);
  const int need = ((threads + 63) / 64 + 3) / 4;
  *out = std::min(nb, per_simd / need);
  return RTS_OK;
}

template <class Real, int H>
int occupancy_h(Plan& P) {
  // per launch, the smallest residency of the plain and the extended sweeps
  // (flux partials, tolerance laps: more registers and a little static LDS)
  P.occupancy_blocks = 1 << 30;
  for (Plan::WidthClass& c : P.wclasses) {
    const void* fns[3] = {c.uni ? sweep_fn<Real, H, true>() : sweep_fn<Real, H, false>(),
                          c.uni ? sweep_fn_ext<Real, H, true>(1) : sweep_fn_ext<Real, H, false>(1),
                          c.uni ? sweep_fn_ext<Real, H, true>(2) : sweep_fn_ext<Real, H, false>(2)};
    c.blocks = 1 << 30;
    for (const void* f : fns) {
      int nb = 0;
      int rc = resident_blocks(f, c.threads, sweep_lds_bytes<Real, H>(c.threads), &nb);
      if (rc) return rc;
      c.blocks = std::min(c.blocks, nb);
    }
    P.occupancy_blocks = std::min(P.occupancy_blocks, c.blocks);
  }
  P.rev_blocks = 1 << 30;
  for (Plan::WidthClass& c : P.rclasses) {
    const bool small = P.rev_small.count(c.threads) && P.rev_small.at(c.threads);
    const void* fn = reverse_fn<Real>(c.threads, small);
    if (!fn) {  // (wider than the reverse sweep supports: no resident block)
      c.blocks = 0;
      continue;
    }
    int rc = resident_blocks(fn, c.threads, reverse_lds_bytes<Real>(c.threads, small), &c.blocks);
    if (rc) return rc;
    P.rev_blocks = std::min(P.rev_blocks, c.blocks);
  }
  return RTS_OK;
}

template <class Real>
int occupancy(Plan& P) {
  switch (P.sched.rows_per_strip) {
    case 2: return occupancy_h<Real, 2>(P);
    case 4: return occupancy_h<Real, 4>(P);
    case 6: if (sizeof(Real) == 4) return occupancy_h<float, 6>(P); break;
    case 8: if (sizeof(Real) == 4) return occupancy_h<float, 8>(P); break;
  }
  return RTS_E_UNSUPPORTED;
}

template <class Real, bool UNI>
hipError_t launch_sweep_u(Plan& P, const SweepArgs& a, int grid, int threads, hipStream_t st) {
  switch (P.sched.rows_per_strip) {
    case 2: return launch_sweep_h<Real, 2, UNI>(a, grid, threads, st);
    case 4: return launch_sweep_h<Real, 4, UNI>(a, grid, threads, st);
    case 6: if (sizeof(Real) == 4) return launch_sweep_h<float, 6, UNI>(a, grid, threads, st); break;
    case 8: if (sizeof(Real) == 4) return launch_sweep_h<float, 8, UNI>(a, grid, threads, st); break;
  }
  return hipErrorInvalidValue;
}

template <class Real>
hipError_t launch_sweep(Plan& P, const Plan::WidthClass& c, const SweepArgs& a, int grid,
                        hipStream_t st) {
  return c.uni ? launch_sweep_u<Real, true>(P, a, grid, c.threads, st)
               : launch_sweep_u<Real, false>(P, a, grid, c.threads, st);
}

int ensure_pinned(Plan& P) {
  const size_t bytes = (P.off_data - P.off_tasks);
  if (P.pinned && P.pinned_bytes >= bytes) return RTS_OK;
  if (P.pinned) P.old_pinned.push_back(P.pinned);
  P.pinned = nullptr;
  RTS_HIP(hipHostMalloc(&P.pinned, bytes, hipHostMallocDefault));
  P.pinned_bytes = bytes;
  std::memset(P.pinned, 0, bytes);
  std::memcpy(P.pinned, P.tasks.data(), sizeof(Task) * P.tasks.size());
  std::memcpy((char*)P.pinned + (P.off_queue - P.off_tasks), P.queue.data(),
              sizeof(int32_t) * P.queue.size());
  std::memcpy((char*)P.pinned + (P.off_atasks - P.off_tasks), P.atasks.data(),
              sizeof(AdjTask) * P.atasks.size());
  std::memcpy((char*)P.pinned + (P.off_rqueue - P.off_tasks), P.rqueue.data(),
              sizeof(int32_t) * P.rqueue.size());
  if (!P.gsg.empty())
    std::memcpy((char*)P.pinned + (P.off_gsg - P.off_tasks), P.gsg.data(),
                sizeof(GsGroup) * P.gsg.size());
  return RTS_OK;
}

hipError_t upload_tables(const Plan& P, char* ws, hipStream_t st) {
  return hipMemcpyAsync(ws + P.off_tasks, P.pinned, P.off_data - P.off_tasks,
                        hipMemcpyHostToDevice, st);
}

// Enqueue one forward solve of all boxes of the plan.
BoxGeo box_geo(const Plan& P, size_t b) {
  const Box& B = P.boxes[b];
  BoxGeo G;
  std::memset(&G, 0, sizeof(G));
  G.nx = B.d.g.nx; G.ny = B.d.g.ny; G.nz = B.d.g.nz; G.nbands = B.d.nbands;
  G.n_up = B.n_up;
  G.tasks_per_band = B.tasks_per_band;
  for (size_t t = 0; t < P.tasks.size(); ++t)
    if (P.tasks[t].box == (int)b) { G.task0 = (int)t; break; }
  for (int k = 0; k < B.d.nbands; ++k) G.qweight[k] = B.qw[k];
  for (int r = 0; r < B.d.nrays; ++r)
    for (int m = 0; m < 3; ++m) G.msum[m] += B.w[r] * B.mu[3 * r + m];
  G.dx = B.d.g.dx; G.dy = B.d.g.dy; G.dz = B.d.g.dz;
  G.chi_off = B.chi_off;
  G.chiT_off = B.chiT_off;
  G.sT_off = B.sT_off;
  // sum_r w_r - 1, compensated (Neumaier), so that weights summing to 1 give
  // an exact 0 whenever their rounded sum is exact
  double s = 0.0, comp = 0.0;
  for (int r = 0; r < B.d.nrays; ++r) {
    const double t = s + B.w[r];
    comp += std::fabs(s) >= std::fabs(B.w[r]) ? (s - t) + B.w[r] : (B.w[r] - t) + s;
    s = t;
  }
  G.wsum1 = (s - 1.0) + comp;
  return G;
}

// With out == nullptr (the forward pass of the adjoint) the sweep also stores
// D of every plane, writes no I_top and the reduce is skipped; with store the
// sweep stores D as well as writing the outputs (rts_solve_for_adjoint).
// Marks 1 and 2 bracket the sweep launches: an eager timed call records its
// events there, a timed graph capture cuts its segments there.
struct Marks {
  hipEvent_t* ev = nullptr;          // eager: events [4], marks record ev[1], ev[2]
  hipStream_t cap = nullptr;         // capture: the capturing stream
  std::vector<hipGraph_t>* segs = nullptr;  // capture: the segments ended so far
  int mark(int i, hipStream_t st) const {
    if (ev) {
      RTS_HIP(hipEventRecord(ev[i], st));
      return RTS_OK;
    }
    if (!segs) return RTS_OK;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &g);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    segs->push_back(g);
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    return RTS_OK;
  }
};

// Scattering with Gauss-Seidel source updates (rts_gs.hip): the state
// initialisation, then per iteration and ray group its ghost plane and one
// launch per plane of each lap, then Q, J and S.  The marks bracket the
// iterations.
int enqueue_gs(Plan& P, const rts_inputs* in, const rts_outputs* out, char* ws, hipStream_t st,
               const Marks* mk) {
  const Box& B = P.boxes[0];
  GsArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ws = ws;
  a.groups = reinterpret_cast<const GsGroup*>(ws + P.off_gsg);
  a.ngroups = (int)P.gsg.size();
  a.nbands = B.d.nbands;
  a.nx = B.d.g.nx; a.ny = B.d.g.ny; a.nz = B.d.g.nz;
  a.bot = B.d.bot; a.top = B.d.top; a.ibot = B.d.i_bot;
  a.N = B.N;
  a.chi_off = B.chi_off;
  a.s_off = P.gs_s; a.j_off = P.gs_j; a.p_off = P.gs_p; a.l_off = P.gs_l; a.i_off = P.gs_i;
  a.chit_off = B.chiT_off; a.st_off = B.sT_off;
  a.B = reinterpret_cast<const double*>(in[0].S);
  a.eps = reinterpret_cast<const double*>(in[0].eps);
  for (int k = 0; k < B.d.nbands; ++k) a.qw[k] = B.qw[k];
  a.Q = out[0].Q;
  a.J = reinterpret_cast<double*>(out[0].J);
  a.I_top = reinterpret_cast<double*>(out[0].I_top);
  a.S = reinterpret_cast<double*>(out[0].S);
  RTS_HIP(launch_gs_init(a, st));
  int mrc = RTS_OK;
  if (mk && (mrc = mk->mark(1, st))) return mrc;
  const int n[3] = {a.nx, a.ny, a.nz};
  const int G = a.ngroups;
  // per iteration: the ghost planes; every group's laps with the iteration's S
  // (all but the last group's last lap), one launch per step over the groups;
  // then the last group's last lap, plane by plane, updating S
  int steps = 0, pcmax = 0;
  for (int g = 0; g < G; ++g) {
    const GsGroup& gg = P.gsg[g];
    steps = std::max(steps, (g == G - 1 ? gg.laps - 1 : gg.laps) * n[gg.axis]);
    pcmax = std::max(pcmax, n[gg.ea] * n[gg.eb]);
  }
  const GsGroup& gl = P.gsg[G - 1];
  const int nal = n[gl.axis], pcl = n[gl.ea] * n[gl.eb];
  for (int it = 0; it < P.gs_iter; ++it) {
    const int top = it == P.gs_iter - 1 ? 1 : 0;
    // the [x][z][y] copy of the iteration's S for the x-dominant groups (and chi
    // again, the same values)
    if (it > 0)
      RTS_HIP(launch_prep<double>(in[0].kappa, in[0].rho, ws + P.gs_s * sizeof(double), ws,
                                  B.chi_off, B.chiT_off, B.sT_off, a.nx, a.ny, a.nz, a.nbands, st));
    for (int g = 0; g < G; ++g) {
      const GsGroup& gg = P.gsg[g];
      if (gg.axis != 2) RTS_HIP(launch_gs_ghost(a, g, n[gg.ea] * n[gg.eb], st));
    }
    for (int t = 0; t < steps; ++t) RTS_HIP(launch_gs_step(a, t, top, pcmax, st));
    for (int t = 0; t < nal; ++t) {
      const int q = gl.sa > 0 ? t : nal - 1 - t;
      RTS_HIP(launch_gs_plane(a, G - 1, q, 1, 1, top, pcl, st));
    }
  }
  if (mk && (mrc = mk->mark(2, st))) return mrc;
  RTS_HIP(launch_gs_finish(a, st));
  return RTS_OK;
}

template <class Real>
int enqueue_forward(Plan& P, const rts_inputs* in, const rts_outputs* out, char* ws,
                    hipStream_t st, const Marks* mk, bool store = false) {
  int mrc = RTS_OK;
  // header and exchange buffers to zero
  RTS_HIP(launch_zero(reinterpret_cast<int*>(ws),
                      (int64_t)((P.off_tasks) / sizeof(int32_t)), st));
  // The task table and queues go up with every call: the same workspace
  // address does not mean the same device bytes (a caller's allocator may have
  // handed the block to other work in between).  They are tens of KB.
  RTS_HIP(upload_tables(P, ws, st));
  for (size_t b = 0; b < P.boxes.size(); ++b) {
    const Box& B = P.boxes[b];
    RTS_HIP(launch_prep<Real>(in[b].kappa, in[b].rho, in[b].S, ws, B.chi_off, B.chiT_off,
                              B.sT_off, B.d.g.nx, B.d.g.ny, B.d.g.nz, B.d.nbands, st));
  }
  if (P.gs_iter > 0) {
    if (!out || store || sizeof(Real) != 8) return RTS_E_UNSUPPORTED;
    return enqueue_gs(P, in, out, ws, st, mk);
  }
  if (P.decomposed) {
    // subdomains with lagged exchange: iteration 0's field, then one launch
    // per iteration (the launch boundary is the exchange), then the reduce
    if (!out || store) return RTS_E_UNSUPPORTED;
    BlockArgs b;
    std::memset(&b, 0, sizeof(b));
    b.ws = ws;
    b.tasks = reinterpret_cast<const Task*>(ws + P.off_tasks);
    b.ntasks = (int)P.tasks.size();
    for (size_t i = 0; i < P.boxes.size(); ++i)
      b.box[i] = BoxPtrs{in[i].kappa, in[i].rho, in[i].S, out[i].Q, out[i].J, out[i].I_top,
                         nullptr, nullptr, nullptr, nullptr};
    RTS_HIP(launch_block_init<Real>(b, P.max_cells, st));
    if (mk && (mrc = mk->mark(1, st))) return mrc;
    // one workgroup of 1024 threads per (block, task): the cells of a block's
    // plane are spread over 16 waves (measured against 256 and 512 threads:
    // faster for 2x2x2 to 8x8x4 blocks of a 288^3 box, 3x for the fewest blocks)
    const int bthreads = 1024;
    for (int it = 0; it < P.max_iter; ++it) {
      b.iter = it;
      RTS_HIP(launch_block_sweep<Real>(b, P.max_blocks, bthreads, st));
    }
    if (mk && (mrc = mk->mark(2, st))) return mrc;
    for (size_t i = 0; i < P.boxes.size(); ++i)
      RTS_HIP(launch_reduce<Real>(ws, b.tasks, box_geo(P, i), b.box[i], st));
    return RTS_OK;
  }
  SweepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ws = ws;
  a.tasks = reinterpret_cast<const Task*>(ws + P.off_tasks);
  a.timeout_ticks = P.timeout_ticks;
  bool warm = false;
  for (size_t b = 0; b < P.boxes.size(); ++b) {
    a.box[b] = out ? BoxPtrs{in[b].kappa, in[b].rho, in[b].S, out[b].Q, out[b].J, out[b].I_top,
                             out[b].F, out[b].QF, in[b].ghost, out[b].ghost}
                   : BoxPtrs{in[b].kappa, in[b].rho, in[b].S, nullptr, nullptr, nullptr, nullptr,
                             nullptr, nullptr, nullptr};
    warm = warm || a.box[b].gin || a.box[b].gout;
  }
  a.store_d = out && !store ? 0 : 1;
  a.flux = 0;
  if (out)
    for (size_t b = 0; b < P.boxes.size(); ++b) a.flux |= out[b].F != nullptr;
  a.ext = a.flux ? 1 : 0;
  for (const Task& T : P.tasks)
    if (T.tol > 0) a.ext = 2;
  if (warm) a.ext = 2;  // (the warm start lives in the extended sweep)
  // One persistent launch per workgroup width, in stream order.  Every strip
  // of a task must be resident together (neighbouring strips wait on each
  // other), so a launch's grid never drops below its largest task's strip
  // count; tickets are claimed in order, hence with that many resident
  // workgroups the tasks being worked on always make progress.
  if (P.wclasses.size() > (size_t)kMaxWidths) return RTS_E_UNSUPPORTED;  // (widths <= kMaxCols)
  if (mk && (mrc = mk->mark(1, st))) return mrc;
  for (size_t k = 0; k < P.wclasses.size(); ++k) {
    const Plan::WidthClass& c = P.wclasses[k];
    a.queue = reinterpret_cast<const int32_t*>(ws + P.off_queue) + 2 * c.q0;
    a.ntasks = c.nq;
    a.total_strips = c.strips;
    a.wclass = (int)k;
    int grid = c.blocks * P.cus;
    if (P.sched.max_workgroups > 0)
      grid = std::min(grid, std::max((int)P.sched.max_workgroups, c.max_strips));
    grid = std::max(1, std::min(grid, c.strips));
    RTS_HIP(launch_sweep<Real>(P, c, a, grid, st));
  }
  if (mk && (mrc = mk->mark(2, st))) return mrc;
  if (!out) return RTS_OK;
  for (size_t b = 0; b < P.boxes.size(); ++b) {
    const BoxGeo G = box_geo(P, b);
    // J, Q and, with F requested, the flux vector and its divergence
    RTS_HIP(launch_reduce<Real>(ws, reinterpret_cast<const Task*>(ws + P.off_tasks), G,
                                a.box[b], st));
  }
  return RTS_OK;
}

// Enqueue one adjoint: the forward sweep storing D, the seeds, one reverse
// launch per workgroup width (every task of every box), the gradient reduce.
// Without run_forward the stored D of an earlier rts_solve_for_adjoint on this
// workspace is used; only the header (reverse ticket, status) is cleared.
template <class Real>
int enqueue_adjoint(Plan& P, const rts_inputs* in, const rts_seeds* g, const rts_grads* d,
                    char* ws, hipStream_t st, bool run_forward = true) {
  if (run_forward) {
    int rc = enqueue_forward<Real>(P, in, nullptr, ws, st, nullptr);
    if (rc) return rc;
  } else {
    RTS_HIP(launch_zero(reinterpret_cast<int*>(ws), (int64_t)(sizeof(WsHeader) / sizeof(int32_t)), st));
    RTS_HIP(upload_tables(P, ws, st));
  }
  RTS_HIP(launch_zero(reinterpret_cast<int*>(ws + P.off_grads),
                      (int64_t)((P.off_xrev_end - P.off_grads) / sizeof(int32_t)), st));
  for (size_t b = 0; b < P.boxes.size(); ++b) {
    const Box& B = P.boxes[b];
    Real* base = reinterpret_cast<Real*>(ws);
    for (int k = 0; k < B.d.nbands; ++k) {
      const int64_t o = (int64_t)k * B.N;
      const double qf = 4.0 * 3.14159265358979323846 * B.qw[k];
      const Real* kap = reinterpret_cast<const Real*>(in[b].kappa) + o;
      const Real* gJ = g[b].gJ ? reinterpret_cast<const Real*>(g[b].gJ) + o : nullptr;
      RTS_HIP(launch_adj_seed<Real>(kap, in[b].rho, g[b].gQ, gJ, base + B.seed_off + o,
                                    base + B.seedT_off + o, qf, B.d.g.nx, B.d.g.ny, B.d.g.nz, st));
    }
  }
  RevArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ws = ws;
  a.tasks = reinterpret_cast<const Task*>(ws + P.off_tasks);
  a.atasks = reinterpret_cast<const AdjTask*>(ws + P.off_atasks);
  a.timeout_ticks = P.timeout_ticks;
  for (size_t b = 0; b < P.boxes.size(); ++b) {
    a.gItop[b] = g[b].gItop;
    a.S[b] = in[b].S;
  }
  // one persistent reverse launch per width, in stream order
  if (P.rclasses.size() > (size_t)kMaxWidths) return RTS_E_UNSUPPORTED;
  for (size_t k = 0; k < P.rclasses.size(); ++k) {
    const Plan::WidthClass& c = P.rclasses[k];
    a.queue = reinterpret_cast<const int32_t*>(ws + P.off_rqueue) + 2 * c.q0;
    a.ntasks = c.nq;
    a.total_strips = c.strips;
    a.wclass = (int)k;
    const int grid = std::max(1, std::min(c.blocks * P.cus, c.strips));
    const bool small = P.rev_small.count(c.threads) && P.rev_small.at(c.threads);
    RTS_HIP(launch_reverse<Real>(a, grid, c.threads, small, st));
  }
  for (size_t b = 0; b < P.boxes.size(); ++b) {
    const BoxGeo G = box_geo(P, b);
    RTS_HIP(launch_adj_reduce<Real>(ws, a.tasks, a.atasks, G, g[b].gQ, g[b].gJ, g[b].gItop,
                                    in[b].S, d[b].dS, d[b].dchi, st));
  }
  return RTS_OK;
}

int check_call(Plan* P, int nbox, const rts_inputs* in, const rts_outputs* out, void* ws,
               size_t ws_bytes) {
  if (!P || !in || !out) return RTS_E_ARG;
  if (nbox != (int)P->boxes.size()) return RTS_E_ARG;
  for (int b = 0; b < nbox; ++b) {
    if (!in[b].kappa || !in[b].rho || !in[b].S || !out[b].Q) return RTS_E_ARG;
    // the flux vector needs the plan's flux partials; its divergence needs F
    if (out[b].F && !P->boxes[b].d.flux) return RTS_E_ARG;
    if (out[b].QF && !out[b].F) return RTS_E_ARG;
    if (P->gs_iter > 0 && !in[b].eps) return RTS_E_ARG;
    if ((in[b].ghost || out[b].ghost) && (P->decomposed || P->gs_iter > 0)) {
      g_last_hip = "ghost planes (warm start) need an undivided plan without scattering";
      return RTS_E_UNSUPPORTED;
    }
  }
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < P->total)
    return RTS_E_WORKSPACE;
  return RTS_OK;
}

// Device state a call needs: the device check, occupancy and the pinned task
// table.  Without may_alloc a missing table is an error, not an allocation.
int prepare(Plan* P, bool may_alloc = true) {
  int rc = dev_init(*P);
  if (rc) return rc;
  if (P->occupancy_blocks == 0) {
    rc = P->prec == RTS_FP32 ? occupancy<float>(*P) : occupancy<double>(*P);
    if (rc) return rc;
    for (const Plan::WidthClass& c : P->wclasses)
      // (decomposed and scattering plans have no co-resident strips: their
      // workgroups never wait)
      if (!P->decomposed && P->gs_iter == 0 && (c.blocks < 1 || c.blocks * P->cus < c.max_strips)) {
        P->occupancy_blocks = 0;
        g_last_hip = "the strips of one sweep task cannot all be resident; use more rows per strip";
        return RTS_E_UNSUPPORTED;
      }
  }
  if (!may_alloc && (!P->pinned || P->pinned_bytes < (P->off_data - P->off_tasks))) {
    g_last_hip = "the plan has no pinned task table (it was created with no GPU visible)";
    return RTS_E_UNSUPPORTED;
  }
  return ensure_pinned(*P);
}

// The pinned task table, allocated when the plan is made or rescheduled if a
// GPU is visible, so that a call of the allocation-free entry point finds it.
void pin_early(Plan* P) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return;
  }
  (void)ensure_pinned(*P);
}

// One set of timing events (call start, sweep start, sweep end, call end) for
// the next timed call, or nullptr once kMaxTimed calls are recorded.
int next_events(Plan* P, hipEvent_t** out) {
  *out = nullptr;
  if (!P->timing || P->ev_used >= kMaxTimed) return RTS_OK;
  if ((int)P->ev.size() <= P->ev_used) {
    std::array<hipEvent_t, 4> e{};
    for (int i = 0; i < 4; ++i) RTS_HIP(hipEventCreate(&e[i]));
    P->ev.push_back(e);
  }
  *out = P->ev[P->ev_used].data();
  return RTS_OK;
}

void drop_graph(Plan* P) {
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->gexec = nullptr;
  P->graph = nullptr;
  for (auto& n : P->ev_nodes) n = nullptr;
}

int solve_impl(Plan* P, int nbox, const rts_inputs* in, const rts_outputs* out, void* ws,
               size_t ws_bytes, void* stream, bool allow_graph) {
  int rc = check_call(P, nbox, in, out, ws, ws_bytes);
  if (rc) return rc;
  if ((rc = prepare(P))) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const bool graph = allow_graph && P->sched.use_graph;
  hipEvent_t* ev = nullptr;
  if ((rc = next_events(P, &ev))) return rc;
  if (!graph) {
    Marks mk;
    mk.ev = ev;
    if (ev) RTS_HIP(hipEventRecord(ev[0], st));
    rc = P->prec == RTS_FP32 ? enqueue_forward<float>(*P, in, out, (char*)ws, st, ev ? &mk : nullptr)
                             : enqueue_forward<double>(*P, in, out, (char*)ws, st, ev ? &mk : nullptr);
    if (rc) return rc;
    if (ev) {
      RTS_HIP(hipEventRecord(ev[3], st));
      ++P->ev_used;
    }
    return RTS_OK;
  }
  // graph path: key on every pointer the captured work uses, and on timing
  // (a timed graph holds event-record nodes around the call and the sweeps)
  const bool timed = ev != nullptr;
  std::vector<const void*> key{ws, reinterpret_cast<const void*>(uintptr_t(timed ? 1 : 0))};
  for (int b = 0; b < nbox; ++b) {
    key.insert(key.end(), {in[b].kappa, in[b].rho, in[b].S, in[b].eps, in[b].ghost, out[b].Q,
                           out[b].J, out[b].I_top, out[b].F, out[b].QF, out[b].S, out[b].ghost});
  }
  if (!P->gexec || key != P->gkey) {
    drop_graph(P);
    if (!P->cap_stream) RTS_HIP(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    if (timed && !P->cap_ev[0])
      for (auto& e : P->cap_ev) RTS_HIP(hipEventCreate(&e));
    // A timed graph is captured in three segments (before, during and after
    // the sweep launches) and assembled as child graphs between explicit
    // event-record nodes; an untimed graph is one capture.
    std::vector<hipGraph_t> segs;
    Marks mk;
    mk.cap = P->cap_stream;
    mk.segs = &segs;
    auto drop_segs = [&]() {
      for (hipGraph_t x : segs) (void)hipGraphDestroy(x);
      segs.clear();
    };
    RTS_HIP(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = P->prec == RTS_FP32
             ? enqueue_forward<float>(*P, in, out, (char*)ws, P->cap_stream, timed ? &mk : nullptr)
             : enqueue_forward<double>(*P, in, out, (char*)ws, P->cap_stream, timed ? &mk : nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(P->cap_stream, &g);
    if (rc || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      drop_segs();
      return rc ? rc : hip_fail(e, "hipStreamEndCapture");
    }
    if (timed) {
      segs.push_back(g);
      g = nullptr;
      if (segs.size() != 3) {
        drop_segs();
        g_last_hip = "timed graph capture: expected three segments";
        return RTS_E_HIP;
      }
      e = hipGraphCreate(&g, 0);
      hipGraphNode_t prev = nullptr;
      for (int i = 0; i < 4 && e == hipSuccess; ++i) {
        hipGraphNode_t n = nullptr;
        e = hipGraphAddEventRecordNode(&n, g, prev ? &prev : nullptr, prev ? 1 : 0, P->cap_ev[i]);
        if (e != hipSuccess) break;
        P->ev_nodes[i] = n;
        prev = n;
        if (i < 3) {  // (the child node holds its own copy of the segment)
          e = hipGraphAddChildGraphNode(&n, g, &prev, 1, segs[i]);
          prev = n;
        }
      }
      drop_segs();
      if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        for (auto& x : P->ev_nodes) x = nullptr;
        return hip_fail(e, "timed graph assembly");
      }
    }
    e = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      for (auto& x : P->ev_nodes) x = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    P->graph = g;  // kept: its nodes address the exec's event-record nodes
    P->gkey = key;
  }
  if (timed) {
    for (int i = 0; i < 4; ++i)
      RTS_HIP(hipGraphExecEventRecordNodeSetEvent(P->gexec, P->ev_nodes[i], ev[i]));
  }
  RTS_HIP(hipGraphLaunch(P->gexec, st));
  if (timed) ++P->ev_used;
  return RTS_OK;
}

}  // namespace

namespace rts {
// The allocation-free forward solve behind rts_solve_static (rts_static.hip):
// the argument checks against a workspace of `cap` bytes, then the eager path
// on `ws` (no graph, no timing events, no staging allocation).
int static_solve_check(void* plan, int nbox, const rts_inputs* in, const rts_outputs* out,
                       size_t cap) {
  if (!plan) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  if (!in || !out || nbox != (int)P->boxes.size()) return RTS_E_ARG;
  if (P->total > cap) return RTS_E_WORKSPACE;
  return RTS_OK;
}

int static_solve(void* plan, int nbox, const rts_inputs* in, const rts_outputs* out, void* ws,
                 size_t cap, void* stream) {
  Plan* P = static_cast<Plan*>(plan);
  try {
    int rc = check_call(P, nbox, in, out, ws, cap);
    if (rc) return rc;
    if ((rc = prepare(P, false))) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    return P->prec == RTS_FP32 ? enqueue_forward<float>(*P, in, out, (char*)ws, st, nullptr)
                               : enqueue_forward<double>(*P, in, out, (char*)ws, st, nullptr);
  } catch (...) {
    return RTS_E_HIP;
  }
}

int static_fail(hipError_t e, const char* where) { return hip_fail(e, where); }
int static_scratch(void** out);  // rts_static.hip
}  // namespace rts

namespace {

// Schedules the autotuner tries: every strip height of the precision, both
// queue orders and, when the sweep planes have more than one padded width,
// both launch forms (one launch per width, one at the widest).
std::vector<rts_schedule> tune_candidates(const Plan& P) {
  std::vector<rts_schedule> c;
  const int hs32[] = {2, 4, 6, 8}, hs64[] = {2, 4};
  const int* hs = P.prec == RTS_FP32 ? hs32 : hs64;
  const int nh = P.prec == RTS_FP32 ? 4 : 2;
  bool mixed = false;
  for (const Task& T : P.tasks)
    mixed = mixed || (T.n_cols + 63) / 64 != (P.tasks[0].n_cols + 63) / 64;
  const int sl0 = mixed ? 0 : P.sched.single_launch, sl1 = mixed ? 1 : P.sched.single_launch;
  for (int sl = sl0; sl <= sl1; ++sl)
    for (int i = 0; i < nh; ++i)
      for (int order = 0; order < 2; ++order)
        c.push_back(rts_schedule{hs[i], 0, order, P.sched.use_graph, sl, P.sched.split_reverse});
  return c;
}

// The problem part of a tuning key: precision and, per box, grid, bands,
// tasks, sweeps and ray grouping.
std::string tune_problem(const Plan& P) {
  std::string k = std::to_string(P.prec);
  for (const Box& B : P.boxes) {
    k += "|" + std::to_string(B.d.g.nx) + "x" + std::to_string(B.d.g.ny) + "x" +
         std::to_string(B.d.g.nz) + "b" + std::to_string(B.d.nbands) + "t" +
         std::to_string(B.tasks_per_band) + "i" + std::to_string(B.d.n_iter);
    for (const auto& g : B.groups)
      for (int r : g) k += "," + std::to_string(r);
  }
  return k;
}

// The process-wide cache of tuned schedules (plans of several threads share
// it), keyed by device index and problem.
std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}
std::map<std::string, rts_schedule>& tune_cache() {
  static std::map<std::string, rts_schedule> m;
  return m;
}

// The persisted cache: a text file named by the environment variable
// RTS_TUNE_CACHE, one line per tuning run,
//   <arch>/<compute units>/<problem> <rows_per_strip> <order> <single_launch>
// (the key has no blanks).  When the variable is set the file is the cache:
// it is read on every tuning call (the last valid line of a key wins) and
// each new choice is appended.  Lines that do not parse, or whose schedule is
// not a candidate of the plan, are ignored.
const char* tune_file() {
  const char* f = std::getenv("RTS_TUNE_CACHE");
  return (f && *f) ? f : nullptr;
}
std::string tune_file_key(const Plan& P) {
  std::string a = P.arch;
  for (char& c : a)
    if (c == ' ' || c == '\t' || c == '\n') c = '_';
  return a + "/" + std::to_string(P.cus) + "/" + tune_problem(P);
}

bool same_choice(const rts_schedule& a, const rts_schedule& b) {
  return a.rows_per_strip == b.rows_per_strip && a.order == b.order &&
         a.single_launch == b.single_launch;
}

bool tune_lookup(const Plan& P, rts_schedule* s) {
  std::lock_guard<std::mutex> lk(tune_mutex());
  if (const char* path = tune_file()) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    const std::string want = tune_file_key(P);
    const std::vector<rts_schedule> cands = tune_candidates(P);
    bool found = false;
    std::vector<char> line(1 << 16);
    while (std::fgets(line.data(), (int)line.size(), f)) {
      const char* sp = std::strchr(line.data(), ' ');
      if (!sp || (size_t)(sp - line.data()) != want.size() ||
          std::strncmp(line.data(), want.data(), want.size()) != 0)
        continue;
      int h = 0, order = 0, sl = 0;
      if (std::sscanf(sp, " %d %d %d", &h, &order, &sl) != 3) continue;
      for (const rts_schedule& c : cands)
        if (same_choice(c, rts_schedule{h, 0, order, 0, sl, 0})) {
          *s = c;
          found = true;
        }
    }
    std::fclose(f);
    return found;
  }
  auto hit = tune_cache().find(std::to_string(P.device) + "/" + tune_problem(P));
  if (hit == tune_cache().end()) return false;
  *s = hit->second;
  return true;
}

void tune_store(const Plan& P, const rts_schedule& s) {
  std::lock_guard<std::mutex> lk(tune_mutex());
  tune_cache()[std::to_string(P.device) + "/" + tune_problem(P)] = s;
  if (const char* path = tune_file()) {
    if (FILE* f = std::fopen(path, "a")) {
      std::fprintf(f, "%s %d %d %d\n", tune_file_key(P).c_str(), s.rows_per_strip, s.order,
                   s.single_launch);
      std::fclose(f);
    }
  }
}

void set_sched(Plan* P, const rts_schedule& s) {
  P->sched = s;
  P->occupancy_blocks = 0;
  if (P->pinned) {
    P->old_pinned.push_back(P->pinned);
    P->pinned = nullptr;
    P->pinned_bytes = 0;
  }
  build_layout(*P);
  pin_early(P);
}

// Time every candidate schedule on the caller's data (HIP events, `reps`
// timed calls after one warm-up call each) and keep the fastest.  Results
// are cached per process by problem shape and device.
int autotune_impl(Plan* P, int nbox, const rts_inputs* in, const rts_outputs* out, void* ws,
                  size_t ws_bytes, hipStream_t st, int reps, int* tried) {
  int rc = check_call(P, nbox, in, out, ws, SIZE_MAX);  // the size is checked per candidate
  if (rc) return rc;
  if ((rc = dev_init(*P))) return rc;
  *tried = 0;
  // a decomposed or scattering plan has no strip schedule to choose: its
  // launches do not depend on it
  if (P->decomposed || P->gs_iter > 0) return RTS_OK;
  rts_schedule cached;
  if (tune_lookup(*P, &cached)) {
    set_sched(P, cached);
    return RTS_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  RTS_HIP(hipEventCreate(&e0));
  RTS_HIP(hipEventCreate(&e1));
  const rts_schedule orig = P->sched;
  rts_schedule best = orig;
  float best_ms = INFINITY;
  int status = RTS_OK;
  for (const rts_schedule& c : tune_candidates(*P)) {
    set_sched(P, c);
    if (P->total > ws_bytes) continue;
    rc = prepare(P);
    if (rc == RTS_E_UNSUPPORTED) continue;
    if (rc) { status = rc; break; }
    auto run = [&]() {
      return P->prec == RTS_FP32 ? enqueue_forward<float>(*P, in, out, (char*)ws, st, nullptr)
                                 : enqueue_forward<double>(*P, in, out, (char*)ws, st, nullptr);
    };
    if ((rc = run())) { status = rc; break; }
    if (hipEventRecord(e0, st) != hipSuccess) { status = RTS_E_HIP; break; }
    for (int i = 0; i < reps && !rc; ++i) rc = run();
    if (rc) { status = rc; break; }
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      status = RTS_E_HIP;
      break;
    }
    int32_t dev_status = 0;
    if (hipMemcpy(&dev_status, ws, sizeof(dev_status), hipMemcpyDeviceToHost) != hipSuccess) {
      status = RTS_E_HIP;
      break;
    }
    if (dev_status) { status = RTS_E_DEADLOCK; break; }
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { status = RTS_E_HIP; break; }
    ms /= reps;
    ++*tried;
    if (ms < best_ms) { best_ms = ms; best = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status == RTS_OK && *tried == 0) status = RTS_E_WORKSPACE;
  set_sched(P, status == RTS_OK ? best : orig);
  if (status == RTS_OK) tune_store(*P, best);
  return status;
}

}  // namespace

extern "C" {

int rts_plan_create(const rts_desc* descs, int32_t nbox, void** out) {
  if (!out) return RTS_E_ARG;
  *out = nullptr;
  if (!descs || nbox < 1) return RTS_E_ARG;
  if (nbox > kMaxBoxes) return RTS_E_UNSUPPORTED;
  try {
    for (int b = 0; b < nbox; ++b) {
      int rc = validate_desc(descs[b]);
      if (rc) return rc;
      if (descs[b].prec != descs[0].prec) return RTS_E_ARG;
    }
    for (int b = 1; b < nbox; ++b)
      if (decomposed(descs[b]) != decomposed(descs[0])) {
        g_last_hip = "a plan's boxes are all decomposed into subdomains or none";
        return RTS_E_UNSUPPORTED;
      }
    for (int b = 0; b < nbox; ++b)
      if (descs[b].gs_iter > 0 && nbox > 1) {
        g_last_hip = "a scattering plan (gs_iter > 0) has one box";
        return RTS_E_UNSUPPORTED;
      }
    Plan* P = new Plan();
    P->prec = descs[0].prec;
    P->gs_iter = descs[0].gs_iter;
    P->decomposed = decomposed(descs[0]);
    P->esz = P->prec == RTS_FP32 ? 4 : 8;
    P->sched.rows_per_strip = P->prec == RTS_FP32 ? 4 : 2;  // measured best on MI355X
    for (int b = 0; b < nbox; ++b) {
      Box B;
      B.d = descs[b];
      B.mu.assign(descs[b].mu, descs[b].mu + 3 * descs[b].nrays);
      B.w.assign(descs[b].w, descs[b].w + descs[b].nrays);
      B.qw.assign(descs[b].nbands, 1.0);
      if (descs[b].qweight) B.qw.assign(descs[b].qweight, descs[b].qweight + descs[b].nbands);
      B.d.mu = nullptr; B.d.w = nullptr; B.d.qweight = nullptr;
      B.N = (int64_t)B.d.g.nx * B.d.g.ny * B.d.g.nz;
      for (int r = 0; r < B.d.nrays; ++r) B.n_up += B.mu[3 * r + 2] > 0;
      // group rays by (dominant axis, direction) in ray order; inside a group a
      // ray takes the slot of its in-plane signs (slot = 2 [col sign < 0] +
      // [row sign < 0]), opening a new task when that slot is taken
      std::map<std::pair<int, int>, std::vector<std::array<int, 4>>> grp;
      std::vector<std::pair<int, int>> keys;
      for (int r = 0; r < B.d.nrays; ++r) {
        RayGeo g = ray_geo(B.d.g, &B.mu[3 * r]);
        auto k = std::make_pair(g.axis, g.sa);
        if (!grp.count(k)) keys.push_back(k);
        const int col_axis = g.axis == 0 ? 1 : 0;
        const int row_axis = g.axis == 2 ? 1 : 2;
        const int slot = (g.mu[col_axis] < 0 ? 2 : 0) + (g.mu[row_axis] < 0 ? 1 : 0);
        auto& tl = grp[k];
        bool placed = false;
        for (auto& a : tl)
          if (a[slot] < 0) { a[slot] = r; placed = true; break; }
        if (!placed) {
          std::array<int, 4> a{-1, -1, -1, -1};
          a[slot] = r;
          tl.push_back(a);
        }
      }
      // with a tolerance the rays of a group stop together: one sweep task each
      // (a decomposed box stops all its rays together)
      if ((B.d.tol > 0 && !decomposed(B.d)) || B.d.gs_iter > 0)
        for (auto& k : keys)
          if ((k.first != 2 || B.d.gs_iter > 0) && grp[k].size() > 1) {
            g_last_hip = "tol > 0 and gs_iter > 0 need at most four rays per dominant axis and "
                         "direction, one per in-plane sign pattern";
            delete P;
            return RTS_E_UNSUPPORTED;
          }
      for (auto& k : keys)
        for (auto& a : grp[k]) B.groups.push_back(a);
      B.tasks_per_band = (int)B.groups.size();
      P->boxes.push_back(std::move(B));
    }
    build_layout(*P);
    pin_early(P);
    *out = P;
    return RTS_OK;
  } catch (...) {
    return RTS_E_ARG;
  }
}

int rts_workspace_bytes(void* plan, int32_t op, size_t* bytes) {
  if (!plan || !bytes) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  if (op == RTS_OP_SOLVE) {
    *bytes = P->total;
    return RTS_OK;
  }
  if (op == RTS_OP_ADJOINT) {
    *bytes = P->total_adj;
    return RTS_OK;
  }
  if (op == RTS_OP_AUTOTUNE) {
    size_t m = 0;
    try {
      for (const rts_schedule& c : tune_candidates(*P)) {
        Plan tmp;
        tmp.boxes = P->boxes;
        tmp.prec = P->prec;
        tmp.esz = P->esz;
        tmp.sched = c;
        build_layout(tmp);
        m = std::max(m, tmp.total);
      }
    } catch (...) {
      return RTS_E_ARG;
    }
    *bytes = m;
    return RTS_OK;
  }
  return RTS_E_ARG;
}

int rts_solve(void* plan, const rts_inputs* in, const rts_outputs* out, void* ws, size_t ws_bytes,
              void* hip_stream) {
  if (!plan) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  if (P->boxes.size() != 1) return RTS_E_ARG;
  try {
    return solve_impl(P, 1, in, out, ws, ws_bytes, hip_stream, true);
  } catch (...) {
    return RTS_E_HIP;
  }
}

int rts_solve_batched(void* plan, int32_t nbox, const rts_inputs* in, const rts_outputs* out,
                      void* ws, size_t ws_bytes, void* hip_stream) {
  if (!plan) return RTS_E_ARG;
  try {
    return solve_impl(static_cast<Plan*>(plan), nbox, in, out, ws, ws_bytes, hip_stream, true);
  } catch (...) {
    return RTS_E_HIP;
  }
}

namespace {
// Argument, tolerance and residency checks shared by the adjoint entry points.
int adjoint_checks(Plan* P, int32_t nbox, const rts_inputs* in, void* ws, size_t ws_bytes) {
  if (nbox != (int)P->boxes.size() || !in) return RTS_E_ARG;
  for (int b = 0; b < nbox; ++b)
    if (!in[b].kappa || !in[b].rho || !in[b].S) return RTS_E_ARG;
  for (int b = 0; b < nbox; ++b)
    if (in[b].ghost) {  // (the reverse sweep replays the cold start's ghost planes)
      g_last_hip = "the adjoint starts from the cold ghost planes (rts_inputs.ghost = NULL)";
      return RTS_E_UNSUPPORTED;
    }
  if (P->decomposed || P->gs_iter > 0) {
    g_last_hip = "no adjoint of a solve decomposed into subdomains or of a scattering solve";
    return RTS_E_UNSUPPORTED;
  }
  for (int b = 0; b < nbox; ++b)
    if (P->boxes[b].d.tol > 0) {  // the reverse sweep replays a fixed number of laps
      g_last_hip = "the adjoint needs a fixed sweep count (tol = 0)";
      return RTS_E_UNSUPPORTED;
    }
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < P->total_adj)
    return RTS_E_WORKSPACE;
  int rc = prepare(P);
  if (rc) return rc;
  for (const Plan::WidthClass& c : P->rclasses)
    if (c.blocks < 1 || c.blocks * P->cus < c.max_strips) {
      g_last_hip = "the strips of one reverse sweep task cannot all be resident";
      return RTS_E_UNSUPPORTED;
    }
  return RTS_OK;
}
}  // namespace

int rts_solve_for_adjoint(void* plan, int32_t nbox, const rts_inputs* in, const rts_outputs* out,
                          void* ws, size_t ws_bytes, void* hip_stream) {
  if (!plan || !in || !out) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  try {
    int rc = check_call(P, nbox, in, out, ws, ws_bytes);
    if (rc) return rc;
    if ((rc = adjoint_checks(P, nbox, in, ws, ws_bytes))) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    return P->prec == RTS_FP32 ? enqueue_forward<float>(*P, in, out, (char*)ws, st, nullptr, true)
                               : enqueue_forward<double>(*P, in, out, (char*)ws, st, nullptr, true);
  } catch (...) {
    return RTS_E_HIP;
  }
}

int rts_adjoint_from_solve(void* plan, int32_t nbox, const rts_inputs* in, const rts_seeds* g,
                           const rts_grads* d, void* ws, size_t ws_bytes, void* hip_stream) {
  if (!plan || !in || !g || !d) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  for (int b = 0; b < nbox && b < (int)P->boxes.size(); ++b)
    if (!d[b].dS || !d[b].dchi) return RTS_E_ARG;
  try {
    int rc = adjoint_checks(P, nbox, in, ws, ws_bytes);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    return P->prec == RTS_FP32 ? enqueue_adjoint<float>(*P, in, g, d, (char*)ws, st, false)
                               : enqueue_adjoint<double>(*P, in, g, d, (char*)ws, st, false);
  } catch (...) {
    return RTS_E_HIP;
  }
}

int rts_adjoint(void* plan, int32_t nbox, const rts_inputs* in, const rts_seeds* g,
                const rts_grads* d, void* ws, size_t ws_bytes, void* hip_stream) {
  if (!plan || !in || !g || !d) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  for (int b = 0; b < nbox && b < (int)P->boxes.size(); ++b)
    if (!d[b].dS || !d[b].dchi) return RTS_E_ARG;
  try {
    int rc = adjoint_checks(P, nbox, in, ws, ws_bytes);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    return P->prec == RTS_FP32 ? enqueue_adjoint<float>(*P, in, g, d, (char*)ws, st)
                               : enqueue_adjoint<double>(*P, in, g, d, (char*)ws, st);
  } catch (...) {
    return RTS_E_HIP;
  }
}

int rts_plan_autotune(void* plan, int32_t nbox, const rts_inputs* in, const rts_outputs* out,
                      void* ws, size_t ws_bytes, void* hip_stream, int32_t reps,
                      rts_schedule* chosen) {
  if (!plan || reps < 1) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  try {
    int tried = 0;
    const int rc = autotune_impl(P, nbox, in, out, ws, ws_bytes,
                                 reinterpret_cast<hipStream_t>(hip_stream), reps, &tried);
    if (rc == RTS_OK && chosen) *chosen = P->sched;
    return rc;
  } catch (...) {
    return RTS_E_HIP;
  }
}

int rts_check_inputs(void* plan, int32_t nbox, const rts_inputs* in, void* ws, size_t ws_bytes,
                     void* hip_stream) {
  if (!plan || !in) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  if (nbox != (int)P->boxes.size()) return RTS_E_ARG;
  for (int b = 0; b < nbox; ++b) {
    if (!in[b].kappa || !in[b].rho || !in[b].S) return RTS_E_ARG;
    if (P->gs_iter > 0 && !in[b].eps) return RTS_E_ARG;
  }
  if (!ws || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0 || ws_bytes < sizeof(WsHeader))
    return RTS_E_WORKSPACE;
  try {
    int rc = dev_init(*P);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    int* flag = &reinterpret_cast<WsHeader*>(ws)->nonfinite;
    RTS_HIP(launch_zero(flag, 1, st));
    auto scan = [&](const void* v, int64_t n) {
      return P->prec == RTS_FP32 ? launch_scan_nonfinite<float>(v, n, flag, P->cus, st)
                                 : launch_scan_nonfinite<double>(v, n, flag, P->cus, st);
    };
    for (int b = 0; b < nbox; ++b) {
      const rts_desc& d = P->boxes[b].d;
      const int64_t N = (int64_t)d.g.nx * d.g.ny * d.g.nz, nb = d.nbands;
      RTS_HIP(scan(in[b].kappa, nb * N));
      RTS_HIP(scan(in[b].rho, N));
      RTS_HIP(scan(in[b].S, nb * N));
      if (P->gs_iter > 0) RTS_HIP(scan(in[b].eps, nb * N));
    }
    RTS_HIP(hipStreamSynchronize(st));
    int32_t bad = 0;
    RTS_HIP(hipMemcpy(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost));
    return bad ? RTS_E_NONFINITE : RTS_OK;
  } catch (...) {
    return RTS_E_HIP;
  }
}

int rts_check_status(void* plan, const void* ws, void* hip_stream) {
  if (!plan) return RTS_E_ARG;
  if (!ws) {  // the array of rts_solve_static on the current device
    void* p = nullptr;
    const int rc = rts::static_scratch(&p);
    if (rc) return rc;
    ws = p;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  RTS_HIP(hipStreamSynchronize(st));
  int32_t s = 0;
  RTS_HIP(hipMemcpy(&s, ws, sizeof(s), hipMemcpyDeviceToHost));
  return s ? RTS_E_DEADLOCK : RTS_OK;
}

int rts_plan_get_schedule(void* plan, rts_schedule* s) {
  if (!plan || !s) return RTS_E_ARG;
  *s = static_cast<Plan*>(plan)->sched;
  return RTS_OK;
}

int rts_plan_set_schedule(void* plan, const rts_schedule* s) {
  if (!plan || !s) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  const int h = s->rows_per_strip;
  const bool ok = P->prec == RTS_FP32 ? (h == 2 || h == 4 || h == 6 || h == 8) : (h == 2 || h == 4);
  if (!ok || s->max_workgroups < 0 || (s->order != 0 && s->order != 1) ||
      (s->single_launch != 0 && s->single_launch != 1) ||
      (s->split_reverse != 0 && s->split_reverse != 1))
    return RTS_E_ARG;
  try {
    set_sched(P, *s);
  } catch (...) {
    return RTS_E_ARG;
  }
  return RTS_OK;
}

int rts_plan_enable_timing(void* plan, int32_t on) {
  if (!plan) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  P->timing = on != 0;
  P->ev_used = 0;
  return RTS_OK;
}

int rts_plan_last_timing(void* plan, double* sweep_ms, double* total_ms) {
  if (!plan || !sweep_ms || !total_ms) return RTS_E_ARG;
  Plan* P = static_cast<Plan*>(plan);
  *sweep_ms = -1;
  *total_ms = -1;
  if (P->ev_used == 0) return RTS_OK;
  double sa = 0, sb = 0;
  RTS_HIP(hipEventSynchronize(P->ev[P->ev_used - 1][3]));
  for (int i = 0; i < P->ev_used; ++i) {
    float a = 0, b = 0;
    RTS_HIP(hipEventElapsedTime(&a, P->ev[i][1], P->ev[i][2]));
    RTS_HIP(hipEventElapsedTime(&b, P->ev[i][0], P->ev[i][3]));
    sa += a;
    sb += b;
  }
  *sweep_ms = sa / P->ev_used;
  *total_ms = sb / P->ev_used;
  return RTS_OK;
}

void rts_plan_destroy(void* plan) {
  if (!plan) return;
  Plan* P = static_cast<Plan*>(plan);
  if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  for (auto& e : P->cap_ev)
    if (e) (void)hipEventDestroy(e);
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
  for (auto& a : P->ev)
    for (auto& e : a)
      if (e) (void)hipEventDestroy(e);
  if (P->pinned) (void)hipHostFree(P->pinned);
  for (void* p : P->old_pinned) (void)hipHostFree(p);
  delete P;
}

const char* rts_status_string(int status) {
  switch (status) {
    case RTS_OK: return "RTS_OK";
    case RTS_E_ARG: return "RTS_E_ARG: invalid argument";
    case RTS_E_UNSUPPORTED: return "RTS_E_UNSUPPORTED: not supported by the library";
    case RTS_E_WORKSPACE: return "RTS_E_WORKSPACE: workspace null, misaligned or too small";
    case RTS_E_HIP: {
      static thread_local std::string s;
      s = "RTS_E_HIP: " + g_last_hip;
      return s.c_str();
    }
    case RTS_E_DEADLOCK: return "RTS_E_DEADLOCK: a sweep neighbour wait timed out";
    case RTS_E_NONFINITE: return "RTS_E_NONFINITE: an input holds a NaN or an infinity";
    case RTS_E_NOT_BUILT: {
      static thread_local std::string s;
      s = "RTS_E_NOT_BUILT: " + g_last_hip;
      return s.c_str();
    }
  }
  return "unknown status";
}

const char* rts_version(void) { return "librts 0.1 (gfx950)"; }

}  // extern "C"
