// gfx950 kernels of the short-characteristics radiation transport solve
// (arXiv 2107.08145, section "Summary of the Radiation Transport Solver",
// RTS core-loop and wavefront-dependency figures).
//
//  * rts_prep      : chi = kappa * rho per band (the opacity part of the
//                    paper's interpolation step) plus [x][z][y] copies of chi
//                    and S so that sweeps along x read contiguous planes (the
//                    role of the paper's transposed arrays).
//  * rts_sweep     : the formal solution.  Persistent workgroups claim
//                    (task, strip) tickets from a device counter.  A task is
//                    up to four rays of one band that share the dominant axis
//                    and its direction; a strip is H rows x all columns of the
//                    task's sweep plane.  Each thread owns one column, keeps
//                    the strip's previous plane in LDS, marches plane by plane
//                    (periodic directions: n_iter laps), and exchanges its
//                    edge rows with the neighbouring strips through tagged
//                    words in the workspace.  It sweeps D = I - S (see rts.h).
//  * rts_reduce_flux, rts_flux_div : the radiative flux vector from the
//                    per-task flux partials (FP64), and its divergence heating.
//  * rts_reduce    : FP64 sum of the per-task partial J - S arrays in a fixed
//                    order, Q, J (the paper's "flux" step).
//  * rts_adj_*, rts_reverse : the adjoint: seeds, the reverse sweep (one
//                    persistent launch over the strips of every task) and the
//                    FP64 gradient reduction.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rts_internal.h"

namespace rts {

// The task table and queue are written by the host before the sweep and only
// read by it.  Reading them through the constant address space lets the
// compiler use scalar loads (and reload instead of spilling): a plain global
// pointer into the workspace, which the sweep also writes, forces vector loads.
#define RTS_CONST __attribute__((address_space(4)))
typedef const Task RTS_CONST CTask;
typedef const int32_t RTS_CONST CInt;

// ---------------------------------------------------------------------------
// small helpers

__device__ inline float rts_exp_neg(float x) { return __builtin_amdgcn_exp2f(-x * 1.4426950408889634f); }
__device__ inline double rts_exp_neg(double x) { return exp(-x); }

// c = (1 - e) / x, power series below x = 0.1 (sum_n (-x)^n / (n+1)!).
__device__ inline float rts_cw(float x, float e) {
  float s = fmaf(fmaf(fmaf(fmaf(x, 1.f / 120.f, -1.f / 24.f), x, 1.f / 6.f), x, -0.5f), x, 1.f);
  float l = (1.f - e) * __builtin_amdgcn_rcpf(x);
  return x < 0.1f ? s : l;
}
__device__ inline double rts_cw(double x, double e) {
  double s = 1.0 / 39916800.0;  // 1/11!
  s = fma(s, -x, 1.0 / 3628800.0);
  s = fma(s, -x, 1.0 / 362880.0);
  s = fma(s, -x, 1.0 / 40320.0);
  s = fma(s, -x, 1.0 / 5040.0);
  s = fma(s, -x, 1.0 / 720.0);
  s = fma(s, -x, 1.0 / 120.0);
  s = fma(s, -x, 1.0 / 24.0);
  s = fma(s, -x, 1.0 / 6.0);
  s = fma(s, -x, 0.5);
  s = fma(s, -x, 1.0);
  if (x < 0.1) return s;
  return (1.0 - e) / x;
}

// a + f (b - a) as one explicit fused multiply-add (the library is built with
// -ffp-contract=off, so every fusion is written out and the arithmetic of a
// cell does not depend on how the compiler schedules a template instance).
__device__ inline float lerp(float a, float b, float f) { return fmaf(f, b - a, a); }
__device__ inline double lerp(double a, double b, double f) { return fma(f, b - a, a); }
__device__ inline float fmad(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fmad(double a, double b, double c) { return fma(a, b, c); }

// Cross-workgroup traffic of the sweep (edge rows and progress flags) uses
// only device-coherent accesses: relaxed agent-scope atomic loads and stores,
// which gfx950 issues with the sc1 bit, so they neither read nor leave stale
// lines in the non-coherent per-XCD L2.  Ordering is explicit: a producer's
// edge-row stores complete (s_waitcnt vmcnt(0)) before the workgroup barrier
// that precedes its flag store; a consumer issues its edge-row loads only
// after its flag load returned the awaited value.  No cache-wide writeback or
// invalidate is needed, which an agent-scope fence would cost at every plane.
// Through the global address space explicitly: a generic pointer would make
// these FLAT instructions, which also count against the LDS wait counter, so
// every LDS-only barrier would wait for the in-flight neighbour loads.
#define RTS_GLOBAL __attribute__((address_space(1)))
// A generic pointer the compiler cannot prove global (loaded from a table or
// picked by a runtime index) becomes FLAT memory instructions; this cast lets
// it emit global ones.
template <class T>
__device__ inline T* gptr(T* p) {
  return (T*)(RTS_GLOBAL T*)(uintptr_t)p;
}
template <class R>
__device__ inline R ld_dev(const R* p) {
  return __hip_atomic_load((const RTS_GLOBAL R*)(uintptr_t)p, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}
template <class R>
__device__ inline void st_dev(R* p, R v) {
  __hip_atomic_store((RTS_GLOBAL R*)(uintptr_t)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Element of a uniform row at a per-lane 32-bit byte offset: lets the
// compiler use the scalar-base + 32-bit lane offset form of global memory
// instructions instead of a 64-bit address add per lane.
template <class T>
__device__ inline T* lane_at(T* row, uint32_t boff) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(row) + boff);
}
template <class T>
__device__ inline const T* lane_at(const T* row, uint32_t boff) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(row) + boff);
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS accesses,
// not for its outstanding global stores (the sweep's global stores are read by
// other workgroups through tags, never by this one).
__device__ inline void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Edge rows are exchanged as self-validating words: every published value
// carries the number of the plane step that produced it (plus one) in the
// same single-copy-atomic 64-bit word.  FP32: (value, tag); FP64: two words
// (low half, tag) and (high half, tag).  A consumer issues its loads early,
// overlaps them with other work, and re-polls only if a tag is stale.
template <class Real>
struct Tagged;
template <>
struct Tagged<float> {
  static constexpr int WORDS = 1;
  __device__ static void put(uint64_t* p, float v, uint32_t tag) {
    st_dev<uint64_t>(p, ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v));
  }
  __device__ static bool fresh(const uint64_t* w, uint32_t tag) { return (uint32_t)(w[0] >> 32) == tag; }
  __device__ static float value(const uint64_t* w) { return __uint_as_float((uint32_t)w[0]); }
};
template <>
struct Tagged<double> {
  static constexpr int WORDS = 2;
  __device__ static void put(uint64_t* p, double v, uint32_t tag) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    st_dev<uint64_t>(p, ((uint64_t)tag << 32) | (b & (uint64_t)0xffffffffu));
    st_dev<uint64_t>(p + 1, ((uint64_t)tag << 32) | (b >> 32));
  }
  __device__ static bool fresh(const uint64_t* w, uint32_t tag) {
    return (uint32_t)(w[0] >> 32) == tag && (uint32_t)(w[1] >> 32) == tag;
  }
  __device__ static double value(const uint64_t* w) {
    return __longlong_as_double((long long)((w[0] & 0xffffffffull) | (w[1] << 32)));
  }
};

// ---------------------------------------------------------------------------
// prep: chi = kappa * rho, chi^T and S^T in [x][z][y]

template <class Real>
__global__ __launch_bounds__(256) void rts_prep(const Real* __restrict__ kappa,
                                               const Real* __restrict__ rho,
                                               const Real* __restrict__ S, Real* __restrict__ chi,
                                               Real* __restrict__ chiT, Real* __restrict__ sT,
                                               int nx, int ny, int nz) {
  __shared__ Real tc[32][33];
  __shared__ Real ts[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
  const int z = blockIdx.z % nz, b = blockIdx.z / nz;
  const int64_t N = (int64_t)nx * ny * nz;
  const Real* kb = kappa + b * N;
  const Real* sb = S + b * N;
  for (int i = 0; i < 4; ++i) {
    const int y = y0 + ty + 8 * i, x = x0 + tx;
    if (x < nx && y < ny) {
      const int64_t p = ((int64_t)z * ny + y) * nx + x;
      const Real c = kb[p] * rho[p];
      chi[b * N + p] = c;
      tc[ty + 8 * i][tx] = c;
      ts[ty + 8 * i][tx] = sb[p];
    }
  }
  __syncthreads();
  for (int i = 0; i < 4; ++i) {
    const int x = x0 + ty + 8 * i, y = y0 + tx;
    if (x < nx && y < ny) {
      const int64_t p = ((int64_t)x * nz + z) * ny + y;
      chiT[b * N + p] = tc[tx][ty + 8 * i];
      sT[b * N + p] = ts[tx][ty + 8 * i];
    }
  }
}

__global__ void rts_zero_ints(int* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ---------------------------------------------------------------------------
// the sweep

template <class Real, int H>
struct Strip {
  // LDS plane state, one column per thread: chi and S of rows -1..H (index
  // 0..H+1), then D of rows 0..H-1 for the four slots.  Stored [column][NQP]
  // with an odd NQP, so that a thread's quantities sit at immediate offsets
  // from its column base and consecutive columns hit distinct banks.
  static constexpr int NQ = 2 * (H + 2) + kMaxRaysPerTask * H;
  static constexpr int NQP = NQ | 1;
  __device__ static constexpr int qc(int j) { return j; }
  __device__ static constexpr int qs(int j) { return H + 2 + j; }
  __device__ static constexpr int qd(int i, int r) { return 2 * (H + 2) + kMaxRaysPerTask * i + r; }
};

// c = (1 - e)/x of the linear-source step, e = exp(-x), by its closed form
// or by its power series (x < 0.1, where 1 - e cancels).  FP32 takes
// xs = x log2(e) (the factor is folded into the scaled opacities) so that e is
// one v_exp_f32; its series has 5 terms (truncation 1.4e-8 relative).  FP64
// takes xs = x and 11 terms.
__device__ inline float rts_exp_step(float xs) { return __builtin_amdgcn_exp2f(-xs); }
__device__ inline double rts_exp_step(double x) { return exp(-x); }
__device__ inline bool rts_small_step(float xs) { return xs < 0.1f * 1.4426950408889634f; }
__device__ inline bool rts_small_step(double x) { return x < 0.1; }
__device__ inline float rts_c_closed(float xs, float e) {
  return (1.f - e) * (__builtin_amdgcn_rcpf(xs) * 1.4426950408889634f);
}
__device__ inline double rts_c_closed(double x, double e) { return (1.0 - e) / x; }
__device__ inline float rts_c_series(float xs) {
  // sum_{n=0}^{4} (-x)^n / (n+1)!  with x = xs ln2
  constexpr float ln2 = 0.69314718055994531f;
  constexpr float a1 = -ln2 / 2.f, a2 = ln2 * ln2 / 6.f, a3 = -ln2 * ln2 * ln2 / 24.f,
                  a4 = ln2 * ln2 * ln2 * ln2 / 120.f;
  return fmaf(fmaf(fmaf(fmaf(xs, a4, a3), xs, a2), xs, a1), xs, 1.f);
}
__device__ inline double rts_c_series(double x) {
  double s = 1.0 / 39916800.0;  // 1/11!
  s = fma(s, -x, 1.0 / 3628800.0);
  s = fma(s, -x, 1.0 / 362880.0);
  s = fma(s, -x, 1.0 / 40320.0);
  s = fma(s, -x, 1.0 / 5040.0);
  s = fma(s, -x, 1.0 / 720.0);
  s = fma(s, -x, 1.0 / 120.0);
  s = fma(s, -x, 1.0 / 24.0);
  s = fma(s, -x, 1.0 / 6.0);
  s = fma(s, -x, 0.5);
  return fma(s, -x, 1.0);
}

// Column-interpolated values of one old row: chi and S (NC variants) and D of
// every slot, at the upwind column of each slot.
template <class Real, int NC>
struct LRow {
  Real c[NC], s[NC], d[kMaxRaysPerTask];
};

// One strip of one task: H rows x all columns of the task's sweep plane,
// marched through every plane (and lap) of the task.
//
// Ray slots are fixed: slot k has its upwind column at c-1 for k < 2 (else
// c+1) and its upwind row at i-1 for even k (else i+1).  With UNI the four
// slots share f1, f2, ds and w, so the column interpolation of chi and S is
// shared by the two slots with the same column direction.  FULL strips have
// exactly H rows (known at compile time); the last strip of a task may not.
//
// The old plane (chi, S of the strip's rows and the two halo rows, D of every
// row and slot) lives in LDS, one column per thread, so that column
// neighbours are plain LDS reads and registers hold only a sliding window of
// interpolated rows.  A step has a read phase (the two edge rows first, which
// need the neighbouring strips' D and are published at once as tagged words,
// then the interior rows) and, after a barrier, a write phase that stores the
// new plane; a second barrier ends the step.  Addresses of global data are a
// uniform row pointer plus the thread's column.
// End of a lap of a tolerance-driven sweep (called by every thread of the
// strip, after the lap's last plane is in LDS: D and S of this thread's column
// are read from there, so the call takes no register arrays and stays out of
// the step's register allocation): compares this strip's rows of the plane
// with the stored previous one (the ghost the lap started from) and stores
// the new one; the
// workgroup's maxima of |change| and |D + S| go to the task's words of this
// lap with device-scope atomic max (non-negative doubles order like their
// bits), then thread 0 counts the strip in and waits until every strip of the
// task has (bounded by the watchdog).  Returns the task's common decision:
// stop after this lap (within tolerance, or the last lap).
// (Task fields come as scalars: `used` has bit r set for a used slot r.)
template <class Real, int H>
__device__ __noinline__ bool lap_end_stop(char* ws, int64_t timeout_ticks, double tol, int laps,
                                          int strips, int64_t gbuf_off, int64_t tolw_off,
                                          int used, int W, int lap, int hr, bool act, int c,
                                          int r0, const Real* lc) {
  using ST = Strip<Real, H>;
  constexpr int R = kMaxRaysPerTask;
  __shared__ double sh_red[2][kMaxCols / 64];
  __shared__ int sh_stop;
  double dmax = 0.0, smax = 0.0;
  if (act) {
    Real* gb = gptr(reinterpret_cast<Real*>(ws) + gbuf_off);
    for (int i = 0; i < hr; ++i) {
      for (int r = 0; r < R; ++r) {
        if (!((used >> r) & 1)) continue;  // unused slot
        const Real d = lc[ST::qd(i, r)];
        Real& g = gb[((int64_t)(r0 + i) * W + c) * R + r];
        dmax = fmax(dmax, (double)fabs(d - g));
        smax = fmax(smax, (double)fabs(d + lc[ST::qs(i + 1)]));
        g = d;
      }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    dmax = fmax(dmax, __shfl_xor(dmax, o));
    smax = fmax(smax, __shfl_xor(smax, o));
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh_red[0][wv] = dmax;
    sh_red[1][wv] = smax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (int)(blockDim.x + 63) / 64;
    for (int w = 1; w < nw; ++w) {
      dmax = fmax(dmax, sh_red[0][w]);
      smax = fmax(smax, sh_red[1][w]);
    }
    unsigned long long* tw =
        gptr(reinterpret_cast<unsigned long long*>(ws) + tolw_off) + 3 * lap;
    int* status = gptr(reinterpret_cast<int*>(ws));
    atomicMax(&tw[0], (unsigned long long)__double_as_longlong(dmax));
    atomicMax(&tw[1], (unsigned long long)__double_as_longlong(smax));
    __hip_atomic_fetch_add((RTS_GLOBAL unsigned long long*)(uintptr_t)&tw[2], 1ull,
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    auto arrived = [&]() {
      return __hip_atomic_load((const RTS_GLOBAL unsigned long long*)(uintptr_t)&tw[2],
                               __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    };
    bool ok = true;
    if (arrived() < (unsigned long long)strips) {
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      while (arrived() < (unsigned long long)strips) {
        __builtin_amdgcn_s_sleep(2);
        if (ld_dev(status) != 0) { ok = false; break; }
        if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > timeout_ticks) {
          st_dev(status, 1);
          ok = false;
          break;
        }
      }
    }
    const double gd = __longlong_as_double((long long)__hip_atomic_load(
        (const RTS_GLOBAL unsigned long long*)(uintptr_t)&tw[0], __ATOMIC_ACQUIRE,
        __HIP_MEMORY_SCOPE_AGENT));
    const double gs = __longlong_as_double((long long)__hip_atomic_load(
        (const RTS_GLOBAL unsigned long long*)(uintptr_t)&tw[1], __ATOMIC_ACQUIRE,
        __HIP_MEMORY_SCOPE_AGENT));
    sh_stop = !ok || gd <= tol * gs || lap + 1 >= laps;
  }
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(sh_stop) != 0;
}

template <class Real, int H, bool UNI, bool FULL, int EXT>
__device__ __forceinline__ void run_strip(const SweepArgs& A, CTask& T, const int strip,
                                          Real* lds) {
  using ST = Strip<Real, H>;
  constexpr int R = kMaxRaysPerTask;
  constexpr int NC = UNI ? 2 : R;  // distinct column-interpolated chi/S per row
  using LR = LRow<Real, NC>;
  using TG = Tagged<Real>;
  constexpr int NW = TG::WORDS;
  const int W = T.n_cols;
  const int c = threadIdx.x;
  const bool act = c < W;
  const int cc = act ? c : W - 1;
  const int cm = cc > 0 ? cc - 1 : W - 1, cp1 = cc + 1 < W ? cc + 1 : 0;
  int r0 = strip * T.rows_per_strip;
  const int hr = FULL ? H : min(T.rows_per_strip, T.n_rows - r0);
  int ps = (int)T.plane_stride, rs = (int)T.row_stride;
  int* status = gptr(reinterpret_cast<int*>(A.ws));

  // per-slot constants; FP32 folds log2(e) into ds/2 (see rts_exp_step)
  const Real kx = sizeof(Real) == 4 ? Real(1.4426950408889634) : Real(1);
  Real f1[R], f2[R], hds[R], wgt[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const TaskRay RTS_CONST& y = T.ray[UNI ? 0 : r];
    f1[r] = (Real)y.f1; f2[r] = (Real)y.f2; hds[r] = (Real)y.hds * kx; wgt[r] = (Real)y.w;
  }
  // scale of the chi values kept in LDS: ds/2 (times log2 e in FP32) when the
  // four slots share ds, so that the optical depth step is one add
  const Real csc = UNI ? hds[0] : Real(1);
  const bool zp = T.z_planes != 0;
  const int bc_up = zp ? -1 : 0, bc_dn = zp ? -1 : T.n_rows - 1;

  const Real* chi = gptr(reinterpret_cast<const Real*>(A.ws) + T.chi_off);
  const Real* Sv = gptr(T.transposed ? reinterpret_cast<const Real*>(A.ws) + T.s_off
                                     : reinterpret_cast<const Real*>(A.box[T.box].S) + T.s_off);
  Real* P = gptr(reinterpret_cast<Real*>(A.ws) + T.part_off);
  // exchange buffer of 64-bit words: [strip][parity][edge][slot][column][NW]
  uint64_t* X = gptr(reinterpret_cast<uint64_t*>(A.ws) + T.xbuf_off);

  const int ns = T.strips;
  const bool per = T.row_periodic != 0;
  const bool has_lo = per || r0 > 0;
  const bool has_hi = per || r0 + hr < T.n_rows;
  const int row_lo = r0 > 0 ? r0 - 1 : T.n_rows - 1;
  const int row_hi = r0 + hr < T.n_rows ? r0 + hr : 0;
  const int st_lo = strip > 0 ? strip - 1 : ns - 1;
  const int st_hi = strip + 1 < ns ? strip + 1 : 0;
  const int xstride = R * W * NW;  // one published edge row, all slots
  const int lrow = has_lo ? row_lo : r0, hrow = has_hi ? row_hi : r0;

  const int na = T.n_planes;
  const int q0 = T.sa > 0 ? 0 : na - 1;
  const int q_last = T.sa > 0 ? na - 1 : 0;
  const int nsteps = zp ? na - 1 : T.laps * na;
  // tolerance-driven laps: outputs written every lap (the last lap run keeps them)
  const bool tolmode = EXT == 2 && !zp && T.tol > 0;
  const int out_from = zp || tolmode ? 0 : (T.laps - 1) * na;
  auto plane_of = [&](int t) {
    return t < 0 ? (zp ? q0 : q_last) : (zp ? q0 + T.sa * (t + 1) : q0 + T.sa * (t % na));
  };
  Real* lc = lds + c * ST::NQP;                         // this column
  const Real* lcc = lds + cc * ST::NQP;                 // this column (clamped)
  const Real* lcm = lds + cm * ST::NQP;                 // column c-1
  const Real* lcp = lds + cp1 * ST::NQP;                // column c+1
  // per-lane byte offsets of this column in a Real row and in an exchange row
  const uint32_t cb = (uint32_t)cc * sizeof(Real), ub = (uint32_t)c * sizeof(Real);
  const uint32_t xb_c = (uint32_t)cc * NW * 8, xb_m = (uint32_t)cm * NW * 8,
                 xb_p = (uint32_t)cp1 * NW * 8, xb_u = (uint32_t)c * NW * 8;
  // uniform row pointer (a readfirstlane'd offset, so the compiler keeps one
  // 32-bit lane offset instead of a 64-bit pointer per row)
  auto urow = [&](auto* base, int off) __attribute__((always_inline)) {
    return base + __builtin_amdgcn_readfirstlane(off);
  };

  // chi and S of a plane, rows -1..H (index 0..H+1)
  Real ncx[H + 2], nsx[H + 2];
  auto load_plane = [&](int q) __attribute__((always_inline)) {
    const int qo = q * ps;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const int o = qo + (r0 + (FULL || i < hr ? i : 0)) * rs;
      ncx[i + 1] = *lane_at(urow(chi, o), cb) * csc;
      nsx[i + 1] = *lane_at(urow(Sv, o), cb);
    }
    ncx[0] = *lane_at(urow(chi, qo + lrow * rs), cb) * csc;
    nsx[0] = *lane_at(urow(Sv, qo + lrow * rs), cb);
    ncx[H + 1] = *lane_at(urow(chi, qo + hrow * rs), cb) * csc;
    nsx[H + 1] = *lane_at(urow(Sv, qo + hrow * rs), cb);
  };
  // outputs of plane q from the new D and S: the pairwise sum of w_r D_r over
  // the task's four slots (the sums over tasks and bands are FP64) and I_top
  auto write_out = [&](int q, const Real (&Dn)[H][R]) __attribute__((always_inline)) {
    if (!act) return;
    const int qo = q * ps;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      if (!FULL && i >= hr) break;
      Real sum;
      if (UNI) {
        sum = wgt[0] * ((Dn[i][0] + Dn[i][1]) + (Dn[i][2] + Dn[i][3]));
      } else {
        sum = fmad(wgt[1], Dn[i][1], wgt[0] * Dn[i][0]) + fmad(wgt[3], Dn[i][3], wgt[2] * Dn[i][2]);
      }
      *lane_at(urow(P, qo + (r0 + i) * rs), ub) = sum;
    }
    if (EXT >= 1 && A.flux && T.flux_off >= 0) {  // (a box without flux partials writes none)
      // flux partials sum_r (w mu_k)_r D_r along k = cols, rows (and the plane
      // axis unless uni), in the layout of the partial sum.  With uni the
      // slots share |w mu_k| and the signs follow the slot order (cols: + for
      // slots 0 and 1; rows: + for even slots).
      Real* Fp = gptr(reinterpret_cast<Real*>(A.ws) + T.flux_off);
#pragma unroll
      for (int i = 0; i < H; ++i) {
        if (!FULL && i >= hr) break;
        const int o = qo + (r0 + i) * rs;
        if (UNI || T.uni) {  // (a uni task in a launch for general tasks too)
          const Real wc = (Real)T.ray[0].wm[0], wr = (Real)T.ray[0].wm[1];
          *lane_at(urow(Fp, o), ub) = wc * ((Dn[i][0] + Dn[i][1]) - (Dn[i][2] + Dn[i][3]));
          *lane_at(urow(Fp + T.n_cells, o), ub) = wr * ((Dn[i][0] + Dn[i][2]) - (Dn[i][1] + Dn[i][3]));
        } else {
#pragma unroll
          for (int m = 0; m < 3; ++m) {
            Real f = Real(0);
#pragma unroll
            for (int r = 0; r < R; ++r) f = fmad((Real)T.ray[r].wm[m], Dn[i][r], f);
            *lane_at(urow(Fp + m * T.n_cells, o), ub) = f;
          }
        }
      }
    }
    Real* Itop = gptr(reinterpret_cast<Real*>(A.box[T.box].I_top));
    const int it_row = T.it_top - r0;
    if (Itop && (zp ? (q == T.it_top) : (it_row >= 0 && it_row < hr))) {
#pragma unroll
      for (int i = 0; i < H; ++i) {
        if (zp ? (!FULL && i >= hr) : (i != it_row)) continue;
        const int gr = r0 + i;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int it = T.ray[r].itop;
          if (it >= 0)
            Itop[T.it_off + it * T.it_ray + (int64_t)q * T.itp + (int64_t)gr * T.itr +
                 (int64_t)c * T.itc] = nsx[i + 1] + Dn[i][r];
        }
      }
    }
  };
  // D of unrolled plane u, kept for the adjoint's reverse sweep
  auto store_d = [&](int u, const Real (&Dn)[H][R]) __attribute__((always_inline)) {
    if (!A.store_d || !act) return;
    Real* ds = gptr(reinterpret_cast<Real*>(A.ws) + T.dstore_off + (int64_t)u * R * T.n_rows * W);
#pragma unroll
    for (int i = 0; i < H; ++i) {
      if (!FULL && i >= hr) break;
#pragma unroll
      for (int r = 0; r < R; ++r) *lane_at(urow(ds, (r * T.n_rows + r0 + i) * W), ub) = Dn[i][r];
    }
  };
  // store the plane (ncx, nsx, Dn) as the next step's old plane
  auto store_plane = [&](const Real (&Dn)[H][R]) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < H + 2; ++j) {
      lc[ST::qc(j)] = ncx[j];
      lc[ST::qs(j)] = nsx[j];
    }
#pragma unroll
    for (int i = 0; i < H; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) lc[ST::qd(i, r)] = Dn[i][r];
  };

  // ---- first upwind plane: the boundary layer (planes are z) or the ghost plane
  {
    load_plane(plane_of(-1));
    const Real pa = (Real)T.pl_a, pb = (Real)T.pl_b;
    const Real ua = (Real)T.bu_a, ub = (Real)T.bu_b, da = (Real)T.bd_a, db = (Real)T.bd_b;
    Real D0[H][R];
#pragma unroll
    for (int i = 0; i < H; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool up = (r & 1) == 0;
        const int br = up ? bc_up : bc_dn;
        D0[i][r] = zp ? fmad(pa, nsx[i + 1], pb)
                      : ((r0 + i == br) ? fmad(up ? ua : da, nsx[i + 1], up ? ub : db) : Real(0));
      }
    lds_barrier();  // the previous strip of this workgroup has finished with the LDS
    store_plane(D0);
    if (zp) write_out(q0, D0);
    if (zp) store_d(0, D0);
    if (tolmode && act) {  // the initial ghost plane's D of this strip's rows
      Real* gb = gptr(reinterpret_cast<Real*>(A.ws) + T.gbuf_off);
#pragma unroll
      for (int i = 0; i < H; ++i) {
        if (!FULL && i >= hr) break;
#pragma unroll
        for (int r = 0; r < R; ++r) gb[((int64_t)(r0 + i) * W + c) * R + r] = D0[i][r];
      }
    }
    if (nsteps > 0) load_plane(plane_of(0));
    lds_barrier();
  }

  // neighbours' tagged edge-row words for the next step: issued at the end of
  // a step (the neighbours publish early in theirs), checked in the next
  uint64_t hw[R][2][NW];
  auto halo_issue = [&](int t) __attribute__((always_inline)) {
    const int par = (t - 1) & 1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool lower = (r & 1) == 0;  // even slots look at the lower halo, odd at the upper
      const bool has = lower ? has_lo : has_hi;
      const int xoff = (((lower ? st_lo : st_hi) * 2 + par) * 2 + (lower ? 1 : 0)) * xstride;
      const uint64_t* rowp = urow(X, xoff + r * W * NW);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const uint32_t colb = k == 0 ? xb_c : (r < 2 ? xb_m : xb_p);
#pragma unroll
        for (int x = 0; x < NW; ++x) hw[r][k][x] = has ? ld_dev(lane_at(rowp, colb) + x) : 0ull;
      }
    }
  };
  // wait until every word of this step is fresh (re-polling, bounded by the watchdog)
  auto halo_wait = [&](int t) __attribute__((always_inline)) {
    const uint32_t tag = (uint32_t)t;
    auto all_fresh = [&]() __attribute__((always_inline)) {
      bool ok = true;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool has = (r & 1) == 0 ? has_lo : has_hi;
#pragma unroll
        for (int k = 0; k < 2; ++k) ok = ok && (!has || TG::fresh(hw[r][k], tag));
      }
      return ok;
    };
    if (__ballot(!all_fresh()) == 0) return;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
      __builtin_amdgcn_s_sleep(1);
      halo_issue(t);
      if (__ballot(!all_fresh()) == 0) break;
      if (__builtin_amdgcn_readfirstlane(ld_dev(status)) != 0) break;
      if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > A.timeout_ticks) {
        st_dev(status, 1);
        break;
      }
    }
  };

  // ---- the march
  for (int t = 0; t < nsteps; ++t) {
    // Launder the strides, the strip origin and the base pointers each step:
    // the address arithmetic derived from them is then recomputed in the loop
    // (scalar ALU) instead of being hoisted as dozens of live row offsets,
    // which would be spilled.
    asm volatile("" : "+s"(rs), "+s"(ps), "+s"(r0), "+s"(chi), "+s"(Sv), "+s"(P), "+s"(X));
    chi = gptr(chi);  // the asm hides the address space again
    Sv = gptr(Sv);
    P = gptr(P);
    X = gptr(X);
    const int q = plane_of(t);
    if (t > 0) halo_wait(t);

    // column interpolation of old LDS row j (own rows, 1..H, carry D of row j-1)
    auto interp = [&](int j, bool own, LR& o) __attribute__((always_inline)) {
      const Real ca = lcc[ST::qc(j)], cl = lcm[ST::qc(j)], cr = lcp[ST::qc(j)];
      const Real sa = lcc[ST::qs(j)], sl = lcm[ST::qs(j)], sr = lcp[ST::qs(j)];
#pragma unroll
      for (int v = 0; v < NC; ++v) {
        const bool lft = UNI ? (v == 0) : (v < 2);
        o.c[v] = lerp(ca, lft ? cl : cr, f1[UNI ? 2 * v : v]);
        o.s[v] = lerp(sa, lft ? sl : sr, f1[UNI ? 2 * v : v]);
      }
      if (own) {
        const int i = j - 1 >= 0 ? (j - 1 < H ? j - 1 : H - 1) : 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const Real a = lcc[ST::qd(i, r)], n = (r < 2 ? lcm : lcp)[ST::qd(i, r)];
          o.d[r] = lerp(a, n, f1[r]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) o.d[r] = Real(0);
      }
    };
    // the formal solution of row i from the interpolated old rows i-1, i, i+1
    auto solve_row = [&](int i, const LR& lp, const LR& lk, const LR& ln, Real* out)
        __attribute__((always_inline)) {
      const Real cpv = ncx[i + 1], spv = nsx[i + 1];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int v = UNI ? (r < 2 ? 0 : 1) : r;
        const bool up = (r & 1) == 0;
        const Real bc = lerp(lk.c[v], up ? lp.c[v] : ln.c[v], f2[r]);
        const Real bs = lerp(lk.s[v], up ? lp.s[v] : ln.s[v], f2[r]);
        const Real bd = lerp(lk.d[r], up ? lp.d[r] : ln.d[r], f2[r]);
        // UNI: chi is stored pre-scaled by ds/2 (and log2 e in FP32)
        const Real xs = UNI ? cpv + bc : hds[r] * (cpv + bc);
        // both forms, then a select (a branch here costs registers)
        const Real e = rts_exp_step(xs);
        const Real c_ser = rts_c_series(xs), c_cl = rts_c_closed(xs, e);
        const Real cw = rts_small_step(xs) ? c_ser : c_cl;
        out[r] = fmad(e, bd, cw * (bs - spv));
      }
      const int gr = r0 + i;  // boundary rows (rows are z): set, not integrated
      if (gr == bc_up) {
        const Real v = fmad((Real)T.bu_a, spv, (Real)T.bu_b);
        out[0] = v; out[2] = v;
      }
      if (gr == bc_dn) {
        const Real v = fmad((Real)T.bd_a, spv, (Real)T.bd_b);
        out[1] = v; out[3] = v;
      }
    };
    // halo D of the slots that look at the halo row (even: lower, odd: upper).
    // On the first plane it is local, an affine function of the halo's S (the
    // column interpolation commutes with it); later it is the neighbour's
    // edge row of the previous plane, a tagged word.
    auto halo_d = [&](bool lower, LR& h) __attribute__((always_inline)) {
      const bool has = lower ? has_lo : has_hi;
      const int hrow_g = lower ? row_lo : row_hi;
      if (t == 0) {
        const Real pa = (Real)T.pl_a, pb = (Real)T.pl_b;
        const Real ua = (Real)T.bu_a, ub = (Real)T.bu_b, da = (Real)T.bd_a, db = (Real)T.bd_b;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (((r & 1) == 0) != lower) continue;
          const int v = UNI ? (r < 2 ? 0 : 1) : r;
          const bool up = (r & 1) == 0;
          const int br = up ? bc_up : bc_dn;
          h.d[r] = !has ? Real(0)
                        : zp ? fmad(pa, h.s[v], pb)
                             : (hrow_g == br ? fmad(up ? ua : da, h.s[v], up ? ub : db) : Real(0));
        }
        return;
      }
      if (!has) return;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (((r & 1) == 0) != lower) continue;
        h.d[r] = lerp(TG::value(hw[r][0]), TG::value(hw[r][1]), f1[r]);
      }
    };

    Real Dn[H][R];
    // ---- edge rows first, published for the neighbouring strips
    {
      LR lo, k0, n0;
      interp(0, false, lo);
      halo_d(true, lo);
      interp(1, true, k0);
      if (hr == 1) {
        interp(H + 1, false, n0);
        halo_d(false, n0);
      } else {
        interp(2, true, n0);
      }
      solve_row(0, lo, k0, n0, Dn[0]);
    }
#pragma unroll
    for (int i = 1; i < H; ++i) {
      if (!(FULL ? (i == H - 1) : (i == hr - 1))) continue;
      LR lp, lk, up_;
      interp(i, true, lp);
      interp(i + 1, true, lk);
      interp(H + 1, false, up_);
      halo_d(false, up_);
      solve_row(i, lp, lk, up_, Dn[i]);
    }
    if (act) {
      const int xe = ((strip * 2 + (t & 1)) * 2) * xstride;
      const uint32_t tag = (uint32_t)(t + 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        Real top = Dn[0][r];
#pragma unroll
        for (int i = 1; i < H; ++i)
          if (FULL ? (i == H - 1) : (i == hr - 1)) top = Dn[i][r];
        if ((r & 1) == 1) TG::put(lane_at(urow(X, xe + r * W * NW), xb_u), Dn[0][r], tag);  // lower: odd slots
        if ((r & 1) == 0) TG::put(lane_at(urow(X, xe + xstride + r * W * NW), xb_u), top, tag);  // upper: even
      }
    }
    // ---- interior rows, sliding window of interpolated old rows
    if (FULL ? (H > 2) : (hr > 2)) {
      LR a, b, d;
      interp(1, true, a);
      interp(2, true, b);
#pragma unroll
      for (int i = 1; i < H - 1; ++i) {
        if (!FULL && i >= hr - 1) break;
        interp(i + 2, true, d);
        solve_row(i, a, b, d, Dn[i]);
        a = b;
        b = d;
      }
    }
    lds_barrier();  // every thread has read the old plane
    store_plane(Dn);
    if (t >= out_from) write_out(q, Dn);
    store_d(zp ? t + 1 : t, Dn);
    if (tolmode && (t % na) == na - 1) {
      // end of a lap: the change of this strip's part of the last plane (the
      // next ghost) and its largest intensity, folded into the task's words;
      // once every strip of the task has arrived all read the same maxima and
      // stop together when the change is within tolerance
      int used = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) used |= (T.ray[r].ray >= 0) << r;
      if (lap_end_stop<Real, H>(A.ws, A.timeout_ticks, T.tol, T.laps, T.strips, T.gbuf_off,
                                T.tolw_off, used, W, t / na, hr, act, c, r0, lc)) {
        lds_barrier();
        break;
      }
    }
    if (t + 1 < nsteps) {
      load_plane(plane_of(t + 1));
      halo_issue(t + 1);
    }
    lds_barrier();  // the new plane is complete
  }
}

// EXT: 0 the plain sweep; 1 also the flux partials (A.flux); 2 also
// tolerance-driven laps (T.tol > 0).  Separate instantiations, so that each
// keeps its own register allocation.
template <class Real, int H, bool UNI, int EXT>
__global__ __launch_bounds__(1024) void rts_sweep(SweepArgs A) {
  extern __shared__ char smem_raw[];
  Real* lds = reinterpret_cast<Real*>(smem_raw);
  __shared__ int sh_ticket;
  WsHeader* hdr = reinterpret_cast<WsHeader*>(A.ws);
  for (;;) {
    if (threadIdx.x == 0) sh_ticket = atomicAdd(&hdr->ticket[A.wclass], 1);
    __syncthreads();
    const int tk = __builtin_amdgcn_readfirstlane(sh_ticket);
    __syncthreads();
    if (tk >= A.total_strips) return;
    CInt* queue = (CInt*)(uintptr_t)A.queue;
    int qi = 0;
    while (qi + 1 < A.ntasks && queue[2 * (qi + 1)] <= tk) ++qi;
    CTask& T = ((CTask*)(uintptr_t)A.tasks)[queue[2 * qi + 1]];
    const int strip = tk - queue[2 * qi];
    if ((strip + 1) * T.rows_per_strip <= T.n_rows) run_strip<Real, H, UNI, true, EXT>(A, T, strip, lds);
    else run_strip<Real, H, UNI, false, EXT>(A, T, strip, lds);
  }
}

// ---------------------------------------------------------------------------
// Radiative flux vector F = sum_b qweight_b 4 pi (sum_tasks flux partial +
// S_b sum_r w_r mu_r) in FP64, fixed order; partials of transposed tasks
// through an LDS tile as in rts_reduce.  F is [3][N].
template <class Real>
__global__ __launch_bounds__(256) void rts_reduce_flux(const char* __restrict__ ws,
                                                      const Task* __restrict__ tasks, BoxGeo G,
                                                      const Real* __restrict__ S,
                                                      double* __restrict__ F) {
  __shared__ Real tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int64_t N = (int64_t)nx * ny * nz;
  double f[3][4] = {};
  // one task array (natural or [x][z][y] layout) at this thread's four cells
  auto load4 = [&](const Real* part, bool transposed, double (&v)[4]) {
    if (!transposed) {
      for (int i = 0; i < 4; ++i) {
        const int y = y0 + ty + 8 * i, x = x0 + tx;
        v[i] = x < nx && y < ny ? (double)part[((int64_t)z * ny + y) * nx + x] : 0.0;
      }
    } else {
      __syncthreads();
      for (int i = 0; i < 4; ++i) {
        const int x = x0 + ty + 8 * i, y = y0 + tx;
        if (x < nx && y < ny) tile[ty + 8 * i][tx] = part[((int64_t)x * nz + z) * ny + y];
      }
      __syncthreads();
      for (int i = 0; i < 4; ++i) {
        const int y = y0 + ty + 8 * i, x = x0 + tx;
        v[i] = x < nx && y < ny ? (double)tile[tx][ty + 8 * i] : 0.0;
      }
    }
  };
  for (int b = 0; b < G.nbands; ++b) {
    double acc[3][4] = {};
    for (int k = 0; k < G.tasks_per_band; ++k) {
      const Task& T = tasks[G.task0 + b * G.tasks_per_band + k];
      const Real* fp = reinterpret_cast<const Real*>(ws) + T.flux_off;
      double v[3][4];
      load4(fp, T.transposed, v[0]);
      load4(fp + N, T.transposed, v[1]);
      if (T.uni) {  // plane-axis component: mu_axis times the partial sum
        load4(reinterpret_cast<const Real*>(ws) + T.part_off, T.transposed, v[2]);
        const double mua = T.ray[0].wm[2] / T.ray[0].w;
        for (int i = 0; i < 4; ++i) v[2][i] *= mua;
      } else {
        load4(fp + 2 * N, T.transposed, v[2]);
      }
      for (int m = 0; m < 3; ++m)
        for (int i = 0; i < 4; ++i) acc[T.frame[m]][i] += v[m][i];
    }
    const double qf = 4.0 * 3.14159265358979323846 * G.qweight[b];
    for (int i = 0; i < 4; ++i) {
      const int y = y0 + ty + 8 * i, x = x0 + tx;
      if (x < nx && y < ny) {
        const double sv = (double)S[b * N + ((int64_t)z * ny + y) * nx + x];
        for (int m = 0; m < 3; ++m) f[m][i] += qf * (acc[m][i] + sv * G.msum[m]);
      }
    }
  }
  for (int i = 0; i < 4; ++i) {
    const int y = y0 + ty + 8 * i, x = x0 + tx;
    if (x < nx && y < ny)
      for (int m = 0; m < 3; ++m) F[m * N + ((int64_t)z * ny + y) * nx + x] = f[m][i];
  }
}

// Heating by the flux divergence, QF = -(dFx/dx + dFy/dy + dFz/dz), FP64:
// central differences, periodic in x and y; second-order one-sided in z in
// the bottom and top layers (first-order when nz = 2).  One thread per cell.
__global__ __launch_bounds__(256) void rts_flux_div(const double* __restrict__ F,
                                                   double* __restrict__ QF, int nx, int ny,
                                                   int nz, double rdx, double rdy, double rdz) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int i = (int)(p % nx);
  const int j = (int)((p / nx) % ny);
  const int k = (int)(p / ((int64_t)nx * ny));
  const int64_t plane = (int64_t)nx * ny;
  const double* Fx = F;
  const double* Fy = F + N;
  const double* Fz = F + 2 * N;
  const int64_t row = p - i, pl = p - (int64_t)j * nx;
  const int ip = i + 1 < nx ? i + 1 : 0, im = i > 0 ? i - 1 : nx - 1;
  const int jp = j + 1 < ny ? j + 1 : 0, jm = j > 0 ? j - 1 : ny - 1;
  const double ddx = (Fx[row + ip] - Fx[row + im]) * (0.5 * rdx);
  const double ddy = (Fy[pl + (int64_t)jp * nx] - Fy[pl + (int64_t)jm * nx]) * (0.5 * rdy);
  double ddz;
  if (nz == 2) {
    ddz = (Fz[p + (k == 0 ? plane : 0)] - Fz[p - (k == 0 ? 0 : plane)]) * rdz;
  } else if (k == 0) {
    ddz = (-3.0 * Fz[p] + 4.0 * Fz[p + plane] - Fz[p + 2 * plane]) * (0.5 * rdz);
  } else if (k == nz - 1) {
    ddz = (3.0 * Fz[p] - 4.0 * Fz[p - plane] + Fz[p - 2 * plane]) * (0.5 * rdz);
  } else {
    ddz = (Fz[p + plane] - Fz[p - plane]) * (0.5 * rdz);
  }
  QF[p] = -(ddx + ddy + ddz);
}

// ---------------------------------------------------------------------------
// reduce: dJ_b = sum of the band's task partials (FP64, fixed order),
// Q = sum_b qweight_b 4 pi chi_b dJ_b, J_b = S_b + dJ_b.

template <class Real>
__global__ __launch_bounds__(256) void rts_reduce(const char* __restrict__ ws,
                                                 const Task* __restrict__ tasks, BoxGeo G,
                                                 BoxPtrs P) {
  __shared__ Real tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int64_t N = (int64_t)nx * ny * nz;
  const Real* kap = reinterpret_cast<const Real*>(P.kappa);
  const Real* rho = reinterpret_cast<const Real*>(P.rho);
  const Real* S = reinterpret_cast<const Real*>(P.S);
  Real* J = reinterpret_cast<Real*>(P.J);
  double q[4] = {0, 0, 0, 0};
  for (int b = 0; b < G.nbands; ++b) {
    double acc[4] = {0, 0, 0, 0};
    for (int k = 0; k < G.tasks_per_band; ++k) {
      const Task& T = tasks[G.task0 + b * G.tasks_per_band + k];
      const Real* part = reinterpret_cast<const Real*>(ws) + T.part_off;
      if (!T.transposed) {
        for (int i = 0; i < 4; ++i) {
          const int y = y0 + ty + 8 * i, x = x0 + tx;
          if (x < nx && y < ny) acc[i] += (double)part[((int64_t)z * ny + y) * nx + x];
        }
      } else {
        __syncthreads();
        for (int i = 0; i < 4; ++i) {
          const int x = x0 + ty + 8 * i, y = y0 + tx;
          if (x < nx && y < ny) tile[ty + 8 * i][tx] = part[((int64_t)x * nz + z) * ny + y];
        }
        __syncthreads();
        for (int i = 0; i < 4; ++i) {
          const int y = y0 + ty + 8 * i, x = x0 + tx;
          if (x < nx && y < ny) acc[i] += (double)tile[tx][ty + 8 * i];
        }
      }
    }
    const double qf = 4.0 * 3.14159265358979323846 * G.qweight[b];
    for (int i = 0; i < 4; ++i) {
      const int y = y0 + ty + 8 * i, x = x0 + tx;
      if (x < nx && y < ny) {
        const int64_t p = ((int64_t)z * ny + y) * nx + x;
        const double chi = (double)kap[b * N + p] * (double)rho[p];
        const double sv = (double)S[b * N + p];
        const double dj = acc[i] + G.wsum1 * sv;  // J - S
        q[i] += qf * chi * dj;
        if (J) J[b * N + p] = (Real)(sv + dj);
      }
    }
  }
  for (int i = 0; i < 4; ++i) {
    const int y = y0 + ty + 8 * i, x = x0 + tx;
    if (x < nx && y < ny) P.Q[((int64_t)z * ny + y) * nx + x] = q[i];
  }
}

// The same reduction with 16-byte accesses, for FP32 and nx a multiple of 4:
// a thread owns four consecutive x of one row; partials of x-sweeps ([x][z][y])
// go through an LDS tile.  Sums in the same order as rts_reduce.
// FLUX: also the flux vector F from the tasks' flux partials (rts_reduce_flux's
// sums, in the same order), reading S once for both.
template <bool FLUX>
__global__ __launch_bounds__(256) void rts_reduce_v4(const char* __restrict__ ws,
                                                    const Task* __restrict__ tasks, BoxGeo G,
                                                    BoxPtrs P) {
  __shared__ float tile[32][33];
  const int t = threadIdx.x;
  const int qx = (t & 7) * 4, ry = t >> 3;  // this thread: x0 + qx .. +3, row y0 + ry
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int64_t N = (int64_t)nx * ny * nz;
  const int x = x0 + qx, y = y0 + ry;
  const bool in = x < nx && y < ny;  // nx % 4 == 0: the four x are all in or all out
  const int64_t p = ((int64_t)z * ny + y) * nx + x;
  const float* kap = gptr(reinterpret_cast<const float*>(P.kappa));
  const float* rho = gptr(reinterpret_cast<const float*>(P.rho));
  const float* S = gptr(reinterpret_cast<const float*>(P.S));
  float* J = P.J ? gptr(reinterpret_cast<float*>(P.J)) : nullptr;
  const float4 r4 = in ? *reinterpret_cast<const float4*>(rho + p) : make_float4(0, 0, 0, 0);
  double q[4] = {0, 0, 0, 0};
  double f[3][4] = {};
  // one partial array of a task (natural or [x][z][y] layout) into acc
  auto add_part = [&](const float* part, bool transposed, double (&acc)[4]) {
    if (!transposed) {
      if (in) {
        const float4 v = *reinterpret_cast<const float4*>(part + p);
        acc[0] += (double)v.x; acc[1] += (double)v.y; acc[2] += (double)v.z; acc[3] += (double)v.w;
      }
    } else {
      __syncthreads();
      // tile[xr][yc] = part[x0 + xr][z][y0 + yc], coalesced along y
      const int yc = t & 31;
      for (int xr = t >> 5; xr < 32; xr += 8) {
        const int xx = x0 + xr, yy = y0 + yc;
        if (xx < nx && yy < ny) tile[xr][yc] = part[((int64_t)xx * nz + z) * ny + yy];
      }
      __syncthreads();
      if (in) {
        acc[0] += (double)tile[qx][ry];
        acc[1] += (double)tile[qx + 1][ry];
        acc[2] += (double)tile[qx + 2][ry];
        acc[3] += (double)tile[qx + 3][ry];
      }
    }
  };
  // f[ax] += sc * v for a uniform grid axis ax: every axis gets sc or an
  // exact zero times v (no dynamic index into the register array)
  auto add_to = [&](int ax, const double (&v)[4], double sc) {
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const double w = ax == m ? sc : 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) f[m][i] += w * v[i];
    }
  };
  for (int b = 0; b < G.nbands; ++b) {
    double acc[4] = {0, 0, 0, 0};
    const double qfb = 4.0 * 3.14159265358979323846 * G.qweight[b];
    for (int k = 0; k < G.tasks_per_band; ++k) {
      const Task& T = tasks[G.task0 + b * G.tasks_per_band + k];
      const float* part = gptr(reinterpret_cast<const float*>(ws) + T.part_off);
      if (!FLUX) {
        add_part(part, T.transposed, acc);
        continue;
      }
      // flux components along (cols, rows, plane axis) of the task, mapped to x, y, z;
      // with uni the plane-axis one is mu_axis times the partial sum
      double v[4] = {0, 0, 0, 0};
      add_part(part, T.transposed, v);
      for (int i = 0; i < 4; ++i) acc[i] += v[i];
      if (T.uni) add_to(T.frame[2], v, qfb * (T.ray[0].wm[2] / T.ray[0].w));
      const float* fp = gptr(reinterpret_cast<const float*>(ws) + T.flux_off);
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        if (m == 2 && T.uni) break;
        for (int i = 0; i < 4; ++i) v[i] = 0.0;
        add_part(fp + m * N, T.transposed, v);
        add_to(T.frame[m], v, qfb);
      }
    }
    if (in) {
      const double qf = 4.0 * 3.14159265358979323846 * G.qweight[b];
      const float4 k4 = *reinterpret_cast<const float4*>(kap + b * N + p);
      const float4 s4 = *reinterpret_cast<const float4*>(S + b * N + p);
      // J - S = sum of the partials + (sum_r w_r - 1) S
      const double dj[4] = {acc[0] + G.wsum1 * (double)s4.x, acc[1] + G.wsum1 * (double)s4.y,
                            acc[2] + G.wsum1 * (double)s4.z, acc[3] + G.wsum1 * (double)s4.w};
      q[0] += qf * ((double)k4.x * (double)r4.x) * dj[0];
      q[1] += qf * ((double)k4.y * (double)r4.y) * dj[1];
      q[2] += qf * ((double)k4.z * (double)r4.z) * dj[2];
      q[3] += qf * ((double)k4.w * (double)r4.w) * dj[3];
      if (J)
        *reinterpret_cast<float4*>(J + b * N + p) =
            make_float4((float)((double)s4.x + dj[0]), (float)((double)s4.y + dj[1]),
                        (float)((double)s4.z + dj[2]), (float)((double)s4.w + dj[3]));
      if (FLUX) {
        const double sv[4] = {(double)s4.x, (double)s4.y, (double)s4.z, (double)s4.w};
        for (int m = 0; m < 3; ++m)
          for (int i = 0; i < 4; ++i) f[m][i] += qf * (sv[i] * G.msum[m]);
      }
    }
  }
  if (in) {
    double* Q = gptr(P.Q);
    *reinterpret_cast<double2*>(Q + p) = make_double2(q[0], q[1]);
    *reinterpret_cast<double2*>(Q + p + 2) = make_double2(q[2], q[3]);
    if (FLUX) {
      double* F = gptr(P.F);
      for (int m = 0; m < 3; ++m) {
        *reinterpret_cast<double2*>(F + m * N + p) = make_double2(f[m][0], f[m][1]);
        *reinterpret_cast<double2*>(F + m * N + p + 2) = make_double2(f[m][2], f[m][3]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint: the reverse sweep.
//
// Forward recursion of cell q of unrolled plane u, slot r: with B the
// bilinear interpolation at the upwind point in plane u-1,
//   x = ds/2 (chi_q + B chi),  e = exp(-x),  c = (1 - e)/x,
//   D_q = e B(D) + c (B(S) - S_q).
// With lambda_q = dL/dD_q, reverse mode gives for every integrated cell
//   A_q = e lambda_q            (flows to the upwind D),
//   Bq  = c lambda_q            (flows to the upwind S; -Bq to S_q),
//   G_q = ds/2 lambda_q dD/dx   (flows to chi_q and the upwind chi),
//   dD/dx = -e B(D) + c' (B(S) - S_q),  c' = dc/dx = (e - c)/x,
// and a cell of plane u collects from plane u+1 with the transposed
// (mirrored) bilinear weights B^T:
//   lambda_q = seed_q + B^T A,  dL/dS_q += B^T B - Bq,  dL/dchi_q += B^T G + G_q.
// A boundary cell (D = a_bc S + b_bc) adds a_bc lambda_q to dL/dS_q and
// passes nothing upwind; the ghost plane of a periodic sweep (u = -1) is such
// a plane, with D = 0 off the boundary row.  The seed of a cell in the last
// lap is w_r (4 pi qweight chi gQ + gJ) (+ gItop in the top layer).
//
// The sweep runs downwind to upwind with the strip machinery of the forward
// sweep: persistent workgroups, strips of kRevRows rows x all columns, the
// state (A, B, G) of the previous (downwind) plane in LDS, the edge rows
// exchanged as tagged words.  B^T reads rows i and i - sr, so even slots
// (upwind row i-1) take the upper neighbour's first row and odd slots the
// lower neighbour's last row.  The forward step of each cell is recomputed
// from the stored D of plane u-1 (D is kept, the weights are not).

// c' = dc/dx, power series below x = 0.1 (sum_{n>=1} n (-x)^(n-1) / (n+1)!, with sign)
__device__ inline float rts_dcw(float x, float e, float c) {
  const float s =
      fmaf(fmaf(fmaf(fmaf(x, -5.f / 720.f, 4.f / 120.f), x, -3.f / 24.f), x, 2.f / 6.f), x, -0.5f);
  const float l = (e - c) * __builtin_amdgcn_rcpf(x);
  return x < 0.1f ? s : l;
}
__device__ inline double rts_dcw(double x, double e, double c) {
  double s = -11.0 / 479001600.0;
  s = fma(s, x, 10.0 / 39916800.0);
  s = fma(s, x, -9.0 / 3628800.0);
  s = fma(s, x, 8.0 / 362880.0);
  s = fma(s, x, -7.0 / 40320.0);
  s = fma(s, x, 6.0 / 5040.0);
  s = fma(s, x, -5.0 / 720.0);
  s = fma(s, x, 4.0 / 120.0);
  s = fma(s, x, -3.0 / 24.0);
  s = fma(s, x, 2.0 / 6.0);
  s = fma(s, x, -0.5);
  if (x < 0.1) return s;
  return (e - c) / x;
}

typedef const AdjTask RTS_CONST CAdjTask;

template <class Real, int H>
struct RevStrip {
  // LDS per column: chi and S of the upwind plane u-1, rows -1..H (index
  // 0..H+1); its D per slot, rows -1..H; the downwind state A, B, G per slot
  // of the strip's rows; the two halo rows of that state (side 0: the lower
  // neighbour's last row, odd slots 1 and 3; side 1: the upper neighbour's
  // first row, even slots 0 and 2).  [column][NQP], NQP odd.
  static constexpr int R = kMaxRaysPerTask;
  static constexpr int NQ = (2 + R) * (H + 2) + 3 * R * H + 12;
  static constexpr int NQP = NQ | 1;
  __device__ static constexpr int qc(int j) { return j; }
  __device__ static constexpr int qs(int j) { return H + 2 + j; }
  __device__ static constexpr int qd(int j, int r) { return 2 * (H + 2) + R * j + r; }
  __device__ static constexpr int qw(int i, int r, int m) {
    return (2 + R) * (H + 2) + 3 * (R * i + r) + m;
  }
  __device__ static constexpr int qh(int side, int s2, int m) {
    return (2 + R) * (H + 2) + 3 * R * H + 6 * side + 3 * s2 + m;
  }
};

// One strip of one task.  SP slots per thread (4, 2 or 1): NH = 4 / SP
// threads share a column; part h takes slots h, h + NH, ... (with NH = 2 the
// even slots, which read the upper halo and publish the strip's first row,
// and the odd slots, lower halo and last row).  Threads of one part form
// whole waves, so the part is wave-uniform.
template <class Real, int H, bool FULL, int SP>
__device__ __forceinline__ void run_rev_strip(const RevArgs& A, CTask& T, CAdjTask& AT,
                                              const int strip, Real* lds) {
  using ST = RevStrip<Real, H>;
  constexpr int R = kMaxRaysPerTask;
  constexpr int NH = R / SP;  // threads per column
  using TG = Tagged<Real>;
  constexpr int NW = TG::WORDS;
  const int W = T.n_cols, nr = T.n_rows;
  const int ncol = blockDim.x / NH;  // padded columns of the block
  const int c = threadIdx.x % ncol;
  const int h = NH == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x / ncol);
  const bool act = c < W;
  const int cc = act ? c : W - 1;
  const int cm = cc > 0 ? cc - 1 : W - 1, cp1 = cc + 1 < W ? cc + 1 : 0;
  const int r0 = strip * H;
  const int hr = FULL ? H : min(H, nr - r0);
  const int ps = (int)T.plane_stride, rs = (int)T.row_stride;
  int* status = gptr(reinterpret_cast<int*>(A.ws));
  const bool zp = T.z_planes != 0;
  const bool per = T.row_periodic != 0;
  const bool has_lo = per || r0 > 0, has_hi = per || r0 + hr < nr;
  const int ns = AT.strips;
  const int st_lo = strip > 0 ? strip - 1 : ns - 1, st_hi = strip + 1 < ns ? strip + 1 : 0;
  const int na = T.n_planes;
  const int q0 = T.sa > 0 ? 0 : na - 1, q_last = T.sa > 0 ? na - 1 : 0;
  const int U = T.n_unrolled, u_init = AT.u_init;
  const int K = U - u_init;
  const int last_from = zp ? 0 : (T.laps - 1) * na;
  auto plane_of = [&](int u) { return u < 0 ? q_last : q0 + T.sa * (zp ? u : u % na); };
  // this thread's slots
  auto slot = [&](int s) { return NH * s + h; };
  Real f1[SP], f2[SP], hds[SP], wgt[SP];
  int itop[SP];
#pragma unroll
  for (int s = 0; s < SP; ++s) {
    const TaskRay RTS_CONST& y = T.ray[slot(s)];
    f1[s] = (Real)y.f1; f2[s] = (Real)y.f2; hds[s] = (Real)y.hds; wgt[s] = (Real)y.w;
    itop[s] = y.itop;
  }
  Real* ws = gptr(reinterpret_cast<Real*>(A.ws));
  const Real* chi = ws + T.chi_off;
  const Real* Sv = gptr(T.transposed ? ws + T.s_off : reinterpret_cast<const Real*>(A.S[T.box]) + T.s_off);
  const Real* Dst = ws + T.dstore_off;
  const Real* seed = ws + AT.seed_off;
  const int64_t N = (int64_t)na * nr * W;
  Real* GS = ws + AT.gs_off + h * N;  // one partial per part
  Real* GC = ws + AT.gc_off + h * N;
  uint64_t* X = gptr(reinterpret_cast<uint64_t*>(A.ws) + AT.xbuf_off);
  const Real* gI = gptr(reinterpret_cast<const Real*>(A.gItop[T.box]));
  const int64_t pc = (int64_t)nr * W;
  const int xstride = 2 * 3 * W * NW;  // one published edge row: 2 slots x 3 quantities
  const uint32_t cb = (uint32_t)cc * sizeof(Real), xb = (uint32_t)cc * NW * 8;
  Real* lc = lds + c * ST::NQP;
  const Real* lcc = lds + cc * ST::NQP;
  const Real* lcm = lds + cm * ST::NQP;
  const Real* lcp = lds + cp1 * ST::NQP;
  auto urow = [&](auto* base, int off) __attribute__((always_inline)) {
    return base + __builtin_amdgcn_readfirstlane(off);
  };
  const Real bua = (Real)T.bu_a, bub = (Real)T.bu_b, bda = (Real)T.bd_a, bdb = (Real)T.bd_b;
  const Real pla = (Real)T.pl_a;
  auto up_row = [&](int j) __attribute__((always_inline)) {
    int g = r0 - 1 + j;
    if (per) g = g < 0 ? g + nr : (g >= nr ? g - nr : g);
    else g = g < 0 ? 0 : (g >= nr ? nr - 1 : g);
    return g;
  };

  // Global inputs of a step, loaded one step ahead: of the upwind plane u-1,
  // rows -1..H of this column (rows outside a bounded plane are clamped: no
  // integrated cell reads them), chi (part 0) and S (part 1; both with one
  // part) and D of this thread's slots; of this plane, chi, S, seeds and
  // gradient partials of the strip's rows.
  constexpr int NQU = NH == 1 ? 2 : 1;
  const bool loads_cs = NH == 1 || h < 2;
  struct StepIn {
    Real upq[NQU][H + 2], upd[H + 2][SP];
    Real cpv[H], spv[H], sdv[H], gsv[H], gcv[H];
  };
  auto load_step = [&](int k, StepIn& L) __attribute__((always_inline)) {
    const int u = U - 1 - k;
    const int uu = u - 1;
    if (u >= 0 && !(zp && u == 0)) {
      const int qo = plane_of(uu) * ps;
#pragma unroll
      for (int j = 0; j < H + 2; ++j) {
        const int o = qo + up_row(j) * rs;
#pragma unroll
        for (int qq = 0; qq < NQU; ++qq) {
          const bool want_s = NH == 1 ? qq == 1 : h == 1;
          if (loads_cs) L.upq[qq][j] = *lane_at(urow(want_s ? Sv : chi, o), cb);
        }
#pragma unroll
        for (int s = 0; s < SP; ++s)
          // unconditional loads (the ghost plane reads plane 0 and ignores it)
          L.upd[j][s] = *lane_at(urow(Dst + (int64_t)(uu >= 0 ? uu : 0) * R * pc,
                                      (slot(s) * nr + up_row(j)) * W), cb);
      }
    }
    const int qp = plane_of(u);
    const bool last_lap = u >= last_from;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const int o = qp * ps + (r0 + (FULL || i < hr ? i : 0)) * rs;
      L.cpv[i] = *lane_at(urow(chi, o), cb);
      L.spv[i] = *lane_at(urow(Sv, o), cb);
      L.sdv[i] = *lane_at(urow(seed, o), cb);  // used in the last lap only
      L.gsv[i] = *lane_at(urow(GS, o), cb);
      L.gcv[i] = *lane_at(urow(GC, o), cb);
    }
  };
  // the upwind plane into LDS; D of the ghost plane is a_bc S + b_bc on the
  // slot's boundary row and 0 elsewhere (it reads S from LDS: after a barrier)
  auto commit_up = [&](int u, const StepIn& L) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < H + 2; ++j) {
#pragma unroll
      for (int qq = 0; qq < NQU; ++qq) {
        const bool is_s = NH == 1 ? qq == 1 : h == 1;
        if (loads_cs) lc[is_s ? ST::qs(j) : ST::qc(j)] = L.upq[qq][j];
      }
      if (u - 1 >= 0) {
#pragma unroll
        for (int s = 0; s < SP; ++s) lc[ST::qd(j, slot(s))] = L.upd[j][s];
      }
    }
  };
  auto ghost_d = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < H + 2; ++j)
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int r = slot(s);
        const bool up = (r & 1) == 0;
        lc[ST::qd(j, r)] = up_row(j) == (up ? 0 : nr - 1)
                               ? fmad(up ? bua : bda, lc[ST::qs(j)], up ? bub : bdb)
                               : Real(0);
      }
  };

  // neighbours' edge words of the downwind state (published at their step
  // k-1), for this thread's slots: odd slots from the lower neighbour's last
  // row (LDS side 0), even slots from the upper neighbour's first row (side 1)
  uint64_t hw[SP][3][NW];
  auto halo_issue = [&](int k) __attribute__((always_inline)) {
    const int par = (k - 1) & 1;
#pragma unroll
    for (int s = 0; s < SP; ++s) {
      const int r = slot(s);
      const int side = (r & 1) ? 0 : 1;
      const bool has = side == 0 ? has_lo : has_hi;
      // without a neighbour the strip reads its own words (ignored): no branch
      const int nb = side == 0 ? st_lo : st_hi;
      const int edge = side == 0 ? 1 : 0;
      const int xoff = ((nb * 2 + par) * 2 + edge) * xstride;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const uint64_t* rowp = urow(X, xoff + ((r >> 1) * 3 + m) * W * NW);
#pragma unroll
        for (int x = 0; x < NW; ++x) hw[s][m][x] = has ? ld_dev(lane_at(rowp, xb) + x) : 0ull;
      }
    }
  };
  auto halo_wait = [&](int k) __attribute__((always_inline)) {
    const uint32_t tag = (uint32_t)k;
    auto all_fresh = [&]() __attribute__((always_inline)) {
      bool ok = true;
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const bool has = (slot(s) & 1) ? has_lo : has_hi;
#pragma unroll
        for (int m = 0; m < 3; ++m) ok = ok && (!has || TG::fresh(hw[s][m], tag));
      }
      return ok;
    };
    if (__ballot(!all_fresh()) != 0) {
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      for (;;) {
        __builtin_amdgcn_s_sleep(1);
        halo_issue(k);
        if (__ballot(!all_fresh()) == 0) break;
        if (__builtin_amdgcn_readfirstlane(ld_dev(status)) != 0) break;
        if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > A.timeout_ticks) {
          st_dev(status, 1);
          break;
        }
      }
    }
#pragma unroll
    for (int s = 0; s < SP; ++s) {
      const int r = slot(s);
      const bool has = (r & 1) ? has_lo : has_hi;
#pragma unroll
      for (int m = 0; m < 3; ++m)
        lc[ST::qh((r & 1) ? 0 : 1, r >> 1, m)] = has ? TG::value(hw[s][m]) : Real(0);
    }
  };

  // ---- the downwind state of plane U (beyond the last plane) is zero
  lds_barrier();  // the previous strip of this workgroup has finished with the LDS
#pragma unroll
  for (int i = 0; i < H; ++i)
#pragma unroll
    for (int s = 0; s < SP; ++s)
#pragma unroll
      for (int m = 0; m < 3; ++m) lc[ST::qw(i, slot(s), m)] = Real(0);
#pragma unroll
  for (int s = 0; s < SP; ++s)
#pragma unroll
    for (int m = 0; m < 3; ++m) lc[ST::qh((slot(s) & 1) ? 0 : 1, slot(s) >> 1, m)] = Real(0);

  const int top = FULL ? H - 1 : hr - 1;
  // one step; the caller alternates the two input buffers (no register copies)
  auto step = [&](const int k, StepIn& cur, StepIn& nxt) __attribute__((always_inline)) {
    const int u = U - 1 - k;
    const int qp = plane_of(u);
    const bool ghost = u < 0;
    const bool bcplane = zp && u == 0;
    const bool last_lap = u >= last_from;
    // the next step's loads are in flight during this one
    if (k + 1 < K) load_step(k + 1, nxt);
    if (k > 0) halo_wait(k);
    if (!ghost && !bcplane) commit_up(u, cur);
    lds_barrier();  // halo rows, upwind plane and downwind state complete
    if (u == 0 && !zp) {
      ghost_d();  // upwind D of the first plane from the ghost plane's S
      lds_barrier();
    }

    Real nst[H][SP][3];
    auto do_row = [&](int i) __attribute__((always_inline)) {
      const int gi = r0 + i;
      const int j = i + 1;  // LDS row of this cell in the upwind plane
      Real gs = 0, gc = 0;
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int r = slot(s);
        const bool up = (r & 1) == 0;  // upwind row i-1 (even slots) or i+1 (odd)
        const Real* cn = r < 2 ? lcp : lcm;  // downwind column c - sc
        // B^T of the downwind state: rows i and i - sr
        Real tq[3];
        const int io = up ? i + 1 : i - 1;
        const bool in_strip = io >= 0 && io < (FULL ? H : hr);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const Real v0 = lerp(lcc[ST::qw(i, r, m)], cn[ST::qw(i, r, m)], f1[s]);
          const int qo_ = in_strip ? ST::qw(in_strip ? io : 0, r, m) : ST::qh(up ? 1 : 0, r >> 1, m);
          const Real v1 = lerp(lcc[qo_], cn[qo_], f1[s]);
          tq[m] = lerp(v0, v1, f2[s]);
        }
        Real lam = fmad(wgt[s], last_lap ? cur.sdv[i] : Real(0), tq[0]);
        if (last_lap && gI && itop[s] >= 0 && (zp ? qp == T.it_top : gi == T.it_top))
          lam += gI[T.it_off + itop[s] * T.it_ray + (int64_t)qp * T.itp + (int64_t)gi * T.itr +
                    (int64_t)cc * T.itc];
        // Branch-free: the forward step is recomputed for every cell (the LDS
        // rows it reads always hold finite values) and selected away for
        // boundary cells, D = coef S + const, which pass coef lambda to S.
        const int br = up ? 0 : nr - 1;
        const Real bca = up ? bua : bda;
        const bool bc_row = !zp && gi == br;
        const bool comp = !ghost && !bcplane && !bc_row;
        const Real coef = ghost ? (gi == br ? bca : Real(0)) : (bcplane ? pla : bca);
        Real a = 0, b = 0, g = 0;
        // (FP64 keeps the branch: its longer recompute would cost registers)
        if (sizeof(Real) == 4 || comp) {
          const int ju = up ? j - 1 : j + 1;
          const Real* cu = r < 2 ? lcm : lcp;  // upwind column c + sc
          const Real bcx = lerp(lerp(lcc[ST::qc(j)], cu[ST::qc(j)], f1[s]),
                                lerp(lcc[ST::qc(ju)], cu[ST::qc(ju)], f1[s]), f2[s]);
          const Real bsx = lerp(lerp(lcc[ST::qs(j)], cu[ST::qs(j)], f1[s]),
                                lerp(lcc[ST::qs(ju)], cu[ST::qs(ju)], f1[s]), f2[s]);
          const Real bdx = lerp(lerp(lcc[ST::qd(j, r)], cu[ST::qd(j, r)], f1[s]),
                                lerp(lcc[ST::qd(ju, r)], cu[ST::qd(ju, r)], f1[s]), f2[s]);
          const Real x = hds[s] * (cur.cpv[i] + bcx);
          const Real e = rts_exp_neg(x);
          const Real cw = rts_cw(x, e);
          const Real dc = rts_dcw(x, e, cw);
          a = comp ? e * lam : Real(0);
          b = comp ? cw * lam : Real(0);
          g = comp ? hds[s] * lam * fmad(-e, bdx, dc * (bsx - cur.spv[i])) : Real(0);
        }
        gs = fmad(comp ? Real(0) : coef, lam, gs) - b + tq[1];
        gc += g + tq[2];
        nst[i][s][0] = a;
        nst[i][s][1] = b;
        nst[i][s][2] = g;
      }
      if (act) {
        const int o = qp * ps + gi * rs;
        *lane_at(urow(GS, o), cb) = cur.gsv[i] + gs;
        *lane_at(urow(GC, o), cb) = cur.gcv[i] + gc;
      }
    };
    // edge rows first (they are published), then the interior
    do_row(0);
    if (top > 0) {
#pragma unroll
      for (int i = 1; i < H; ++i)
        if (i == top) do_row(i);
    }
    if (act && k + 1 < K) {
      const int xe = ((strip * 2 + (k & 1)) * 2) * xstride;
      const uint32_t tag = (uint32_t)(k + 1);
#pragma unroll
      for (int s = 0; s < SP; ++s) {
        const int r = slot(s);
        const bool even = (r & 1) == 0;
        Real v[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          v[m] = nst[0][s][m];
          if (!even) {
#pragma unroll
            for (int i = 1; i < H; ++i)
              if (i == top) v[m] = nst[i][s][m];
          }
          // edge 0: first row, even slots; edge 1: last row, odd slots
          TG::put(lane_at(urow(X, xe + (even ? 0 : xstride) + ((r >> 1) * 3 + m) * W * NW), xb), v[m], tag);
        }
      }
    }
#pragma unroll
    for (int i = 1; i < H - 1; ++i)
      if (i < top) do_row(i);
    lds_barrier();  // every thread has read the downwind state and the upwind plane
#pragma unroll
    for (int i = 0; i < H; ++i)
#pragma unroll
      for (int s = 0; s < SP; ++s)
#pragma unroll
        for (int m = 0; m < 3; ++m)
          lc[ST::qw(i, slot(s), m)] = (FULL || i < hr) ? nst[i][s][m] : Real(0);
    // the neighbours publish their edge rows of this step at about the same
    // time as this strip (two-row strips have no interior rows in between):
    // their words are loaded last, so that they are fresh more often
    if (k + 1 < K) halo_issue(k + 1);
  };
  StepIn s0, s1;
  load_step(0, s0);
  for (int k = 0; k < K; k += 2) {
    step(k, s0, s1);
    if (k + 1 < K) step(k + 1, s1, s0);
  }
}

// MAXT: the block-size bound; SP: slots per thread (2: two threads per column)
template <class Real, int MAXT, int SP>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(1, 1024 / MAXT * 2)))
void rts_reverse(RevArgs A) {
  extern __shared__ char smem_raw[];
  Real* lds = reinterpret_cast<Real*>(smem_raw);
  __shared__ int sh_ticket;
  WsHeader* hdr = reinterpret_cast<WsHeader*>(A.ws);
  constexpr int H = kRevRows;
  for (;;) {
    if (threadIdx.x == 0) sh_ticket = atomicAdd(&hdr->ticket_rev[A.wclass], 1);
    __syncthreads();
    const int tk = __builtin_amdgcn_readfirstlane(sh_ticket);
    __syncthreads();
    if (tk >= A.total_strips) return;
    CInt* queue = (CInt*)(uintptr_t)A.queue;
    int qi = 0;
    while (qi + 1 < A.ntasks && queue[2 * (qi + 1)] <= tk) ++qi;
    const int ai = queue[2 * qi + 1];
    CAdjTask& AT = ((CAdjTask*)(uintptr_t)A.atasks)[ai];
    CTask& T = ((CTask*)(uintptr_t)A.tasks)[AT.task];
    const int strip = tk - queue[2 * qi];
    if ((strip + 1) * H <= T.n_rows) run_rev_strip<Real, H, true, SP>(A, T, AT, strip, lds);
    else run_rev_strip<Real, H, false, SP>(A, T, AT, strip, lds);
  }
}

// Seeds of one band, w_r aside: 4 pi qweight chi gQ + gJ, in [z][y][x] and
// in the [x][z][y] layout of the x-sweeps.
template <class Real>
__global__ __launch_bounds__(256) void rts_adj_seed(const Real* __restrict__ kappa,
                                                   const Real* __restrict__ rho,
                                                   const double* __restrict__ gQ,
                                                   const Real* __restrict__ gJ,
                                                   Real* __restrict__ seed, Real* __restrict__ seedT,
                                                   double qf, int nx, int ny, int nz) {
  __shared__ Real tl[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
  for (int i = 0; i < 4; ++i) {
    const int y = y0 + ty + 8 * i, x = x0 + tx;
    if (x < nx && y < ny) {
      const int64_t p = ((int64_t)z * ny + y) * nx + x;
      double v = 0;
      if (gQ) v = qf * (double)(kappa[p] * rho[p]) * gQ[p];
      if (gJ) v += (double)gJ[p];
      seed[p] = (Real)v;
      tl[ty + 8 * i][tx] = (Real)v;
    }
  }
  __syncthreads();
  for (int i = 0; i < 4; ++i) {
    const int x = x0 + ty + 8 * i, y = y0 + tx;
    if (x < nx && y < ny) seedT[((int64_t)x * nz + z) * ny + y] = tl[tx][ty + 8 * i];
  }
}

// Gradients of one box: the task partials (one per part of the reverse
// sweep's threads of a column) summed in a fixed order (FP64),
// plus the direct terms dL/dS_b += gJ_b (+ sum_r gItop_b,r in the top layer)
// and dL/dchi_b += 4 pi qweight_b (J_b - S_b) gQ, where J_b - S_b is the sum
// of the forward partials.
template <class Real>
__global__ __launch_bounds__(256) void rts_adj_reduce(const char* __restrict__ ws,
                                                     const Task* __restrict__ tasks,
                                                     const AdjTask* __restrict__ atasks, BoxGeo G,
                                                     const double* __restrict__ gQ,
                                                     const Real* __restrict__ gJ,
                                                     const Real* __restrict__ gItop,
                                                     const Real* __restrict__ S,
                                                     Real* __restrict__ dS, Real* __restrict__ dchi) {
  __shared__ double t0[32][33], t1[32][33], t2[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int64_t N = (int64_t)nx * ny * nz;
  const Real* w = reinterpret_cast<const Real*>(ws);
  const Real* chi = w + G.chi_off;
  for (int b = 0; b < G.nbands; ++b) {
    double as[4] = {0, 0, 0, 0}, ac[4] = {0, 0, 0, 0}, aj[4] = {0, 0, 0, 0};
    for (int k = 0; k < G.tasks_per_band; ++k) {
      const int ti = G.task0 + b * G.tasks_per_band + k;
      const Task& T = tasks[ti];
      const AdjTask& AT = atasks[ti];
      const Real* gs = w + AT.gs_off;
      const Real* gc = w + AT.gc_off;
      const Real* pj = w + T.part_off;
      if (!T.transposed) {
        for (int i = 0; i < 4; ++i) {
          const int y = y0 + ty + 8 * i, x = x0 + tx;
          if (x < nx && y < ny) {
            const int64_t p = ((int64_t)z * ny + y) * nx + x;
            for (int h = 0; h < AT.nparts; ++h) {
              as[i] += (double)gs[p + h * N];
              ac[i] += (double)gc[p + h * N];
            }
            aj[i] += (double)pj[p];
          }
        }
      } else {
        __syncthreads();
        for (int i = 0; i < 4; ++i) {
          const int x = x0 + ty + 8 * i, y = y0 + tx;
          if (x < nx && y < ny) {
            const int64_t p = ((int64_t)x * nz + z) * ny + y;
            double vs = 0, vc = 0;
            for (int h = 0; h < AT.nparts; ++h) {
              vs += (double)gs[p + h * N];
              vc += (double)gc[p + h * N];
            }
            t0[ty + 8 * i][tx] = vs;
            t1[ty + 8 * i][tx] = vc;
            t2[ty + 8 * i][tx] = (double)pj[p];
          }
        }
        __syncthreads();
        for (int i = 0; i < 4; ++i) {
          const int y = y0 + ty + 8 * i, x = x0 + tx;
          if (x < nx && y < ny) {
            as[i] += t0[tx][ty + 8 * i];
            ac[i] += t1[tx][ty + 8 * i];
            aj[i] += t2[tx][ty + 8 * i];
          }
        }
      }
    }
    const double qf = 4.0 * 3.14159265358979323846 * G.qweight[b];
    for (int i = 0; i < 4; ++i) {
      const int y = y0 + ty + 8 * i, x = x0 + tx;
      if (x < nx && y < ny) {
        const int64_t p = ((int64_t)z * ny + y) * nx + x;
        double vs = as[i], vc = ac[i];
        // direct terms of J_b = (1 + wsum1) S_b + sum_r w_r D_r and
        // Q = sum_b 4 pi qw_b chi_b (wsum1 S_b + sum_r w_r D_r)
        const double sv = G.wsum1 != 0.0 ? (double)S[b * N + p] : 0.0;
        const double cv = G.wsum1 != 0.0 ? (double)chi[b * N + p] : 0.0;
        if (gJ) vs += (1.0 + G.wsum1) * (double)gJ[b * N + p];
        if (gItop && z == nz - 1)
          for (int r = 0; r < G.n_up; ++r)
            vs += (double)gItop[(((int64_t)b * G.n_up + r) * ny + y) * nx + x];
        if (gQ) {
          vc += qf * (aj[i] + G.wsum1 * sv) * gQ[p];
          vs += qf * G.wsum1 * cv * gQ[p];
        }
        dS[b * N + p] = (Real)vs;
        dchi[b * N + p] = (Real)vc;
      }
    }
  }
}

// The same with 16-byte accesses, for FP32 and nx a multiple of 4: a thread
// owns four consecutive x of one row; partials of x-sweeps go through LDS.
__global__ __launch_bounds__(256) void rts_adj_reduce_v4(const char* __restrict__ ws,
                                                        const Task* __restrict__ tasks,
                                                        const AdjTask* __restrict__ atasks,
                                                        BoxGeo G, const double* __restrict__ gQ,
                                                        const float* __restrict__ gJ,
                                                        const float* __restrict__ gItop,
                                                        const float* __restrict__ S,
                                                        float* __restrict__ dS,
                                                        float* __restrict__ dchi) {
  __shared__ double t0[32][33], t1[32][33], t2[32][33];
  const int t = threadIdx.x;
  const int qx = (t & 7) * 4, ry = t >> 3;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int64_t N = (int64_t)nx * ny * nz;
  const int x = x0 + qx, y = y0 + ry;
  const bool in = x < nx && y < ny;
  const int64_t p = ((int64_t)z * ny + y) * nx + x;
  const float* w = gptr(reinterpret_cast<const float*>(ws));
  for (int b = 0; b < G.nbands; ++b) {
    double as[4] = {0, 0, 0, 0}, ac[4] = {0, 0, 0, 0}, aj[4] = {0, 0, 0, 0};
    for (int k = 0; k < G.tasks_per_band; ++k) {
      const int ti = G.task0 + b * G.tasks_per_band + k;
      const Task& T = tasks[ti];
      const AdjTask& AT = atasks[ti];
      const float* gs = w + AT.gs_off;
      const float* gc = w + AT.gc_off;
      const float* pj = w + T.part_off;
      if (!T.transposed) {
        if (in) {
          for (int h = 0; h < AT.nparts; ++h) {
            const float4 a = *reinterpret_cast<const float4*>(gs + p + h * N);
            const float4 c = *reinterpret_cast<const float4*>(gc + p + h * N);
            as[0] += (double)a.x; as[1] += (double)a.y; as[2] += (double)a.z; as[3] += (double)a.w;
            ac[0] += (double)c.x; ac[1] += (double)c.y; ac[2] += (double)c.z; ac[3] += (double)c.w;
          }
          const float4 j = *reinterpret_cast<const float4*>(pj + p);
          aj[0] += (double)j.x; aj[1] += (double)j.y; aj[2] += (double)j.z; aj[3] += (double)j.w;
        }
      } else {
        __syncthreads();
        const int yc = t & 31;
        for (int xr = t >> 5; xr < 32; xr += 8) {
          const int xx = x0 + xr, yy = y0 + yc;
          if (xx < nx && yy < ny) {
            const int64_t q = ((int64_t)xx * nz + z) * ny + yy;
            double vs = 0, vc = 0;
            for (int h = 0; h < AT.nparts; ++h) {
              vs += (double)gs[q + h * N];
              vc += (double)gc[q + h * N];
            }
            t0[xr][yc] = vs;
            t1[xr][yc] = vc;
            t2[xr][yc] = (double)pj[q];
          }
        }
        __syncthreads();
        if (in) {
          for (int e = 0; e < 4; ++e) {
            as[e] += t0[qx + e][ry];
            ac[e] += t1[qx + e][ry];
            aj[e] += t2[qx + e][ry];
          }
        }
      }
    }
    if (in) {
      const double qf = 4.0 * 3.14159265358979323846 * G.qweight[b];
      double vs[4] = {as[0], as[1], as[2], as[3]}, vc[4] = {ac[0], ac[1], ac[2], ac[3]};
      // direct terms of J_b = (1 + wsum1) S_b + sum_r w_r D_r and
      // Q = sum_b 4 pi qw_b chi_b (wsum1 S_b + sum_r w_r D_r)
      const double wj = 1.0 + G.wsum1;
      double sv[4] = {0, 0, 0, 0}, cv[4] = {0, 0, 0, 0};
      if (G.wsum1 != 0.0) {
        const float4 s4 = *reinterpret_cast<const float4*>(S + b * N + p);
        const float4 c4 = *reinterpret_cast<const float4*>(w + G.chi_off + b * N + p);
        sv[0] = s4.x; sv[1] = s4.y; sv[2] = s4.z; sv[3] = s4.w;
        cv[0] = c4.x; cv[1] = c4.y; cv[2] = c4.z; cv[3] = c4.w;
      }
      if (gJ) {
        const float4 j = *reinterpret_cast<const float4*>(gJ + b * N + p);
        vs[0] += wj * (double)j.x; vs[1] += wj * (double)j.y;
        vs[2] += wj * (double)j.z; vs[3] += wj * (double)j.w;
      }
      if (gItop && z == nz - 1)
        for (int r = 0; r < G.n_up; ++r) {
          const float4 g = *reinterpret_cast<const float4*>(gItop + (((int64_t)b * G.n_up + r) * ny + y) * nx + x);
          vs[0] += (double)g.x; vs[1] += (double)g.y; vs[2] += (double)g.z; vs[3] += (double)g.w;
        }
      if (gQ) {
        const double2 q01 = *reinterpret_cast<const double2*>(gQ + p);
        const double2 q23 = *reinterpret_cast<const double2*>(gQ + p + 2);
        const double gq[4] = {q01.x, q01.y, q23.x, q23.y};
        for (int e = 0; e < 4; ++e) {
          vc[e] += qf * (aj[e] + G.wsum1 * sv[e]) * gq[e];
          vs[e] += qf * G.wsum1 * cv[e] * gq[e];
        }
      }
      *reinterpret_cast<float4*>(dS + b * N + p) =
          make_float4((float)vs[0], (float)vs[1], (float)vs[2], (float)vs[3]);
      *reinterpret_cast<float4*>(dchi + b * N + p) =
          make_float4((float)vc[0], (float)vc[1], (float)vc[2], (float)vc[3]);
    }
  }
}

}  // namespace rts

// ---------------------------------------------------------------------------
// launch wrappers used by the host planner

namespace rts {

template <class Real>
hipError_t launch_prep(const void* kappa, const void* rho, const void* S, void* ws, int64_t chi_off,
                       int64_t chiT_off, int64_t sT_off, int nx, int ny, int nz, int nb,
                       hipStream_t st) {
  dim3 grid((nx + 31) / 32, (ny + 31) / 32, nz * nb);
  Real* base = reinterpret_cast<Real*>(ws);
  hipLaunchKernelGGL(rts_prep<Real>, grid, dim3(256), 0, st, (const Real*)kappa, (const Real*)rho,
                     (const Real*)S, base + chi_off, base + chiT_off, base + sT_off, nx, ny, nz);
  return hipGetLastError();
}

hipError_t launch_zero(int* p, int64_t n, hipStream_t st) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(rts_zero_ints, dim3(blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

template <class Real, int H>
size_t sweep_lds_bytes(int threads) {
  return (size_t)Strip<Real, H>::NQP * threads * sizeof(Real);
}

template <class Real, int H, bool UNI>
const void* sweep_fn() {
  return reinterpret_cast<const void*>(&rts_sweep<Real, H, UNI, 0>);
}

template <class Real, int H, bool UNI>
const void* sweep_fn_ext(int ext) {
  return ext == 2 ? reinterpret_cast<const void*>(&rts_sweep<Real, H, UNI, 2>)
                  : reinterpret_cast<const void*>(&rts_sweep<Real, H, UNI, 1>);
}

template <class Real, int H, bool UNI>
hipError_t launch_sweep_h(const SweepArgs& a, int grid, int threads, hipStream_t st) {
  // (the occupancy estimate takes the smallest of the three variants)
  const size_t lds = sweep_lds_bytes<Real, H>(threads);
  if (a.ext == 2) rts_sweep<Real, H, UNI, 2><<<dim3(grid), dim3(threads), lds, st>>>(a);
  else if (a.ext == 1) rts_sweep<Real, H, UNI, 1><<<dim3(grid), dim3(threads), lds, st>>>(a);
  else rts_sweep<Real, H, UNI, 0><<<dim3(grid), dim3(threads), lds, st>>>(a);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_reduce(const char* ws, const Task* tasks, const BoxGeo& g, const BoxPtrs& p,
                         hipStream_t st) {
  dim3 grid((g.nx + 31) / 32, (g.ny + 31) / 32, g.nz);
  const uintptr_t al = (uintptr_t)p.kappa | (uintptr_t)p.rho | (uintptr_t)p.S |
                       (uintptr_t)p.J | (uintptr_t)p.Q | (uintptr_t)p.F;
  if (sizeof(Real) == 4 && g.nx % 4 == 0 && al % 16 == 0) {
    // 16-byte accesses; with F, the flux sums in the same pass
    if (p.F) hipLaunchKernelGGL(rts_reduce_v4<true>, grid, dim3(256), 0, st, ws, tasks, g, p);
    else hipLaunchKernelGGL(rts_reduce_v4<false>, grid, dim3(256), 0, st, ws, tasks, g, p);
  } else {
    hipLaunchKernelGGL(rts_reduce<Real>, grid, dim3(256), 0, st, ws, tasks, g, p);
    if (p.F)
      hipLaunchKernelGGL(rts_reduce_flux<Real>, grid, dim3(256), 0, st, ws, tasks, g,
                         reinterpret_cast<const Real*>(p.S), p.F);
  }
  if (p.F && p.QF)
    hipLaunchKernelGGL(rts_flux_div, dim3((unsigned)(((int64_t)g.nx * g.ny * g.nz + 255) / 256)),
                       dim3(256), 0, st, p.F, p.QF, g.nx, g.ny, g.nz, 1.0 / g.dx, 1.0 / g.dy,
                       1.0 / g.dz);
  return hipGetLastError();
}

// Reverse sweep launch shape for `cols` padded columns: up to 256 columns,
// two threads per column (two slots each) in a block of at most 512 threads;
// up to 512 columns, one thread per column (four slots) in 512 threads; above,
// one thread per column in 1024 threads.  A block bound of 512 allows 256
// VGPRs per lane, which the four-slot state nearly fills; 1024 allows 128 and
// spills.
template <class Real>
size_t reverse_lds_bytes(int cols) {
  return (size_t)RevStrip<Real, kRevRows>::NQP * cols * sizeof(Real);
}

int reverse_parts(int cols) { return cols <= 256 ? 2 : 1; }
int reverse_threads(int cols) { return reverse_parts(cols) * cols; }

template <class Real>
const void* reverse_fn(int cols) {
  if (cols <= 256) return reinterpret_cast<const void*>(&rts_reverse<Real, 512, 2>);
  if (cols <= 512) return reinterpret_cast<const void*>(&rts_reverse<Real, 512, 4>);
  return reinterpret_cast<const void*>(&rts_reverse<Real, 1024, 4>);
}

template <class Real>
hipError_t launch_reverse(const RevArgs& a, int grid, int cols, hipStream_t st) {
  const size_t lds = reverse_lds_bytes<Real>(cols);
  const dim3 b(reverse_threads(cols));
  if (cols <= 256) rts_reverse<Real, 512, 2><<<dim3(grid), b, lds, st>>>(a);
  else if (cols <= 512) rts_reverse<Real, 512, 4><<<dim3(grid), b, lds, st>>>(a);
  else rts_reverse<Real, 1024, 4><<<dim3(grid), b, lds, st>>>(a);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_adj_seed(const void* kappa, const void* rho, const double* gQ, const void* gJ,
                           void* seed, void* seedT, double qf, int nx, int ny, int nz,
                           hipStream_t st) {
  dim3 grid((nx + 31) / 32, (ny + 31) / 32, nz);
  hipLaunchKernelGGL(rts_adj_seed<Real>, grid, dim3(256), 0, st, (const Real*)kappa,
                     (const Real*)rho, gQ, (const Real*)gJ, (Real*)seed, (Real*)seedT, qf, nx, ny,
                     nz);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_adj_reduce(const char* ws, const Task* tasks, const AdjTask* atasks,
                             const BoxGeo& g, const double* gQ, const void* gJ, const void* gItop,
                             const void* S, void* dS, void* dchi, hipStream_t st) {
  dim3 grid((g.nx + 31) / 32, (g.ny + 31) / 32, g.nz);
  const uintptr_t al = (uintptr_t)gQ | (uintptr_t)gJ | (uintptr_t)gItop | (uintptr_t)S |
                       (uintptr_t)dS | (uintptr_t)dchi;
  if (sizeof(Real) == 4 && g.nx % 4 == 0 && al % 16 == 0)
    hipLaunchKernelGGL(rts_adj_reduce_v4, grid, dim3(256), 0, st, ws, tasks, atasks, g, gQ,
                       (const float*)gJ, (const float*)gItop, (const float*)S, (float*)dS,
                       (float*)dchi);
  else
    hipLaunchKernelGGL(rts_adj_reduce<Real>, grid, dim3(256), 0, st, ws, tasks, atasks, g, gQ,
                       (const Real*)gJ, (const Real*)gItop, (const Real*)S, (Real*)dS,
                       (Real*)dchi);
  return hipGetLastError();
}


// explicit instantiations
template hipError_t launch_prep<float>(const void*, const void*, const void*, void*, int64_t,
                                       int64_t, int64_t, int, int, int, int, hipStream_t);
template hipError_t launch_prep<double>(const void*, const void*, const void*, void*, int64_t,
                                        int64_t, int64_t, int, int, int, int, hipStream_t);
template hipError_t launch_reduce<float>(const char*, const Task*, const BoxGeo&, const BoxPtrs&,
                                         hipStream_t);
template hipError_t launch_reduce<double>(const char*, const Task*, const BoxGeo&, const BoxPtrs&,
                                          hipStream_t);

#define RTS_ADJ_INST(Real)                                                                      \
  template size_t reverse_lds_bytes<Real>(int);                                                 \
  template const void* reverse_fn<Real>(int);                                                   \
  template hipError_t launch_reverse<Real>(const RevArgs&, int, int, hipStream_t);              \
  template hipError_t launch_adj_seed<Real>(const void*, const void*, const double*, const void*, \
                                            void*, void*, double, int, int, int, hipStream_t);  \
  template hipError_t launch_adj_reduce<Real>(const char*, const Task*, const AdjTask*,          \
                                              const BoxGeo&, const double*, const void*,         \
                                              const void*, const void*, void*, void*, hipStream_t);
RTS_ADJ_INST(float)
RTS_ADJ_INST(double)
#undef RTS_ADJ_INST
#define RTS_INST(Real, H)                                                                   \
  template hipError_t launch_sweep_h<Real, H, true>(const SweepArgs&, int, int, hipStream_t); \
  template hipError_t launch_sweep_h<Real, H, false>(const SweepArgs&, int, int, hipStream_t); \
  template size_t sweep_lds_bytes<Real, H>(int);                                            \
  template const void* sweep_fn<Real, H, true>();                                           \
  template const void* sweep_fn<Real, H, false>();                                          \
  template const void* sweep_fn_ext<Real, H, true>(int);                                    \
  template const void* sweep_fn_ext<Real, H, false>(int);
RTS_INST(float, 2)
RTS_INST(float, 4)
RTS_INST(float, 6)
RTS_INST(float, 8)
RTS_INST(double, 2)
RTS_INST(double, 4)
#undef RTS_INST

}  // namespace rts
