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
//                    task's sweep plane.  Each thread owns one column and H
//                    rows in registers, marches plane by plane (periodic
//                    directions: n_iter laps), and exchanges its edge rows
//                    with the neighbouring strips through the workspace and
//                    per-strip progress flags.  Column neighbours come from
//                    DPP lane shifts, with the wave-edge lanes patched from a
//                    small LDS table.  It sweeps D = I - S (see rts.h).
//  * rts_reduce    : FP64 sum of the per-task partial J - S arrays in a fixed
//                    order, Q, J (the paper's "flux" step).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rts_internal.h"

namespace rts {

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

// DPP whole-wave shifts: lane i receives lane i-1 (shr) or lane i+1 (shl);
// the lane with no source keeps `old`.
__device__ inline float dpp_shr(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ inline float dpp_shl(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ inline double dpp_shr(double old, double v) {
  int2 o = *reinterpret_cast<int2*>(&old), s = *reinterpret_cast<int2*>(&v);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(o.x, s.x, 0x138, 0xf, 0xf, false);
  r.y = __builtin_amdgcn_update_dpp(o.y, s.y, 0x138, 0xf, 0xf, false);
  return *reinterpret_cast<double*>(&r);
}
__device__ inline double dpp_shl(double old, double v) {
  int2 o = *reinterpret_cast<int2*>(&old), s = *reinterpret_cast<int2*>(&v);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(o.x, s.x, 0x130, 0xf, 0xf, false);
  r.y = __builtin_amdgcn_update_dpp(o.y, s.y, 0x130, 0xf, 0xf, false);
  return *reinterpret_cast<double*>(&r);
}

// a + f (b - a) as one explicit fused multiply-add (the library is built with
// -ffp-contract=off, so every fusion is written out and the arithmetic of a
// cell does not depend on how the compiler schedules a template instance).
__device__ inline float lerp(float a, float b, float f) { return fmaf(f, b - a, a); }
__device__ inline double lerp(double a, double b, double f) { return fma(f, b - a, a); }
__device__ inline float fmad(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline double fmad(double a, double b, double c) { return fma(a, b, c); }

// Error-free sum s + t = u + err (Knuth).
template <class R>
__device__ inline void two_sum(R s, R t, R& u, R& err) {
  u = s + t;
  R bp = u - s;
  err = (s - (u - bp)) + (t - bp);
}

// Cross-workgroup traffic of the sweep (edge rows and progress flags) uses
// only device-coherent accesses: relaxed agent-scope atomic loads and stores,
// which gfx950 issues with the sc1 bit, so they neither read nor leave stale
// lines in the non-coherent per-XCD L2.  Ordering is explicit: a producer's
// edge-row stores complete (s_waitcnt vmcnt(0)) before the workgroup barrier
// that precedes its flag store; a consumer issues its edge-row loads only
// after its flag load returned the awaited value.  No cache-wide writeback or
// invalidate is needed, which an agent-scope fence would cost at every plane.
template <class R>
__device__ inline R ld_dev(const R* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class R>
__device__ inline void st_dev(R* p, R v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void vmem_drain() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ inline int ld_flag(const int* p) { return ld_dev(p); }

// Wait until the given flags reach `need` (null flags are skipped).  Bounded:
// after `limit` ticks of the constant real-time clock the device status is set
// and every later wait returns at once, so every wave always finishes.
__device__ inline void wait_flags(const int* fa, const int* fb, int need, int* status,
                                  int64_t limit) {
  uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (;;) {
    int ok = 1;
    if (fa) ok &= __builtin_amdgcn_readfirstlane(ld_flag(fa)) >= need;
    if (fb) ok &= __builtin_amdgcn_readfirstlane(ld_flag(fb)) >= need;
    if (ok) break;
    if (__builtin_amdgcn_readfirstlane(ld_flag(status)) != 0) break;
    if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > limit) {
      st_dev(status, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  asm volatile("" ::: "memory");
}

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
  // LDS table entry of one lane: chi and S of rows -1..H, then D of rows 0..H-1 per ray
  static constexpr int NS = 2 * (H + 2) + kMaxRaysPerTask * H;
};

// One strip of one task: H rows x all columns of the task's sweep plane,
// marched through every plane (and lap) of the task.
//
// Ray slots are fixed: slot k has its upwind column at c-1 for k < 2 (else
// c+1) and its upwind row at i-1 for even k (else i+1).  With UNI the four
// slots share f1, f2, ds and w, so the column interpolation of chi and S is
// shared by the two slots with the same column direction.
//
// State carried from plane to plane is raw: chi and S of the strip's rows and
// of the two halo rows, and D of every row and slot.  The interpolation to the
// upwind point of the next plane is done at step time, row by row: along the
// columns with DPP lane shifts (wave-edge lanes patched from the LDS table),
// along the rows from registers (halo rows: chi and S loaded, D from the
// neighbouring strips' published edge rows).
template <class Real, int H, bool UNI>
__device__ __forceinline__ void run_strip(const SweepArgs& A, const Task& T, const int strip,
                                          Real* tab, int& phase) {
  constexpr int R = kMaxRaysPerTask;
  constexpr int NS = Strip<Real, H>::NS;
  constexpr int NC = UNI ? 2 : R;  // distinct column-interpolated chi/S per row
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int W = T.n_cols;
  const int c = threadIdx.x;
  const bool act = c < W;
  const int cc = act ? c : W - 1;
  const int nwt = (W + 63) >> 6;  // waves that hold columns of this task
  const int last_lane = (wv == nwt - 1) ? (W - 1 - 64 * (nwt - 1)) : 63;
  const int r0 = strip * T.rows_per_strip;
  const int hr = min(T.rows_per_strip, T.n_rows - r0);
  const int64_t ps = T.plane_stride, rs = T.row_stride;
  int* status = reinterpret_cast<int*>(A.ws);

  Real f1[R], f2[R], hds[R], wgt[R];
  int itop[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const TaskRay& y = T.ray[UNI ? 0 : r];
    f1[r] = (Real)y.f1; f2[r] = (Real)y.f2; hds[r] = (Real)y.hds; wgt[r] = (Real)y.w;
    itop[r] = T.ray[r].itop;
  }
  // boundary values D = a S + b: boundary plane (planes are z), or the boundary
  // row of the up (even slots, row 0) and down (odd slots, last row) rays
  const Real pla = (Real)T.pl_a, plb = (Real)T.pl_b;
  const Real bua = (Real)T.bu_a, bub = (Real)T.bu_b;
  const Real bda = (Real)T.bd_a, bdb = (Real)T.bd_b;
  const bool zp = T.z_planes != 0;
  const int bc_up = zp ? -1 : 0, bc_dn = zp ? -1 : T.n_rows - 1;

  const Real* chi = reinterpret_cast<const Real*>(A.ws) + T.chi_off;
  const Real* Sv = T.transposed ? reinterpret_cast<const Real*>(A.ws) + T.s_off
                                : reinterpret_cast<const Real*>(A.box[T.box].S) + T.s_off;
  Real* P = reinterpret_cast<Real*>(A.ws) + T.part_off;
  Real* X = reinterpret_cast<Real*>(A.ws) + T.xbuf_off;
  int* flags = reinterpret_cast<int*>(A.ws) + T.flag_off;
  Real* Itop = reinterpret_cast<Real*>(A.box[T.box].I_top);

  const int ns = T.strips;
  const bool per = T.row_periodic != 0;
  const bool has_lo = per || r0 > 0;
  const bool has_hi = per || r0 + hr < T.n_rows;
  const int row_lo = r0 > 0 ? r0 - 1 : T.n_rows - 1;
  const int row_hi = r0 + hr < T.n_rows ? r0 + hr : 0;
  const int st_lo = strip > 0 ? strip - 1 : ns - 1;
  const int st_hi = strip + 1 < ns ? strip + 1 : 0;
  const int* flag_lo = has_lo ? flags + st_lo : nullptr;
  const int* flag_hi = has_hi ? flags + st_hi : nullptr;
  const int64_t xstride = (int64_t)R * W;  // one published edge row, all slots

  const int na = T.n_planes;
  const int q0 = T.sa > 0 ? 0 : na - 1;
  const int q_last = T.sa > 0 ? na - 1 : 0;
  const int nsteps = zp ? na - 1 : T.laps * na;
  const int out_from = zp ? 0 : (T.laps - 1) * na;
  const int wl = wv > 0 ? wv - 1 : nwt - 1, wr = wv + 1 < nwt ? wv + 1 : 0;
  const int cm = cc > 0 ? cc - 1 : W - 1, cp1 = cc + 1 < W ? cc + 1 : 0;

  // raw state of the last computed plane (index 0: lower halo, 1..H: rows, H+1: upper halo)
  Real cx[H + 2], sx[H + 2], D[H][R];
#pragma unroll
  for (int i = 0; i < H + 2; ++i) cx[i] = sx[i] = Real(0);
#pragma unroll
  for (int i = 0; i < H; ++i)
#pragma unroll
    for (int r = 0; r < R; ++r) D[i][r] = Real(0);

  for (int t = -1; t < nsteps; ++t) {
    const int q = t < 0 ? (zp ? q0 : q_last) : (zp ? q0 + T.sa * (t + 1) : q0 + T.sa * (t % na));
    // ---- chi and S of plane q
    Real ncx[H + 2], nsx[H + 2];
    {
      const int64_t base = (int64_t)q * ps + cc;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const int64_t o = base + (int64_t)(r0 + (i < hr ? i : 0)) * rs;
        ncx[i + 1] = chi[o];
        nsx[i + 1] = Sv[o];
      }
      const int64_t ol = base + (int64_t)(has_lo ? row_lo : r0) * rs;
      const int64_t oh = base + (int64_t)(has_hi ? row_hi : r0) * rs;
      ncx[0] = chi[ol];
      nsx[0] = Sv[ol];
      ncx[H + 1] = chi[oh];
      nsx[H + 1] = Sv[oh];
    }
    if (t < 0) {
      // first upwind plane: the boundary layer (planes are z) or the ghost plane
#pragma unroll
      for (int i = 0; i < H + 2; ++i) { cx[i] = ncx[i]; sx[i] = nsx[i]; }
#pragma unroll
      for (int i = 0; i < H; ++i)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const bool up = (r & 1) == 0;
          const int br = up ? bc_up : bc_dn;
          D[i][r] = zp ? fmad(pla, sx[i + 1], plb)
                       : ((r0 + i == br) ? fmad(up ? bua : bda, sx[i + 1], up ? bub : bdb) : Real(0));
        }
    } else {
      const int pold = (phase - 1) & 1;  // table of the previous plane
      const Real* tl = tab + ((pold * 2 * 16 + wl * 2 + 1) * NS);   // left wave, last lane
      const Real* trt = tab + ((pold * 2 * 16 + wr * 2 + 0) * NS);  // right wave, first lane
      const Real* t0 = tab + ((pold * 2 * 16 + 0 * 2 + 0) * NS);    // column 0
      auto left = [&](int k, Real v) { return dpp_shr(tl[k], v); };
      auto right = [&](int k, Real v) {
        const Real r = dpp_shl(trt[k], v);
        return c == W - 1 ? t0[k] : r;
      };
      // column-interpolated chi and S of old row index idx (NC variants)
      auto lcs = [&](int idx, Real* lc, Real* ls) {
        const Real cl = left(idx, cx[idx]), cr = right(idx, cx[idx]);
        const Real sl = left(H + 2 + idx, sx[idx]), sr = right(H + 2 + idx, sx[idx]);
#pragma unroll
        for (int v = 0; v < NC; ++v) {
          const bool lft = UNI ? (v == 0) : (v < 2);
          lc[v] = lerp(cx[idx], lft ? cl : cr, f1[v]);
          ls[v] = lerp(sx[idx], lft ? sl : sr, f1[v]);
        }
      };
      auto ldd = [&](int i, Real* ld) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int k = 2 * (H + 2) + i * R + r;
          const Real n = r < 2 ? left(k, D[i][r]) : right(k, D[i][r]);
          ld[r] = lerp(D[i][r], n, f1[r]);
        }
      };
      // halo rows: column-interpolated chi and S, and D
      Real hlc[NC], hls[NC], huc[NC], hus[NC], hld[R], hud[R];
      lcs(0, hlc, hls);
      lcs(H + 1, huc, hus);
      if (t == 0) {
        // first plane: the halo D is known locally, an affine function of S
        // (the column interpolation commutes with it: its weights sum to 1)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int v = UNI ? (r < 2 ? 0 : 1) : r;
          const bool up = (r & 1) == 0;
          const int br = up ? bc_up : bc_dn;
          const Real a = up ? bua : bda, b = up ? bub : bdb;
          hld[r] = zp ? fmad(pla, hls[v], plb) : (row_lo == br ? fmad(a, hls[v], b) : Real(0));
          hud[r] = zp ? fmad(pla, hus[v], plb) : (row_hi == br ? fmad(a, hus[v], b) : Real(0));
        }
      } else {
        wait_flags(flag_lo, flag_hi, t, status, A.timeout_ticks);
        const int par = (t - 1) & 1;
        const Real* xl = X + ((int64_t)(st_lo * 2 + par) * 2 + 1) * xstride;
        const Real* xh = X + ((int64_t)(st_hi * 2 + par) * 2 + 0) * xstride;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int cn = r < 2 ? cm : cp1;
          // only the slots whose upwind row is the halo need it
          if ((r & 1) == 0) {
            const Real a = has_lo ? ld_dev(xl + r * W + cc) : Real(0);
            const Real b = has_lo ? ld_dev(xl + r * W + cn) : Real(0);
            hld[r] = lerp(a, b, f1[r]);
            hud[r] = Real(0);
          } else {
            const Real a = has_hi ? ld_dev(xh + r * W + cc) : Real(0);
            const Real b = has_hi ? ld_dev(xh + r * W + cn) : Real(0);
            hud[r] = lerp(a, b, f1[r]);
            hld[r] = Real(0);
          }
        }
      }
      // ---- formal solution, row by row, with a sliding window of the
      // interpolated old rows i-1 (p*), i (k*) and i+1 (n*)
      Real pc[NC], pS[NC], pd[R], kc[NC], kS[NC], kd[R], nc[NC], nS[NC], nd[R];
#pragma unroll
      for (int v = 0; v < NC; ++v) { pc[v] = hlc[v]; pS[v] = hls[v]; }
#pragma unroll
      for (int r = 0; r < R; ++r) pd[r] = hld[r];
      lcs(1, kc, kS);
      ldd(0, kd);
#pragma unroll
      for (int i = 0; i < H; ++i) {
        if (i >= hr) break;
        const bool last = (i == hr - 1);
        if (last || i + 1 >= H) {
#pragma unroll
          for (int v = 0; v < NC; ++v) { nc[v] = huc[v]; nS[v] = hus[v]; }
#pragma unroll
          for (int r = 0; r < R; ++r) nd[r] = hud[r];
        } else {
          lcs(i + 2 < H + 2 ? i + 2 : H + 1, nc, nS);
          ldd(i + 1 < H ? i + 1 : H - 1, nd);
        }
        const int gr = r0 + i;
        const Real cpv = ncx[i + 1], spv = nsx[i + 1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int v = UNI ? (r < 2 ? 0 : 1) : r;
          const bool up = (r & 1) == 0;
          const Real uc = up ? pc[v] : nc[v];
          const Real us = up ? pS[v] : nS[v];
          const Real ud = up ? pd[r] : nd[r];
          const Real bc = lerp(kc[v], uc, f2[r]);
          const Real bs = lerp(kS[v], us, f2[r]);
          const Real bd = lerp(kd[r], ud, f2[r]);
          const Real x = hds[r] * (cpv + bc);
          const Real e = rts_exp_neg(x);
          const Real cw = rts_cw(x, e);
          const Real dn = fmad(e, bd, cw * (bs - spv));
          const int br = up ? bc_up : bc_dn;
          D[i][r] = (gr == br) ? fmad(up ? bua : bda, spv, up ? bub : bdb) : dn;
        }
#pragma unroll
        for (int v = 0; v < NC; ++v) { pc[v] = kc[v]; pS[v] = kS[v]; kc[v] = nc[v]; kS[v] = nS[v]; }
#pragma unroll
        for (int r = 0; r < R; ++r) { pd[r] = kd[r]; kd[r] = nd[r]; }
      }
#pragma unroll
      for (int i = 0; i < H + 2; ++i) { cx[i] = ncx[i]; sx[i] = nsx[i]; }
      // ---- publish the edge rows for the neighbouring strips
      if (act) {
        Real* xe = X + ((int64_t)(strip * 2 + (t & 1)) * 2) * xstride;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          Real top = D[0][r];
#pragma unroll
          for (int i = 1; i < H; ++i)
            if (i == hr - 1) top = D[i][r];
          if ((r & 1) == 1) st_dev(xe + r * W + c, D[0][r]);        // lower neighbour: its odd slots
          if ((r & 1) == 0) st_dev(xe + xstride + r * W + c, top);  // upper neighbour: its even slots
        }
      }
      vmem_drain();
    }
    // ---- outputs of plane q: partial sum of w_r D_r (compensated) and I_top
    if (act && (t < 0 ? zp : t >= out_from)) {
#pragma unroll
      for (int i = 0; i < H; ++i) {
        if (i >= hr) break;
        Real s = wgt[0] * D[i][0], comp = 0;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          Real u, e;
          two_sum(s, wgt[r] * D[i][r], u, e);
          s = u;
          comp += e;
        }
        P[(int64_t)q * ps + (int64_t)(r0 + i) * rs + c] = s + comp;
        if (Itop) {
          const int gr = r0 + i;
          if (zp ? (q == T.it_top) : (gr == T.it_top)) {
#pragma unroll
            for (int r = 0; r < R; ++r)
              if (itop[r] >= 0)
                Itop[T.it_off + itop[r] * T.it_ray + (int64_t)q * T.itp + (int64_t)gr * T.itr +
                     (int64_t)c * T.itc] = sx[i + 1] + D[i][r];
          }
        }
      }
    }
    // ---- LDS edge table of this plane, then the step barrier
    {
      const int par = phase & 1;
      if (lane == 0 || lane == last_lane) {
        Real* te = tab + ((par * 2 * 16 + wv * 2 + (lane == 0 ? 0 : 1)) * NS);
#pragma unroll
        for (int i = 0; i < H + 2; ++i) {
          te[i] = cx[i];
          te[H + 2 + i] = sx[i];
        }
#pragma unroll
        for (int i = 0; i < H; ++i)
#pragma unroll
          for (int r = 0; r < R; ++r) te[2 * (H + 2) + i * R + r] = D[i][r];
        if (lane == 0 && last_lane == 0) {  // one-lane wave: both sides
          Real* t1 = tab + ((par * 2 * 16 + wv * 2 + 1) * NS);
#pragma unroll
          for (int k = 0; k < NS; ++k) t1[k] = te[k];
        }
      }
    }
    __syncthreads();
    if (t >= 0 && threadIdx.x == 0) st_dev(flags + strip, t + 1);
    ++phase;
  }
}

template <class Real, int H, bool UNI>
__global__ __launch_bounds__(1024) void rts_sweep(SweepArgs A) {
  extern __shared__ char smem_raw[];
  Real* tab = reinterpret_cast<Real*>(smem_raw);
  __shared__ int sh_ticket;
  WsHeader* hdr = reinterpret_cast<WsHeader*>(A.ws);
  int phase = 0;
  for (;;) {
    if (threadIdx.x == 0) sh_ticket = atomicAdd(&hdr->ticket, 1);
    __syncthreads();
    const int tk = __builtin_amdgcn_readfirstlane(sh_ticket);
    __syncthreads();
    if (tk >= A.total_strips) return;
    int qi = 0;
    while (qi + 1 < A.ntasks && A.queue[2 * (qi + 1)] <= tk) ++qi;
    const Task& T = A.tasks[A.queue[2 * qi + 1]];
    run_strip<Real, H, UNI>(A, T, tk - A.queue[2 * qi], tab, phase);
  }
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
        q[i] += qf * chi * acc[i];
        if (J) J[b * N + p] = (Real)((double)S[b * N + p] + acc[i]);
      }
    }
  }
  for (int i = 0; i < 4; ++i) {
    const int y = y0 + ty + 8 * i, x = x0 + tx;
    if (x < nx && y < ny) P.Q[((int64_t)z * ny + y) * nx + x] = q[i];
  }
}

// DPP lane-layout self test: out[i] = in[i-1] (shr, lane 0 keeps -1) and
// out[64 + i] = in[i+1] (shl, lane 63 keeps -2) for one wave.
__global__ void rts_dpp_selftest(const float* in, float* out) {
  const int l = threadIdx.x;
  const float v = in[l];
  out[l] = dpp_shr(-1.f, v);
  out[64 + l] = dpp_shl(-2.f, v);
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
  (void)threads;
  return (size_t)2 * 16 * 2 * Strip<Real, H>::NS * sizeof(Real);
}

template <class Real, int H, bool UNI>
const void* sweep_fn() {
  return reinterpret_cast<const void*>(&rts_sweep<Real, H, UNI>);
}

template <class Real, int H, bool UNI>
hipError_t launch_sweep_h(const SweepArgs& a, int grid, int threads, hipStream_t st) {
  rts_sweep<Real, H, UNI><<<dim3(grid), dim3(threads), sweep_lds_bytes<Real, H>(threads), st>>>(a);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_reduce(const char* ws, const Task* tasks, const BoxGeo& g, const BoxPtrs& p,
                         hipStream_t st) {
  dim3 grid((g.nx + 31) / 32, (g.ny + 31) / 32, g.nz);
  hipLaunchKernelGGL(rts_reduce<Real>, grid, dim3(256), 0, st, ws, tasks, g, p);
  return hipGetLastError();
}

hipError_t launch_dpp_selftest(const float* in, float* out, hipStream_t st) {
  hipLaunchKernelGGL(rts_dpp_selftest, dim3(1), dim3(64), 0, st, in, out);
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
#define RTS_INST(Real, H)                                                                   \
  template hipError_t launch_sweep_h<Real, H, true>(const SweepArgs&, int, int, hipStream_t); \
  template hipError_t launch_sweep_h<Real, H, false>(const SweepArgs&, int, int, hipStream_t); \
  template size_t sweep_lds_bytes<Real, H>(int);                                            \
  template const void* sweep_fn<Real, H, true>();                                           \
  template const void* sweep_fn<Real, H, false>();
RTS_INST(float, 2)
RTS_INST(float, 4)
RTS_INST(float, 6)
RTS_INST(float, 8)
RTS_INST(double, 2)
RTS_INST(double, 4)
#undef RTS_INST

}  // namespace rts
