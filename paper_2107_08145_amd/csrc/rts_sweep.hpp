// The forward sweep kernel (rts_sweep) and its launch wrappers, as templates;
// rts_sweep_<precision><rows>.hip instantiate one precision and strip height
// each (separate translation units, compiled in parallel).
#pragma once
#include "rts_device.hpp"

namespace rts {

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
          st_dev(status, 3);  // (3: a lap-end wait)
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

  // warm start (the extended sweep only): the caller's initial ghost planes,
  // I of slot r at (row, column) of the task's plane
  const Real* gin = EXT == 2 && !zp ? reinterpret_cast<const Real*>(A.box[T.box].gin) : nullptr;
  const bool warm = gin != nullptr;
  auto ghost_in = [&](int r, int row, int col) __attribute__((always_inline)) {
    return gptr(gin)[T.gh_off + ((int64_t)T.ray[r].ray * T.n_rows + row) * T.gh_M + col];
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
        if (EXT == 2 && warm && r0 + i != br && T.ray[r].ray >= 0)  // the given ghost intensity
          D0[i][r] = ghost_in(r, FULL || i < hr ? r0 + i : r0, cc) - nsx[i + 1];
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
    // the formal solution of row i from the interpolated old rows i-1, i, i+1.
    // With UNI the four slots share f2, and the row interpolations of chi and
    // S are taken as lk + f2 (lp - lk) or lk + f2 (ln - lk) with the current
    // cell's chi added to (S subtracted from) lk once per column direction;
    // du holds lp - lk of chi (both column directions) and S, dn receives
    // ln - lk, which is the next row's du negated.
    auto solve_row = [&](int i, const LR& lp, const LR& lk, const LR& ln, const Real (&du)[4],
                         Real (&dn)[4], Real* out) __attribute__((always_inline)) {
      const Real cpv = ncx[i + 1], spv = nsx[i + 1];
      if constexpr (UNI) {
        Real tc[2], ts[2];
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          tc[v] = cpv + lk.c[v];  // chi is stored pre-scaled by ds/2 (and log2 e in FP32)
          ts[v] = lk.s[v] - spv;
          dn[v] = ln.c[v] - lk.c[v];
          dn[2 + v] = ln.s[v] - lk.s[v];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int v = r < 2 ? 0 : 1;
          const bool up = (r & 1) == 0;
          const Real xs = fmad(f2[0], up ? du[v] : dn[v], tc[v]);
          const Real bsd = fmad(f2[0], up ? du[2 + v] : dn[2 + v], ts[v]);  // B(S) - S
          const Real bd = lerp(lk.d[r], up ? lp.d[r] : ln.d[r], f2[0]);
          // both forms, then a select (a branch here costs registers)
          const Real e = rts_exp_step(xs);
          const Real c_ser = rts_c_series(xs), c_cl = rts_c_closed(xs, e);
          const Real cw = rts_small_step(xs) ? c_ser : c_cl;
          out[r] = fmad(e, bd, cw * bsd);
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const bool up = (r & 1) == 0;
          const Real bc = lerp(lk.c[r], up ? lp.c[r] : ln.c[r], f2[r]);
          const Real bs = lerp(lk.s[r], up ? lp.s[r] : ln.s[r], f2[r]);
          const Real bd = lerp(lk.d[r], up ? lp.d[r] : ln.d[r], f2[r]);
          const Real xs = hds[r] * (cpv + bc);
          const Real e = rts_exp_step(xs);
          const Real c_ser = rts_c_series(xs), c_cl = rts_c_closed(xs, e);
          const Real cw = rts_small_step(xs) ? c_ser : c_cl;
          out[r] = fmad(e, bd, cw * (bs - spv));
        }
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
          // warm start: the given ghost intensities, interpolated along the
          // columns, minus the interpolated S (the interpolation is linear)
          if (EXT == 2 && warm && has && hrow_g != br && T.ray[r].ray >= 0)
            h.d[r] = lerp(ghost_in(r, hrow_g, cc), ghost_in(r, hrow_g, r < 2 ? cm : cp1), f1[r]) -
                     h.s[v];
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

    // lp - lk of chi (both column directions) and S (UNI only)
    auto row_diff = [&](const LR& lp, const LR& lk, Real (&du)[4]) __attribute__((always_inline)) {
      if constexpr (UNI) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          du[v] = lp.c[v] - lk.c[v];
          du[2 + v] = lp.s[v] - lk.s[v];
        }
      }
    };

    Real Dn[H][R];
    // ---- edge rows first, published for the neighbouring strips: the top
    // row (of a strip of more than one row), then row 0.  (The interior rows
    // interpolate rows 1 and 2 again: keeping row 0's copies across the
    // publication measured slower, by the register allocation it leads to.)
#pragma unroll
    for (int i = 1; i < H; ++i) {
      if (!(FULL ? (i == H - 1) : (i == hr - 1))) continue;
      LR lp, lk, up_;
      Real du[4], dn[4];
      interp(i, true, lp);
      interp(i + 1, true, lk);
      interp(H + 1, false, up_);
      halo_d(false, up_);
      row_diff(lp, lk, du);
      solve_row(i, lp, lk, up_, du, dn, Dn[i]);
    }
    {
      LR lo, k0, n0;
      Real du[4], dn[4];
      interp(0, false, lo);
      halo_d(true, lo);
      interp(1, true, k0);
      if (hr == 1) {
        interp(H + 1, false, n0);
        halo_d(false, n0);
      } else {
        interp(2, true, n0);
      }
      row_diff(lo, k0, du);
      solve_row(0, lo, k0, n0, du, dn, Dn[0]);
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
    // ---- interior rows, sliding window of interpolated old rows (lp - lk of
    // a row is ln - lk of the row below negated, exactly)
    if (FULL ? (H > 2) : (hr > 2)) {
      LR wa, wb, d;  // interpolated LDS rows i, i + 1, i + 2
      Real dw[4];    // ln - lk of the last row solved
      interp(1, true, wa);
      interp(2, true, wb);
      row_diff(wb, wa, dw);
#pragma unroll
      for (int i = 1; i < H - 1; ++i) {
        if (!FULL && i >= hr - 1) break;
        Real du[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) du[m] = -dw[m];
        interp(i + 2, true, d);
        solve_row(i, wa, wb, d, du, dw, Dn[i]);
        wa = wb;
        wb = d;
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
  // the final ghost planes (the outflow plane, in LDS after the last step), as I
  if (EXT == 2 && !zp && A.box[T.box].gout && act) {
    Real* go = gptr(reinterpret_cast<Real*>(A.box[T.box].gout));
    for (int i = 0; i < hr; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (T.ray[r].ray >= 0)
          go[T.gh_off + ((int64_t)T.ray[r].ray * T.n_rows + r0 + i) * T.gh_M + c] =
              lc[ST::qd(i, r)] + lc[ST::qs(i + 1)];
  }
}

// EXT: 0 the plain sweep; 1 also the flux partials (A.flux); 2 also
// tolerance-driven laps (T.tol > 0) and the warm start (given initial ghost
// planes, final ones out).  Separate instantiations, so that each
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
    // a full strip has the template's H rows (a task with fewer rows than H has
    // one strip of all its rows: not full)
    if (T.rows_per_strip == H && (strip + 1) * H <= T.n_rows)
      run_strip<Real, H, UNI, true, EXT>(A, T, strip, lds);
    else run_strip<Real, H, UNI, false, EXT>(A, T, strip, lds);
  }
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


#define RTS_INST(Real, H)                                                                   \
  template hipError_t launch_sweep_h<Real, H, true>(const SweepArgs&, int, int, hipStream_t); \
  template hipError_t launch_sweep_h<Real, H, false>(const SweepArgs&, int, int, hipStream_t); \
  template size_t sweep_lds_bytes<Real, H>(int);                                            \
  template const void* sweep_fn<Real, H, true>();                                           \
  template const void* sweep_fn<Real, H, false>();                                          \
  template const void* sweep_fn_ext<Real, H, true>(int);                                    \
  template const void* sweep_fn_ext<Real, H, false>(int);

}  // namespace rts
