// The adjoint's reverse sweep kernel (rts_reverse) and its launch wrappers,
// as templates; rts_reverse_<precision>.hip instantiate them.
#pragma once
#include "rts_device.hpp"

namespace rts {

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
// The recursion itself gives e B(D) = D_q - c (B(S) - S_q), so
//   dD/dx = -D_q + (c + c') (B(S) - S_q)
// needs the cell's own stored D and no interpolation of the upwind plane's D.
// A boundary cell (D = a_bc S + b_bc) adds a_bc lambda_q to dL/dS_q and
// passes nothing upwind; the ghost plane of a periodic sweep (u = -1) is such
// a plane, with D = 0 off the boundary row.  The seed of a cell in the last
// lap is w_r (4 pi qweight chi gQ + gJ) (+ gItop in the top layer).
//
// The rays of a task are independent in reverse (their gradients only add),
// so every task is reversed as two slot-pair passes: slots 0 and 2 (upwind
// row i-1 in the forward) and slots 1 and 3 (upwind row i+1).  A pass's B^T
// reads downwind rows i and i + 1 (even pass) or i and i - 1 (odd pass): its
// strips depend on one neighbour only (the upper one, or the lower one),
// which may run ahead.  The sweep runs downwind to upwind with persistent
// workgroups, one per strip of H rows x all columns (one thread per column);
// the state (A, B, G) of the downwind plane and chi, S of the upwind plane
// are in LDS; the neighbour's edge row arrives as tagged words through a ring
// of kRevRing steps per strip, and a strip does not overwrite a ring entry
// before its reader has taken it (the reader's progress word).  The forward
// step of each cell is recomputed from chi and S; D is kept, the weights are
// not.

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

// LDS per column of a strip of H rows in one pass: chi and S of the upwind
// plane u-1, rows -1..H (index 0..H+1); the downwind state A, B, G of the
// pass's two slots for the strip's rows; the halo row of that state (the
// neighbour's edge row).  [column][NQP], NQP odd (conflict-free columns).
template <class Real, int H>
struct RevStrip {
  static constexpr int NQ = 2 * (H + 2) + 6 * H + 6;
  static constexpr int NQP = NQ | 1;
  __device__ static constexpr int qc(int j) { return j; }
  __device__ static constexpr int qs(int j) { return H + 2 + j; }
  __device__ static constexpr int qw(int i, int s, int m) { return 2 * (H + 2) + 3 * (2 * i + s) + m; }
  __device__ static constexpr int qh(int s, int m) { return 2 * (H + 2) + 6 * H + 3 * s + m; }
};

// One strip of one pass (UP: the even pass, slots 0 and 2; FULL: the strip
// has H rows).
template <class Real, int H, bool FULL, bool UP>
__device__ __forceinline__ void run_rev_strip(const RevArgs& A, CTask& T, CAdjTask& AT,
                                              const int strip, Real* lds) {
  using ST = RevStrip<Real, H>;
  constexpr int R = kMaxRaysPerTask;
  using TG = Tagged<Real>;
  constexpr int NW = TG::WORDS;
  const int W = T.n_cols, nr = T.n_rows;
  const int c = threadIdx.x;
  constexpr int part = UP ? 0 : 1;  // slots part and part + 2
  constexpr bool up = UP;           // upwind row i-1 in the forward: B^T reads rows i, i+1
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
  // the neighbour whose edge row this strip reads, and the one that reads this strip's
  const bool has_src = up ? has_hi : has_lo, has_dst = up ? has_lo : has_hi;
  const int src = up ? st_hi : st_lo, dst = up ? st_lo : st_hi;
  const int na = T.n_planes;
  const int q0 = T.sa > 0 ? 0 : na - 1, q_last = T.sa > 0 ? na - 1 : 0;
  const int U = T.n_unrolled, u_init = AT.u_init;
  const int K = U - u_init;
  const int last_from = zp ? 0 : (T.laps - 1) * na;
  // the plane before plane q in the sweep (planes of unrolled u-1 from u; a
  // periodic sweep's first plane is preceded by its last, the ghost plane)
  auto prev_plane = [&](int q) { return (!zp && q == q0) ? q_last : q - T.sa; };
  Real f1[2], f2[2], hds[2], wgt[2];
  int itop[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const TaskRay RTS_CONST& y = T.ray[part + 2 * s];
    f1[s] = (Real)y.f1; f2[s] = (Real)y.f2; hds[s] = (Real)y.hds; wgt[s] = (Real)y.w;
    itop[s] = y.itop;
  }
  Real* ws = gptr(reinterpret_cast<Real*>(A.ws));
  const Real* chi = ws + T.chi_off;
  const Real* Sv = gptr(T.transposed ? ws + T.s_off : reinterpret_cast<const Real*>(A.S[T.box]) + T.s_off);
  const Real* Dst = ws + T.dstore_off;
  const Real* seed = ws + AT.seed_off;
  const int64_t N = (int64_t)na * nr * W;
  Real* GS = ws + AT.gs_off + part * N;  // one partial per pass
  Real* GC = ws + AT.gc_off + part * N;
  uint64_t* X = gptr(reinterpret_cast<uint64_t*>(A.ws) + AT.xbuf_off);
  int* progress = gptr(reinterpret_cast<int*>(X + rev_ring_words(ns, W, NW)));
  const Real* gI = gptr(reinterpret_cast<const Real*>(A.gItop[T.box]));
  const int64_t pc = (int64_t)nr * W;
  const int xstride = 6 * W * NW;  // one ring entry: 2 slots x 3 quantities
  const uint32_t cb = (uint32_t)cc * sizeof(Real), xb = (uint32_t)cc * NW * 8;
  Real* lc = lds + c * ST::NQP;
  const Real* lcc = lds + cc * ST::NQP;
  const Real* lcm = lds + cm * ST::NQP;
  const Real* lcp = lds + cp1 * ST::NQP;
  auto urow = [&](auto* base, int off) __attribute__((always_inline)) {
    return base + __builtin_amdgcn_readfirstlane(off);
  };
  // buffer resources of the arrays this strip reads and writes per row
  const Rsrc rC = rts_rsrc(chi), rS = rts_rsrc(Sv), rSeed = rts_rsrc(seed);
  const Rsrc rGS = rts_rsrc(GS), rGC = rts_rsrc(GC);
  const Real bua = (Real)T.bu_a, bub = (Real)T.bu_b, bda = (Real)T.bd_a, bdb = (Real)T.bd_b;
  const Real pla = (Real)T.pl_a;
  (void)bub; (void)bdb;
  auto up_row = [&](int j) __attribute__((always_inline)) {
    int g = r0 - 1 + j;
    if (per) g = g < 0 ? g + nr : (g >= nr ? g - nr : g);
    else g = g < 0 ? 0 : (g >= nr ? nr - 1 : g);
    return g;
  };
  // the strip's own rows (clamped for a partial strip: such rows are neither
  // read nor written)
  auto own_row = [&](int i) __attribute__((always_inline)) { return r0 + (FULL || i < hr ? i : 0); };

  // Per step k (unrolled plane u = U-1-k): chi and S of the upwind plane
  // u-1, rows -1..H of this column, loaded during the previous step and put
  // into LDS at the start of this one; and per own row, D of the two slots,
  // the seed (last lap) and the old gradient partials (other laps), loaded
  // during the previous step as its rows retire.  chi and S of the own rows
  // are the previous step's upwind rows 1..H, read back from LDS.
  Real upc[H + 2], ups[H + 2];
  Real dq[H][2], sdv[H], gsv[H], gcv[H], cpv[H], spv[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {  // (a ghost or boundary step reads them unused)
    dq[i][0] = dq[i][1] = sdv[i] = gsv[i] = gcv[i] = cpv[i] = spv[i] = Real(0);
  }
  // (k: the step; q: the plane the loads are of).  Branch-free: a load that a
  // step does not need (beyond the last step, the ghost or boundary plane, a
  // seed outside the last lap, a partial at its first visit) reads row 0 of
  // its array instead (in cache after the first time) and is not used; the
  // branches would split the step into small blocks that each reload the
  // buffer resources from spilled SGPRs.
  constexpr uint32_t ES = sizeof(Real);
  auto load_up = [&](int k, int q) __attribute__((always_inline)) {
    const int u = U - 1 - k;
    const bool live = k < K && u >= 0 && !(zp && u == 0);
    const int qo = live ? q * ps : 0;
#pragma unroll
    for (int j = 0; j < H + 2; ++j) {
      const uint32_t o = live ? (uint32_t)(qo + up_row(j) * rs) * ES : 0u;
      upc[j] = buf_load<Real>(rC, cb, o);
      ups[j] = buf_load<Real>(rS, cb, o);
    }
  };
  auto load_own = [&](int k, int i, int q) __attribute__((always_inline)) {
    const int u = U - 1 - k;
    const bool live = k < K && u >= 0;  // (the ghost plane is not in the last lap: no seed)
    const bool dlive = live && !(zp && u == 0);  // (the boundary plane: no recompute)
    const int gi = own_row(i);
    const uint32_t o = (uint32_t)(q * ps + gi * rs) * ES;
    sdv[i] = buf_load<Real>(rSeed, cb, live && u >= last_from ? o : 0u);
    const Rsrc rD = rts_rsrc(Dst + (int64_t)(dlive ? u : 0) * R * pc);
#pragma unroll
    for (int s = 0; s < 2; ++s)
      dq[i][s] = buf_load<Real>(rD, cb, dlive ? (uint32_t)(((part + 2 * s) * nr + gi) * W) * ES : 0u);
  };
  auto load_part = [&](int k, int i, int q) __attribute__((always_inline)) {
    const int u = U - 1 - k;
    const bool live = k < K && u < last_from;  // the first visit of a cell writes its partial
    const uint32_t o = live ? (uint32_t)(q * ps + own_row(i) * rs) * ES : 0u;
    gsv[i] = buf_load<Real>(rGS, cb, o);
    gcv[i] = buf_load<Real>(rGC, cb, o);
  };

  // the neighbour's edge words of the downwind state, published at its step k-1 (tag k)
  uint64_t hw[2][3][NW];
  auto halo_issue = [&](int k) __attribute__((always_inline)) {
    const int xoff = (src * kRevRing + (k % kRevRing)) * xstride;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const uint64_t* rowp = urow(X, xoff + (s * 3 + m) * W * NW);
#pragma unroll
        for (int x = 0; x < NW; ++x) hw[s][m][x] = has_src ? ld_dev(lane_at(rowp, xb) + x) : 0ull;
      }
  };
  auto timed_out = [&](uint64_t t0) __attribute__((always_inline)) {
    if (__builtin_amdgcn_readfirstlane(ld_dev(status)) != 0) return true;
    if ((int64_t)(__builtin_amdgcn_s_memrealtime() - t0) > A.timeout_ticks) {
      st_dev(status, 2);  // (2: a reverse-sweep wait)
      return true;
    }
    return false;
  };
  auto halo_wait = [&](int k) __attribute__((always_inline)) {
    const uint32_t tag = (uint32_t)k;
    auto all_fresh = [&]() __attribute__((always_inline)) {
      bool ok = true;
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int m = 0; m < 3; ++m) ok = ok && (!has_src || TG::fresh(hw[s][m], tag));
      return ok;
    };
    if (__ballot(!all_fresh()) != 0) {
      const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
      for (;;) {
        __builtin_amdgcn_s_sleep(1);
        halo_issue(k);
        if (__ballot(!all_fresh()) == 0) break;
        if (timed_out(t0)) break;
      }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int m = 0; m < 3; ++m) lc[ST::qh(s, m)] = has_src ? TG::value(hw[s][m]) : Real(0);
  };
  // before overwriting ring entry (k+1) % kRevRing (tag k+1-kRevRing), its
  // reader must have taken it: its progress word is at least k+1-kRevRing.
  // Progress only grows, so the last value read stands until a step needs
  // more (a device-scope load costs a memory round trip: once per several
  // steps instead of every step).
  int seen = 0;
  auto ring_free = [&](int k) __attribute__((always_inline)) {
    const int need = k + 1 - kRevRing;
    if (!has_dst || need <= seen) return;
    seen = __builtin_amdgcn_readfirstlane(ld_dev(progress + dst));
    if (seen >= need) return;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (;;) {
      __builtin_amdgcn_s_sleep(1);
      seen = __builtin_amdgcn_readfirstlane(ld_dev(progress + dst));
      if (seen >= need) break;
      if (timed_out(t0)) break;
    }
  };

  // ---- the downwind state of plane U (beyond the last plane) is zero
  lds_barrier();  // the previous strip of this workgroup has finished with the LDS
#pragma unroll
  for (int i = 0; i < H; ++i)
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int m = 0; m < 3; ++m) lc[ST::qw(i, s, m)] = Real(0);
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int m = 0; m < 3; ++m) lc[ST::qh(s, m)] = Real(0);

  const int top = FULL ? H - 1 : hr - 1;
  // the plane of the first step (unrolled plane U-1)
  int qp = q0 + T.sa * (zp ? U - 1 : (U - 1) % na);
  // first step: its own rows' chi and S from memory
  {
    const int u = U - 1;
    if (u >= 0 && !(zp && u == 0)) {
      const int qo = qp * ps;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const int o = qo + own_row(i) * rs;
        cpv[i] = buf_load<Real>(rC, cb, (uint32_t)o * sizeof(Real));
        spv[i] = buf_load<Real>(rS, cb, (uint32_t)o * sizeof(Real));
      }
    }
  }
  load_up(0, prev_plane(qp));
#pragma unroll
  for (int i = 0; i < H; ++i) {
    load_own(0, i, qp);
    load_part(0, i, qp);
  }

  for (int k = 0; k < K; ++k) {
    const int u = U - 1 - k;
    const int qn = prev_plane(qp);  // the plane of u - 1 (the next step's)
    const bool ghost = u < 0;
    const bool bcplane = zp && u == 0;
    const bool last_lap = u >= last_from;
    if (k > 0) halo_wait(k);
    if (!ghost && !bcplane) {
#pragma unroll
      for (int j = 0; j < H + 2; ++j) {
        lc[ST::qc(j)] = upc[j];
        lc[ST::qs(j)] = ups[j];
      }
    }
    load_up(k + 1, prev_plane(qn));  // in flight during this step
    lds_barrier();   // halo row, upwind plane and downwind state complete
    // every wave has its copy of ring entry k: the producer may reuse it
    if (k > 0 && threadIdx.x == 0) st_dev(progress + strip, k);

    Real nst[H][2][3];
    auto do_row = [&](int i) __attribute__((always_inline)) {
      // rows are scheduled one at a time: hoisting every row's LDS reads to
      // the barrier would hold them all in registers
      __builtin_amdgcn_sched_barrier(0);
      const int gi = r0 + i;
      const int j = i + 1;  // LDS row of this cell in the upwind plane
      Real gs = 0, gc = 0;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int r = part + 2 * s;
        const Real* cn = r < 2 ? lcp : lcm;  // downwind column c - sc
        // B^T of the downwind state: rows i and i - sr
        Real tq[3];
        const int io = up ? i + 1 : i - 1;
        const bool in_strip = io >= 0 && io < (FULL ? H : hr);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const Real v0 = lerp(lcc[ST::qw(i, s, m)], cn[ST::qw(i, s, m)], f1[s]);
          const int qo_ = in_strip ? ST::qw(in_strip ? io : 0, s, m) : ST::qh(s, m);
          const Real v1 = lerp(lcc[qo_], cn[qo_], f1[s]);
          tq[m] = lerp(v0, v1, f2[s]);
        }
        Real lam = fmad(wgt[s], last_lap ? sdv[i] : Real(0), tq[0]);
        if (last_lap && gI && itop[s] >= 0 && (zp ? qp == T.it_top : gi == T.it_top))
          lam += gI[T.it_off + itop[s] * T.it_ray + (int64_t)qp * T.itp + (int64_t)gi * T.itr +
                    (int64_t)cc * T.itc];
        // Branch-free in FP32: the forward step is recomputed for every cell
        // (the LDS rows it reads always hold finite values) and selected away
        // for boundary cells, D = coef S + const, which pass coef lambda to S.
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
          const Real x = hds[s] * (cpv[i] + bcx);
          const Real e = rts_exp_neg(x);
          const Real cw = rts_cw(x, e);
          const Real dc = rts_dcw(x, e, cw);
          a = comp ? e * lam : Real(0);
          b = comp ? cw * lam : Real(0);
          g = comp ? hds[s] * lam * fmad(cw + dc, bsx - spv[i], -dq[i][s]) : Real(0);
        }
        gs = fmad(comp ? Real(0) : coef, lam, gs) - b + tq[1];
        gc += g + tq[2];
        nst[i][s][0] = a;
        nst[i][s][1] = b;
        nst[i][s][2] = g;
      }
      if (act && (FULL || i < hr)) {
        const int o = qp * ps + gi * rs;
        buf_store(rGS, cb, (uint32_t)o * sizeof(Real), last_lap ? gs : gsv[i] + gs);
        buf_store(rGC, cb, (uint32_t)o * sizeof(Real), last_lap ? gc : gcv[i] + gc);
      }
      // this row's registers are free: the next step's own-row loads
      load_own(k + 1, i, qn);
      load_part(k + 1, i, qn);
      __builtin_amdgcn_sched_barrier(0);
    };
    // the published edge row first (even pass: the first row; odd: the last), then the rest
    if constexpr (UP) do_row(0);
    else {
#pragma unroll
      for (int i = 0; i < H; ++i)
        if (i == top) do_row(i);
    }
    if (k + 1 < K) ring_free(k);  // (every wave: the check is uniform)
    if (act && k + 1 < K) {
      const int xe = (strip * kRevRing + ((k + 1) % kRevRing)) * xstride;
      const uint32_t tag = (uint32_t)(k + 1);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        Real v[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          v[m] = nst[0][s][m];
          if constexpr (!UP) {
#pragma unroll
            for (int i = 1; i < H; ++i)
              if (i == top) v[m] = nst[i][s][m];
          }
          TG::put(lane_at(urow(X, xe + (s * 3 + m) * W * NW), xb), v[m], tag);
        }
      }
    }
    if constexpr (UP) {
#pragma unroll
      for (int i = 1; i < H; ++i)
        if (FULL || i < hr) do_row(i);
    } else {
#pragma unroll
      for (int i = 0; i < H - 1; ++i)
        if (i < top) do_row(i);
    }
    lds_barrier();  // every thread has read the downwind state and the upwind plane
#pragma unroll
    for (int i = 0; i < H; ++i)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int m = 0; m < 3; ++m)
          lc[ST::qw(i, s, m)] = (FULL || i < hr) ? nst[i][s][m] : Real(0);
    // the next step's own rows: this step's upwind rows 1..H (this column,
    // written by this thread only)
    if (!ghost && !bcplane) {
#pragma unroll
      for (int i = 0; i < H; ++i) {
        cpv[i] = lc[ST::qc(i + 1)];
        spv[i] = lc[ST::qs(i + 1)];
      }
    }
    if (k + 1 < K) halo_issue(k + 1);
    qp = qn;
  }
}

// H: rows per strip; MAXT: the block-size bound; WMIN, WMAX: waves per SIMD.
template <class Real, int H, int MAXT, int WMIN, int WMAX>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(WMIN, WMAX)))
void rts_reverse(RevArgs A) {
  extern __shared__ char smem_raw[];
  Real* lds = reinterpret_cast<Real*>(smem_raw);
  __shared__ int sh_ticket;
  WsHeader* hdr = reinterpret_cast<WsHeader*>(A.ws);
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
    const bool full = (strip + 1) * H <= T.n_rows;
    if (AT.part == 0) {
      if (full) run_rev_strip<Real, H, true, true>(A, T, AT, strip, lds);
      else run_rev_strip<Real, H, false, true>(A, T, AT, strip, lds);
    } else {
      if (full) run_rev_strip<Real, H, true, false>(A, T, AT, strip, lds);
      else run_rev_strip<Real, H, false, false>(A, T, AT, strip, lds);
    }
  }
}


// Launch shapes of the reverse sweep by padded width (classes up to 128, 256,
// 512, 768 and 1024 columns): one thread per column, strips of H rows, as tall
// as the registers of a block of that many waves allow without spilling (the
// LDS state of every column, RevStrip, fits with room to spare), with the
// waves-per-SIMD bounds (W0, W1) of the kernel:
//   FP32: 4 rows up to 128 columns (three waves per SIMD; a few registers
//         spill), 6 up to 512, 3 up to 768, 2 up to 1024;
//   FP64: 2 rows up to 512 columns, 1 up to 768 (wider: not supported).
// Taller strips amortise a step's fixed costs (barriers, the exchange, the
// loads' latency) over more cells; on planes of up to 128 columns the extra
// resident waves of 4-row strips win over 6 rows (measured on the 96^2 x 512
// box and at 128^3; 3 and 4 rows lose to 6 from 192 columns on).
template <class Real, int C, bool SMALL = false>
struct RevShape;
template <> struct RevShape<float, 0> { static constexpr int H = 4, T = 128, W0 = 3, W1 = 3; };
template <> struct RevShape<float, 1> { static constexpr int H = 6, T = 256, W0 = 2, W1 = 2; };
template <> struct RevShape<float, 2> { static constexpr int H = 6, T = 512, W0 = 1, W1 = 2; };
template <> struct RevShape<float, 3> { static constexpr int H = 4, T = 768, W0 = 3, W1 = 3; };
template <> struct RevShape<float, 4> { static constexpr int H = 2, T = 1024, W0 = 4, W1 = 4; };
template <> struct RevShape<double, 0> { static constexpr int H = 2, T = 128, W0 = 2, W1 = 2; };
template <> struct RevShape<double, 1> { static constexpr int H = 2, T = 256, W0 = 2, W1 = 2; };
template <> struct RevShape<double, 2> { static constexpr int H = 2, T = 512, W0 = 1, W1 = 2; };
template <> struct RevShape<double, 3> { static constexpr int H = 1, T = 768, W0 = 3, W1 = 3; };
// Small problems (a launch whose tall strips would leave the SIMDs with
// fewer than two waves each): FP32 planes up to 256 columns in 2-row strips
// (126 VGPRs, four waves per SIMD), so that there are twice or thrice as many.
template <> struct RevShape<float, 0, true> { static constexpr int H = 2, T = 128, W0 = 4, W1 = 4; };
template <> struct RevShape<float, 1, true> { static constexpr int H = 2, T = 256, W0 = 4, W1 = 4; };

constexpr int rev_class(int cols) {
  return cols <= 128 ? 0 : cols <= 256 ? 1 : cols <= 512 ? 2 : cols <= 768 ? 3 : 4;
}

// Calls f(shape) for the shape of `cols` (the small one if asked and there is
// one); false when the width is not supported.
template <class Real, class F>
bool rev_dispatch(int cols, bool small, F&& f) {
  constexpr bool f32 = sizeof(Real) == 4;
  switch (rev_class(cols)) {
    case 0:
      if constexpr (f32) {
        if (small) { f(RevShape<Real, 0, true>{}); return true; }
      }
      f(RevShape<Real, 0>{});
      return true;
    case 1:
      if constexpr (f32) {
        if (small) { f(RevShape<Real, 1, true>{}); return true; }
      }
      f(RevShape<Real, 1>{});
      return true;
    case 2: f(RevShape<Real, 2>{}); return true;
    case 3: f(RevShape<Real, 3>{}); return true;
    case 4:
      if constexpr (f32) {
        f(RevShape<Real, 4>{});
        return true;
      }
      return false;
  }
  return false;
}

template <class Real>
size_t reverse_lds_bytes(int cols, bool small) {
  size_t b = 0;
  rev_dispatch<Real>(cols, small, [&](auto S) {
    b = (size_t)RevStrip<Real, decltype(S)::H>::NQP * cols * sizeof(Real);
  });
  return b;
}

template <class Real>
const void* reverse_fn(int cols, bool small) {
  const void* fn = nullptr;
  rev_dispatch<Real>(cols, small, [&](auto S) {
    using Sh = decltype(S);
    fn = reinterpret_cast<const void*>(&rts_reverse<Real, Sh::H, Sh::T, Sh::W0, Sh::W1>);
  });
  return fn;
}

template <class Real>
hipError_t launch_reverse(const RevArgs& a, int grid, int cols, bool small, hipStream_t st) {
  const size_t lds = reverse_lds_bytes<Real>(cols, small);
  const bool ok = rev_dispatch<Real>(cols, small, [&](auto S) {
    using Sh = decltype(S);
    rts_reverse<Real, Sh::H, Sh::T, Sh::W0, Sh::W1><<<dim3(grid), dim3(cols), lds, st>>>(a);
  });
  return ok ? hipGetLastError() : hipErrorInvalidValue;
}

// the host's view of the launch shape: rows per strip (0: not supported)
template <class Real>
int reverse_rows(int cols, bool small) {
  int h = 0;
  rev_dispatch<Real>(cols, small, [&](auto S) { h = decltype(S)::H; });
  return h;
}

#define RTS_REV_INST(Real)                                                 \
  template size_t reverse_lds_bytes<Real>(int, bool);                      \
  template const void* reverse_fn<Real>(int, bool);                        \
  template int reverse_rows<Real>(int, bool);                              \
  template hipError_t launch_reverse<Real>(const RevArgs&, int, int, bool, hipStream_t);

}  // namespace rts
