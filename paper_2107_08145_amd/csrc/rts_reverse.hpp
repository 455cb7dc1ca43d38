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

template <class Real, int H, int RL = kMaxRaysPerTask>
struct RevStrip {
  // LDS per column: chi and S of the upwind plane u-1, rows -1..H (index
  // 0..H+1); its D per slot, rows -1..H; the downwind state A, B, G per slot
  // of the strip's rows; the halo rows of that state (side 0: the lower
  // neighbour's last row, odd slots 1 and 3; side 1: the upper neighbour's
  // first row, even slots 0 and 2).  [column][NQP], NQP odd.  RL = 4 holds
  // every slot; RL = 2 one slot pair of one parity (slots h and h + 2, at
  // index r >> 1), whose halo is one side only.
  static constexpr int R = RL;
  static constexpr int NQ = (2 + R) * (H + 2) + 3 * R * H + 3 * R;
  static constexpr int NQP = NQ | 1;
  __device__ static constexpr int li(int r) { return R == 4 ? r : (r >> 1); }
  __device__ static constexpr int qc(int j) { return j; }
  __device__ static constexpr int qs(int j) { return H + 2 + j; }
  __device__ static constexpr int qd(int j, int r) { return 2 * (H + 2) + R * j + li(r); }
  __device__ static constexpr int qw(int i, int r, int m) {
    return (2 + R) * (H + 2) + 3 * (R * i + li(r)) + m;
  }
  __device__ static constexpr int qh(int side, int s2, int m) {
    return (2 + R) * (H + 2) + 3 * R * H + (R == 4 ? 6 * side : 0) + 3 * s2 + m;
  }
};

// One strip of one task.  SP slots per thread (4, 2 or 1): NH = 4 / SP
// threads share a column; part h takes slots h, h + NH, ... (with NH = 2 the
// even slots, which read the upper halo and publish the strip's first row,
// and the odd slots, lower halo and last row).  Threads of one part form
// whole waves, so the part is wave-uniform.  SPLIT: the two parts are two
// passes in different workgroups (the adjoint task's `part`), one thread per
// column, and the LDS holds only the pass's slot pair.
template <class Real, int H, bool FULL, int SP, bool SPLIT>
__device__ __forceinline__ void run_rev_strip(const RevArgs& A, CTask& T, CAdjTask& AT,
                                              const int strip, Real* lds) {
  using ST = RevStrip<Real, H, SPLIT ? 2 : kMaxRaysPerTask>;
  constexpr int R = kMaxRaysPerTask;
  static_assert(!SPLIT || SP == 2, "a split pass holds one slot pair");
  constexpr int NH = SPLIT ? 1 : R / SP;  // threads per column
  constexpr int PS = SPLIT ? 2 : NH;      // slot stride of a thread's slots
  using TG = Tagged<Real>;
  constexpr int NW = TG::WORDS;
  const int W = T.n_cols, nr = T.n_rows;
  const int ncol = blockDim.x / NH;  // padded columns of the block
  const int c = threadIdx.x % ncol;
  const int h = SPLIT ? AT.part : NH == 1 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x / ncol);
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
  auto slot = [&](int s) { return PS * s + h; };
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
      // (a split pass keeps every step's words: its strips depend on one
      // neighbour only, so a neighbour may run more than a step ahead)
      const int xoff = SPLIT ? (nb * K + (k - 1)) * xstride : ((nb * 2 + par) * 2 + edge) * xstride;
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
          st_dev(status, 2);  // (2: a reverse-sweep wait)
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
      const int xe = SPLIT ? (strip * K + k) * xstride : ((strip * 2 + (k & 1)) * 2) * xstride;
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
          TG::put(lane_at(urow(X, xe + (even || SPLIT ? 0 : xstride) + ((r >> 1) * 3 + m) * W * NW), xb),
                  v[m], tag);
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

// MAXT: the block-size bound; SP: slots per thread (2: two threads per
// column, or one slot pair of a split pass); H: rows per strip; SPLIT: the
// adjoint tasks are slot-pair passes.  WMIN, WMAX: waves per SIMD (a split
// block of up to 768 threads, one per CU, needs three).
template <class Real, int MAXT, int SP, int H, bool SPLIT, int WMIN, int WMAX>
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
    if ((strip + 1) * H <= T.n_rows) run_rev_strip<Real, H, true, SP, SPLIT>(A, T, AT, strip, lds);
    else run_rev_strip<Real, H, false, SP, SPLIT>(A, T, AT, strip, lds);
  }
}


// Reverse sweep launch shape for `cols` padded columns: up to 256 columns,
// two threads per column (two slots each) in a block of at most 512 threads;
// up to 512 columns, one thread per column (four slots) in 512 threads; above,
// one thread per column in 1024 threads.  A block bound of 512 allows 256
// VGPRs per lane, which the four-slot state nearly fills; 1024 allows 128 and
// spills.  Split passes (tasks too wide or too tall for the four-slot LDS
// state of two-row strips with every strip resident): one thread per column,
// one slot pair, strips of rev_rows(true) rows (four in FP32, two in FP64),
// blocks of at most 768 threads.
template <class Real>
constexpr int rev_rows(bool split) {
  return split ? (sizeof(Real) == 4 ? 4 : 2) : kRevRows;
}

template <class Real>
size_t reverse_lds_bytes(int cols, bool split) {
  const int np = split ? RevStrip<Real, rev_rows<Real>(true), 2>::NQP
                       : RevStrip<Real, kRevRows>::NQP;
  return (size_t)np * cols * sizeof(Real);
}

int reverse_parts(int cols);    // (rts_misc.hip)
int reverse_threads(int cols);

// split passes: up to 512 columns in a 512-thread bound (256 VGPRs), above
// in a 768-thread one (three waves per SIMD: 168 VGPRs)
#define RTS_REV_SPLIT(Real) rts_reverse<Real, 768, 2, rev_rows<Real>(true), true, 3, 3>
#define RTS_REV_SPLIT_N(Real) rts_reverse<Real, 512, 2, rev_rows<Real>(true), true, 1, 4>

template <class Real>
const void* reverse_fn(int cols, bool split) {
  if (split && cols <= 512) return reinterpret_cast<const void*>(&RTS_REV_SPLIT_N(Real));
  if (split) return reinterpret_cast<const void*>(&RTS_REV_SPLIT(Real));
  if (cols <= 256) return reinterpret_cast<const void*>(&rts_reverse<Real, 512, 2, kRevRows, false, 1, 4>);
  if (cols <= 512) return reinterpret_cast<const void*>(&rts_reverse<Real, 512, 4, kRevRows, false, 1, 4>);
  return reinterpret_cast<const void*>(&rts_reverse<Real, 1024, 4, kRevRows, false, 1, 2>);
}

template <class Real>
hipError_t launch_reverse(const RevArgs& a, int grid, int cols, bool split, hipStream_t st) {
  const size_t lds = reverse_lds_bytes<Real>(cols, split);
  if (split) {
    if (cols > 768) return hipErrorInvalidValue;
    if (cols <= 512) RTS_REV_SPLIT_N(Real)<<<dim3(grid), dim3(cols), lds, st>>>(a);
    else RTS_REV_SPLIT(Real)<<<dim3(grid), dim3(cols), lds, st>>>(a);
    return hipGetLastError();
  }
  const dim3 b(reverse_threads(cols));
  if (cols <= 256) rts_reverse<Real, 512, 2, kRevRows, false, 1, 4><<<dim3(grid), b, lds, st>>>(a);
  else if (cols <= 512) rts_reverse<Real, 512, 4, kRevRows, false, 1, 4><<<dim3(grid), b, lds, st>>>(a);
  else rts_reverse<Real, 1024, 4, kRevRows, false, 1, 2><<<dim3(grid), b, lds, st>>>(a);
  return hipGetLastError();
}


#define RTS_REV_INST(Real)                                                          \
  template size_t reverse_lds_bytes<Real>(int, bool);                               \
  template const void* reverse_fn<Real>(int, bool);                                 \
  template hipError_t launch_reverse<Real>(const RevArgs&, int, int, bool, hipStream_t);

}  // namespace rts
