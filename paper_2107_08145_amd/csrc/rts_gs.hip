// Scattering with Gauss-Seidel source updates along the rays (the paper's
// proposed variation of the radiation transport solver for strongly
// scattering media, section "RTS Integration and Interpolation Merge", after
// Trujillo Bueno & Fabiani Bendicho 1995): S = (1 - eps) J + eps B, with the
// source function of each point updated as the rays are integrated and the
// new value used for the next point along the ray.
//
// The launch boundary orders the planes of a sweep; inside a plane the cells
// are independent.  Only the last ray group updates S, so within one
// iteration every other group, and the last group's laps before its last,
// sweep with the S of the iteration's start and run concurrently: one launch
// per step over (cells of a plane, band, group), then one launch per plane of
// the last group's last lap.  FP64, natural [z][y][x] layout:
//   rts_gs_init  : the local operator L(p) = sum_r w_r dI_r(p)/dS_p over every
//                  ray (w0 of the ray's linear-source step, or 1 / 0 on a
//                  boundary cell), S = B, the group contributions
//                  P_g = (sum_{r in g} w_r) S;
//   rts_gs_ghost : the ghost plane of a periodic group, I = S of the current S
//                  (boundary cells at their value), written into the group's
//                  outflow plane (the first plane reads it as its upwind plane);
//   rts_gs_step  : step t of every group (its lap and plane), each slot's step
//                  from the upwind plane with the current S; in a group's last
//                  lap its contribution P_g (the last group's last lap is not a
//                  step of this launch);
//   rts_gs_plane : one plane of the last group's last lap: each slot's step,
//                  then the update
//                    J' = sum_{g' != g} P_g' + (this group's new sum),
//                    dS = ((1 - eps) J' + eps B - S) / (1 - (1 - eps) L),
//                    S += dS,  I_r += (dI_r/dS_p) dS,
//                  and the group's contribution;
//   rts_gs_finish: J = sum_g P_g (in group order), Q = sum_b qw_b 4 pi chi_b
//                  (J_b - S_b), J and S out.
// Each group keeps its own intensities [group][slot][band][N], each block in
// the group's plane layout [plane][eb][ea] (contiguous along its planes); the
// x-dominant groups' steps read chi and S from copies in the [x][z][y] layout
// (S copied at the start of every iteration), where their planes are
// contiguous too; the last group's last lap reads and updates S in place.
#include "rts_device.hpp"

namespace rts {

namespace {

// Linear-source weights e = exp(-x), w0 = (x - 1 + e)/x, w1 = (1 - e (1 + x))/x;
// below x = 0.5 their power series, where the closed forms cancel:
//   w0 = sum_{m>=1} c_m x^m,  w1 = sum_{m>=1} m c_m x^m,  c_m = (-1)^(m+1) / (m+1)!,
// in Horner form over m = 1..18 (the first omitted term is below 1e-22 of w0).
__device__ inline void gs_weights(double x, double& e, double& w0, double& w1) {
  e = exp(-x);
  if (x < 0.5) {
    constexpr int M = 18;
    double a = 0.0, b = 0.0;
    // c_m for m = M down to 1
    constexpr double c[M + 1] = {
        0.0,
        1.0 / 2.0, -1.0 / 6.0, 1.0 / 24.0, -1.0 / 120.0, 1.0 / 720.0, -1.0 / 5040.0,
        1.0 / 40320.0, -1.0 / 362880.0, 1.0 / 3628800.0, -1.0 / 39916800.0,
        1.0 / 479001600.0, -1.0 / 6227020800.0, 1.0 / 87178291200.0,
        -1.0 / 1307674368000.0, 1.0 / 20922789888000.0, -1.0 / 355687428096000.0,
        1.0 / 6402373705728000.0, -1.0 / 121645100408832000.0};
#pragma unroll
    for (int m = M; m >= 1; --m) {
      a = fma(a, x, c[m]);
      b = fma(b, x, (double)m * c[m]);
    }
    w0 = a * x;
    w1 = b * x;
  } else {
    w0 = (x - 1.0 + e) / x;
    w1 = (1.0 - e * (1.0 + x)) / x;
  }
}

__device__ inline int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

struct GsCell {
  int c[3];
  __device__ int64_t at(int nx, int ny) const { return ((int64_t)c[2] * ny + c[1]) * nx + c[0]; }
  // the [x][z][y] layout
  __device__ int64_t at_t(int ny, int nz) const { return ((int64_t)c[0] * nz + c[2]) * ny + c[1]; }
};

// The boundary value of slot y at a boundary-layer cell with source s, and
// its derivative in s.
__device__ inline double gs_bc(const GsArgs& A, const GsRay& y, double s, double* ds) {
  if (y.up) {
    *ds = A.bot == 0 ? 1.0 : 0.0;
    return A.bot == 0 ? s : A.ibot;
  }
  *ds = A.top == 0 ? 0.0 : 1.0;
  return A.top == 0 ? 0.0 : s;
}

}  // namespace

// grid.x over cells, grid.y = band
__global__ __launch_bounds__(256) void rts_gs_init(GsArgs A) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.N) return;
  const int b = blockIdx.y;
  const int n[3] = {A.nx, A.ny, A.nz};
  double* ws = reinterpret_cast<double*>(A.ws);
  const double* chi = ws + A.chi_off + (int64_t)b * A.N;
  GsCell me;
  me.c[0] = (int)(p % A.nx);
  me.c[1] = (int)((p / A.nx) % A.ny);
  me.c[2] = (int)(p / ((int64_t)A.nx * A.ny));
  double L = 0.0;
  for (int g = 0; g < A.ngroups; ++g) {
    const GsGroup& G = A.groups[g];
    for (int k = 0; k < kMaxRaysPerTask; ++k) {
      const GsRay& y = G.ray[k];
      if (!y.used) continue;
      double d;
      if (y.up ? me.c[2] == 0 : me.c[2] == A.nz - 1) {
        gs_bc(A, y, 0.0, &d);
      } else {
        GsCell u = me;
        u.c[G.axis] = wrapi(me.c[G.axis] - G.sa, n[G.axis]);
        const int a1 = G.ea == 2 ? me.c[G.ea] - y.sea : wrapi(me.c[G.ea] - y.sea, n[G.ea]);
        const int b1 = G.eb == 2 ? me.c[G.eb] - y.seb : wrapi(me.c[G.eb] - y.seb, n[G.eb]);
        GsCell u10 = u, u01 = u, u11 = u;
        u10.c[G.ea] = a1;
        u01.c[G.eb] = b1;
        u11.c[G.ea] = a1;
        u11.c[G.eb] = b1;
        const double b00 = (1 - y.fa) * (1 - y.fb), b10 = y.fa * (1 - y.fb);
        const double b01 = (1 - y.fa) * y.fb, b11 = y.fa * y.fb;
        const double cu = b00 * chi[u.at(A.nx, A.ny)] + b10 * chi[u10.at(A.nx, A.ny)] +
                          b01 * chi[u01.at(A.nx, A.ny)] + b11 * chi[u11.at(A.nx, A.ny)];
        double e, w0, w1;
        gs_weights(y.hds * (chi[p] + cu), e, w0, w1);
        d = w0;
      }
      L += y.w * d;
    }
  }
  const int64_t bo = (int64_t)b * A.N + p;
  ws[A.l_off + bo] = L;
  const double s = A.B[bo];
  ws[A.s_off + bo] = s;
  for (int g = 0; g < A.ngroups; ++g)
    ws[A.p_off + ((int64_t)g * A.nbands + b) * A.N + p] = A.groups[g].wsum * s;
}

// The ghost plane of group g: grid.x over the plane's cells, grid.y = band.
__global__ __launch_bounds__(256) void rts_gs_ghost(GsArgs A, int g) {
  const GsGroup& G = A.groups[g];
  const int n[3] = {A.nx, A.ny, A.nz};
  const int nA = n[G.ea], nB = n[G.eb];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nA * nB) return;
  const int b = blockIdx.y;
  double* ws = reinterpret_cast<double*>(A.ws);
  GsCell me;
  me.c[G.axis] = G.sa > 0 ? n[G.axis] - 1 : 0;
  me.c[G.ea] = idx % nA;
  me.c[G.eb] = idx / nA;
  const int64_t p = me.at(A.nx, A.ny);
  const int64_t pi = ((int64_t)me.c[G.axis] * nB + me.c[G.eb]) * nA + me.c[G.ea];
  const double s = ws[A.s_off + (int64_t)b * A.N + p];
  for (int k = 0; k < kMaxRaysPerTask; ++k) {
    const GsRay& y = G.ray[k];
    if (!y.used) continue;
    double d;
    const bool bcl = y.up ? me.c[2] == 0 : me.c[2] == A.nz - 1;
    ws[A.i_off + (((int64_t)g * kMaxRaysPerTask + k) * A.nbands + b) * A.N + pi] =
        bcl ? gs_bc(A, y, s, &d) : s;
  }
}

// Cell idx of plane q of group g, band b.  contribute: the group's last lap
// (its contribution P_g); update: also the Gauss-Seidel update (the last lap
// of the last group); top: write I_top.
// tr: read chi and S from the [x][z][y] copies (x-dominant groups' steps).
__device__ inline void gs_plane_cell(const GsArgs& A, int g, int q, bool contribute, bool update,
                                     bool top, int idx, int b, bool tr) {
  const GsGroup& G = A.groups[g];
  const int n[3] = {A.nx, A.ny, A.nz};
  const int nA = n[G.ea], nB = n[G.eb];
  if (idx >= nA * nB) return;
  const int64_t N = A.N;
  double* ws = reinterpret_cast<double*>(A.ws);
  const double* chi = ws + (tr ? A.chit_off : A.chi_off) + (int64_t)b * N;
  double* S = ws + A.s_off + (int64_t)b * N;  // (updated in place: natural layout)
  const double* Sr = tr ? ws + A.st_off + (int64_t)b * N : S;
  double* Ig = ws + A.i_off + (int64_t)g * kMaxRaysPerTask * A.nbands * N;  // the group's
  auto at = [&](const GsCell& c) { return tr ? c.at_t(A.ny, A.nz) : c.at(A.nx, A.ny); };
  auto at_i = [&](const GsCell& c) {
    return ((int64_t)c.c[G.axis] * nB + c.c[G.eb]) * nA + c.c[G.ea];
  };
  GsCell me;
  me.c[G.axis] = q;
  me.c[G.ea] = idx % nA;
  me.c[G.eb] = idx / nA;
  const int64_t p = me.at(A.nx, A.ny), pr = at(me), pi = at_i(me);
  GsCell u = me;
  u.c[G.axis] = wrapi(q - G.sa, n[G.axis]);
  const double sp = Sr[pr];
  double v[kMaxRaysPerTask], dv[kMaxRaysPerTask];
  double pn = 0.0;
  for (int k = 0; k < kMaxRaysPerTask; ++k) {
    const GsRay& y = G.ray[k];
    v[k] = 0.0;
    dv[k] = 0.0;
    if (!y.used) continue;
    const double* I = Ig + ((int64_t)k * A.nbands + b) * N;
    if (y.up ? me.c[2] == 0 : me.c[2] == A.nz - 1) {
      v[k] = gs_bc(A, y, sp, &dv[k]);
    } else {
      const int a1 = G.ea == 2 ? me.c[G.ea] - y.sea : wrapi(me.c[G.ea] - y.sea, nA);
      const int b1 = G.eb == 2 ? me.c[G.eb] - y.seb : wrapi(me.c[G.eb] - y.seb, nB);
      GsCell u10 = u, u01 = u, u11 = u;
      u10.c[G.ea] = a1;
      u01.c[G.eb] = b1;
      u11.c[G.ea] = a1;
      u11.c[G.eb] = b1;
      const int64_t c00 = at(u), c10 = at(u10), c01 = at(u01), c11 = at(u11);
      const int64_t i00 = at_i(u), i10 = at_i(u10), i01 = at_i(u01), i11 = at_i(u11);
      const double b00 = (1 - y.fa) * (1 - y.fb), b10 = y.fa * (1 - y.fb);
      const double b01 = (1 - y.fa) * y.fb, b11 = y.fa * y.fb;
      const double iu = b00 * I[i00] + b10 * I[i10] + b01 * I[i01] + b11 * I[i11];
      const double su = b00 * Sr[c00] + b10 * Sr[c10] + b01 * Sr[c01] + b11 * Sr[c11];
      const double cu = b00 * chi[c00] + b10 * chi[c10] + b01 * chi[c01] + b11 * chi[c11];
      double e, w0, w1;
      gs_weights(y.hds * (chi[pr] + cu), e, w0, w1);
      v[k] = e * iu + w0 * sp + w1 * su;
      dv[k] = w0;
    }
    pn += y.w * v[k];
  }
  const int64_t bo = (int64_t)b * N + p;
  double* P = ws + A.p_off;
  if (update) {
    double jn = 0.0;  // J' with this group's new sum
    for (int gg = 0; gg < A.ngroups; ++gg)
      jn += gg == g ? pn : P[((int64_t)gg * A.nbands + b) * N + p];
    const double ep = A.eps[bo];
    const double om = 1.0 - ep;
    const double ds = (om * jn + ep * A.B[bo] - sp) / (1.0 - om * ws[A.l_off + bo]);
    S[p] = sp + ds;
    pn = 0.0;
    for (int k = 0; k < kMaxRaysPerTask; ++k) {
      if (!G.ray[k].used) continue;
      v[k] += dv[k] * ds;
      pn += G.ray[k].w * v[k];
    }
  }
  for (int k = 0; k < kMaxRaysPerTask; ++k)
    if (G.ray[k].used) Ig[((int64_t)k * A.nbands + b) * N + pi] = v[k];
  if (contribute) P[((int64_t)g * A.nbands + b) * N + p] = pn;
  if (top && A.I_top && me.c[2] == A.nz - 1) {
    const int nup_plane = A.nx * A.ny;
    int nup = 0;
    for (int gg = 0; gg < A.ngroups; ++gg)
      for (int k = 0; k < kMaxRaysPerTask; ++k) nup += A.groups[gg].ray[k].used && A.groups[gg].ray[k].up;
    for (int k = 0; k < kMaxRaysPerTask; ++k) {
      const GsRay& y = G.ray[k];
      if (y.used && y.up)
        A.I_top[((int64_t)b * nup + y.itop) * nup_plane + (int64_t)me.c[1] * A.nx + me.c[0]] = v[k];
    }
  }
}

// Plane q of the last group's last lap: grid.x over the plane's cells, grid.y = band.
__global__ __launch_bounds__(256) void rts_gs_plane(GsArgs A, int g, int q, int contribute,
                                                    int update, int top) {
  gs_plane_cell(A, g, q, contribute != 0, update != 0, top != 0,
                blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y, false);
}

// Step t of every group (grid.z): the group's lap t / na and its plane; the
// last group runs its laps before the last here.  top: the iteration is the
// last (I_top of the groups' last laps).
__global__ __launch_bounds__(256) void rts_gs_step(GsArgs A, int t, int top) {
  const int g = blockIdx.z;
  const GsGroup& G = A.groups[g];
  const int n[3] = {A.nx, A.ny, A.nz};
  const int na = n[G.axis];
  const int laps = g == A.ngroups - 1 ? G.laps - 1 : G.laps;
  if (t >= laps * na) return;
  const int lap = t / na, tt = t - lap * na;
  const int q = G.sa > 0 ? tt : na - 1 - tt;
  const bool contribute = g != A.ngroups - 1 && lap == G.laps - 1;
  gs_plane_cell(A, g, q, contribute, false, top != 0 && contribute,
                blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y, G.axis == 0);
}

// grid.x over cells: Q over the bands in order, J and S out
__global__ __launch_bounds__(256) void rts_gs_finish(GsArgs A) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.N) return;
  const double* ws = reinterpret_cast<const double*>(A.ws);
  double q = 0.0;
  for (int b = 0; b < A.nbands; ++b) {
    const int64_t bo = (int64_t)b * A.N + p;
    double j = 0.0;
    for (int g = 0; g < A.ngroups; ++g) j += ws[A.p_off + ((int64_t)g * A.nbands + b) * A.N + p];
    const double s = ws[A.s_off + bo];
    q += 4.0 * 3.14159265358979323846 * A.qw[b] * ws[A.chi_off + bo] * (j - s);
    if (A.J) A.J[bo] = j;
    if (A.S) A.S[bo] = s;
  }
  A.Q[p] = q;
}

hipError_t launch_gs_init(const GsArgs& a, hipStream_t st) {
  rts_gs_init<<<dim3((unsigned)((a.N + 255) / 256), (unsigned)a.nbands), dim3(256), 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_gs_ghost(const GsArgs& a, int g, int plane_cells, hipStream_t st) {
  rts_gs_ghost<<<dim3((unsigned)((plane_cells + 255) / 256), (unsigned)a.nbands), dim3(256), 0, st>>>(
      a, g);
  return hipGetLastError();
}

hipError_t launch_gs_plane(const GsArgs& a, int g, int q, int contribute, int update, int top,
                           int plane_cells, hipStream_t st) {
  rts_gs_plane<<<dim3((unsigned)((plane_cells + 255) / 256), (unsigned)a.nbands), dim3(256), 0, st>>>(
      a, g, q, contribute, update, top);
  return hipGetLastError();
}

hipError_t launch_gs_step(const GsArgs& a, int t, int top, int plane_cells, hipStream_t st) {
  rts_gs_step<<<dim3((unsigned)((plane_cells + 255) / 256), (unsigned)a.nbands, (unsigned)a.ngroups),
                dim3(256), 0, st>>>(a, t, top);
  return hipGetLastError();
}

hipError_t launch_gs_finish(const GsArgs& a, hipStream_t st) {
  rts_gs_finish<<<dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rts
